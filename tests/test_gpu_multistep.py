"""Multi-step GPU parity against the FP64 oracle on grids that span several
tiles and tile groups, in FP64, FP32 and FP32_COMP.

* 3D m = 2 from the start-up on a 65 x 9 x 3 grid: two x-tiles and two tile
  groups in y of the default 64 x 4 launch (groups of 2 tile rows), 17 steps
  (one replayed 16-step graph plus an eager step), with the default, an
  explicit (128 x 2, groups of 4) and the autotuned tile shape;
* FP32 over many steps of smooth data (2D m = 3 standing mode, 100 steps;
  3D m = 2 pulse, 50 steps) against the bound of tolerances.fp32_steps;
* the 3D pulse workload's recipe (m = 2, nu = 0.5, width 0.05, seeded
  centre, start-up) on a reduced 12^3 grid for 48 steps.

Every oracle trajectory is computed once per module and shared by the
precisions and tile shapes that compare with it.
"""

import functools
import sys

import numpy as np
import pytest

import oracle
from oracle.diagnostics import rel_l2
from paper_1808_10481_amd import inputs
from tolerances import _close, comp_steps, fp32_steps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1808_10481_amd import hl  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pulse(K, width=0.05, seed=2):
    centre = tuple(float(v) for v in np.random.default_rng(seed).random(3))
    return inputs.gaussian_pulse(3, 2, K, (1.0,) * 3, centre, width)


@functools.lru_cache(maxsize=None)
def _oracle_pulse(K, checkpoints):
    """Oracle trajectory of the pulse from the start-up (nu = 0.5): states
    after each step count in `checkpoints`."""
    d, m = 3, 2
    P = _pulse(K)
    prob = oracle.Problem(d, m, K, (1.0,) * d, 0.5 / max(K), 1.0)
    U = oracle.startup(prob, P, np.zeros((d,) + P.shape))
    out, done = {}, 0
    for n in checkpoints:
        P, U = oracle.step(prob, P, U, n - done)
        done = n
        out[n] = (P, U)
    return out


def _run(plan, P0, nsteps, startup=True, U0=None, tile=None):
    p, u = plan.alloc()
    if tile == "tuned":
        plan.init(p, u, P0, U0, startup=startup)
        picked = plan.tune(p, u, reps=1)
        _say(f"[multistep] tuned tile {picked}")
    elif tile is not None:
        plan.set_tile(*tile)
    plan.init(p, u, P0, U0, startup=startup)
    plan.step(p, u, nsteps)
    return plan.export(p, u)


@pytest.mark.parametrize("tile", [None, (128, 2, 4), "tuned"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_3d_multitile_steps_from_startup(prec, tile):
    K, n = (65, 9, 3), 17
    _say(f"[multistep] 3D m=2 K={K} {n} steps {prec} tile={tile}")
    ref = _oracle_pulse(K, (n, 50))[n]
    plan = hl.Plan(3, 2, K, dt=0.5 / max(K), c=1.0, precision=prec)
    Pg, Ug = _run(plan, _pulse(K), n, tile=tile)
    plan.close()
    if prec == "fp64":
        _close(Pg, ref[0], 2e-12 * n, 1e-11 * n)
        _close(Ug, ref[1], 2e-12 * n, 1e-11 * n)
    else:
        t = fp32_steps(3, 2, 2 * n + 1)
        _close(Pg, ref[0], *t)
        _close(Ug, ref[1], *t)


def test_3d_fp32_fifty_steps():
    K, n = (65, 9, 3), 50
    _say(f"[multistep] 3D m=2 K={K} {n} steps fp32")
    ref = _oracle_pulse(K, (17, n))[n]
    plan = hl.Plan(3, 2, K, dt=0.5 / max(K), c=1.0, precision="fp32")
    Pg, Ug = _run(plan, _pulse(K), n)
    plan.close()
    t = fp32_steps(3, 2, 2 * n + 1)
    rp = _close(Pg, ref[0], *t)
    ru = _close(Ug, ref[1], *t)
    _say(f"[multistep] 3D fp32 {n} steps: rel L2 p {rp:.2e} u {ru:.2e}, bound {t[0]:.2e}")


@pytest.mark.parametrize("prec", ["fp32", "fp32_comp"])
def test_2d_m3_hundred_steps(prec):
    """The 2D standing mode (waves (3, 2), exact U at dt/2) for 100 steps on a
    grid of two x-tiles and three tile rows."""
    d, m, K, n = 2, 3, (70, 12), 100
    _say(f"[multistep] 2D m=3 K={K} {n} steps {prec}")
    plan = hl.Plan(d, m, K, cfl=0.5, c=1.0, precision=prec)
    P0, U0 = inputs.standing_mode(d, m, K, (1.0, 1.0), (3, 2), 0.0, plan.dt / 2)
    Pg, Ug = _run(plan, P0, n, startup=False, U0=U0)
    prob = oracle.Problem(d, m, K, (1.0, 1.0), plan.dt, 1.0)
    plan.close()
    Pr, Ur = oracle.step(prob, P0, U0, n)
    t = fp32_steps(d, m, 2 * n) if prec == "fp32" else comp_steps(d, m, 2 * n)
    rp = _close(Pg, Pr, *t)
    ru = _close(Ug, Ur, *t)
    _say(f"[multistep] 2D {prec} {n} steps: rel L2 p {rp:.2e} u {ru:.2e}, bound {t[0]:.2e}")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
def test_pulse_workload_recipe_on_reduced_grid(prec):
    """The 3D workload's recipe (m = 2, nu = 0.5, pulse width 0.05 at the
    seeded centre, start-up from u = 0) on 12^3 cells for 48 steps (3
    replayed graphs)."""
    K, n = (12, 12, 12), 48
    _say(f"[multistep] 3D pulse recipe K={K} {n} steps {prec}")
    ref = _oracle_pulse(K, (n,))[n]
    plan = hl.Plan(3, 2, K, cfl=0.5, c=1.0, precision=prec)
    assert abs(plan.dt - 0.5 / 12) < 1e-15
    Pg, Ug = _run(plan, _pulse(K), n)
    plan.close()
    if prec == "fp64":
        t = (2e-12 * n, 1e-11 * n)
    elif prec == "fp32":
        t = fp32_steps(3, 2, 2 * n + 1)
    else:
        t = comp_steps(3, 2, 2 * n + 1)
    rp = _close(Pg, ref[0], *t)
    ru = _close(Ug, ref[1], *t)
    _say(f"[multistep] pulse recipe {prec}: rel L2 p {rp:.2e} u {ru:.2e}")
    assert rel_l2(Pg, _pulse(K)) > 0.1                     # the pulse has moved
