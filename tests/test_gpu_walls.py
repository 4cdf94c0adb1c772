"""GPU parity of the reflecting-wall boundary (Sec. 5, "Imposing reflective
boundary conditions") against the FP64 oracle, through the C ABI: the ghost
refresh, both half-steps, stepping (graph replay included), the start-up and
the norms.  Tolerances as in test_gpu_parity.py."""

import sys

import numpy as np
import pytest

import oracle
from paper_1808_10481_amd import inputs

from tolerances import COMP_TOL, _close, tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1808_10481_amd import hl  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _wprob(d, m, K, dt, length, kappa=1.0):
    return oracle.Problem(d, m, tuple(K), tuple(length), dt, kappa, bc="walls")


CASES = ([(1, m, (37,)) for m in (0, 1, 3, 7)] + [(1, 2, (2,))]
         + [(2, m, (70, 9)) for m in (0, 2, 3, 5)] + [(2, 1, (2, 3))]
         + [(3, m, (67, 5, 3)) for m in (0, 1, 2, 3)] + [(3, 2, (2, 2, 2))])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("d,m,K", CASES)
def test_walls_half_steps_match_oracle(d, m, K, prec):
    _say(f"[walls] half-steps d={d} m={m} K={K} {prec}")
    rng = np.random.default_rng(2000 + 100 * d + 10 * m + len(K))
    L = (1.0, 0.7, 1.3)[:d]
    kappa = 1.3
    plan = hl.Plan(d, m, K, length=L, dt=0.0, cfl=0.6, c=np.sqrt(kappa), precision=prec, boundary="walls")
    prob = _wprob(d, m, K, plan.dt, L, kappa)
    ps, us = plan.host_shapes()
    assert ps == prob.p_shape() and us == prob.u_shape()
    P = inputs.zero_on_walls(inputs.random_data(rng, d, m, prob.p_nodes()), d)
    U = inputs.random_data(rng, d, m, prob.u_nodes(), ncomp=d)
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    P_in, U_in = plan.export(p, u)
    plan.p_half(p, u)
    Pg, Ug0 = plan.export(p, u)
    assert np.array_equal(Ug0, U_in)                 # the ghost refresh leaves the dual nodes alone
    _close(Pg, oracle.p_half(prob, P_in, U_in), *tol(prec, d, m))
    plan.u_half(u, p)
    _, Ug = plan.export(p, u)
    _close(Ug, oracle.u_half(prob, U_in, Pg), *tol(prec, d, m))
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_comp"])
@pytest.mark.parametrize("d,m,K,n", [(1, 3, (40,), 40), (2, 3, (33, 20), 20), (3, 2, (9, 8, 7), 17)])
def test_walls_multistep(d, m, K, n, prec):
    """n >= 16 steps go through the captured graph (ghost refresh included)."""
    _say(f"[walls] {n} steps d={d} m={m} K={K} {prec}")
    rng = np.random.default_rng(17 + d + m)
    L = (1.0,) * d
    plan = hl.Plan(d, m, K, length=L, cfl=0.9, precision=prec, boundary="walls")
    prob = _wprob(d, m, K, plan.dt, L)
    P = inputs.zero_on_walls(inputs.random_data(rng, d, m, prob.p_nodes()), d)
    U = inputs.random_data(rng, d, m, prob.u_nodes(), ncomp=d)
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    P_in, U_in = plan.export(p, u)
    plan.step(p, u, n)
    Pg, Ug = plan.export(p, u)
    Pr, Ur = oracle.step(prob, P_in, U_in, n)
    t = 1e-12 if prec == "fp64" else COMP_TOL
    _close(Pg, Pr, 2 * t * n, 10 * t * n)
    _close(Ug, Ur, 2 * t * n, 10 * t * n)


def test_walls_startup_and_norms():
    _say("[walls] start-up and norms")
    d, m, K = 2, 2, (12, 9)
    L = (1.2, 0.9)
    plan = hl.Plan(d, m, K, length=L, cfl=0.5, precision="fp64", boundary="walls")
    prob = _wprob(d, m, K, plan.dt, L)
    P0, _ = inputs.box_mode(d, m, K, L, (1, 2), 0.0, 0.0)
    p, u = plan.alloc()
    plan.init(p, u, P0, None, startup=True)
    Pg, Ug = plan.export(p, u)
    _close(Ug, oracle.startup(prob, P0, np.zeros(prob.u_shape())), 1e-12, 1e-11)
    plan.p_half(p, u)                                 # fills the ghost shell
    sp, su = plan.norms(p, u)                         # ghosts are not counted
    Pg, Ug = plan.export(p, u)
    assert abs(sp - np.sum(Pg * Pg)) <= 1e-12 * sp and abs(su - np.sum(Ug * Ug)) <= 1e-12 * su


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gaussian_pulse_walls_2d_full_size_sampled(prec):
    """The walled 2D m=3 1024^2 pulse after the start-up and 60 steps, then one
    more step checked on sampled nodes, walls and corners included."""
    _say(f"[walls] gaussian_pulse_walls_2d 1024^2 m=3 sampled {prec}")
    wl = inputs.gaussian_pulse_walls_2d(seed=3, K=1024, m=3)
    plan = hl.Plan(2, 3, wl.K, length=wl.length, dt=wl.dt, c=1.0, precision=prec, boundary="walls")
    p, u = plan.alloc()
    plan.init(p, u, wl.P0, None, startup=True)
    plan.step(p, u, 60)
    P_in, U_in = plan.export(p, u)
    prob = _wprob(2, 3, wl.K, plan.dt, wl.length)
    rng = np.random.default_rng(5)
    nodes = np.stack([rng.integers(0, 1025, 300), rng.integers(0, 1025, 300)], axis=1)
    nodes[:4] = [[0, 0], [1024, 1024], [0, 517], [1024, 3]]
    plan.p_half(p, u)
    Pg, _ = plan.export(p, u, want_u=False)
    ref = oracle.p_half(prob, P_in, U_in, nodes=nodes)
    _close(Pg[nodes[:, 0], nodes[:, 1]], ref, *tol(prec, 2, 3))
    qn = np.minimum(nodes, 1023)
    plan.u_half(u, p)
    _, Ug = plan.export(p, u)
    refu = oracle.u_half(prob, U_in, Pg, nodes=qn)
    _close(np.stack([Ug[i][qn[:, 0], qn[:, 1]] for i in range(2)]), refu, *tol(prec, 2, 3))
