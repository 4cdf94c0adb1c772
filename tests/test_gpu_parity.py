"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle,
element by element on the same seeded inputs.  Tolerances: tolerances.py.
"""

import sys

import numpy as np
import pytest

import oracle
from oracle.diagnostics import rel_l2
from paper_1808_10481_amd import inputs
from tolerances import COMP_TOL, _close, tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1808_10481_amd import hl  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _prob(d, m, K, dt, kappa=1.0):
    return oracle.Problem(d, m, tuple(K), tuple(1.0 for _ in K), dt, kappa)


CASES = (
    [(1, m, (37,)) for m in range(0, 8)] + [(1, 1, (200,)), (1, 3, (2,))]
    + [(2, m, (70, 9)) for m in range(0, 6)] + [(2, 2, (2, 3))]
    + [(3, m, (67, 5, 3)) for m in range(0, 4)] + [(3, 1, (2, 2, 2))]
)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("d,m,K", CASES)
def test_half_steps_match_oracle(d, m, K, prec):
    _say(f"[parity] half-steps d={d} m={m} K={K} {prec}")
    rng = np.random.default_rng(1000 + 100 * d + 10 * m + len(K))
    P = inputs.random_data(rng, d, m, K)
    U = inputs.random_data(rng, d, m, K, ncomp=d)
    kappa = 1.7
    plan = hl.Plan(d, m, K, dt=0.0, cfl=0.6, c=np.sqrt(kappa), precision=prec)
    prob = _prob(d, m, K, plan.dt, kappa)
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    P_in, U_in = plan.export(p, u)          # inputs as rounded to the plan precision
    plan.p_half(p, u)
    Pg, _ = plan.export(p, u)
    Pr = oracle.p_half(prob, P_in, U_in)
    _close(Pg, Pr, *tol(prec, d, m))
    plan.u_half(u, p)
    _, Ug = plan.export(p, u)
    Ur = oracle.u_half(prob, U_in, Pg)
    _close(Ug, Ur, *tol(prec, d, m))
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_comp"])
@pytest.mark.parametrize("d,m,K,n", [(1, 3, (50,), 40), (2, 3, (33, 20), 10), (3, 1, (12, 10, 9), 6),
                                     (3, 2, (10, 9, 8), 4)])
def test_multistep(d, m, K, n, prec):
    """n steps from the stored (rounded) initial data; FP32_COMP rounds the
    state once per half-step, 2n roundings of at most 2^-33 relative each."""
    _say(f"[parity] {n} steps d={d} m={m} K={K} {prec}")
    rng = np.random.default_rng(7 + d + m)
    P = inputs.random_data(rng, d, m, K)
    U = inputs.random_data(rng, d, m, K, ncomp=d)
    plan = hl.Plan(d, m, K, cfl=0.9, precision=prec)
    prob = _prob(d, m, K, plan.dt)
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    P_in, U_in = plan.export(p, u)
    plan.step(p, u, n)
    Pg, Ug = plan.export(p, u)
    Pr, Ur = oracle.step(prob, P_in, U_in, n)
    t = 1e-12 if prec == "fp64" else COMP_TOL
    _close(Pg, Pr, 2 * t * n, 10 * t * n)
    _close(Ug, Ur, 2 * t * n, 10 * t * n)


def test_comp_storage_round_trip():
    """FP32_COMP stores x as hi + lo within 2^-33 |x| (and exactly for values
    that fit in FP32 + BF16); exported values are exactly hi + lo."""
    d, m, K = 2, 2, (40, 7)
    rng = np.random.default_rng(21)
    P = inputs.random_data(rng, d, m, K)
    U = inputs.random_data(rng, d, m, K, ncomp=d)
    plan = hl.Plan(d, m, K, precision="fp32_comp")
    assert plan.info.word_bytes == 2 and plan.info.p_words == 3 * plan.info.nc * plan.info.nodes
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    Pg, Ug = plan.export(p, u)
    for got, ref in ((Pg, P), (Ug, U)):
        assert np.all(np.abs(got - ref) <= 2.0 ** -33 * np.abs(ref) + 1e-300)
        assert rel_l2(got, ref) > 0                        # not FP64 storage
    # values representable as FP32 + BF16 survive exactly
    P2 = (P.astype(np.float32).astype(np.float64))
    plan.init(p, u, P2, None)
    assert np.array_equal(plan.export(p, u)[0], P2)
    # norms see the stored values
    plan.init(p, u, P, U)
    sp, su = plan.norms(p, u)
    assert abs(sp - np.sum(Pg * Pg)) <= 1e-12 * sp and abs(su - np.sum(Ug * Ug)) <= 1e-12 * su


def test_standing_wave_1d_full_run():
    """The 1D standing-wave workload (m=1, 200 cells, nu = 0.5, to T = 1) run
    in full on both sides."""
    _say("[parity] standing_wave_1d 200 cells 400 steps")
    wl = inputs.standing_wave_1d(K=200, m=1, nu=0.5, T=1.0)
    plan = hl.Plan(1, 1, wl.K, dt=wl.dt, c=1.0, precision="fp64")
    p, u = plan.alloc()
    plan.init(p, u, wl.P0, wl.U0)
    plan.step(p, u, wl.steps)
    Pg, Ug = plan.export(p, u)
    prob = _prob(1, 1, wl.K, wl.dt)
    Pr, Ur = oracle.step(prob, wl.P0, wl.U0, wl.steps)
    _close(Pg, Pr, 1e-12, 1e-11)
    _close(Ug, Ur, 1e-12, 1e-11)
    # and the discretisation error is what the scheme gives (rate-2 regime)
    err = oracle.diagnostics.nodal_l2(prob, Pg[..., 0], wl.exact(wl.steps * wl.dt)[..., 0])
    assert err < 1e-3


def test_startup_matches_oracle():
    _say("[parity] start-up")
    d, m, K = 3, 1, (9, 8, 7)
    wl_c = (0.3, 0.6, 0.2)
    P0 = inputs.gaussian_pulse(d, m, K, (1.0,) * 3, wl_c, 0.2)
    plan = hl.Plan(d, m, K, cfl=0.5, precision="fp64")
    p, u = plan.alloc()
    plan.init(p, u, P0, None, startup=True)
    _, Ug = plan.export(p, u)
    prob = _prob(d, m, K, plan.dt)
    Ur = oracle.startup(prob, P0, np.zeros((d,) + P0.shape))
    _close(Ug, Ur, 1e-12, 1e-11)


def test_deterministic_and_zero_steps():
    d, m, K = 2, 3, (64, 16)
    rng = np.random.default_rng(9)
    P = inputs.random_data(rng, d, m, K)
    U = inputs.random_data(rng, d, m, K, ncomp=d)
    plan = hl.Plan(d, m, K, cfl=0.5, precision="fp64")
    outs = []
    for _ in range(2):
        p, u = plan.alloc()
        plan.init(p, u, P, U)
        plan.step(p, u, 0)
        P0g, U0g = plan.export(p, u)
        assert np.array_equal(P0g, P) and np.array_equal(U0g, U)
        plan.step(p, u, 5)
        outs.append(plan.export(p, u))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_norms_and_nonfinite_flag():
    d, m, K = 2, 1, (16, 16)
    rng = np.random.default_rng(11)
    P = inputs.random_data(rng, d, m, K)
    U = inputs.random_data(rng, d, m, K, ncomp=d)
    plan = hl.Plan(d, m, K, precision="fp64")
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    sp, su = plan.norms(p, u)
    assert abs(sp - np.sum(P * P)) <= 1e-12 * sp and abs(su - np.sum(U * U)) <= 1e-12 * su
    P[3, 4, 0, 1] = np.nan
    plan.init(p, u, P, U)
    with pytest.raises(hl.HLError) as ei:
        plan.norms(p, u)
    assert ei.value.status == hl.HL_ERR_NONFINITE


def _sampled_check(wl, prec, nsamp, tol):
    """One full step at full size; sampled nodes recomputed by the oracle."""
    rng = np.random.default_rng(123)
    plan = hl.Plan(wl.d, wl.m, wl.K, dt=wl.dt, c=1.0, precision=prec)
    p, u = plan.alloc()
    plan.init(p, u, wl.P0, wl.U0, startup=wl.startup)
    P_in, U_in = plan.export(p, u)
    prob = _prob(wl.d, wl.m, wl.K, plan.dt)
    nodes = np.stack([rng.integers(0, k, nsamp) for k in wl.K], axis=1)
    nodes[0] = 0
    nodes[1] = np.array(wl.K) - 1                       # wrap-around corners
    if wl.startup:
        U0 = np.zeros((wl.d,) + wl.P0.shape) if wl.U0 is None else wl.U0
        refs = oracle.u_half(prob, U0, P_in, nodes=nodes, weight_scale=0.5)
        gots = np.stack([U_in[i][tuple(nodes[:, k] for k in range(wl.d))] for i in range(wl.d)])
        _close(gots, refs, *tol)
    plan.p_half(p, u)
    Pg, _ = plan.export(p, u)
    ref = oracle.p_half(prob, P_in, U_in, nodes=nodes)
    got = Pg[tuple(nodes[:, k] for k in range(wl.d))]
    _close(got, ref, *tol)
    plan.u_half(u, p)
    _, Ug = plan.export(p, u)
    refu = oracle.u_half(prob, U_in, Pg, nodes=nodes)
    gotu = np.stack([Ug[i][tuple(nodes[:, k] for k in range(wl.d))] for i in range(wl.d)])
    _close(gotu, refu, *tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
def test_standing_mode_2d_full_size_sampled(prec):
    """2D m=3 1024^2 (the benchmark workload): sampled parity of one step."""
    _say(f"[parity] standing_mode_2d 1024^2 m=3 sampled {prec}")
    wl = inputs.standing_mode_2d(seed=1, K=1024, m=3)
    _sampled_check(wl, prec, 300, tol(prec, 2, 3))


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp32_comp"])
def test_gaussian_pulse_3d_full_size_sampled(prec):
    """3D m=2 256^3 Gaussian pulse with the start-up: sampled parity of the
    start-up and one step at full size."""
    _say(f"[parity] gaussian_pulse_3d 256^3 m=2 sampled {prec}")
    wl = inputs.gaussian_pulse_3d(seed=2, K=256, m=2)
    wl.U0 = None
    _sampled_check(wl, prec, 200, tol(prec, 3, 2))


@pytest.mark.parametrize("d,m,K,prec", [(1, 1, (200,), "fp64"), (2, 3, (64, 32), "fp32"), (3, 2, (16, 12, 8), "fp64"),
                                        (2, 2, (40, 24), "fp32_comp")])
def test_graph_replay_matches_eager(d, m, K, prec):
    """hl_step replays a captured graph for >= 16 steps: its results equal the
    eager half-step launches bit for bit, on every replay, with eager work and
    host synchronisation in between, and after the buffers change."""
    _say(f"[parity] graph replay d={d} m={m} K={K} {prec}")
    rng = np.random.default_rng(5)
    P = inputs.random_data(rng, d, m, K) * 0.1
    U = inputs.random_data(rng, d, m, K, ncomp=d) * 0.1
    plan = hl.Plan(d, m, K, cfl=0.7, precision=prec)
    pe, ue = plan.alloc()
    pg, ug = plan.alloc()
    plan.init(pe, ue, P, U)
    plan.init(pg, ug, P, U)
    for rep in range(3):
        for _ in range(37):
            plan.p_half(pe, ue)
            plan.u_half(ue, pe)
        plan.step(pg, ug, 37)               # 2 graph replays + 5 eager steps
        Pe, Ue = plan.export(pe, ue)
        Pg, Ug = plan.export(pg, ug)
        assert np.array_equal(Pe, Pg) and np.array_equal(Ue, Ug), rep
    # new buffers: the plan must re-capture for them
    p2, u2 = plan.alloc()
    plan.init(p2, u2, P, U)
    plan.step(p2, u2, 16)
    plan.init(pe, ue, P, U)
    for _ in range(16):
        plan.p_half(pe, ue)
        plan.u_half(ue, pe)
    assert np.array_equal(plan.export(p2, u2)[0], plan.export(pe, ue)[0])
