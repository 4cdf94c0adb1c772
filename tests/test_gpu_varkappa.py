"""GPU parity of the variable-coefficient half-steps (hl_set_kappa; Sec. 4,
"Smoothly varying wave speed") against the oracle, through the C ABI."""

import sys

import numpy as np
import pytest

import oracle
from paper_1808_10481_amd import inputs
from tolerances import _close, tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1808_10481_amd import hl  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def vtol(prec, d, m):
    """FP32: the recurrence multiplies by kappa up to kmax times on top of the
    constant-coefficient contraction, so the bound is 4x the constant one.
    FP32_COMP: FP64 arithmetic on hi + lo data and hi + lo kappa data (each
    within 2^-33 of its value), so 4x the constant bound as well."""
    t2, tm = tol(prec, d, m)
    return (t2, tm) if prec == "fp64" else (4 * t2, 4 * tm)


def _kappa(d, m, K, rng, smooth):
    if smooth:
        amps = tuple(rng.uniform(0.1, 0.3, d))
        waves = tuple(int(w) for w in rng.integers(1, 4, d))
        return (inputs.kappa_sines(d, m, K, (1.0,) * d, amps, waves, "primal"),
                inputs.kappa_sines(d, m, K, (1.0,) * d, amps, waves, "dual"))
    shape = tuple(K) + (2 * m + 2,) * d
    kp, ku = rng.uniform(-0.2, 0.2, shape), rng.uniform(-0.2, 0.2, shape)
    kp[(Ellipsis,) + (0,) * d] += 1.5
    ku[(Ellipsis,) + (0,) * d] += 1.5
    return kp, ku


CASES = ([(1, m, (37,)) for m in (0, 1, 3, 5, 7)] + [(1, 2, (2,))] + [(2, m, (41, 9)) for m in (0, 1, 2, 3, 4)]
         + [(2, 5, (20, 7)), (2, 1, (2, 3)), (3, 0, (9, 7, 5)), (3, 1, (70, 6, 5)), (3, 1, (2, 3, 2)),
            (3, 2, (5, 4, 3)), (3, 2, (2, 2, 2)), (3, 3, (3, 3, 2))])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("d,m,K", CASES)
def test_varkappa_half_steps_match_oracle(d, m, K, prec):
    _say(f"[varkappa] half-steps d={d} m={m} K={K} {prec}")
    rng = np.random.default_rng(900 + 10 * d + m)
    plan = hl.Plan(d, m, K, cfl=0.5, c=np.sqrt(2.0), precision=prec)
    prob = oracle.Problem(d, m, tuple(K), (1.0,) * d, plan.dt, 1.0)
    kp, ku = _kappa(d, m, K, rng, smooth=(m % 2 == 0))
    plan.set_kappa(kp, ku)
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    P_in, U_in = plan.export(p, u)
    plan.p_half(p, u)
    Pg, _ = plan.export(p, u)
    _close(Pg, oracle.p_half_var(prob, P_in, U_in, kp), *vtol(prec, d, m))
    plan.u_half(u, p)
    _, Ug = plan.export(p, u)
    _close(Ug, oracle.u_half_var(prob, U_in, Pg, ku), *vtol(prec, d, m))


@pytest.mark.parametrize("d,m,K,n", [(1, 3, (40,), 20), (2, 2, (24, 18), 17), (3, 2, (6, 5, 4), 17)])
def test_varkappa_multistep_and_startup(d, m, K, n):
    """Start-up with half weights, then n >= 16 steps (graph replay) in FP64."""
    _say(f"[varkappa] start-up + {n} steps d={d} m={m}")
    rng = np.random.default_rng(31 + d)
    plan = hl.Plan(d, m, K, cfl=0.6, c=np.sqrt(1.5), precision="fp64")
    prob = oracle.Problem(d, m, tuple(K), (1.0,) * d, plan.dt, 1.0)
    kp, ku = _kappa(d, m, K, rng, smooth=True)
    plan.set_kappa(kp, ku)
    P0 = inputs.random_data(rng, d, m, K)
    p, u = plan.alloc()
    plan.init(p, u, P0, None, startup=True)
    _, Ug = plan.export(p, u)
    U = oracle.u_half_var(prob, np.zeros((d,) + P0.shape), P0, ku, weight_scale=0.5)
    _close(Ug, U, 1e-12, 1e-11)
    plan.step(p, u, n)
    Pg, Ug = plan.export(p, u)
    Pr, Ur = oracle.step_var(prob, P0, U, kp, ku, n)
    _close(Pg, Pr, 2e-12 * n, 1e-11 * n)
    _close(Ug, Ur, 2e-12 * n, 1e-11 * n)


def test_set_kappa_none_restores_constant_and_adjoint_refuses():
    d, m, K = 2, 1, (16, 12)
    rng = np.random.default_rng(2)
    plan = hl.Plan(d, m, K, cfl=0.5, precision="fp64")
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    plan.step(p, u, 3)
    ref = plan.export(p, u)
    kp, ku = _kappa(d, m, K, rng, smooth=True)
    plan.set_kappa(kp, ku)
    with pytest.raises(hl.HLError) as ei:
        plan.adjoint_step(p, u, 1)
    assert ei.value.status == hl.HL_ERR_UNSUPPORTED
    plan.set_kappa(None, None)
    plan.init(p, u, P, U)
    plan.step(p, u, 3)
    got = plan.export(p, u)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


WALL_CASES = [(1, 3, (37,)), (1, 0, (5,)), (1, 7, (20,)), (2, 1, (70, 9)), (2, 3, (41, 10)), (2, 2, (3, 2)),
              (2, 4, (20, 9)), (2, 5, (12, 7)), (3, 1, (9, 6, 5)), (3, 2, (4, 3, 3)), (3, 3, (2, 2, 2))]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("d,m,K", WALL_CASES)
def test_varkappa_walls_half_steps_match_oracle(d, m, K, prec):
    """Reflecting walls with variable kappa (kappa even about every wall):
    the ghost refresh, then the variable-kappa half-steps on the walled grids."""
    _say(f"[varkappa] walls half-steps d={d} m={m} K={K} {prec}")
    rng = np.random.default_rng(950 + 10 * d + m)
    plan = hl.Plan(d, m, K, cfl=0.5, c=np.sqrt(1.6), precision=prec, boundary="walls")
    prob = oracle.Problem(d, m, tuple(K), (1.0,) * d, plan.dt, 1.0, bc="walls")
    amps = tuple(rng.uniform(0.1, 0.3, d))
    kp = inputs.kappa_box(d, m, K, (1.0,) * d, amps, "primal")
    ku = inputs.kappa_box(d, m, K, (1.0,) * d, amps, "dual")
    plan.set_kappa(kp, ku)
    P = inputs.zero_on_walls(inputs.random_data(rng, d, m, prob.p_nodes()), d)
    U = inputs.random_data(rng, d, m, prob.u_nodes(), ncomp=d)
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    P_in, U_in = plan.export(p, u)
    plan.p_half(p, u)
    Pg, _ = plan.export(p, u)
    _close(Pg, oracle.p_half_var(prob, P_in, U_in, kp), *vtol(prec, d, m))
    plan.u_half(u, p)
    _, Ug = plan.export(p, u)
    _close(Ug, oracle.u_half_var(prob, U_in, Pg, ku), *vtol(prec, d, m))


def test_varkappa_walls_multistep_fp64():
    """20 steps (graph replay) of the walled variable-kappa step against the
    oracle; p stays zero on the walls (even coefficients at wall nodes)."""
    _say("[varkappa] walls 20 steps 2D m=2 (24, 18) fp64")
    d, m, K = 2, 2, (24, 18)
    rng = np.random.default_rng(977)
    plan = hl.Plan(d, m, K, cfl=0.5, c=np.sqrt(1.6), precision="fp64", boundary="walls")
    prob = oracle.Problem(d, m, K, (1.0, 1.0), plan.dt, 1.0, bc="walls")
    kp = inputs.kappa_box(d, m, K, (1.0, 1.0), (0.3, 0.2), "primal")
    ku = inputs.kappa_box(d, m, K, (1.0, 1.0), (0.3, 0.2), "dual")
    plan.set_kappa(kp, ku)
    P = inputs.zero_on_walls(inputs.random_data(rng, d, m, prob.p_nodes()), d)
    U = inputs.random_data(rng, d, m, prob.u_nodes(), ncomp=d)
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    P_in, U_in = plan.export(p, u)
    plan.step(p, u, 20)
    Pg, Ug = plan.export(p, u)
    Po, Uo = oracle.step_var(prob, P_in, U_in, kp, ku, 20)
    _close(Pg, Po, *vtol("fp64", d, m))
    _close(Ug, Uo, *vtol("fp64", d, m))
    for k in range(d):
        for j in (0, Pg.shape[k] - 1):
            idx = [slice(None)] * (2 * d)
            idx[k] = j
            idx[d + k] = slice(0, None, 2)
            assert np.abs(Pg[tuple(idx)]).max() <= 1e-11 * np.abs(Pg).max()


def test_varkappa_2d_m3_1024_sampled_fp32():
    """The batched-shot grid shape at its largest (2D m=3 1024^2, FP32, smooth
    kappa in [~0.4, ~1.6]): one step checked on sampled nodes."""
    _say("[varkappa] 2D m=3 1024^2 fp32 sampled")
    d, m, K = 2, 3, (1024, 1024)
    rng = np.random.default_rng(12)
    plan = hl.Plan(d, m, K, cfl=0.5, c=np.sqrt(1.6), precision="fp32")
    prob = oracle.Problem(d, m, K, (1.0, 1.0), plan.dt, 1.0)
    kp = inputs.kappa_sines(d, m, K, (1.0, 1.0), (0.35, 0.25), (2, 3), "primal")
    ku = inputs.kappa_sines(d, m, K, (1.0, 1.0), (0.35, 0.25), (2, 3), "dual")
    plan.set_kappa(kp, ku)
    P0, U0 = inputs.standing_mode(d, m, K, (1.0, 1.0), (3, 2), 0.0, plan.dt / 2)
    p, u = plan.alloc()
    plan.init(p, u, P0, U0)
    P_in, U_in = plan.export(p, u)
    nodes = np.stack([rng.integers(0, 1024, 200), rng.integers(0, 1024, 200)], axis=1)
    nodes[0], nodes[1] = (0, 0), (1023, 1023)
    plan.p_half(p, u)
    Pg, _ = plan.export(p, u, want_u=False)
    _close(Pg[nodes[:, 0], nodes[:, 1]], oracle.p_half_var(prob, P_in, U_in, kp, nodes=nodes), *vtol("fp32", d, m))
    plan.u_half(u, p)
    _, Ug = plan.export(p, u)
    ref = oracle.u_half_var(prob, U_in, Pg, ku, nodes=nodes)
    _close(np.stack([Ug[i][nodes[:, 0], nodes[:, 1]] for i in range(d)]), ref, *vtol("fp32", d, m))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_varkappa_3d_m2_sampled(prec):
    """3D m=2 (one wavefront per node) on a grid of many workgroups per XCD
    run (80 x 36 x 30, smooth kappa): one step checked on sampled nodes,
    corners and faces included."""
    _say(f"[varkappa] 3D m=2 (80, 36, 30) {prec} sampled")
    d, m, K = 3, 2, (80, 36, 30)
    rng = np.random.default_rng(13)
    plan = hl.Plan(d, m, K, cfl=0.5, c=np.sqrt(1.6), precision=prec)
    prob = oracle.Problem(d, m, K, (1.0,) * 3, plan.dt, 1.0)
    kp = inputs.kappa_sines(d, m, K, (1.0,) * 3, (0.35, 0.25, 0.2), (2, 3, 1), "primal")
    ku = inputs.kappa_sines(d, m, K, (1.0,) * 3, (0.35, 0.25, 0.2), (2, 3, 1), "dual")
    plan.set_kappa(kp, ku)
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    P_in, U_in = plan.export(p, u)
    nodes = np.stack([rng.integers(0, k, 150) for k in K], axis=1)
    nodes[0], nodes[1], nodes[2] = (0, 0, 0), (79, 35, 29), (79, 0, 29)
    idx = tuple(nodes[:, k] for k in range(d))
    plan.p_half(p, u)
    Pg, _ = plan.export(p, u)
    _close(Pg[idx], oracle.p_half_var(prob, P_in, U_in, kp, nodes=nodes), *vtol(prec, d, m))
    plan.u_half(u, p)
    _, Ug = plan.export(p, u)
    ref = oracle.u_half_var(prob, U_in, Pg, ku, nodes=nodes)
    _close(np.stack([Ug[i][idx] for i in range(d)]), ref, *vtol(prec, d, m))
