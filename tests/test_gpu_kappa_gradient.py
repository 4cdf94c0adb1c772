"""GPU parity of the variable-kappa adjoint (hl_adjoint_step_var) and of the
gradient with respect to the kappa data (hl_kappa_grad) against the oracle,
through the C ABI; the checkpointed receiver-trace gradient (autograd) against
the oracle, and against fourth-order central differences of the GPU forward
along random kappa directions (also at the 512^2, m = 2 size)."""

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

from paper_1808_10481_amd import autograd as hag  # noqa: E402
from paper_1808_10481_amd import hl  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def gtol(prec, d, m):
    """FP64: the adjoint sums kmax + 1 recurrence terms of (2m+2)^d products
    per node (cancellation in the gradient): 1e-11 relative L2.  FP32: the
    forward half-step bound times 16 (the gradient pairs two FP32 series and
    the recomputed forward terms, each within 4x the constant-coefficient
    bound).  FP32_COMP: FP64 arithmetic, the outputs and the scratch of
    d/d(interpolant) rounded to hi + lo: 16x its half-step bound."""
    if prec == "fp64":
        return (1e-11, 1e-10)
    t2, tm = tol(prec, d, m)
    return (16 * t2, 16 * tm)


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


def _setup(d, m, K, prec, seed, smooth, c=np.sqrt(2.0), cfl=0.5):
    rng = np.random.default_rng(seed)
    plan = hl.Plan(d, m, K, cfl=cfl, c=c, precision=prec)
    prob = oracle.Problem(d, m, tuple(K), (1.0,) * d, plan.dt, 1.0)
    kp, ku = _kappa(d, m, K, rng, smooth)
    plan.set_kappa(kp, ku)
    return rng, plan, prob, kp, ku


CASES = ([(1, m, (37,)) for m in (0, 1, 3, 7)] + [(2, m, (70, 9)) for m in (0, 1, 2)] + [(2, 1, (2, 3))]
         + [(2, 3, (66, 5)), (3, 0, (5, 4, 3)), (3, 1, (70, 3, 3)), (3, 1, (2, 2, 2))])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("d,m,K", CASES)
def test_adjoint_step_var_matches_oracle(d, m, K, prec):
    _say(f"[kgrad] one step d={d} m={m} K={K} {prec}")
    rng, plan, prob, kp, ku = _setup(d, m, K, prec, 1200 + 10 * d + m, smooth=(m % 2 == 1))
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Pb, Ub = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    P_in, U_in = plan.export(p, u)
    p_next, u_prev = p.clone(), u.clone()
    plan.p_half(p_next, u_prev)                       # P' = P_{t+1}
    pb, ub = plan.alloc()
    plan.init(pb, ub, Pb, Ub)
    Pb_in, Ub_in = plan.export(pb, ub)
    plan.kappa_grad(reset=True)
    plan.adjoint_step_var(pb, ub, p_next, u_prev)
    gp, gu = plan.kappa_grad(reset=True)
    Pa, Ua = plan.export(pb, ub)
    ogp, ogu, oPb, oUb = oracle.kappa_field_gradient(prob, P_in, U_in, kp, ku, Pb_in, Ub_in, 1)
    t = gtol(prec, d, m)
    _close(Pa, oPb, *t)
    _close(Ua, oUb, *t)
    _close(gp, ogp, *t)
    _close(gu, ogu, *t)
    # the accumulators were reset: a second read is zero
    zp, zu = plan.kappa_grad()
    assert not np.any(zp) and not np.any(zu)


def _receivers(rng, K, n):
    return [tuple(int(rng.integers(0, k)) for k in K) for _ in range(n)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("d,m,K,nsteps,seg", [(1, 3, (40,), 7, 3), (2, 2, (24, 18), 9, None), (2, 1, (66, 10), 5, 2),
                                                (2, 3, (12, 10), 4, 2), (3, 1, (5, 4, 3), 4, 2)])
def test_checkpointed_receiver_gradient_matches_oracle(d, m, K, nsteps, seg, prec):
    _say(f"[kgrad] receivers d={d} m={m} K={K} n={nsteps} seg={seg} {prec}")
    rng, plan, prob, kp, ku = _setup(d, m, K, prec, 1300 + 10 * d + m, smooth=True)
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Pd, Ud = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    rec = _receivers(rng, K, 3)
    data = rng.normal(size=(nsteps, len(rec)))
    p, u = plan.alloc()
    plan.init(p, u, P, U)
    P_in, U_in = plan.export(p, u)
    pd, ud = plan.alloc()
    plan.init(pd, ud, Pd, Ud)
    Pd_in, Ud_in = plan.export(pd, ud)
    kpt = torch.tensor(kp, dtype=torch.float64, requires_grad=True)
    kut = torch.tensor(ku, dtype=torch.float64, requires_grad=True)
    p.requires_grad_(True)
    u.requires_grad_(True)
    tr, p_n, u_n = hag.receiver_traces(kpt, kut, p, u, plan, nsteps, rec, seg=seg)
    dt_ = torch.tensor(data, dtype=tr.dtype, device=tr.device)
    loss = 0.5 * ((tr - dt_) ** 2).sum() + (p_n * pd).sum() + (u_n * ud).sum()
    loss.backward()
    Pg, Ug = plan.export(p.grad, u.grad)
    # oracle: the same loss through its own trajectory
    z = (0,) * d
    Ps, Us = np.array(P_in), np.array(U_in)
    src = []
    for t in range(nsteps):
        Ps, Us = oracle.step_var(prob, Ps, Us, kp, ku, 1)
        s = np.zeros_like(Ps)
        for r_i, r in enumerate(rec):
            s[tuple(r) + z] += Ps[tuple(r) + z] - data[t, r_i]
        src.append(s)
    ogp, ogu, oPb, oUb = oracle.kappa_field_gradient(prob, P_in, U_in, kp, ku, Pd_in, Ud_in, nsteps, p_sources=src)
    t = gtol(prec, d, m)
    t = (4 * t[0], 4 * t[1]) if prec == "fp32" else t   # nsteps of accumulated rounding
    _close(kpt.grad.numpy(), ogp, *t)
    _close(kut.grad.numpy(), ogu, *t)
    _close(Pg, oPb, *t)
    _close(Ug, oUb, *t)


def _fd_check(plan, kp, ku, p0, u0, nsteps, rec, data, ndir, rng, eps, rtol):
    """Directional derivatives of the receiver misfit along ndir random kappa
    directions (smooth: each direction is a random field's scaled Taylor data,
    here random coefficients decaying with degree) against fourth-order central
    differences of the GPU forward."""
    kpt = torch.tensor(kp, dtype=torch.float64, requires_grad=True)
    kut = torch.tensor(ku, dtype=torch.float64, requires_grad=True)
    dtd = torch.tensor(data, dtype=torch.float64, device="cuda")

    def misfit(a, b, grad):
        with torch.set_grad_enabled(grad):
            tr, _, _ = hag.receiver_traces(a, b, p0, u0, plan, nsteps, rec)
            return 0.5 * ((tr.double() - dtd) ** 2).sum()

    loss = misfit(kpt, kut, True)
    loss.backward()
    gp, gu = kpt.grad.numpy(), kut.grad.numpy()
    d, m = plan.d, plan.m
    decay = np.ones((2 * m + 2,) * d)
    for idx in np.ndindex(*decay.shape):
        decay[idx] = 0.5 ** sum(idx)
    worst = 0.0
    for _ in range(ndir):
        dp = rng.normal(size=kp.shape) * decay
        du = rng.normal(size=ku.shape) * decay

        def L(s):
            return float(misfit(torch.tensor(kp + s * dp), torch.tensor(ku + s * du), False))

        fd = (-L(2 * eps) + 8 * L(eps) - 8 * L(-eps) + L(-2 * eps)) / (12 * eps)
        an = float(np.sum(gp * dp) + np.sum(gu * du))
        err = abs(fd - an) / max(abs(fd), 1e-300)
        worst = max(worst, err)
        assert err <= rtol, (fd, an)
    return worst


def test_gradient_matches_central_differences_on_8_directions():
    _say("[kgrad] FD, 8 directions, 2D m=2 (32, 24) FP64")
    d, m, K = 2, 2, (32, 24)
    rng, plan, prob, kp, ku = _setup(d, m, K, "fp64", 1400, smooth=True)
    p0, u0 = plan.alloc()
    centre = tuple(rng.uniform(0.3, 0.7, d))
    plan.init(p0, u0, inputs.gaussian_pulse(d, m, K, (1.0,) * d, centre, 0.1), np.zeros(plan.host_shapes()[1]))
    nsteps = 12
    rec = _receivers(rng, K, 4)
    data = rng.normal(size=(nsteps, len(rec))) * 0.01
    _fd_check(plan, kp, ku, p0, u0, nsteps, rec, data, 8, rng, 1e-3, 1e-7)


def test_gradient_m3_central_differences_on_4_directions():
    """2D m = 3 (the batched workload's order), FP64: the kappa-data gradient
    against central differences of the GPU forward on 4 directions."""
    _say("[kgrad] FD, 4 directions, 2D m=3 (20, 16) FP64")
    d, m, K = 2, 3, (20, 16)
    rng, plan, prob, kp, ku = _setup(d, m, K, "fp64", 1450, smooth=True)
    p0, u0 = plan.alloc()
    centre = tuple(rng.uniform(0.3, 0.7, d))
    plan.init(p0, u0, inputs.gaussian_pulse(d, m, K, (1.0,) * d, centre, 0.1), np.zeros(plan.host_shapes()[1]))
    nsteps = 8
    rec = _receivers(rng, K, 4)
    data = rng.normal(size=(nsteps, len(rec))) * 0.01
    _fd_check(plan, kp, ku, p0, u0, nsteps, rec, data, 4, rng, 1e-3, 1e-7)


def test_gradient_full_size_512_m2_central_differences():
    """The adjoint workload's grid (512^2, m = 2) in FP64: two random
    directions against central differences (a property at any size)."""
    _say("[kgrad] FD, 2 directions, 2D m=2 512^2 FP64")
    d, m, K = 2, 2, (512, 512)
    rng, plan, prob, kp, ku = _setup(d, m, K, "fp64", 1500, smooth=True)
    p0, u0 = plan.alloc()
    plan.init(p0, u0, inputs.random_data(rng, d, m, K) * 0.1, np.zeros(plan.host_shapes()[1]))
    nsteps = 6
    rec = [(int(x), 256) for x in np.linspace(16, 496, 16)]   # 16 receivers on a line
    data = np.zeros((nsteps, len(rec)))
    _fd_check(plan, kp, ku, p0, u0, nsteps, rec, data, 2, rng, 1e-3, 1e-6)


WALL_VAR_CASES = [(1, 3, (10,)), (2, 1, (6, 5)), (2, 2, (4, 3)), (2, 3, (3, 3)), (3, 1, (3, 2, 2))]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("d,m,K", WALL_VAR_CASES)
def test_walls_adjoint_step_var_matches_oracle(d, m, K, prec):
    """Reflecting walls: the transposed variable-kappa step (B^T from the K
    dual nodes, G^T A^T with the ghost fold, A_kappa on the ghost-refreshed
    U_t) against the oracle's transpose read off unit responses of its walled
    step, and sampled kappa-gradient entries against central differences of
    that step."""
    _say(f"[kgrad] walls one step d={d} m={m} K={K} {prec}")
    rng = np.random.default_rng(1500 + 10 * d + m)
    plan = hl.Plan(d, m, K, cfl=0.5, c=np.sqrt(2.0), precision=prec, boundary="walls")
    prob = oracle.Problem(d, m, tuple(K), (1.0,) * d, plan.dt, 1.0, "walls")
    N2 = 2 * m + 2
    kap = []
    for nodes in (prob.p_nodes(), prob.u_nodes()):
        kd = rng.uniform(-0.2, 0.2, nodes + (N2,) * d)
        kd[(Ellipsis,) + (0,) * d] += 1.5
        kap.append(kd)
    kp, ku = kap
    plan.set_kappa(kp, ku)
    ps, us = plan.host_shapes()
    p, u = plan.alloc()
    plan.init(p, u, inputs.zero_on_walls(rng.uniform(-1, 1, ps), d), rng.uniform(-1, 1, us))
    P_in, U_in = plan.export(p, u)
    p_next, u_prev = p.clone(), u.clone()
    plan.p_half(p_next, u_prev)                       # P' = P_{t+1} (ghost refresh first)
    pb, ub = plan.alloc()
    plan.init(pb, ub, rng.uniform(-1, 1, ps), rng.uniform(-1, 1, us))
    Pb_in, Ub_in = plan.export(pb, ub)
    plan.kappa_grad(reset=True)
    plan.adjoint_step_var(pb, ub, p_next, u_prev)
    gp, gu = plan.kappa_grad(reset=True)
    Pa, Ua = plan.export(pb, ub)
    oPb, oUb = oracle.adjoint_step_var_bruteforce(prob, Pb_in, Ub_in, kp, ku, 1)
    t = gtol(prec, d, m)
    _close(Pa, oPb, *t)
    _close(Ua, oUb, *t)
    ent = [(0, int(i)) for i in rng.choice(kp.size, 8, replace=False)] + \
          [(1, int(i)) for i in rng.choice(ku.size, 8, replace=False)]
    # kappa_0 of the nodes next to a wall and of an interior node
    ent += [(0, 0), (1, 0), (0, kp.size - N2 ** d), (1, ku.size - N2 ** d)]
    fd = oracle.kappa_field_gradient_fd(prob, P_in, U_in, kp, ku, Pb_in, Ub_in, 1, ent)
    got = np.array([(gp if f == 0 else gu).reshape(-1)[i] for f, i in ent])
    scale = np.max(np.abs(fd))
    rt = 1e-8 if prec == "fp64" else max(1e-8, 16 * t[1])
    assert np.max(np.abs(got - fd)) <= rt * scale, (got, fd)


def test_walls_receiver_gradient_matches_central_differences():
    """Reflecting walls, 2D m = 2 FP64: the checkpointed receiver-trace
    gradient (walled transposed steps) against central differences of the
    GPU's walled forward on 4 random kappa directions."""
    _say("[kgrad] FD, 4 directions, walls 2D m=2 (16, 12) FP64")
    d, m, K = 2, 2, (16, 12)
    rng = np.random.default_rng(1600)
    plan = hl.Plan(d, m, K, cfl=0.5, c=np.sqrt(2.0), precision="fp64", boundary="walls")
    amps = tuple(rng.uniform(0.1, 0.3, d))
    kp = inputs.kappa_box(d, m, K, (1.0,) * d, amps, "primal")
    ku = inputs.kappa_box(d, m, K, (1.0,) * d, amps, "dual")
    p0, u0 = plan.alloc()
    ps, us = plan.host_shapes()
    plan.init(p0, u0, inputs.zero_on_walls(rng.uniform(-1, 1, ps) * 0.1, d), np.zeros(us))
    nsteps = 10
    rec = [tuple(int(rng.integers(1, k)) for k in K) for _ in range(4)]
    data = rng.normal(size=(nsteps, len(rec))) * 0.01
    _fd_check(plan, kp, ku, p0, u0, nsteps, rec, data, 4, rng, 1e-3, 1e-7)


def test_adjoint_step_var_3d_m2_unsupported():
    """3D m = 2 has the variable-kappa forward (one wavefront per node) but no
    transposed step: the adjoint and the kappa gradient refuse it."""
    rng, plan, prob, kp, ku = _setup(3, 2, (4, 4, 4), "fp32", 7, smooth=False)
    p, u = plan.alloc()
    pb, ub = plan.alloc()
    with pytest.raises(hl.HLError) as ei:
        plan.adjoint_step_var(pb, ub, p, u)
    assert ei.value.status == hl.HL_ERR_UNSUPPORTED
    with pytest.raises(hl.HLError) as ei:
        plan.kappa_grad()
    assert ei.value.status == hl.HL_ERR_UNSUPPORTED
