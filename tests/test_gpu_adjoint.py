"""GPU parity of the discrete adjoint (hl_adjoint_step) against the oracle's
transpose, periodic and with reflecting walls, the kappa gradient, the
dot-product identity at a larger size and the autograd wrapper.  FP32_COMP
storage runs the same transposed half-steps in FP64 arithmetic on its hi + lo
data."""

import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_1808_10481_amd import inputs
from tolerances import _close, comp_steps, tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1808_10481_amd import hl  # noqa: E402
from paper_1808_10481_amd.autograd import hermite_steps  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def atol(prec, d, m, n):
    """n transposed steps: FP64/FP32 n times the one-step bound; FP32_COMP
    rounds each transposed half-step's output to hi + lo exactly as the
    forward step does, so its bound is the forward one over 2n half-steps."""
    if prec == "fp32_comp":
        return comp_steps(d, m, 2 * n)
    t2, tm = tol(prec, d, m)
    return n * t2, n * tm


def _prob(d, m, K, dt, kappa):
    return oracle.Problem(d, m, tuple(K), tuple(1.0 for _ in K), dt, kappa)


# nc > 27 (2D m >= 5, 3D m = 3) runs the dense blocks in passes of 16 rows
CASES = [(1, 0, (9,)), (1, 3, (37,)), (1, 7, (11,)), (2, 1, (19, 6)), (2, 3, (13, 7)), (2, 4, (6, 5)),
         (2, 5, (7, 5)), (3, 1, (9, 5, 4)), (3, 2, (7, 4, 3)), (3, 2, (2, 2, 2)), (3, 3, (5, 4, 3)),
         (3, 3, (2, 2, 2))]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("d,m,K", CASES)
def test_adjoint_matches_oracle(d, m, K, prec):
    _say(f"[adjoint] d={d} m={m} K={K} {prec}")
    rng = np.random.default_rng(300 + 10 * d + m)
    kappa = 1.4
    plan = hl.Plan(d, m, K, cfl=0.7, c=np.sqrt(kappa), precision=prec)
    prob = _prob(d, m, K, plan.dt, kappa)
    Pb, Ub = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    pb, ub = plan.alloc()
    plan.init(pb, ub, Pb, Ub)
    Pb_in, Ub_in = plan.export(pb, ub)
    n = 3
    plan.adjoint_step(pb, ub, n)
    Pg, Ug = plan.export(pb, ub)
    Pr, Ur = oracle.adjoint_step(prob, Pb_in, Ub_in, n)
    _close(Pg, Pr, *atol(prec, d, m, n))
    _close(Ug, Ur, *atol(prec, d, m, n))


def test_dot_product_identity_2d_m3_256():
    """<step^n x, y> = <x, adjoint^n y> on the device state, 2D m=3 256^2."""
    _say("[adjoint] dot-product identity 2D m=3 256^2")
    d, m, K, n = 2, 3, (256, 256), 20
    rng = np.random.default_rng(11)
    plan = hl.Plan(d, m, K, cfl=0.8, precision="fp64")
    x = [torch.tensor(inputs.random_data(rng, d, m, K)), torch.tensor(inputs.random_data(rng, d, m, K, ncomp=d))]
    p, u = plan.alloc()
    pb, ub = plan.alloc()
    plan.init(p, u, x[0].numpy(), x[1].numpy())
    plan.init(pb, ub, inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d))
    p0, u0, pb0, ub0 = p.clone(), u.clone(), pb.clone(), ub.clone()
    plan.step(p, u, n)
    plan.adjoint_step(pb, ub, n)
    lhs = float(torch.dot(p, pb0) + torch.dot(u, ub0))
    rhs = float(torch.dot(p0, pb) + torch.dot(u0, ub))
    scale = float(torch.sqrt(torch.dot(p, p) + torch.dot(u, u)) * torch.sqrt(torch.dot(pb0, pb0) + torch.dot(ub0, ub0)))
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)


def test_autograd_backward_is_the_adjoint():
    _say("[adjoint] autograd")
    d, m, K, n = 2, 2, (33, 20), 7
    rng = np.random.default_rng(5)
    plan = hl.Plan(d, m, K, cfl=0.6, precision="fp64")
    prob = _prob(d, m, K, plan.dt, 1.0)
    p, u = plan.alloc()
    plan.init(p, u, inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d))
    p.requires_grad_(True)
    u.requires_grad_(True)
    wp = torch.randn(p.shape, dtype=p.dtype, device=p.device)
    p_n, u_n = hermite_steps(p, u, plan, n)
    loss = torch.dot(wp, p_n) + 0.5 * torch.dot(u_n, u_n)
    loss.backward()
    # reference: adjoint of (wp, u_n) through the library, and the oracle in host layout
    pb, ub = wp.clone(), u_n.detach().clone()
    plan.adjoint_step(pb, ub, n)
    assert torch.equal(p.grad, pb) and torch.equal(u.grad, ub)
    Wp, Un = plan.export(wp, u_n.detach())
    Pr, Ur = oracle.adjoint_step(prob, Wp, Un, n)
    Pg, Ug = plan.export(p.grad, u.grad)
    _close(Pg, Pr, 1e-12 * n, 1e-11 * n)
    _close(Ug, Ur, 1e-12 * n, 1e-11 * n)


WALL_CASES = [(1, 2, (9,)), (2, 1, (11, 6)), (2, 3, (7, 5)), (2, 5, (5, 4)), (3, 1, (5, 4, 3)), (3, 2, (4, 3, 3)),
              (3, 2, (2, 2, 2)), (3, 3, (3, 2, 2))]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("d,m,K", WALL_CASES)
def test_walls_adjoint_matches_oracle(d, m, K, prec):
    """The walled transpose: B^T from the K dual nodes, A^T on the padded
    array and the ghost fold, against the oracle's (pinned by the dot-product
    identity with the oracle's walled step)."""
    _say(f"[adjoint] walls d={d} m={m} K={K} {prec}")
    rng = np.random.default_rng(500 + 10 * d + m)
    kappa = 1.3
    plan = hl.Plan(d, m, K, cfl=0.6, c=np.sqrt(kappa), precision=prec, boundary="walls")
    prob = oracle.Problem(d, m, tuple(K), (1.0,) * d, plan.dt, kappa, "walls")
    ps, us = plan.host_shapes()
    pb, ub = plan.alloc()
    plan.init(pb, ub, rng.uniform(-1, 1, ps), rng.uniform(-1, 1, us))
    Pb_in, Ub_in = plan.export(pb, ub)
    n = 3
    plan.adjoint_step(pb, ub, n)
    Pg, Ug = plan.export(pb, ub)
    Pr, Ur = oracle.adjoint_step(prob, Pb_in, Ub_in, n)
    _close(Pg, Pr, *atol(prec, d, m, n))
    _close(Ug, Ur, *atol(prec, d, m, n))


def test_walls_dot_product_identity_2d_m3_128():
    """<step^n x, y> = <x, adjoint^n y> with walls, 2D m=3 128 x 96, FP64,
    on the exported states (the K dual nodes are the variables)."""
    _say("[adjoint] walls dot-product identity 2D m=3")
    d, m, K, n = 2, 3, (128, 96), 12
    rng = np.random.default_rng(13)
    plan = hl.Plan(d, m, K, cfl=0.8, precision="fp64", boundary="walls")
    ps, us = plan.host_shapes()
    X = (rng.uniform(-1, 1, ps), rng.uniform(-1, 1, us))
    Y = (rng.uniform(-1, 1, ps), rng.uniform(-1, 1, us))
    p, u = plan.alloc()
    pb, ub = plan.alloc()
    plan.init(p, u, *X)
    plan.init(pb, ub, *Y)
    plan.step(p, u, n)
    plan.adjoint_step(pb, ub, n)
    SX, AY = plan.export(p, u), plan.export(pb, ub)
    lhs = np.sum(SX[0] * Y[0]) + np.sum(SX[1] * Y[1])
    rhs = np.sum(X[0] * AY[0]) + np.sum(X[1] * AY[1])
    scale = np.sqrt(np.sum(SX[0] ** 2) + np.sum(SX[1] ** 2)) * np.sqrt(np.sum(Y[0] ** 2) + np.sum(Y[1] ** 2))
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("d,m,K,n", [(1, 3, (20,), 20), (2, 2, (14, 11), 10), (3, 1, (7, 5, 4), 5)])
def test_walls_kappa_gradient_matches_oracle(d, m, K, n, prec):
    """The kappa gradient with walls (the walled step walked back, the ghost
    refresh before the pressure-side operators) and the adjoint state against
    the oracle's (pinned by central differences of its walled step)."""
    _say(f"[adjoint] walls kappa gradient d={d} m={m} K={K} n={n} {prec}")
    rng = np.random.default_rng(90 + d + m)
    kappa = 1.2
    plan = hl.Plan(d, m, K, cfl=0.7, c=np.sqrt(kappa), precision=prec, boundary="walls")
    prob = oracle.Problem(d, m, tuple(K), (1.0,) * d, plan.dt, kappa, "walls")
    ps, us = plan.host_shapes()
    p, u = plan.alloc()
    pb, ub = plan.alloc()
    plan.init(p, u, inputs.zero_on_walls(rng.uniform(-1, 1, ps), d), rng.uniform(-1, 1, us))
    plan.init(pb, ub, rng.uniform(-1, 1, ps), rng.uniform(-1, 1, us))
    P0, U0 = plan.export(p, u)
    Pb, Ub = plan.export(pb, ub)
    plan.step(p, u, n)
    g = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.adjoint_step(pb, ub, n, p=p, u=u, grad_kappa=g)
    gr, Pr, Ur = oracle.kappa_gradient(prob, P0, U0, Pb, Ub, n)
    rt = {"fp64": 1e-9, "fp32": 3e-4, "fp32_comp": 1e-6}[prec]
    assert abs(float(g) - gr) <= rt * abs(gr), (float(g), gr)
    Pa, Ua = plan.export(pb, ub)
    _close(Pa, Pr, *atol(prec, d, m, n))
    _close(Ua, Ur, *atol(prec, d, m, n))
    plan.close()


def test_gradient_needs_forward_state():
    plan = hl.Plan(1, 1, (16,))
    p, u = plan.alloc()
    g = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = hl.lib().hl_adjoint_step(plan._h, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(u.data_ptr()), None, None,
                                  ctypes.c_void_p(g.data_ptr()), 1, None)
    assert st == hl.HL_ERR_ARG


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("d,m,K,n", [(1, 3, (24,), 30), (2, 2, (16, 12), 12), (3, 1, (8, 6, 5), 6), (3, 3, (4, 3, 3), 2)])
def test_kappa_gradient_matches_oracle(d, m, K, n, prec):
    """d/dkappa of <Pb, P_n> + <Ub, U_n> and the adjoint state against the
    oracle (stored trajectory); the library recomputes the trajectory by the
    reversed step, so FP64 agrees to rounding growth over n steps."""
    _say(f"[adjoint] kappa gradient d={d} m={m} K={K} n={n} {prec}")
    rng = np.random.default_rng(70 + d + m)
    kappa = 1.2
    plan = hl.Plan(d, m, K, cfl=0.7, c=np.sqrt(kappa), precision=prec)
    prob = _prob(d, m, K, plan.dt, kappa)
    p, u = plan.alloc()
    pb, ub = plan.alloc()
    plan.init(p, u, inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d))
    plan.init(pb, ub, inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d))
    P0, U0 = plan.export(p, u)
    Pb, Ub = plan.export(pb, ub)
    plan.step(p, u, n)
    g = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.adjoint_step(pb, ub, n, p=p, u=u, grad_kappa=g)
    gr, Pr, Ur = oracle.kappa_gradient(prob, P0, U0, Pb, Ub, n)
    rt = {"fp64": 1e-9, "fp32": 3e-4, "fp32_comp": 1e-6}[prec]
    assert abs(float(g) - gr) <= rt * abs(gr), (float(g), gr)
    Pa, Ua = plan.export(pb, ub)
    _close(Pa, Pr, *atol(prec, d, m, n))
    _close(Ua, Ur, *atol(prec, d, m, n))


def test_autograd_kappa_gradient_matches_finite_differences():
    """The kappa gradient through the autograd wrapper against a central
    difference of GPU forward runs (plans at kappa +- dk, +- 2 dk, dt fixed)."""
    _say("[adjoint] autograd kappa gradient vs finite differences")
    d, m, K, n = 2, 3, (64, 48), 40
    rng = np.random.default_rng(8)
    kappa, dt = 1.1, 0.4 / 64
    P0, U0 = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    plan = hl.Plan(d, m, K, dt=dt, c=np.sqrt(kappa), precision="fp64")
    p, u = plan.alloc()
    plan.init(p, u, P0, U0)
    w = torch.randn(p.shape, dtype=p.dtype, device=p.device)
    kt = torch.tensor(kappa, dtype=torch.float64, requires_grad=True)
    p_n, u_n = hermite_steps(p, u, plan, n, kappa=kt)
    loss = torch.dot(w, p_n) + 0.5 * torch.dot(u_n, u_n)
    loss.backward()

    def J(kap):
        pl = hl.Plan(d, m, K, dt=dt, c=np.sqrt(kap), precision="fp64")
        q, v = pl.alloc()
        pl.init(q, v, P0, U0)
        pl.step(q, v, n)
        return float(torch.dot(w, q) + 0.5 * torch.dot(v, v))

    # fourth-order central difference (random high-order data makes J stiff
    # in kappa: a second-order difference at this step is off by ~4e-6)
    dk = 1e-4 * kappa
    fd = (-J(kappa + 2 * dk) + 8 * J(kappa + dk) - 8 * J(kappa - dk) + J(kappa - 2 * dk)) / (12 * dk)
    assert abs(float(kt.grad) - fd) <= 1e-7 * abs(fd), (float(kt.grad), fd)
