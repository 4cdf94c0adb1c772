"""Pins of the oracle's variable-kappa adjoint and of its gradient with respect
to the kappa data (per-node transposed blocks; complex-step derivatives of the
cell updates):

* the transposed step is the transpose of step_var: <step(x), y> = <x, adj(y)>
  on random states and random (non-smooth) kappa data, one half-step at a time
  and over several steps;
* constant kappa data reduce it to the constant-coefficient adjoint, and the
  kappa_0 gradients summed over every node to the scalar kappa derivative
  (both pinned by their own tests against the forward step and differences);
* directional derivatives of <Pb, P_n> + <Ub, U_n>, and of a misfit of the
  pressure at receiver nodes after every step, match fourth-order central
  differences of step_var along random kappa directions.

The definitions used with reflecting walls (the transpose read off unit
responses of step_var, the gradient by central differences per kappa entry)
are pinned on the periodic grid against the structured adjoint and gradient
above, and on the walled box by their reduction, for constant kappa data, to
the constant-coefficient walled adjoint and scalar gradient (pinned by the
dot-product identity and central differences of the walled step).
"""

import numpy as np
import pytest

import oracle
from oracle import hermite_lf as H
from paper_1808_10481_amd import inputs


def _prob(d, m, K, nu=0.6):
    pr = oracle.Problem(d, m, tuple(K), tuple(1.0 + 0.2 * k for k in range(d)), 0.0, 1.0)
    return pr.with_dt(nu * min(pr.h) / np.sqrt(1.6))


def _kappa(rng, d, m, K, amp=0.1):
    """Random kappa data: kappa_0 in [1, 1.4], every other coefficient
    uniform in [-amp, amp] (the step is a polynomial map of these for any
    values)."""
    N2 = 2 * m + 2
    Kd = rng.uniform(-amp, amp, size=tuple(K) + (N2,) * d)
    Kd[(Ellipsis,) + (0,) * d] = rng.uniform(1.0, 1.4, size=tuple(K))
    return Kd


CASES = [(1, 1, (6,)), (1, 3, (5,)), (2, 1, (4, 5)), (2, 2, (4, 3))]


def _dot(a, b):
    return float(np.sum(a * b))


@pytest.mark.parametrize("d,m,K", CASES)
def test_transposed_half_steps(d, m, K):
    rng = np.random.default_rng(500 + 10 * d + m)
    prob = _prob(d, m, K)
    Kp, Ku = _kappa(rng, d, m, K), _kappa(rng, d, m, K)
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Pb, Ub = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    AU = P - H.p_half_var(prob, P, U, Kp)                       # A U
    ATPb = Ub - H.u_half_var_adjoint(prob, Ub, Pb, Kp)          # A^T Pb
    assert abs(_dot(AU, Pb) - _dot(U, ATPb)) <= 1e-12 * np.linalg.norm(AU) * np.linalg.norm(Pb)
    BP = U - H.u_half_var(prob, U, P, Ku)                       # B P
    BTUb = Pb - H.p_half_var_adjoint(prob, Pb, Ub, Ku)          # B^T Ub
    assert abs(_dot(BP, Ub) - _dot(P, BTUb)) <= 1e-12 * np.linalg.norm(BP) * np.linalg.norm(Ub)


@pytest.mark.parametrize("d,m,K", CASES)
def test_dot_product_identity(d, m, K):
    rng = np.random.default_rng(600 + 10 * d + m)
    prob = _prob(d, m, K)
    Kp, Ku = _kappa(rng, d, m, K), _kappa(rng, d, m, K)
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Pb, Ub = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    P1, U1 = H.step_var(prob, P, U, Kp, Ku, 3)
    Pa, Ua = H.adjoint_step_var(prob, Pb, Ub, Kp, Ku, 3)
    lhs, rhs = _dot(P1, Pb) + _dot(U1, Ub), _dot(P, Pa) + _dot(U, Ua)
    scale = np.sqrt(_dot(P1, P1) + _dot(U1, U1)) * np.sqrt(_dot(Pb, Pb) + _dot(Ub, Ub))
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)


@pytest.mark.parametrize("d,m,K", [(1, 2, (5,)), (2, 1, (4, 3))])
def test_constant_kappa_data_reduce_to_the_scalar_gradient(d, m, K):
    rng = np.random.default_rng(700 + d + m)
    kappa = 1.3
    prob = oracle.Problem(d, m, tuple(K), (1.0,) * d, 0.0, kappa).with_dt(0.6 / max(K) / np.sqrt(kappa))
    Kc = np.zeros(tuple(K) + (2 * m + 2,) * d)
    Kc[(Ellipsis,) + (0,) * d] = kappa
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Pb, Ub = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    n = 3
    Pa, Ua = H.adjoint_step_var(prob, Pb, Ub, Kc, Kc, n)
    Pc, Uc = H.adjoint_step(prob, Pb, Ub, n)
    assert np.max(np.abs(Pa - Pc)) <= 1e-12 * np.max(np.abs(Pc))
    assert np.max(np.abs(Ua - Uc)) <= 1e-12 * np.max(np.abs(Uc))
    P1, U1 = H.step(prob, P, U, n)
    gp, gu, P0b, U0b = H.kappa_field_gradient(prob, P, U, Kc, Kc, Pb, Ub, n)
    g, Ps, Us = H.kappa_gradient(prob, P, U, Pb, Ub, n)
    z = (Ellipsis,) + (0,) * d
    assert abs(np.sum(gp[z]) + np.sum(gu[z]) - g) <= 1e-11 * max(1.0, abs(g)), (np.sum(gp[z]) + np.sum(gu[z]), g)
    assert np.max(np.abs(P0b - Ps)) <= 1e-12 * np.max(np.abs(Ps))
    assert np.max(np.abs(U0b - Us)) <= 1e-12 * np.max(np.abs(Us))


def _misfit(prob, P0, U0, Kp, Ku, Pb, Ub, n, rec, data):
    """<Pb, P_n> + <Ub, U_n> + 1/2 sum_t sum_r (P_{t+1}[rec_r][0] - data[t, r])^2."""
    P, U = np.array(P0), np.array(U0)
    loss = 0.0
    z = (0,) * prob.d
    for t in range(n):
        P, U = H.step_var(prob, P, U, Kp, Ku, 1)
        tr = np.array([P[tuple(r) + z] for r in rec])
        loss += 0.5 * np.sum((tr - data[t]) ** 2)
    return loss + _dot(Pb, P) + _dot(Ub, U)


def _sources(prob, P0, U0, Kp, Ku, n, rec, data):
    """Adjoint sources of the receiver misfit: d/dP_{t+1} = residual at the
    receivers' coefficient 0."""
    P, U = np.array(P0), np.array(U0)
    src = []
    z = (0,) * prob.d
    for t in range(n):
        P, U = H.step_var(prob, P, U, Kp, Ku, 1)
        s = np.zeros_like(P)
        for r_i, r in enumerate(rec):
            s[tuple(r) + z] += P[tuple(r) + z] - data[t, r_i]
        src.append(s)
    return src


@pytest.mark.parametrize("d,m,K", [(1, 1, (6,)), (1, 3, (4,)), (2, 1, (4, 3)), (2, 2, (3, 4))])
def test_directional_derivatives_match_central_differences(d, m, K):
    rng = np.random.default_rng(800 + 10 * d + m)
    prob = _prob(d, m, K)
    Kp, Ku = _kappa(rng, d, m, K, amp=0.05), _kappa(rng, d, m, K, amp=0.05)
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Pb, Ub = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    n = 3
    rec = [tuple(int(rng.integers(0, k)) for k in K) for _ in range(2)]
    data = rng.normal(size=(n, len(rec)))
    src = _sources(prob, P, U, Kp, Ku, n, rec, data)
    gp, gu, _, _ = H.kappa_field_gradient(prob, P, U, Kp, Ku, Pb, Ub, n, p_sources=src)
    for trial in range(2):
        dp, du = rng.normal(size=Kp.shape), rng.normal(size=Ku.shape)
        if trial == 1:
            dp[...] = 0.0   # the velocity-side coefficient alone
        eps = 1e-3

        def L(s):
            return _misfit(prob, P, U, Kp + s * dp, Ku + s * du, Pb, Ub, n, rec, data)

        fd = (-L(2 * eps) + 8 * L(eps) - 8 * L(-eps) + L(-2 * eps)) / (12 * eps)
        an = _dot(gp, dp) + _dot(gu, du)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(fd)), (trial, fd, an)


def _walls_prob(d, m, K, kappa=1.0, nu=0.6):
    pr = oracle.Problem(d, m, tuple(K), (1.0,) * d, 0.0, kappa, "walls")
    return pr.with_dt(nu * min(pr.h) / np.sqrt(1.6))


def _walls_kappa(rng, prob, amp=0.1):
    N2 = 2 * prob.m + 2
    out = []
    for nodes in (prob.p_nodes(), prob.u_nodes()):
        Kd = rng.uniform(-amp, amp, size=nodes + (N2,) * prob.d)
        Kd[(Ellipsis,) + (0,) * prob.d] = rng.uniform(1.0, 1.4, size=nodes)
        out.append(Kd)
    return out


@pytest.mark.parametrize("d,m,K", [(1, 2, (5,)), (2, 1, (3, 4))])
def test_bruteforce_transpose_and_fd_gradient_match_the_structured_ones(d, m, K):
    """Periodic grid: the transpose from unit responses equals the structured
    adjoint, and the central-difference gradient entries equal the
    complex-step ones."""
    rng = np.random.default_rng(800 + 10 * d + m)
    prob = _prob(d, m, K)
    Kp, Ku = _kappa(rng, d, m, K), _kappa(rng, d, m, K)
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Pb, Ub = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    n = 2
    Pa, Ua = H.adjoint_step_var_bruteforce(prob, Pb, Ub, Kp, Ku, n)
    Ps, Us = H.adjoint_step_var(prob, Pb, Ub, Kp, Ku, n)
    assert np.max(np.abs(Pa - Ps)) <= 1e-12 * np.max(np.abs(Ps))
    assert np.max(np.abs(Ua - Us)) <= 1e-12 * np.max(np.abs(Us))
    gp, gu, _, _ = H.kappa_field_gradient(prob, P, U, Kp, Ku, Pb, Ub, n)
    entries = [(0, int(i)) for i in rng.choice(Kp.size, 6, replace=False)] + \
              [(1, int(i)) for i in rng.choice(Ku.size, 6, replace=False)]
    fd = H.kappa_field_gradient_fd(prob, P, U, Kp, Ku, Pb, Ub, n, entries)
    ref = np.array([(gp if f == 0 else gu).reshape(-1)[i] for f, i in entries])
    assert np.max(np.abs(fd - ref)) <= 1e-8 * np.max(np.abs(ref)), (fd, ref)


@pytest.mark.parametrize("d,m,K", [(1, 3, (5,)), (2, 1, (3, 4))])
def test_walls_bruteforce_reduces_to_the_constant_coefficient_walled_adjoint(d, m, K):
    rng = np.random.default_rng(900 + 10 * d + m)
    kappa = 1.3
    prob = _walls_prob(d, m, K, kappa)
    Kp = np.zeros(prob.p_nodes() + (2 * m + 2,) * d)
    Ku = np.zeros(prob.u_nodes() + (2 * m + 2,) * d)
    z = (Ellipsis,) + (0,) * d
    Kp[z], Ku[z] = kappa, kappa
    P, U = rng.uniform(-1, 1, prob.p_shape()), rng.uniform(-1, 1, prob.u_shape())
    Pb, Ub = rng.uniform(-1, 1, prob.p_shape()), rng.uniform(-1, 1, prob.u_shape())
    n = 2
    Pa, Ua = H.adjoint_step_var_bruteforce(prob, Pb, Ub, Kp, Ku, n)
    Pc, Uc = H.adjoint_step(prob, Pb, Ub, n)
    assert np.max(np.abs(Pa - Pc)) <= 1e-12 * np.max(np.abs(Pc))
    assert np.max(np.abs(Ua - Uc)) <= 1e-12 * np.max(np.abs(Uc))
    # the kappa_0 entries summed over every node of both grids: the scalar kappa derivative
    ent = [(0, i) for i in range(0, Kp.size, (2 * m + 2) ** d)] + [(1, i) for i in range(0, Ku.size, (2 * m + 2) ** d)]
    fd = H.kappa_field_gradient_fd(prob, P, U, Kp, Ku, Pb, Ub, n, ent)
    g, _, _ = H.kappa_gradient(prob, P, U, Pb, Ub, n)
    assert abs(np.sum(fd) - g) <= 1e-8 * max(1.0, abs(g)), (np.sum(fd), g)


def test_walls_bruteforce_transpose_with_variable_kappa():
    """Non-constant kappa data on the walled box: the transpose satisfies the
    dot-product identity with the walled step_var, and a planted error (one
    kappa entry changed in the transpose only) breaks it."""
    rng = np.random.default_rng(950)
    prob = _walls_prob(2, 2, (3, 2))
    Kp, Ku = _walls_kappa(rng, prob)
    P, U = rng.uniform(-1, 1, prob.p_shape()), rng.uniform(-1, 1, prob.u_shape())
    Pb, Ub = rng.uniform(-1, 1, prob.p_shape()), rng.uniform(-1, 1, prob.u_shape())
    P1, U1 = H.step_var(prob, P, U, Kp, Ku, 2)
    Pa, Ua = H.adjoint_step_var_bruteforce(prob, Pb, Ub, Kp, Ku, 2)
    lhs, rhs = _dot(P1, Pb) + _dot(U1, Ub), _dot(P, Pa) + _dot(U, Ua)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)
    Kbad = np.array(Kp)
    Kbad.reshape(-1)[0] += 0.05  # kappa_0 at the corner node
    Pw, Uw = H.adjoint_step_var_bruteforce(prob, Pb, Ub, Kbad, Ku, 2)
    assert abs(lhs - (_dot(P, Pw) + _dot(U, Uw))) > 1e-6 * (abs(lhs) + 1.0)
