"""Pins of the oracle's discrete adjoint: the defining identity
<step(x), y> = <x, adjoint_step(y)> on random states (brute-force transposes
of the pinned forward operators must satisfy it to rounding), the half-step
identities one at a time, and the structure the adjoint must have (linearity,
composition over steps, A and B blocks matching the forward half-steps)."""

import numpy as np
import pytest

import oracle
from oracle import hermite_lf as H
from paper_1808_10481_amd import inputs


def _prob(d, m, K, nu=0.7, kappa=1.3):
    pr = oracle.Problem(d, m, tuple(K), tuple(1.0 + 0.2 * k for k in range(d)), 0.0, kappa)
    return pr.with_dt(nu * min(pr.h) / np.sqrt(kappa))


CASES = [(1, 0, (7,)), (1, 3, (6,)), (2, 1, (5, 4)), (2, 3, (4, 3)), (3, 1, (3, 4, 2)), (3, 2, (2, 3, 2))]


@pytest.mark.parametrize("d,m,K", CASES)
def test_dot_product_identity(d, m, K):
    rng = np.random.default_rng(100 + 10 * d + m)
    prob = _prob(d, m, K)
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Pb, Ub = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    for n in (1, 3):
        P1, U1 = H.step(prob, P, U, n)
        Pa, Ua = H.adjoint_step(prob, Pb, Ub, n)
        lhs = np.sum(P1 * Pb) + np.sum(U1 * Ub)
        rhs = np.sum(P * Pa) + np.sum(U * Ua)
        scale = np.sqrt(np.sum(P1 ** 2) + np.sum(U1 ** 2)) * np.sqrt(np.sum(Pb ** 2) + np.sum(Ub ** 2))
        assert abs(lhs - rhs) <= 1e-12 * scale, (n, lhs, rhs)


@pytest.mark.parametrize("d,m,K", CASES[:4])
def test_half_step_transposes(d, m, K):
    """<P - A U, Pb> = <P, Pb> + <U, -A^T Pb> and the same for B."""
    rng = np.random.default_rng(7 + d + m)
    prob = _prob(d, m, K)
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Pb, Ub = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    AU = P - H.p_half(prob, P, U)                         # A U
    ATPb = Ub - H.u_half_adjoint(prob, Ub, Pb)            # A^T Pb
    assert abs(np.sum(AU * Pb) - np.sum(U * ATPb)) <= 1e-12 * np.linalg.norm(AU) * np.linalg.norm(Pb)
    BP = U - H.u_half(prob, U, P)                         # B P
    BTUb = Pb - H.p_half_adjoint(prob, Pb, Ub)            # B^T Ub
    assert abs(np.sum(BP * Ub) - np.sum(P * BTUb)) <= 1e-12 * np.linalg.norm(BP) * np.linalg.norm(Ub)


def test_blocks_reproduce_the_forward_half_steps():
    d, m, K = 2, 2, (5, 4)
    rng = np.random.default_rng(3)
    prob = _prob(d, m, K)
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    A, B = H.p_operator_blocks(prob), H.u_operator_blocks(prob)
    nc = prob.nc
    Uf, Pf = U.reshape((d,) + K + (nc,)), P.reshape(K + (nc,))
    AU = np.zeros(K + (nc,))
    BP = np.zeros((d,) + K + (nc,))
    for e in [(0, 0), (0, 1), (1, 0), (1, 1)]:
        AU += np.einsum("sia,i...a->...s", A[e], np.roll(Uf, shift=(1 - e[0], 1 - e[1]), axis=(1, 2)))
        BP += np.einsum("isa,...a->i...s", B[e], np.roll(Pf, shift=(-e[0], -e[1]), axis=(0, 1)))
    assert np.allclose(P - AU.reshape(P.shape), H.p_half(prob, P, U), rtol=0, atol=1e-13)
    assert np.allclose(U - BP.reshape(U.shape), H.u_half(prob, U, P), rtol=0, atol=1e-13)


@pytest.mark.parametrize("d,m,K,n", [(1, 2, (8,), 6), (2, 1, (5, 4), 4), (2, 3, (4, 3), 3)])
def test_kappa_gradient_matches_finite_differences(d, m, K, n):
    """d/dkappa of <Pb, P_n> + <Ub, U_n> at fixed dt against a central
    difference of the forward oracle (the misfit is a polynomial in kappa;
    the step 1e-4 kappa leaves a relative error far below the bound)."""
    rng = np.random.default_rng(60 + d + m)
    prob = _prob(d, m, K)
    P0, U0 = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Pb, Ub = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    g, Pa, Ua = H.kappa_gradient(prob, P0, U0, Pb, Ub, n)

    def J(kappa):
        Pn, Un = H.step(oracle.Problem(prob.d, prob.m, prob.K, prob.length, prob.dt, kappa), P0, U0, n)
        return np.sum(Pn * Pb) + np.sum(Un * Ub)

    dk = 1e-4 * prob.kappa
    fd = (J(prob.kappa + dk) - J(prob.kappa - dk)) / (2 * dk)
    assert abs(g - fd) <= 1e-6 * max(abs(fd), 1e-12), (g, fd)
    # the adjoint state it returns is adjoint_step's
    Pr, Ur = H.adjoint_step(prob, Pb, Ub, n)
    assert np.allclose(Pa, Pr, rtol=0, atol=1e-12 * np.abs(Pr).max())
    assert np.allclose(Ua, Ur, rtol=0, atol=1e-12 * np.abs(Ur).max())


# Reflecting walls: the adjoint of the walled step (ghost padding, then the
# pressure half-step, then the velocity half-step) against the same identity.

def _walled(d, m, K, nu=0.6, kappa=1.2):
    pr = oracle.Problem(d, m, tuple(K), tuple(1.0 + 0.3 * k for k in range(d)), 0.0, kappa, "walls")
    return pr.with_dt(nu * min(pr.h) / np.sqrt(kappa))


WALL_CASES = [(1, 0, (5,)), (1, 2, (4,)), (2, 1, (4, 3)), (2, 3, (3, 2)), (3, 1, (2, 3, 2)), (3, 2, (2, 2, 3))]


@pytest.mark.parametrize("d,m,K", WALL_CASES)
def test_ghost_pad_adjoint_identity(d, m, K):
    rng = np.random.default_rng(40 + d + m)
    prob = _walled(d, m, K)
    U = rng.uniform(-1, 1, prob.u_shape())
    W = rng.uniform(-1, 1, (d,) + tuple(k + 2 for k in K) + (m + 1,) * d)
    lhs = np.sum(H.ghost_pad(prob, U) * W)
    rhs = np.sum(U * H.ghost_pad_adjoint(prob, W))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(W) * np.linalg.norm(U) * 8


@pytest.mark.parametrize("d,m,K", WALL_CASES)
def test_walled_dot_product_identity(d, m, K):
    """<step(x), y> = <x, adjoint_step(y)> for the walled step on random data
    (any data, including nonzero pressure on the walls: the step is linear)."""
    rng = np.random.default_rng(200 + 10 * d + m)
    prob = _walled(d, m, K)
    P, U = rng.uniform(-1, 1, prob.p_shape()), rng.uniform(-1, 1, prob.u_shape())
    Pb, Ub = rng.uniform(-1, 1, prob.p_shape()), rng.uniform(-1, 1, prob.u_shape())
    for n in (1, 2):
        P1, U1 = H.step(prob, P, U, n)
        Pa, Ua = H.adjoint_step(prob, Pb, Ub, n)
        lhs = np.sum(P1 * Pb) + np.sum(U1 * Ub)
        rhs = np.sum(P * Pa) + np.sum(U * Ua)
        scale = np.sqrt(np.sum(P1 ** 2) + np.sum(U1 ** 2)) * np.sqrt(np.sum(Pb ** 2) + np.sum(Ub ** 2))
        assert abs(lhs - rhs) <= 1e-12 * scale, (n, lhs, rhs)


def test_walled_adjoint_with_a_planted_sign_error_fails():
    """The identity sees a wrong mirror parity in the ghost fold."""
    d, m, K = 2, 2, (3, 3)
    rng = np.random.default_rng(9)
    prob = _walled(d, m, K)
    P, U = rng.uniform(-1, 1, prob.p_shape()), rng.uniform(-1, 1, prob.u_shape())
    Pb, Ub = rng.uniform(-1, 1, prob.p_shape()), rng.uniform(-1, 1, prob.u_shape())
    P1, U1 = H.step(prob, P, U, 1)
    orig = H.mirror_sign
    try:
        H.mirror_sign = lambda i, k: -orig(i, k)
        # only the adjoint's fold sees the planted sign (the forward result is already computed)
        Pa, Ua = H.adjoint_step(prob, Pb, Ub, 1)
    finally:
        H.mirror_sign = orig
    lhs = np.sum(P1 * Pb) + np.sum(U1 * Ub)
    rhs = np.sum(P * Pa) + np.sum(U * Ua)
    assert abs(lhs - rhs) > 1e-6 * abs(lhs)


@pytest.mark.parametrize("d,m,K,n", [(1, 2, (6,), 5), (2, 1, (4, 3), 4), (3, 1, (2, 3, 2), 2)])
def test_walled_kappa_gradient_matches_finite_differences(d, m, K, n):
    """The kappa derivative with walls against a central difference of the
    oracle's walled step (dt fixed)."""
    rng = np.random.default_rng(80 + d + m)
    prob = _walled(d, m, K)
    P0, U0 = rng.uniform(-1, 1, prob.p_shape()), rng.uniform(-1, 1, prob.u_shape())
    Pb, Ub = rng.uniform(-1, 1, prob.p_shape()), rng.uniform(-1, 1, prob.u_shape())
    g, Pa, Ua = H.kappa_gradient(prob, P0, U0, Pb, Ub, n)

    def J(kappa):
        Pn, Un = H.step(oracle.Problem(prob.d, prob.m, prob.K, prob.length, prob.dt, kappa, "walls"), P0, U0, n)
        return np.sum(Pn * Pb) + np.sum(Un * Ub)

    dk = 1e-4 * prob.kappa
    fd = (J(prob.kappa + dk) - J(prob.kappa - dk)) / (2 * dk)
    assert abs(g - fd) <= 1e-6 * max(abs(fd), 1e-12), (g, fd)
    Pr, Ur = H.adjoint_step(prob, Pb, Ub, n)
    assert np.allclose(Pa, Pr, rtol=0, atol=1e-12 * np.abs(Pr).max())
    assert np.allclose(Ua, Ur, rtol=0, atol=1e-12 * np.abs(Ur).max())
