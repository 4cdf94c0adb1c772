"""Pins of the oracle's reflecting-wall boundary (Sec. 5, "Imposing reflective
boundary conditions"): p = 0 on the faces of the box, imposed through ghost
dual nodes that mirror the velocity polynomials.

What fixes it, independently of the ghost code:
* the ghost layer equals the closed-form velocity of a box mode evaluated at
  the ghost positions (the mirror rule against the PDE's own solution);
* the walled step equals the periodic step (pinned elsewhere) on the doubled
  box holding the odd/even image extension, written here from the image
  positions, not from the ghost rule;
* p stays zero on the walls over many steps (eq. (Boundary), first line),
  which a wrong mirror parity breaks (checked with a planted flip);
* a box standing mode converges at the periodic scheme's rates.
"""

import numpy as np
import pytest

import oracle
from oracle import hermite_lf as H
from paper_1808_10481_amd import inputs


def _wprob(d, m, K, dt, length=None, kappa=1.0):
    length = length or (1.0,) * d
    return oracle.Problem(d, m, tuple(K), tuple(length), dt, kappa, bc="walls")


@pytest.mark.parametrize("d,m", [(1, 1), (1, 3), (2, 2), (3, 1)])
def test_ghost_layer_is_the_mirrored_solution(d, m):
    K = (5, 4, 3)[:d]
    L = (1.0, 0.8, 1.3)[:d]
    waves = (1, 2, 1)[:d]
    _, Uin = inputs.box_mode(d, m, K, L, waves, 0.0, 0.37)
    _, Ugh = inputs.box_mode(d, m, K, L, waves, 0.0, 0.37, ghosts=True)
    prob = _wprob(d, m, K, 0.01, L)
    pad = H.ghost_pad(prob, Uin)
    assert pad.shape == Ugh.shape
    assert np.allclose(pad, Ugh, rtol=0, atol=1e-13 * np.abs(Ugh).max())


def _extend_images(prob, P, U):
    """Odd (p) / even-normal, odd-tangential (u) image extension of walled data
    on [0, L] to the periodic box [0, 2L) with 2K cells."""
    d, m, K = prob.d, prob.m, prob.K
    sgn_a = (-1.0) ** np.arange(m + 1)
    Pe = np.zeros(tuple(2 * k for k in K) + (m + 1,) * d)
    Ue = np.zeros((d,) + tuple(2 * k for k in K) + (m + 1,) * d)
    import itertools
    for je in itertools.product(*[range(2 * k) for k in K]):
        src, fac = [], np.ones((m + 1,) * d)
        for k in range(d):
            if je[k] <= K[k]:
                src.append(je[k])
            else:                                   # image of j = 2K - je across x = L
                src.append(2 * K[k] - je[k])
                shape = [1] * d
                shape[k] = m + 1
                fac = fac * (-sgn_a).reshape(shape)
        Pe[je] = fac * P[tuple(src)]
    for i in range(d):
        for qe in itertools.product(*[range(2 * k) for k in K]):
            src, fac = [], np.ones((m + 1,) * d)
            for k in range(d):
                if qe[k] < K[k]:
                    src.append(qe[k])
                else:                               # image of q = 2K - 1 - qe
                    src.append(2 * K[k] - 1 - qe[k])
                    shape = [1] * d
                    shape[k] = m + 1
                    fac = fac * ((sgn_a if i == k else -sgn_a).reshape(shape))
            Ue[(i,) + qe] = fac * U[(i,) + tuple(src)]
    return Pe, Ue


@pytest.mark.parametrize("d,m,K", [(1, 2, (6,)), (2, 1, (4, 5)), (2, 3, (3, 4)), (3, 1, (3, 2, 3))])
def test_walls_equal_periodic_step_on_image_extension(d, m, K):
    rng = np.random.default_rng(40 + d + m)
    L = (1.0, 1.5, 0.7)[:d]
    prob = _wprob(d, m, K, 0.0, L)
    dt = 0.5 * min(prob.h)
    prob = prob.with_dt(dt)
    P = inputs.zero_on_walls(inputs.random_data(rng, d, m, prob.p_nodes()), d)
    U = inputs.random_data(rng, d, m, prob.u_nodes(), ncomp=d)
    Pw, Uw = H.step(prob, P, U, 3)
    per = oracle.Problem(d, m, tuple(2 * k for k in K), tuple(2 * l for l in L), dt)
    Pe, Ue = _extend_images(prob, P, U)
    Pp, Up = H.step(per, Pe, Ue, 3)
    sl = tuple(slice(0, k + 1) for k in K)
    tol = 1e-13 * max(np.abs(Pp).max(), np.abs(Up).max())      # summation order only
    assert np.allclose(Pw, Pp[sl], rtol=0, atol=tol)
    assert np.allclose(Uw, Up[(slice(None),) + tuple(slice(0, k) for k in K)], rtol=0, atol=tol)


def _wall_even_coefs(P, d):
    out = []
    for k in range(d):
        for j in (0, P.shape[k] - 1):
            idx = [slice(None)] * (2 * d)
            idx[k] = j
            idx[d + k] = slice(0, None, 2)
            out.append(P[tuple(idx)].ravel())
    return np.concatenate(out)


@pytest.mark.parametrize("d,m,K", [(1, 3, (9,)), (2, 2, (6, 5))])
def test_pressure_stays_zero_on_walls(d, m, K, monkeypatch):
    rng = np.random.default_rng(7)
    prob = _wprob(d, m, K, 0.0)
    prob = prob.with_dt(0.8 * min(prob.h))
    P = inputs.zero_on_walls(inputs.random_data(rng, d, m, prob.p_nodes()), d)
    U = inputs.random_data(rng, d, m, prob.u_nodes(), ncomp=d)
    Pn, _ = H.step(prob, P, U, 25)
    assert np.abs(_wall_even_coefs(Pn, d)).max() <= 1e-12 * np.abs(Pn).max()
    # planted mistake: treat the normal component as odd across its wall
    monkeypatch.setattr(H, "mirror_sign", lambda i, k: -1.0)
    Pb, _ = H.step(prob, P, U, 25)
    assert np.abs(_wall_even_coefs(Pb, d)).max() > 1e-3 * np.abs(Pb).max()



def _box_err(d, m, K, T, waves):
    prob = _wprob(d, m, (K,) * d, 0.0)
    n = int(np.ceil(T / (0.5 * min(prob.h))))
    prob = prob.with_dt(T / n)
    P0, U0 = inputs.box_mode(d, m, (K,) * d, (1.0,) * d, waves, 0.0, prob.dt / 2)
    Pn, _ = H.step(prob, P0, U0, n)
    Pex, _ = inputs.box_mode(d, m, (K,) * d, (1.0,) * d, waves, T, T)
    v = (0,) * d
    diff = Pn[(Ellipsis,) + v] - Pex[(Ellipsis,) + v]
    return np.sqrt(np.prod(prob.h) * np.sum(diff ** 2))


@pytest.mark.parametrize("d,m,Ks,T,rate_min", [(1, 1, (16, 32), 0.6, 1.5), (1, 2, (8, 16), 0.6, 4.5),
                                               (2, 2, (8, 16), 0.3, 4.5)])
def test_box_mode_converges(d, m, Ks, T, rate_min):
    waves = (1, 2)[:d]
    e1, e2 = (_box_err(d, m, K, T, waves) for K in Ks)
    rate = np.log2(e1 / e2)
    assert rate >= rate_min, (e1, e2, rate)


def _extend_kappa(K, Kap, grid):
    """Even image extension of walled kappa data to the doubled periodic box
    (a coefficient of order b_k mirrored across x_k picks up (-1)^{b_k})."""
    import itertools
    d = len(K)
    n = Kap.shape[-1]
    sgn = (-1.0) ** np.arange(n)
    out = np.zeros(tuple(2 * k for k in K) + (n,) * d)
    for je in itertools.product(*[range(2 * k) for k in K]):
        src, fac = [], np.ones((n,) * d)
        for k in range(d):
            lim = K[k] if grid == "primal" else K[k] - 1
            if je[k] <= lim:
                src.append(je[k])
            else:
                src.append((2 * K[k] if grid == "primal" else 2 * K[k] - 1) - je[k])
                shape = [1] * d
                shape[k] = n
                fac = fac * sgn.reshape(shape)
        out[je] = fac * Kap[tuple(src)]
    return out


@pytest.mark.parametrize("d,m,K", [(1, 2, (7,)), (2, 1, (5, 4)), (2, 3, (4, 3))])
def test_variable_kappa_walls_equal_periodic_step_on_image_extension(d, m, K):
    """Walls with variable kappa (even about every wall): the walled step equals
    the periodic variable-kappa step on the doubled box holding the image
    extension of P, U and kappa (written from image positions, not the ghost
    rule); constant kappa data reproduce the constant walled step."""
    rng = np.random.default_rng(90 + d + m)
    L = (1.0, 1.5)[:d]
    prob = _wprob(d, m, K, 0.0, L)
    dt = 0.4 * min(prob.h) / np.sqrt(1.3)
    prob = prob.with_dt(dt)
    P = inputs.zero_on_walls(inputs.random_data(rng, d, m, prob.p_nodes()), d)
    U = inputs.random_data(rng, d, m, prob.u_nodes(), ncomp=d)
    amps = tuple(rng.uniform(0.1, 0.3, d))
    Kp, Ku = inputs.kappa_box(d, m, K, L, amps, "primal"), inputs.kappa_box(d, m, K, L, amps, "dual")
    Pw, Uw = H.step_var(prob, P, U, Kp, Ku, 3)
    per = oracle.Problem(d, m, tuple(2 * k for k in K), tuple(2 * l for l in L), dt)
    Pe, Ue = _extend_images(prob, P, U)
    Pp, Up = H.step_var(per, Pe, Ue, _extend_kappa(K, Kp, "primal"), _extend_kappa(K, Ku, "dual"), 3)
    sl = tuple(slice(0, k + 1) for k in K)
    tol = 1e-13 * max(np.abs(Pp).max(), np.abs(Up).max())
    assert np.allclose(Pw, Pp[sl], rtol=0, atol=tol)
    assert np.allclose(Uw, Up[(slice(None),) + tuple(slice(0, k) for k in K)], rtol=0, atol=tol)
    # constant kappa data: the constant-coefficient walled step
    kap = 1.3
    pc = _wprob(d, m, K, dt, L, kappa=kap)
    Kc = np.zeros(prob.p_nodes() + (2 * m + 2,) * d)
    Kc[(Ellipsis,) + (0,) * d] = kap
    Kcu = np.zeros(prob.u_nodes() + (2 * m + 2,) * d)
    Kcu[(Ellipsis,) + (0,) * d] = kap
    P1, U1 = H.step_var(pc, P, U, Kc, Kcu, 2)
    P2, U2 = H.step(pc, P, U, 2)
    assert np.allclose(P1, P2, rtol=0, atol=1e-13 * np.abs(P2).max())
    assert np.allclose(U1, U2, rtol=0, atol=1e-13 * np.abs(U2).max())
