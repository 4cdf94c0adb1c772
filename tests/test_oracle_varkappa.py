"""Pins of the oracle's variable-coefficient step (Sec. 4, "Smoothly varying
wave speed": kappa expanded about every node in a Taylor polynomial of degree
2m+1; the recurrence's reading is in the oracle's header).

* constant kappa data reproduce the constant-coefficient step (pinned
  elsewhere) to rounding;
* one half-step is exact for polynomial solutions with an affine kappa
  (the exact solution from the PDE's own time recurrence, tests/polyutil.py),
  data of total degree <= 2m so that no truncated product is cut;
* the paper's 1D variable-speed case (kappa = 1 + sin(x)/2 on [0, 2 pi])
  converges at high order (self-convergence against a 4x finer grid; the
  paper's rates: 1.98, 1.97, 5.99, 5.88 for m = 0..3 with a forcing term).
"""

import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import hermite_lf as H
from paper_1808_10481_amd import inputs

import polyutil as pu


@pytest.mark.parametrize("d,m,K", [(1, 2, (7,)), (2, 1, (5, 4)), (2, 3, (4, 3)), (3, 1, (3, 3, 2)), (3, 2, (3, 2, 2))])
def test_constant_kappa_data_reproduce_constant_step(d, m, K):
    rng = np.random.default_rng(d + 10 * m)
    kappa = 1.7
    prob = oracle.Problem(d, m, K, (1.0,) * d, 0.0, kappa).with_dt(0.6 / max(K) / np.sqrt(kappa))
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    Kc = np.zeros(K + (2 * m + 2,) * d)
    Kc[(Ellipsis,) + (0,) * d] = kappa
    Pv, Uv = H.step_var(prob, P, U, Kc, Kc, 3)
    Pc, Uc = H.step(prob, P, U, 3)
    scale = max(np.abs(Pc).max(), np.abs(Uc).max())
    assert np.abs(Pv - Pc).max() <= 1e-13 * scale and np.abs(Uv - Uc).max() <= 1e-13 * scale


def _corners(polys, centre, h, m, d):
    out = []
    for q in polys:
        arr = np.empty((2,) * d + (1,) + (m + 1,) * d)
        for e in itertools.product((0, 1), repeat=d):
            pt = [centre[k] + (e[k] - 0.5) * h[k] for k in range(d)]
            arr[e + (0,)] = pu.scaled_data(q, pt, h, m)
        out.append(arr)
    return out


def _kappa_data(k0, kgrad, centre, h, m, d):
    kap = np.zeros((2 * m + 2,) * d)
    kap[(0,) * d] = k0 + float(np.dot(kgrad, centre))
    for k in range(d):
        idx = [0] * d
        idx[k] = 1
        kap[tuple(idx)] = kgrad[k] * h[k]
    return kap[None]


@pytest.mark.parametrize("d,m", [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1)])
def test_half_steps_exact_for_affine_kappa(d, m):
    rng = np.random.default_rng(500 + 10 * d + m)
    deg = 2 * m                                          # total degree <= 2m
    def poly():
        c = pu.random_poly(rng, d, deg)
        for idx in itertools.product(range(deg + 1), repeat=d):
            if sum(idx) > deg:
                c[idx] = 0.0
        return c
    p0, u0 = poly(), [poly() for _ in range(d)]
    k0, kgrad = 1.3, rng.uniform(-0.3, 0.3, size=d)
    h = rng.uniform(0.2, 0.4, size=d)
    centre = rng.uniform(-0.3, 0.3, size=d)
    dt = 0.5 * h.min()
    P, U = pu.time_series_affine(p0, u0, k0, kgrad)
    prob = oracle.Problem(d, m, (4,) * d, tuple(4 * h), dt, 1.0)
    t0 = 0.1
    # pressure half-step at a primal node (kappa about it)
    pv = pu.scaled_data(pu.at_time(P, t0), centre, h, m)[None]
    uc = _corners(pu.at_time(U, t0 + dt / 2), centre, h, m, d)
    got = H.p_update_cells_var(prob, pv, uc, _kappa_data(k0, kgrad, centre, h, m, d))[0]
    want = pu.scaled_data(pu.at_time(P, t0 + dt), centre, h, m)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * max(1.0, np.abs(want).max()))
    # velocity half-step at a dual node
    uv = np.stack([pu.scaled_data(q, centre, h, m) for q in pu.at_time(U, t0 - dt / 2)])[:, None]
    pc = _corners([pu.at_time(P, t0)], centre, h, m, d)[0]
    got = H.u_update_cells_var(prob, uv, pc, _kappa_data(k0, kgrad, centre, h, m, d))[:, 0]
    want = np.stack([pu.scaled_data(q, centre, h, m) for q in pu.at_time(U, t0 + dt / 2)])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * max(1.0, np.abs(want).max()))


def _run_1d(m, K, T):
    L = 2 * np.pi
    prob = oracle.Problem(1, m, (K,), (L,), 0.0, 1.0)
    n = int(np.ceil(T / (0.5 * prob.h[0] / np.sqrt(1.5))))
    prob = prob.with_dt(T / n)
    Kp = inputs.kappa_sines(1, m, (K,), (L,), (0.5,), (1,), "primal")
    Ku = inputs.kappa_sines(1, m, (K,), (L,), (0.5,), (1,), "dual")
    P0, _ = inputs.standing_mode(1, m, (K,), (L,), (1,), 0.0, 0.0)   # p0 = sin x, u0 = 0
    U = H.u_half_var(prob, np.zeros((1,) + P0.shape), P0, Ku, weight_scale=0.5)
    P, U = H.step_var(prob, P0, U, Kp, Ku, n)
    return P[:, 0]


def _paper_rate(m):
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_rates.txt")
    for line in open(path):
        f = line.split()
        if f and f[0] == "varspeed_1d" and float(f[1]) == 0.5:
            return float(f[2 + m])
    raise KeyError


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_variable_speed_1d_converges_at_the_paper_rates(m):
    """Self-convergence (K = 16, 32 against K = 128) at nu = 0.5 matches the
    paper's printed rates for this coefficient within 0.5."""
    T = 1.6
    fine = _run_1d(m, 128, T)
    errs = []
    for K in (16, 32):
        coarse = _run_1d(m, K, T)
        errs.append(np.sqrt(np.mean((coarse - fine[:: 128 // K]) ** 2)))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - _paper_rate(m)) <= 0.5, (errs, rate, _paper_rate(m))


@pytest.mark.parametrize("d,m", [(1, 3), (2, 1), (2, 3), (3, 1), (3, 2)])
def test_laplacian_powers_of_a_cell_polynomial_end_at_d_m(d, m):
    """Lap^k of a polynomial of degree 2m+1 in each of d variables vanishes
    for k > d m and not before (each D_l^2 lowers one variable's degree by
    two), so the variable-kappa series length kmax_var = d m is the last k
    at which the constant-coefficient series has a nonzero term."""
    rng = np.random.default_rng(40 + 10 * d + m)
    c = rng.uniform(-1.0, 1.0, size=(1,) + (2 * m + 2,) * d)
    h = rng.uniform(0.5, 2.0, size=d)
    assert H.kmax_var(d, m) == d * m
    for _ in range(d * m):
        c = H._laplacian(c, h, d, 1)
    assert np.abs(c).max() > 0.0                   # Lap^{dm} of a full cell polynomial
    assert not np.any(H._laplacian(c, h, d, 1))    # Lap^{dm+1} == 0 exactly


@pytest.mark.parametrize("d,m,K", [(2, 1, (4, 3)), (2, 2, (3, 3)), (3, 1, (3, 3, 2))])
def test_variable_kappa_updates_sum_exactly_kmax_terms(d, m, K, monkeypatch):
    """With non-constant kappa the recurrence does not terminate, so the
    series length changes the result: the half-steps sum k = 0..kmax_var
    (one term fewer or more gives a different update)."""
    rng = np.random.default_rng(60 + 10 * d + m)
    L = (1.0,) * d
    prob = oracle.Problem(d, m, K, L, 0.0, 1.0).with_dt(0.5 / max(K) / np.sqrt(1.6))
    Kp = inputs.kappa_sines(d, m, K, L, (0.35, 0.25, 0.2)[:d], (1, 1, 1)[:d], "primal")
    Ku = inputs.kappa_sines(d, m, K, L, (0.35, 0.25, 0.2)[:d], (1, 1, 1)[:d], "dual")
    P, U = inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d)
    ref_p, ref_u = H.p_half_var(prob, P, U, Kp), H.u_half_var(prob, U, P, Ku)
    for km in (d * m - 1, d * m + 1):
        monkeypatch.setattr(H, "kmax_var", lambda dd, mm, km=km: km)
        assert np.abs(H.p_half_var(prob, P, U, Kp) - ref_p).max() > 1e-14 * np.abs(ref_p).max()
        assert np.abs(H.u_half_var(prob, U, P, Ku) - ref_u).max() > 1e-14 * np.abs(ref_u).max()
