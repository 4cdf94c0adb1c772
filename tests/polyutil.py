"""Test-side polynomial tools, written independently of the oracle.

* Dense monomial tensors (numpy.polynomial): exact solutions of
  p_t = -kappa div u, u_t = -grad p for polynomial data, obtained by running
  the PDE's time-derivative recurrence (the series terminates), and sampling
  of scaled Taylor data at points.
* Exact rational polynomials (dict exponent -> Fraction) for brute force on
  tiny grids: direct multivariate Hermite interpolation by solving the full
  interpolation system, and the exact leapfrog difference of the PDE solution.
"""

from __future__ import annotations

import itertools
from fractions import Fraction
from math import comb, factorial

import numpy as np
from numpy.polynomial import polynomial as npp


# ---------------------------------------------------------------------------
# Dense FP64 monomial tensors c[i_1, ..., i_d] x_1^{i_1} ... x_d^{i_d}
# ---------------------------------------------------------------------------
def pder(c, axis, order=1):
    """Derivative along an axis, padded back to the same shape."""
    if order == 0:
        return np.array(c, copy=True)
    out = np.zeros_like(c)
    dc = npp.polyder(c, m=order, axis=axis)
    sl = [slice(None)] * c.ndim
    sl[axis] = slice(0, dc.shape[axis])
    out[tuple(sl)] = dc
    return out


def peval(c, point):
    """Evaluate sum_i c[i] prod_k x_k^{i_k} at a point."""
    v = np.asarray(c, dtype=float)
    for k, x in enumerate(point):
        pw = float(x) ** np.arange(v.shape[0])
        v = np.tensordot(pw, v, axes=(0, 0))
    return float(v)


def scaled_data(c, point, h, m):
    """(m+1,)*d array: prod_k h_k^{a_k}/a_k! * d^a q(point)."""
    d = c.ndim
    out = np.empty((m + 1,) * d)
    for a in itertools.product(range(m + 1), repeat=d):
        q = c
        for k in range(d):
            q = pder(q, k, a[k])
        scale = np.prod([h[k] ** a[k] / factorial(a[k]) for k in range(d)])
        out[a] = scale * peval(q, point)
    return out


def random_poly(rng, d, deg):
    return rng.uniform(-1.0, 1.0, size=(deg + 1,) * d)


def time_series(p0, u0, kappa):
    """Time derivatives at t = 0 of the exact solution, from the PDE:
    P_{j+1} = -kappa sum_i d_i U_{i,j},  U_{i,j+1} = -d_i P_j."""
    d = p0.ndim
    P, U = [np.array(p0, dtype=float)], [[np.array(u, dtype=float) for u in u0]]
    while True:
        Pn = -kappa * sum(pder(U[-1][i], i) for i in range(d))
        Un = [-pder(P[-1], i) for i in range(d)]
        if not np.any(Pn) and not any(np.any(x) for x in Un):
            break
        P.append(Pn)
        U.append(Un)
    return P, U


def at_time(series, t):
    """sum_j t^j / j! S_j (series of arrays, or of lists of arrays)."""
    out = None
    for j, s in enumerate(series):
        f = t ** j / factorial(j)
        term = [f * x for x in s] if isinstance(s, list) else f * s
        if out is None:
            out = term
        elif isinstance(term, list):
            out = [a + b for a, b in zip(out, term)]
        else:
            out = out + term
    return out


# ---------------------------------------------------------------------------
# Exact rational polynomials in local variables xi_k = (x_k - centre_k)/h_k
# ---------------------------------------------------------------------------
def _fr(x):
    return x if isinstance(x, Fraction) else Fraction(x)


def solve_exact(A, b):
    """Gaussian elimination in Fractions (A square, nonsingular)."""
    n = len(A)
    M = [list(map(_fr, A[i])) + [_fr(b[i])] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(col + 1, n):
            if M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    x = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        s = M[r][n] - sum(M[r][c] * x[c] for c in range(r + 1, n))
        x[r] = s / M[r][r]
    return x


def hermite_interpolant_exact(corner_data, d, m):
    """Direct multivariate Hermite interpolation on one cell.

    corner_data[e][a] (e in {0,1}^d corner of the cell at xi = e - 1/2,
    a in {0..m}^d) are scaled data (1/a!) d^a_xi q at the corner.  Solves the
    full (2m+2)^d square system for q = sum_b c_b xi^b; returns {b: c_b}.
    """
    n = 2 * m + 2
    betas = list(itertools.product(range(n), repeat=d))
    rows, rhs = [], []
    for e in itertools.product((0, 1), repeat=d):
        xi0 = [Fraction(2 * ek - 1, 2) for ek in e]
        for a in itertools.product(range(m + 1), repeat=d):
            row = []
            for b in betas:
                v = Fraction(1)
                for k in range(d):
                    if b[k] < a[k]:
                        v = Fraction(0)
                        break
                    v *= comb(b[k], a[k]) * xi0[k] ** (b[k] - a[k])
                row.append(v)
            rows.append(row)
            rhs.append(corner_data[e][a])
    sol = solve_exact(rows, rhs)
    return {b: c for b, c in zip(betas, sol) if c != 0}


def rpoly_deriv(p, k, h_k):
    """d/dx_k of a polynomial in xi (xi_k = (x_k - c_k)/h_k)."""
    out = {}
    for b, c in p.items():
        if b[k] > 0:
            nb = b[:k] + (b[k] - 1,) + b[k + 1:]
            out[nb] = out.get(nb, Fraction(0)) + c * b[k] / h_k
    return {b: c for b, c in out.items() if c != 0}


def rpoly_add(p, q, s=Fraction(1)):
    out = dict(p)
    for b, c in q.items():
        out[b] = out.get(b, Fraction(0)) + s * c
    return {b: c for b, c in out.items() if c != 0}


def leapfrog_difference_exact(p_mid, u_mid, h, kappa, dt):
    """For the exact PDE solution with p(tau) = p_mid, u(tau) = u_mid
    (polynomials in xi), return (p(tau + dt/2) - p(tau - dt/2),
    [u_i(tau + dt/2) - u_i(tau - dt/2)]), from the terminating time series."""
    d = len(h)
    P, U = [p_mid], [list(u_mid)]
    while True:
        Pn = {}
        for i in range(d):
            Pn = rpoly_add(Pn, rpoly_deriv(U[-1][i], i, h[i]), -_fr(kappa))
        Un = [{b: -c for b, c in rpoly_deriv(P[-1], i, h[i]).items()} for i in range(d)]
        if not Pn and not any(Un):
            break
        P.append(Pn)
        U.append(Un)
    half = _fr(dt) / 2
    dp, du = {}, [{} for _ in range(d)]
    for j in range(len(P)):
        f = (half ** j - (-half) ** j) / factorial(j)
        if f == 0:
            continue
        dp = rpoly_add(dp, P[j], f)
        for i in range(d):
            du[i] = rpoly_add(du[i], U[j][i], f)
    return dp, du


def mul_affine(c, k0, kgrad):
    """(k0 + sum_k kgrad_k x_k) * q for a dense monomial tensor q, grown by
    one in every axis that kgrad touches (padded shape: +1 per axis)."""
    d = c.ndim
    out = np.zeros(tuple(n + 1 for n in c.shape))
    out[tuple(slice(0, n) for n in c.shape)] += k0 * c
    for k in range(d):
        if kgrad[k] != 0.0:
            sl = [slice(0, n) for n in c.shape]
            sl[k] = slice(1, c.shape[k] + 1)
            out[tuple(sl)] += kgrad[k] * c
    return out


def time_series_affine(p0, u0, k0, kgrad, nmax=64):
    """Time derivatives at t = 0 of the exact solution of
    p_t = -kappa div u, u_t = -grad p with kappa = k0 + kgrad . x, from the
    PDE's own recurrence on monomials; terminates when the data have total
    degree low enough (every kappa-multiplication is followed by derivatives
    that lower the total degree)."""
    d = p0.ndim
    size = p0.shape[0] + nmax

    def pad(c):
        out = np.zeros((size,) * d)
        out[tuple(slice(0, n) for n in c.shape)] = c
        return out

    P, U = [pad(p0)], [[pad(u) for u in u0]]
    for _ in range(nmax):
        div = sum(pder(U[-1][i], i) for i in range(d))
        Pn = -mul_affine(div, k0, kgrad)[tuple(slice(0, size) for _ in range(d))]
        Un = [-pder(P[-1], i) for i in range(d)]
        if not np.any(Pn) and not any(np.any(x) for x in Un):
            return P, U
        P.append(Pn)
        U.append(Un)
    raise RuntimeError("series did not terminate")
