"""Diagnostics for the oracle (test infrastructure only).

* ``rel_l2``        relative L2 over all coefficients.
* ``nodal_l2``      grid L2 norm of the nodal function values (the "L2 error"
                    of Sec. 4 is never defined in the paper; this reading uses
                    the value coefficient at every node, weighted by the cell
                    volume).
* ``conserved_1d``  the one-dimensional conserved quantity of Sec. 3.1.1,
                    eqs. (Ppmdef)-(Vpmdef), (Qdef)-(Rdef), (fullcons1d),
                    evaluated exactly by Gauss-Legendre quadrature on the
                    pieces of the piecewise-polynomial interpolants.
"""

from __future__ import annotations

from math import factorial

import numpy as np

from .hermite_lf import Problem, hermite_matrix


def rel_l2(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((x - ref).ravel()) / (den if den > 0 else 1.0))


def nodal_l2(prob: Problem, values, exact) -> float:
    """sqrt(prod h * sum_j (values_j - exact_j)^2) over nodes."""
    vol = float(np.prod(prob.h))
    diff = np.asarray(values, dtype=np.float64) - np.asarray(exact, dtype=np.float64)
    return float(np.sqrt(vol * np.sum(diff * diff)))


def _poly_deriv_values(c, order, xi, h):
    """order-th x-derivative of sum_s c[..., s] xi^s at xi (vector over pieces)."""
    n = c.shape[-1]
    out = np.zeros(xi.shape, dtype=np.float64)
    for s in range(order, n):
        fac = factorial(s) / factorial(s - order)
        out = out + c[..., s] * fac * xi ** (s - order)
    return out / h ** order


def conserved_1d(prob: Problem, P: np.ndarray, U: np.ndarray, which: str = "R") -> float:
    """Sobolev (m+1)-seminorm conserved quantity of the 1D scheme.

    The paper writes the system as p_t = c v_x, v_t = c p_x (Sec. 2); the
    system here is p_t = -kappa u_x, u_t = -p_x, so v = -c u with c =
    sqrt(kappa).  With S_pm f(x) = f(x pm c dt/2) (Sec. 3.1, eq. (Sdef)):

      which="R": state (P^n, U^{n+1/2}),
          R = |c u^h + S_+ p^h|^2_{m+1} + |c u^h - S_- p^h|^2_{m+1}
      which="Q": state (P^n, U^{n-1/2}),
          Q = |p^h + c S_+ u^h|^2_{m+1} + |p^h - c S_- u^h|^2_{m+1}

    p^h is the piecewise Hermite interpolant of the primal data (pieces
    [x_j, x_{j+1}]), u^h that of the dual data (pieces [x_{j-1/2}, x_{j+1/2}]).
    Q(n) = R(n+1/2) = Q(0) for all n (eq. (fullcons1d)).
    """
    assert prob.d == 1
    m, K = prob.m, prob.K[0]
    h = prob.h[0]
    c = np.sqrt(prob.kappa)
    a = c * prob.dt / 2.0                      # shift of S_pm
    H = hermite_matrix(m)
    # Piece coefficients in xi = (x - centre)/h.
    # p^h piece j: cell [x_j, x_{j+1}], centre x_{j+1/2}, corners P[j], P[j+1].
    Pn = np.asarray(P, dtype=np.float64)
    Un = np.asarray(U, dtype=np.float64)[0]
    cp = np.concatenate([Pn, np.roll(Pn, -1, axis=0)], axis=1) @ H.T
    # u^h piece j: cell [x_{j-1/2}, x_{j+1/2}], centre x_j, corners U[j-1], U[j].
    cu = np.concatenate([np.roll(Un, 1, axis=0), Un], axis=1) @ H.T
    gx, gw = np.polynomial.legendre.leggauss(m + 1)
    x = np.arange(K, dtype=np.float64) * h     # primal nodes, lo = 0 (shift-invariant)

    def field(kind, xs):
        """Evaluate the (m+1)-th derivative of p^h or u^h at points xs (periodic)."""
        L = K * h
        if kind == "p":                        # piece j covers [x_j, x_{j+1})
            j = np.floor(np.mod(xs, L) / h).astype(np.int64) % K
            xi = (np.mod(xs, L) - (j + 0.5) * h) / h
            return _poly_deriv_values(cp[j], m + 1, xi, h)
        # u piece j covers [x_j - h/2, x_j + h/2)
        xsh = np.mod(xs + 0.5 * h, L)
        j = np.floor(xsh / h).astype(np.int64) % K
        xi = (xsh - 0.5 * h - j * h) / h
        return _poly_deriv_values(cu[j], m + 1, xi, h)

    def seminorm_sq(f_of_x, breaks):
        """integral over one period of f^2, f piecewise polynomial of degree m
        between consecutive sorted breakpoints (exact with m+1 Gauss points)."""
        b = np.sort(np.mod(breaks, K * h))
        b = np.concatenate([b, [b[0] + K * h]])
        lo, hi = b[:-1], b[1:]
        keep = hi - lo > 1e-15 * h
        lo, hi = lo[keep], hi[keep]
        mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
        pts = mid[:, None] + half[:, None] * gx[None, :]
        vals = f_of_x(pts.ravel()).reshape(pts.shape)
        return float(np.sum(half[:, None] * gw[None, :] * vals * vals))

    dual_breaks = x + 0.5 * h
    if which == "R":
        f1 = lambda xs: c * field("u", xs) + field("p", xs + a)   # noqa: E731
        f2 = lambda xs: c * field("u", xs) - field("p", xs - a)   # noqa: E731
        b1 = np.concatenate([dual_breaks, x - a])
        b2 = np.concatenate([dual_breaks, x + a])
    elif which == "Q":
        f1 = lambda xs: field("p", xs) + c * field("u", xs + a)   # noqa: E731
        f2 = lambda xs: field("p", xs) - c * field("u", xs - a)   # noqa: E731
        b1 = np.concatenate([x, dual_breaks - a])
        b2 = np.concatenate([x, dual_breaks + a])
    else:
        raise ValueError(which)
    return seminorm_sq(f1, b1) + seminorm_sq(f2, b2)
