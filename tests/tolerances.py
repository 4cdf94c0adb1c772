"""Tolerances of the GPU parity tests (HIP path against the FP64 oracle).

FP64: relative L2 <= 1e-12 and max |diff| <= 1e-11 max |ref|
(only summation order differs).  FP32: every output is the input minus a
sum of n ~ (2m+2)^d rounded products (tables rounded to FP32 too); with
random rounding the sum's error grows like sqrt(n) u, u = 2^-24, times the
size of the terms, which for random (non-smooth) data exceeds the result by
a factor up to ~16.  Bound used: relative L2 <= 16 sqrt(n) u_32 * 16 =
256 sqrt(n) 2^-24 (about 1.2e-5 for d = 2, m = 5), max <= 4x that.
FP32_COMP: FP64 arithmetic, then the result is stored as hi + lo with
|x - hi| <= 2^-24 |x| and lo the BF16 rounding of x - hi (relative error
2^-9), so every stored entry is within 2^-33 |x| of the FP64 result; bound
used: relative L2 and max |diff| / max |ref| <= 2^-32 + 1e-12.
"""

import numpy as np

from oracle.diagnostics import rel_l2


def _close(got, ref, tol_l2, tol_max):
    r = rel_l2(got, ref)
    mx = np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)
    assert r <= tol_l2 and mx <= tol_max, (r, mx)
    return r


TOL = {"fp64": (1e-12, 1e-11), "fp32": (3e-6, 1e-5)}


COMP_TOL = 2.0 ** -32 + 1e-12


def tol(prec, d, m):
    if prec == "fp64":
        return TOL["fp64"]
    if prec == "fp32_comp":
        return (COMP_TOL, COMP_TOL)
    t = 256.0 * np.sqrt((2 * m + 2) ** d) * 2.0 ** -24
    return (t, 4 * t)


def fp32_steps(d, m, nhalf):
    """FP32 after `nhalf` half-steps of smooth data (closed-form fields well
    resolved by the grid, nu <= 1).  Each half-step adds to the stored state
    x the sum of n = (2m+2)^d rounded products whose total is the increment;
    for smooth data the products and the increment are no larger than x, so
    one half-step contributes at most u (rounding the stored result) plus
    sqrt(n) u (the sum, random rounding, tables rounded to FP32), relative
    to the state, u = 2^-24.  The scheme is neutral (its step matrix has
    unit-modulus eigenvalues, nothing is damped), so the contributions of
    the half-steps add up rather than decay: bound nhalf (1 + sqrt(n)) u,
    times 4 for the spread of the scaled coefficients' sizes; max |diff|
    4x that."""
    t = 4.0 * nhalf * (1.0 + np.sqrt((2 * m + 2) ** d)) * 2.0 ** -24
    return (t, 4 * t)


def comp_steps(d, m, nhalf):
    """FP32_COMP after `nhalf` half-steps of smooth data.  The arithmetic is
    FP64, so each half-step's error is the storage rounding of its result:
    every entry within 2^-33 of its value (hi the FP32 rounding, lo the BF16
    rounding of the residual), plus an FP64 sum of n = (2m+2)^d products.  As
    for FP32 the neutral scheme adds these up over the half-steps: bound
    4 nhalf (2^-33 + sqrt(n) 2^-53), the factor 4 for the spread of the scaled
    coefficients' sizes; max |diff| 4x that."""
    t = 4.0 * nhalf * (2.0 ** -33 + np.sqrt((2 * m + 2) ** d) * 2.0 ** -53)
    return (t, 4 * t)

