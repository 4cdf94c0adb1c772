"""Pins of the oracle's Hermite-Birkhoff interpolation (Sec. 2, eq. (interp);
Sec. 5 tensor-product reconstruction)."""

import itertools
import os
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import oracle
from oracle import hermite_lf as hl
import polyutil as pu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hermite_matrices.txt")


def _load_golden():
    mats, cur, m = {}, None, None
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if line.startswith("m "):
            m = int(line.split()[1])
            cur = mats.setdefault(m, [])
        else:
            cur.append([Fraction(x) for x in line.split()])
    return mats


@pytest.mark.parametrize("m", [0, 1])
def test_H_matches_hand_derived(m):
    """P1: H_0 and H_1 equal the matrices derived by hand from eq. (interp)."""
    assert oracle.hermite_matrix_exact(m) == _load_golden()[m]


@pytest.mark.parametrize("m", range(0, 8))
def test_H_inverts_interpolation_conditions(m):
    """P1: [C^L; C^R] H = I exactly, with C_{ls} = binom(s,l) xi0^{s-l}
    built here by substitution of the end points into the derivatives."""
    H = oracle.hermite_matrix_exact(m)
    n = 2 * m + 2
    for side, xi0 in enumerate((Fraction(-1, 2), Fraction(1, 2))):
        for l in range(m + 1):
            row = [comb(s, l) * xi0 ** (s - l) if s >= l else 0 for s in range(n)]
            for col in range(n):
                val = sum(row[s] * H[s][col] for s in range(n))
                assert val == (1 if col == side * (m + 1) + l else 0)


@pytest.mark.parametrize("m", range(0, 8))
def test_H_fp64_is_correctly_rounded(m):
    """Each FP64 entry is within half an ulp of the exact rational."""
    Hx = oracle.hermite_matrix_exact(m)
    Hf = oracle.hermite_matrix(m)
    for i, j in itertools.product(range(2 * m + 2), repeat=2):
        err = abs(Fraction(float(Hf[i, j])) - Hx[i][j])
        assert err <= Fraction(float(np.spacing(abs(Hf[i, j])))) / 2


@pytest.mark.parametrize("m", range(0, 6))
def test_H_parity_structure(m):
    """Symmetry xi -> -xi: even coefficients depend only on v^R_l + (-1)^l v^L_l
    type combinations; checked as H[s, L_l] = (-1)^(s+l) H[s, R_l]."""
    H = oracle.hermite_matrix_exact(m)
    for s in range(2 * m + 2):
        for l in range(m + 1):
            assert H[s][l] == (-1) ** (s + l) * H[s][m + 1 + l]


@pytest.mark.parametrize("d,m", [(1, 0), (1, 1), (1, 2), (1, 3), (1, 5),
                                 (2, 0), (2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_polynomial_reproduction(d, m):
    """P2: the tensor interpolant of corner data sampled from a polynomial of
    degree <= 2m+1 per variable reproduces it: the cell coefficients equal
    the polynomial's scaled Taylor coefficients at the cell centre."""
    rng = np.random.default_rng(100 + 10 * d + m)
    q = pu.random_poly(rng, d, 2 * m + 1)
    h = rng.uniform(0.2, 0.6, size=d)
    centre = rng.uniform(-0.5, 0.5, size=d)
    B = np.empty((2,) * d + (1,) + (m + 1,) * d)
    for e in itertools.product((0, 1), repeat=d):
        pt = centre + (np.array(e) - 0.5) * h
        B[e + (0,)] = pu.scaled_data(q, pt, h, m)
    c = hl._interpolate(B, oracle.hermite_matrix(m), d, 1)[0]
    expect = pu.scaled_data(q, centre, h, 2 * m + 1)
    np.testing.assert_allclose(c, expect, rtol=0, atol=1e-12 * np.abs(expect).max())


@pytest.mark.parametrize("m", [1, 2, 3])
def test_degree_2m_plus_2_is_not_reproduced(m):
    """The interpolant is exact only up to degree 2m+1: x^{2m+2} is not."""
    q = np.zeros(2 * m + 3)
    q[-1] = 1.0
    h = np.array([0.5])
    B = np.empty((2, 1, m + 1))
    for e in (0, 1):
        B[e, 0] = pu.scaled_data(q, np.array([e - 0.5]) * h, h, m)
    c = hl._interpolate(B, oracle.hermite_matrix(m), 1, 1)[0]
    assert abs(c[0]) > 1e-6   # x^{2m+2} has zero value at the centre
