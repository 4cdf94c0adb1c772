"""Pins of the source-term reading (midpoint rule, oracle step_with_source):
a spatially uniform source reproduces the exact solution p = int r dt, u = 0
(exactly for constant r, at second order in dt for r = cos(w t), which fails
with the source evaluated at t_n instead of t_n + dt/2)."""

import numpy as np

import oracle
from oracle import hermite_lf as H


def _uniform_g(prob):
    G = np.zeros(prob.p_shape())
    G[(Ellipsis,) + (0,) * prob.d] = 1.0          # g = 1: value 1, derivatives 0
    return G


def test_constant_uniform_source_is_exact():
    prob = oracle.Problem(2, 2, (6, 5), (1.0, 1.0), 0.03, 1.3)
    G = _uniform_g(prob)
    P, U = H.step_with_source(prob, np.zeros(prob.p_shape()), np.zeros(prob.u_shape()), G, lambda t: 2.0, 0.0, 7)
    assert np.allclose(P[..., 0, 0], 2.0 * 7 * prob.dt, rtol=0, atol=1e-14)
    assert np.abs(P[..., 1:, :]).max() < 1e-14 and np.abs(P[..., :, 1:]).max() < 1e-14
    assert np.abs(U).max() < 1e-14


def test_time_dependent_uniform_source_is_second_order():
    w, T = 3.0, 1.0
    errs = []
    for n in (10, 20, 40):
        prob = oracle.Problem(1, 1, (4,), (1.0,), T / n, 1.0)
        G = _uniform_g(prob)
        P, _ = H.step_with_source(prob, np.zeros(prob.p_shape()), np.zeros(prob.u_shape()), G,
                                  lambda t: np.cos(w * t), 0.0, n)
        errs.append(abs(P[0, 0] - np.sin(w * T) / w))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.9) and np.all(rates < 2.1), (errs, rates)
