"""The exact solution of the 3D Gaussian-pulse workload (the reference for
its FP64 discretization error): spherical means summed over periodic images.

* at t = 0 it is the workload's initial pressure (the minimum-image product
  Gaussian of gaussian_pulse);
* it solves p_tt = Lap p (fourth-order finite differences in t and x);
* p_t(0) = 0 (the workload starts with u = 0);
* at the centre it matches the closed form (1 - 2 t^2/w^2) exp(-t^2/w^2)
  and is continuous there.
"""

import numpy as np

from paper_1808_10481_amd import inputs

W = 0.05
C = (0.31, 0.62, 0.47)


def _pts(rng, n):
    return rng.uniform(0.0, 1.0, size=(n, 3))


def test_initial_value_is_the_workload_pulse():
    K, m = 16, 2
    P0 = inputs.gaussian_pulse(3, m, (K,) * 3, (1.0,) * 3, C, W)
    x = np.arange(K) / K
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1)
    ex = inputs.pulse_exact_3d(X, C, W, 0.0)
    np.testing.assert_allclose(ex, P0[..., 0, 0, 0], rtol=0, atol=1e-14)


def test_solves_the_wave_equation():
    rng = np.random.default_rng(3)
    pts = np.array(C) + rng.uniform(-0.15, 0.15, size=(40, 3))
    e = 1e-3
    for t in (0.05, 0.3, 0.9):
        f = lambda s, q=pts: inputs.pulse_exact_3d(q, C, W, s)
        ptt = (-f(t + 2 * e) + 16 * f(t + e) - 30 * f(t) + 16 * f(t - e) - f(t - 2 * e)) / (12 * e * e)
        lap = np.zeros(len(pts))
        for k in range(3):
            dk = np.zeros(3)
            dk[k] = e
            g = lambda s: inputs.pulse_exact_3d(pts + s * dk / e, C, W, t)
            lap += (-g(2 * e) + 16 * g(e) - 30 * g(0.0) + 16 * g(-e) - g(-2 * e)) / (12 * e * e)
        scale = np.abs(ptt).max() + 1.0
        assert np.abs(ptt - lap).max() < 2e-4 * scale, (t, np.abs(ptt - lap).max(), scale)


def test_starts_at_rest_and_is_regular_at_the_centre():
    rng = np.random.default_rng(4)
    pts = _pts(rng, 50)
    e = 1e-4
    pt0 = (inputs.pulse_exact_3d(pts, C, W, e) - inputs.pulse_exact_3d(pts, C, W, -e)) / (2 * e)
    assert np.abs(pt0).max() < 1e-9
    t = 0.04
    centre = inputs.pulse_exact_3d(np.array([C]), C, W, t)[0]
    near = inputs.pulse_exact_3d(np.array([C]) + np.array([[1e-6, 0, 0]]), C, W, t)[0]
    assert abs(centre - (1 - 2 * t * t / W ** 2) * np.exp(-t * t / W ** 2)) < 1e-12
    assert abs(near - centre) < 1e-6
