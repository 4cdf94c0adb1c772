"""The layered-medium kappa generator (seeded input of the batched-shot
workload): Taylor data of c(y)^2 for a sum of smoothed tanh steps.

* the first three tanh derivatives match their closed forms;
* the Taylor polynomial about each node predicts c(y + delta)^2 with an error
  falling like delta^(2m+2) (the data are the exact scaled derivatives);
* zero jumps give the constant c0^2; the data depend on y only.
"""

import numpy as np

from paper_1808_10481_amd import inputs


def test_tanh_derivatives_closed_forms():
    s = np.linspace(-0.3, 0.3, 9)
    w, h = 0.1, 0.01
    T = inputs.scaled_tanh(s, w, h, 5)
    th = np.tanh(s / w)
    se2 = 1.0 - th ** 2
    r = h / w
    assert np.allclose(T[:, 0], th, rtol=0, atol=1e-15)
    assert np.allclose(T[:, 1], r * se2, rtol=0, atol=1e-15)
    assert np.allclose(T[:, 2], r ** 2 / 2 * (-2 * th * se2), rtol=0, atol=1e-15)
    assert np.allclose(T[:, 3], r ** 3 / 6 * (-2 * se2 * (se2 - 2 * th ** 2)), rtol=0, atol=1e-15)


def _c(y, med):
    c = np.full_like(y, med["c0"])
    for dj, yi in zip(med["jumps"], med["positions"]):
        c += 0.5 * dj * (1 + np.tanh((y - yi) / med["width"]))
    return c


def test_taylor_data_predict_the_field_to_order_2m_plus_2():
    med = inputs.layered_speed(1.0, [1.2, 0.8, -2.0], [0.3, 0.55, 0.8], 0.04)
    m, K = 2, 64
    h = 1.0 / K
    kp = inputs.kappa_layers(2, m, (8, K), (1.0, 1.0), med, "primal")
    ku = inputs.kappa_layers(2, m, (8, K), (1.0, 1.0), med, "dual")
    assert np.all(kp[:, :, 1:, :] == 0) and np.all(kp[0] == kp[5])
    for data, off in ((kp, 0.0), (ku, 0.5)):
        coef = data[0, :, 0, :]                      # (K, 2m+2) along y
        y0 = (np.arange(K) + off) * h
        errs = []
        for frac in (0.1, 0.05):
            dlt = frac * h
            pred = sum(coef[:, k] * (dlt / h) ** k for k in range(2 * m + 2))
            errs.append(np.max(np.abs(pred - _c(y0 + dlt, med) ** 2)))
        rate = np.log2(errs[0] / errs[1])
        assert rate > 2 * m + 2 - 0.3, rate


def test_no_jumps_is_constant():
    med = inputs.layered_speed(1.7, [], [], 0.05)
    k = inputs.kappa_layers(2, 3, (5, 7), (1.0, 1.0), med)
    assert np.allclose(k[..., 0, 0], 1.7 ** 2) and np.count_nonzero(k) == 35
