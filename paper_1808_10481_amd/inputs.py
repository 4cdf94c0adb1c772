"""Seeded synthetic inputs: closed-form fields sampled as scaled Taylor data.

This module holds no arithmetic of the time-stepping method itself; it only
samples given closed-form functions and their exact derivatives at grid nodes
in the data format of the scheme (value and first m derivatives per
dimension, scaled by h^a / a!; Sec. 2 and Sec. 5 of the paper).  Both the HIP
path's tests and the oracle's tests take their inputs from here.

Host layout of every array: C order, node axes (x_1..x_d) then coefficient
axes (a_1..a_d); velocity arrays have a leading component axis.  Primal node
j sits at x = j*h, dual node q at x = (q + 1/2)*h, on the periodic box
[0, length) (K nodes per grid), or on the walled box [0, length] (primal
j = 0..K, dual q = 0..K-1).
"""

from __future__ import annotations

from dataclasses import dataclass
from math import factorial, pi, sqrt

import numpy as np


# ---------------------------------------------------------------------------
# 1D scaled derivative data of elementary functions
# ---------------------------------------------------------------------------
def scaled_sin(x, a, phase, h, m):
    """Rows n = 0..m of (h^n / n!) d^n/dx^n sin(a x + phase) at points x."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape + (m + 1,), dtype=np.float64)
    for n in range(m + 1):
        out[..., n] = (h * a) ** n / factorial(n) * np.sin(a * x + phase + n * pi / 2)
    return out


def scaled_gauss(s, w, h, m):
    """Rows n = 0..m of (h^n/n!) d^n/ds^n exp(-(s/w)^2), via the physicists'
    Hermite polynomials: d^n/ds^n e^{-y^2} = (-1)^n H_n(y) e^{-y^2}, y = s/w."""
    y = np.asarray(s, dtype=np.float64) / w
    g = np.exp(-y * y)
    out = np.empty(y.shape + (m + 1,), dtype=np.float64)
    Hm1, H0 = np.zeros_like(y), np.ones_like(y)
    for n in range(m + 1):
        out[..., n] = (h / w) ** n / factorial(n) * (-1) ** n * H0 * g
        Hm1, H0 = H0, 2 * y * H0 - 2 * n * Hm1
    return out


def outer(factors):
    """Tensor product of per-dimension data f_k with shape (K_k, m+1):
    result[j_1..j_d, a_1..a_d] = prod_k f_k[j_k, a_k]."""
    d = len(factors)
    res = np.ones((1,) * (2 * d), dtype=np.float64)
    for k, f in enumerate(factors):
        shape = [1] * (2 * d)
        shape[k] = f.shape[0]
        shape[d + k] = f.shape[1]
        res = res * f.reshape(shape)
    return np.ascontiguousarray(res)


# ---------------------------------------------------------------------------
# Closed-form solutions of p_t = -kappa div u, u_t = -grad p
# ---------------------------------------------------------------------------
def standing_mode(d, m, K, length, waves, t_p, t_u, kappa=1.0):
    """Product standing mode  p = cos(w t) prod_k sin(a_k x_k),
    u_i = -(sin(w t)/w) a_i cos(a_i x_i) prod_{k!=i} sin(a_k x_k),
    a_k = 2 pi waves_k / length_k, w = sqrt(kappa) |a|.
    Returns (P at t_p on primal nodes, U at t_u on dual nodes)."""
    K = tuple(int(k) for k in K)
    length = tuple(float(v) for v in length)
    h = [length[k] / K[k] for k in range(d)]
    a = [2 * pi * waves[k] / length[k] for k in range(d)]
    w = sqrt(kappa) * sqrt(sum(x * x for x in a))
    xp = [np.arange(K[k]) * h[k] for k in range(d)]
    xd = [(np.arange(K[k]) + 0.5) * h[k] for k in range(d)]
    P = np.cos(w * t_p) * outer([scaled_sin(xp[k], a[k], 0.0, h[k], m) for k in range(d)])
    U = np.empty((d,) + P.shape, dtype=np.float64)
    for i in range(d):
        fac = [scaled_sin(xd[k], a[k], pi / 2 if k == i else 0.0, h[k], m) for k in range(d)]
        U[i] = -(np.sin(w * t_u) / w) * a[i] * outer(fac)
    return P, U


def box_mode(d, m, K, length, waves, t_p, t_u, kappa=1.0, ghosts=False):
    """Standing mode of the box with p = 0 on its faces:
    p = cos(w t) prod_k sin(a_k x_k),
    u_i = -(sin(w t)/w) a_i cos(a_i x_i) prod_{k!=i} sin(a_k x_k),
    a_k = pi waves_k / length_k, w = sqrt(kappa) |a|.  P at t_p on the K+1
    primal nodes, U at t_u on the K dual nodes (with ghosts: on q = -1..K,
    the closed form evaluated at the ghost positions)."""
    K = tuple(int(k) for k in K)
    length = tuple(float(v) for v in length)
    h = [length[k] / K[k] for k in range(d)]
    a = [pi * waves[k] / length[k] for k in range(d)]
    w = sqrt(kappa) * sqrt(sum(x * x for x in a))
    xp = [np.arange(K[k] + 1) * h[k] for k in range(d)]
    g = 1 if ghosts else 0
    xd = [(np.arange(-g, K[k] + g) + 0.5) * h[k] for k in range(d)]
    P = np.cos(w * t_p) * outer([scaled_sin(xp[k], a[k], 0.0, h[k], m) for k in range(d)])
    U = np.empty((d,) + tuple(len(x) for x in xd) + (m + 1,) * d, dtype=np.float64)
    for i in range(d):
        fac = [scaled_sin(xd[k], a[k], pi / 2 if k == i else 0.0, h[k], m) for k in range(d)]
        U[i] = -(np.sin(w * t_u) / w) * a[i] * outer(fac)
    return P, U


def gaussian_pulse(d, m, K, length, center, width):
    """p0 = prod_k exp(-(s_k/width)^2), s_k the minimum-image distance of x_k to
    center_k on the periodic box; returned as primal scaled data."""
    K = tuple(int(k) for k in K)
    fac = []
    for k in range(d):
        L = float(length[k])
        h = L / K[k]
        x = np.arange(K[k]) * h
        s = np.mod(x - center[k] + 0.5 * L, L) - 0.5 * L
        fac.append(scaled_gauss(s, width, h, m))
    return outer(fac)


def pulse_exact_3d(points, center, width, t, length=1.0, images=2):
    """Exact pressure at time t for p_t = -div u, u_t = -grad p in 3D with
    p(0) = exp(-r^2/width^2), u(0) = 0 (so p_t(0) = 0), unit speed.  The
    radial solution r p(r, t) solves the 1D wave equation (spherical means),
        p(r, t) = [(r - t) G(r - t) + (r + t) G(r + t)] / (2 r),
        G(s) = exp(-s^2/width^2),  p(0, t) = (1 - 2 t^2/width^2) G(t),
    and the periodic box's solution is its sum over the images of the centre
    within `images` box lengths per axis (the Gaussian's overlap with the box
    boundary, exp(-(L/2w)^2), is below rounding for the widths used here).
    points: array (..., 3) of positions."""
    pts = np.asarray(points, dtype=np.float64)
    c = np.asarray(center, dtype=np.float64)
    out = np.zeros(pts.shape[:-1], dtype=np.float64)
    w2 = float(width) ** 2
    rng = range(-images, images + 1)
    for n0 in rng:
        for n1 in rng:
            for n2 in rng:
                dx = pts - (c + length * np.array([n0, n1, n2], dtype=np.float64))
                r = np.sqrt(np.sum(dx * dx, axis=-1))
                a, b = r - t, r + t
                with np.errstate(divide="ignore", invalid="ignore"):
                    v = (a * np.exp(-a * a / w2) + b * np.exp(-b * b / w2)) / (2.0 * r)
                small = r < 1e-12
                if np.any(small):
                    v[small] = (1.0 - 2.0 * t * t / w2) * np.exp(-t * t / w2)
                out += v
    return out


def point_source(d, m, K, length, center, width):
    """A compactly supported stand-in for a point source: the Gaussian of
    gaussian_pulse with a narrow width, kept on the primal nodes where its data
    are not negligible (1e-12 of the peak).  Returns (node tuples (k, d), their
    scaled data (k,) + (m+1,)*d)."""
    G = gaussian_pulse(d, m, K, length, center, width)
    mag = np.abs(G).reshape(G.shape[:d] + (-1,)).max(-1)
    mask = mag > 1e-12 * mag.max()
    return np.argwhere(mask), G[mask]


def ricker(f0, t0):
    """Ricker wavelet r(t) = (1 - 2 a) exp(-a), a = (pi f0 (t - t0))^2."""
    def r(t):
        a = (np.pi * f0 * (t - t0)) ** 2
        return (1.0 - 2.0 * a) * np.exp(-a)
    return r


def kappa_sines(d, m, K, length, amps, waves, grid="primal"):
    """Taylor data of kappa(x) = 1 + sum_k amps_k sin(2 pi waves_k x_k / length_k)
    (periodic, smooth, positive for sum |amps| < 1) to degree 2m+1 per
    variable, about the primal (x = j h) or dual (x = (q + 1/2) h) nodes:
    (K,)*d + (2m+2,)*d, kappa~_b = prod_k h_k^{b_k}/b_k! d^b kappa (node)."""
    K = tuple(int(k) for k in K)
    n = 2 * m + 2
    h = [float(length[k]) / K[k] for k in range(d)]
    off = 0.0 if grid == "primal" else 0.5
    out = np.zeros(K + (n,) * d)
    out[(Ellipsis,) + (0,) * d] = 1.0
    for k in range(d):
        x = (np.arange(K[k]) + off) * h[k]
        a = 2 * pi * waves[k] / float(length[k])
        f = amps[k] * scaled_sin(x, a, 0.0, h[k], 2 * m + 1)          # (K_k, n)
        shape = [1] * (2 * d)
        shape[k] = K[k]
        shape[d + k] = n
        sl = [slice(None)] * d + [0] * d
        sl[d + k] = slice(None)
        out[tuple(sl)] += f.reshape([K[k] if j == k else 1 for j in range(d)] + [n])
    return out


def scaled_tanh(s, w, h, n):
    """Rows k = 0..n of (h^k / k!) d^k/ds^k tanh(s / w), by the Taylor-series
    recurrence of T' = 1 - T^2: with T = sum_k t_k u^k about u = s/w,
    (k + 1) t_{k+1} = [k = 0] - sum_{j <= k} t_j t_{k-j}; the scaled
    coefficient of order k is t_k (h/w)^k."""
    t = [np.tanh(np.asarray(s, dtype=np.float64) / w)]
    for k in range(n):
        conv = sum(t[j] * t[k - j] for j in range(k + 1))
        t.append(((1.0 if k == 0 else 0.0) - conv) / (k + 1))
    return np.stack([t[k] * (h / w) ** k for k in range(n + 1)], axis=-1)


def _series_mul(a, b):
    """Truncated product of Taylor rows (last axis = order, same scaling)."""
    n = a.shape[-1]
    out = np.zeros(np.broadcast_shapes(a.shape, b.shape))
    for i in range(n):
        out[..., i:] += a[..., i:i + 1] * b[..., :n - i]
    return out


def layered_speed(c0, jumps, positions, width):
    """A smooth layered medium in the last coordinate y:
    c(y) = c0 + sum_i jumps_i (1 + tanh((y - y_i) / width)) / 2; jumps summing
    to zero make it periodic on [0, 1) up to the tanh tails."""
    return dict(c0=float(c0), jumps=[float(v) for v in jumps], positions=[float(v) for v in positions],
                width=float(width))


def kappa_layers(d, m, K, length, medium, grid="primal"):
    """Taylor data of kappa = c(y)^2 (c from layered_speed, y = x_d) to degree
    2m+1 per variable about the primal or dual nodes: (K,)*d + (2m+2,)*d; the
    coefficients of order > 0 in the other variables are zero."""
    K = tuple(int(k) for k in K)
    n = 2 * m + 2
    L = float(length[d - 1])
    h = L / K[d - 1]
    off = 0.0 if grid == "primal" else 0.5
    y = (np.arange(K[d - 1]) + off) * h
    c = np.zeros((K[d - 1], n))
    c[:, 0] = medium["c0"]
    for dj, yi in zip(medium["jumps"], medium["positions"]):
        th = scaled_tanh(y - yi * L, medium["width"] * L, h, n - 1)
        c[:, 0] += 0.5 * dj
        c += 0.5 * dj * th
    kap = _series_mul(c, c)                                             # (K_d, n)
    out = np.zeros(K + (n,) * d)
    idx = (slice(None),) * d + (0,) * (d - 1) + (slice(None),)
    out[idx] = kap.reshape((1,) * (d - 1) + (K[d - 1], n))
    return out


def kappa_box(d, m, K, length, amps, grid="primal"):
    """Taylor data of kappa(x) = 1 + sum_k amps_k cos(pi x_k / length_k) on the
    walled box [0, length] (even about every wall, so the odd reflection of p
    stays a solution): about the K+1 primal nodes x = j h or the K dual nodes
    x = (q + 1/2) h per dimension, to degree 2m+1 per variable."""
    K = tuple(int(k) for k in K)
    n = 2 * m + 2
    h = [float(length[k]) / K[k] for k in range(d)]
    cnt = [k + 1 if grid == "primal" else k for k in K]
    off = 0.0 if grid == "primal" else 0.5
    out = np.zeros(tuple(cnt) + (n,) * d)
    out[(Ellipsis,) + (0,) * d] = 1.0
    for k in range(d):
        x = (np.arange(cnt[k]) + off) * h[k]
        f = amps[k] * scaled_sin(x, pi / float(length[k]), pi / 2, h[k], 2 * m + 1)
        sl = [slice(None)] * d + [0] * d
        sl[d + k] = slice(None)
        out[tuple(sl)] += f.reshape([cnt[k] if j == k else 1 for j in range(d)] + [n])
    return out


def random_data(rng, d, m, K, ncomp=None):
    """Uniform[-1,1] scaled data (any data is valid input to the linear scheme)."""
    shape = tuple(int(k) for k in K) + (m + 1,) * d
    if ncomp is not None:
        shape = (ncomp,) + shape
    return rng.uniform(-1.0, 1.0, size=shape)


def zero_on_walls(P, d):
    """Pressure data on the K+1 primal nodes of a walled box with p = 0 on the
    faces: at a node on the wall normal to x_k every coefficient of even order
    a_k is zero (p odd across the wall).  Returns a copy."""
    P = np.array(P, dtype=np.float64, copy=True)
    for k in range(d):
        for j in (0, P.shape[k] - 1):
            idx = [slice(None)] * (2 * d)
            idx[k] = j
            idx[d + k] = slice(0, None, 2)
            P[tuple(idx)] = 0.0
    return P


# ---------------------------------------------------------------------------
# Workloads (seeded recipes)
# ---------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    d: int
    m: int
    K: tuple
    length: tuple
    nu: float
    kappa: float
    steps: int
    P0: np.ndarray | None = None
    U0: np.ndarray | None = None      # U at t0 + dt/2, or U(t0) when startup
    startup: bool = False
    exact: object = None              # callable(t) -> P at time t, or None
    boundary: str = "periodic"        # or "walls" (p = 0 on the box faces)

    @property
    def h(self):
        return tuple(self.length[k] / self.K[k] for k in range(self.d))

    @property
    def dt(self):
        return self.nu * min(self.h) / sqrt(self.kappa)

    @property
    def cells(self):
        return int(np.prod(self.K))


def standing_wave_1d(K=200, m=1, nu=0.5, T=1.0, make_data=True):
    """p_t + u_x = 0, u_t + p_x = 0 on periodic [0,1); p0 = sin(2 pi x),
    u at dt/2 from the exact standing wave; run to T."""
    wl = Workload("standing_wave_1d", 1, m, (K,), (1.0,), nu, 1.0, 0)
    wl.steps = int(round(T / wl.dt))
    if make_data:
        wl.P0, wl.U0 = standing_mode(1, m, wl.K, wl.length, (1,), 0.0, wl.dt / 2)
        wl.exact = lambda t: standing_mode(1, m, wl.K, wl.length, (1,), t, t)[0]
    return wl


def standing_mode_2d(seed=1, K=1024, m=3, nu=0.5, steps=1000, make_data=True):
    """sin(2 pi k x) sin(2 pi l y) standing mode on the periodic unit square,
    (k, l) seeded in [1, 8]."""
    rng = np.random.default_rng(seed)
    kl = tuple(int(v) for v in rng.integers(1, 9, 2))
    wl = Workload("standing_mode_2d", 2, m, (K, K), (1.0, 1.0), nu, 1.0, steps)
    wl.waves = kl
    if make_data:
        wl.P0, wl.U0 = standing_mode(2, m, wl.K, wl.length, kl, 0.0, wl.dt / 2)
        wl.exact = lambda t: standing_mode(2, m, wl.K, wl.length, kl, t, t)[0]
    return wl


def gaussian_pulse_walls_2d(seed=3, K=1024, m=3, nu=0.5, steps=1000, make_data=True):
    """Gaussian pressure pulse exp(-r^2/0.002) in the walled square [0, 2]^2
    (the [-1, 1]^2 box shifted), centre 0.3 from the centre of the box plus a
    seeded offset of at most 0.05 per axis, u(t0) = 0 (start-up builds u at
    dt/2).  At the walls the pulse is below 1e-100; its even coefficients on
    the wall nodes are set to zero so the data satisfy p = 0 there exactly."""
    rng = np.random.default_rng(seed)
    center = tuple(1.3 + 0.05 * float(v) for v in rng.uniform(-1, 1, 2))
    wl = Workload("gaussian_pulse_walls_2d", 2, m, (K, K), (2.0, 2.0), nu, 1.0, steps)
    wl.center = center
    wl.startup = True
    wl.boundary = "walls"
    if make_data:
        h = 2.0 / K
        x = np.arange(K + 1) * h
        width = sqrt(0.002)
        P = outer([scaled_gauss(x - center[k], width, h, m) for k in range(2)])
        wl.P0 = zero_on_walls(P, 2)
        wl.U0 = np.zeros((2, K, K) + (m + 1,) * 2)
    return wl


def gaussian_pulse_3d(seed=2, K=256, m=2, nu=0.5, steps=500, width=0.05, make_data=True):
    """Gaussian pressure pulse of the given width at a seeded centre of the
    periodic unit cube, u(t0) = 0 (the start-up builds u at dt/2)."""
    rng = np.random.default_rng(seed)
    center = tuple(float(v) for v in rng.random(3))
    wl = Workload("gaussian_pulse_3d", 3, m, (K, K, K), (1.0, 1.0, 1.0), nu, 1.0, steps)
    wl.center = center
    wl.startup = True
    if make_data:
        wl.P0 = gaussian_pulse(3, m, wl.K, wl.length, center, width)
        wl.U0 = np.zeros((3,) + wl.P0.shape)
    return wl
