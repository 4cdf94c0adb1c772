"""FP64 CPU oracle of the Hermite-leapfrog scheme (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.  Nothing here is shared with the HIP path.

System (the paper's pressure-velocity form, Sec. 4 and Sec. 5, with kappa = c^2
constant):

    p_t = -kappa * div(u),      u_t = -grad(p).

Data (Sec. 2 and Sec. 5): every node stores scaled Taylor data
    f~_alpha = prod_k h_k^{alpha_k} / alpha_k!  *  d^alpha f (node),
    alpha in {0..m}^d.
Pressure lives on the primal grid x_j = lo + j*h at integer time levels, every
velocity component on the dual grid x_{j+1/2} at half-integer levels (Sec. 2,
eqs. (pGrid), (dGrid); Sec. 5).  Dual index q sits at x_{q+1/2}.

Boundaries: periodic, or reflecting walls (Sec. 5, "Imposing reflective
boundary conditions", eq. (Boundary)): p = 0 on every face of the box
[0, L_1] x ... x [0, L_d].  Then the primal grid has K+1 nodes per dimension
(j = 0..K, the end nodes on the walls), the dual grid K (q = 0..K-1).  Before
the pressure half-step one layer of ghost dual nodes (q = -1 and q = K) is
filled by mirroring the velocity polynomials across the wall: p odd across the
wall makes grad p's normal component even and its tangential components odd,
so by u_t = -grad p the normal velocity component is mirrored evenly and the
tangential ones oddly.  Mirroring a scaled Taylor coefficient across a wall
normal to x_k multiplies it by (-1)^{a_k}, times -1 for an odd mirror.  The
velocity half-step reads primal nodes only and needs no ghosts.

One step (P^n, U^{n+1/2}) -> (P^{n+1}, U^{n+3/2}) is a p half-step followed by
a u half-step:

* p half-step at primal node j: the 2^d dual nodes q = j - 1 + eps
  (eps in {0,1}^d) are the corners of the cell centred on x_j.  Each velocity
  component is interpolated on that cell by the tensor-product Hermite-Birkhoff
  interpolant of degree 2m+1 per variable (Sec. 2, eq. (interp); Sec. 5
  dimension-by-dimension reconstruction).  The leapfrog difference keeps only
  odd time derivatives (Sec. 2, eq. (update1)); Cauchy-Kowalevsky turns them
  into space derivatives (Sec. 2, eq. (LFloop); Sec. 3.1.2, eq. (pdup)):
      d_t^{2k+1} p = -kappa^{k+1} Lap^k div u,
  so  P~_s <- P~_s - sum_k w_k kappa^{k+1} [Lap^k div c]_s,
      w_k = 2 (dt/2)^{2k+1} / (2k+1)!,   s in {0..m}^d.
* u half-step at dual node q: primal corners j = q + eps, interpolate p, and
  (Sec. 3.1.2, eq. (vdup))  d_t^{2k+1} u = -kappa^k grad Lap^k p, so
      U~_{i,s} <- U~_{i,s} - sum_k w_k kappa^k [D_i Lap^k c]_s.

Readings of the paper taken here (each is listed in the design notes):
the interpolant matches value and first m derivatives at each end (Sec. 2,
text after eq. (interp)); the sum over odd j runs until the term vanishes
(Sec. 2, after eq. (update1)); grad^{j-1} in eqs. (pdup)/(vdup) is read as
Lap^{(j-1)/2}; the system signs of Sec. 4 are used in every dimension; a
step is the p half-step then the u half-step.

Arrays use the boundary's host layout: C order, node axes (x_1..x_d) then
coefficient axes (a_1..a_d); U has a leading component axis (u_1..u_d).
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, replace
from fractions import Fraction
from math import comb, factorial

import numpy as np

__all__ = [
    "Problem", "hermite_matrix_exact", "hermite_matrix", "p_half", "u_half",
    "step", "startup", "p_update_cells", "u_update_cells", "ghost_pad", "mirror_sign",
    "p_operator_blocks", "u_operator_blocks", "p_half_adjoint", "u_half_adjoint", "adjoint_step",
    "kappa_gradient", "kmax_var", "p_update_cells_var", "u_update_cells_var", "p_half_var", "u_half_var",
    "step_var", "step_with_source", "p_operator_blocks_var", "u_operator_blocks_var",
    "p_half_var_adjoint", "u_half_var_adjoint", "adjoint_step_var", "kappa_field_gradient",
]

_CHUNK = 1 << 14  # nodes per vectorised batch (bounds memory, not arithmetic)


# ---------------------------------------------------------------------------
# Problem description
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Problem:
    """Constant-coefficient problem: dimension d, Hermite order m, cells per
    dimension K, box (or period) length per dimension, time step dt,
    kappa = c^2 (system of Sec. 4 / Sec. 5 with constant coefficient) and the
    boundary, "periodic" or "walls" (p = 0 on the box faces)."""

    d: int
    m: int
    K: tuple
    length: tuple
    dt: float
    kappa: float = 1.0
    bc: str = "periodic"

    @property
    def walls(self):
        return self.bc == "walls"

    def p_nodes(self):
        """Primal nodes per dimension."""
        return tuple(int(k) + (1 if self.walls else 0) for k in self.K)

    def u_nodes(self):
        """Dual nodes per dimension."""
        return tuple(int(k) for k in self.K)

    @property
    def h(self):
        return tuple(float(L) / int(k) for L, k in zip(self.length, self.K))

    @property
    def nc(self):
        return (self.m + 1) ** self.d

    def with_dt(self, dt):
        return replace(self, dt=dt)

    def p_shape(self):
        return self.p_nodes() + (self.m + 1,) * self.d

    def u_shape(self):
        return (self.d,) + self.u_nodes() + (self.m + 1,) * self.d


# ---------------------------------------------------------------------------
# Hermite-Birkhoff interpolation matrix (Sec. 2, eq. (interp))
# ---------------------------------------------------------------------------
def hermite_matrix_exact(m: int):
    """H_m = [C^L; C^R]^{-1} in exact rationals (Sec. 2, eq. (interp)).

    The interpolant on a cell is q(xi) = sum_{s=0}^{2m+1} c_s xi^s with
    xi = (x - centre)/h.  Its scaled l-th derivative at xi0 is
    sum_s binom(s, l) xi0^{s-l} c_s, which is C_{ls} of the paper with
    xi0 = -1/2 (left end, C^L) and +1/2 (right end, C^R).  Rows of the
    returned matrix are the coefficients c_s; columns are the data
    (v^L_0..v^L_m, v^R_0..v^R_m).
    """
    n = 2 * m + 2
    A = [[Fraction(0)] * n for _ in range(n)]
    for side, xi0 in enumerate((Fraction(-1, 2), Fraction(1, 2))):
        for l in range(m + 1):
            for s in range(l, n):
                A[side * (m + 1) + l][s] = comb(s, l) * xi0 ** (s - l)
    # Gauss-Jordan elimination on [A | I] in exact arithmetic.
    aug = [row[:] + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        pv = aug[col][col]
        aug[col] = [x / pv for x in aug[col]]
        for r in range(n):
            if r != col and aug[r][col] != 0:
                f = aug[r][col]
                aug[r] = [x - f * y for x, y in zip(aug[r], aug[col])]
    return [row[n:] for row in aug]


def hermite_matrix(m: int) -> np.ndarray:
    """FP64 H_m: each entry is the correctly rounded exact rational."""
    return np.array([[float(x) for x in row] for row in hermite_matrix_exact(m)],
                    dtype=np.float64)


# ---------------------------------------------------------------------------
# Coefficient-space operators on cell polynomials
# ---------------------------------------------------------------------------
def _interpolate(B: np.ndarray, H: np.ndarray, d: int, ns: int) -> np.ndarray:
    """Tensor-product interpolation, one dimension at a time (Sec. 5).

    B has shape (2,)*d + S + (m+1,)*d: corner e (left/right per dimension) of
    a batch S of cells, scaled data alpha.  Returns c with shape
    S + (2m+2,)*d, the coefficients of the interpolant in xi.
    """
    for k in range(d):
        L, R = B[0], B[1]                 # consume the corner axis of dim k
        ax = (d - k - 1) + ns + k         # data axis of dim k inside L / R
        both = np.concatenate([L, R], axis=ax)
        B = np.moveaxis(np.tensordot(H, np.moveaxis(both, ax, 0), axes=(1, 0)), 0, ax)
    return B


def _deriv(c: np.ndarray, i: int, h_i: float, ns: int) -> np.ndarray:
    """x_i-derivative in coefficient space: (D_i c)_b = (b_i + 1) c_{b+e_i} / h_i."""
    ax = ns + i
    n = c.shape[ax]
    out = np.zeros_like(c)
    src = [slice(None)] * c.ndim
    dst = [slice(None)] * c.ndim
    src[ax] = slice(1, n)
    dst[ax] = slice(0, n - 1)
    shape = [1] * c.ndim
    shape[ax] = n - 1
    fac = np.arange(1, n, dtype=np.float64).reshape(shape)
    out[tuple(dst)] = c[tuple(src)] * fac / h_i
    return out


def _laplacian(c: np.ndarray, h, d: int, ns: int) -> np.ndarray:
    out = np.zeros_like(c)
    for i in range(d):
        out = out + _deriv(_deriv(c, i, h[i], ns), i, h[i], ns)
    return out


def _truncate(c: np.ndarray, m: int, d: int, ns: int) -> np.ndarray:
    """Keep the coefficients s in {0..m}^d: the new nodal data are the Taylor
    coefficients of the updated polynomial at the cell centre (Sec. 2)."""
    idx = [slice(None)] * ns + [slice(0, m + 1)] * d
    return c[tuple(idx)]


def _w(k: int, dt: float) -> float:
    """w_k = 2 (dt/2)^{2k+1} / (2k+1)!  (Sec. 2, eq. (update1), j = 2k+1)."""
    return 2.0 * (dt / 2.0) ** (2 * k + 1) / factorial(2 * k + 1)


def _is_zero(a: np.ndarray) -> bool:
    return not np.any(a)


# ---------------------------------------------------------------------------
# Cell-level updates (batched over cells)
# ---------------------------------------------------------------------------
def _kw(k: int, j: int, kappa: float, dkappa: bool) -> float:
    """kappa^j, or its derivative j kappa^(j-1) with respect to kappa."""
    if not dkappa:
        return kappa ** j
    return j * kappa ** (j - 1) if j > 0 else 0.0


def p_update_cells(prob: Problem, p_vals: np.ndarray, u_corners, dt=None, dkappa: bool = False) -> np.ndarray:
    """New pressure data at a batch of primal nodes.

    p_vals: (n,) + (m+1,)*d, pressure data at the nodes at time t.
    u_corners: sequence of d arrays, each (2,)*d + (n,) + (m+1,)*d: velocity
    component i at the 2^d dual corners of each node's cell, time t + dt/2.
    Returns p data at t + dt (Sec. 2, eq. (final1); Sec. 3.1.2, eq. (pdup)).
    With ``dkappa`` every kappa^(k+1) is replaced by its kappa-derivative, so
    the result is p_vals minus the kappa-derivative of the increment.
    """
    d, m = prob.d, prob.m
    dt = prob.dt if dt is None else dt
    h = prob.h
    H = hermite_matrix(m)
    r = None
    for i in range(d):
        ci = _interpolate(np.asarray(u_corners[i], dtype=np.float64), H, d, 1)
        di = _deriv(ci, i, h[i], 1)
        r = di if r is None else r + di            # div of the interpolant
    incr = np.zeros_like(r)
    term = r
    k = 0
    while not _is_zero(term):
        incr = incr + _w(k, dt) * _kw(k, k + 1, prob.kappa, dkappa) * term
        term = _laplacian(term, h, d, 1)
        k += 1
    return p_vals - _truncate(incr, m, d, 1)


def u_update_cells(prob: Problem, u_vals: np.ndarray, p_corners: np.ndarray,
                   dt=None, weight_scale: float = 1.0, dkappa: bool = False) -> np.ndarray:
    """New velocity data at a batch of dual nodes.

    u_vals: (d, n) + (m+1,)*d at time t - dt/2 (or t for the start-up).
    p_corners: (2,)*d + (n,) + (m+1,)*d, pressure at the 2^d primal corners of
    each dual node's cell at time t.  Returns u at t + dt/2 (Sec. 3.1.2,
    eq. (vdup)); ``weight_scale`` multiplies every w_k (1/2 for the start-up).
    """
    d, m = prob.d, prob.m
    dt = prob.dt if dt is None else dt
    h = prob.h
    c = _interpolate(np.asarray(p_corners, dtype=np.float64), hermite_matrix(m), d, 1)
    out = np.array(u_vals, dtype=np.float64, copy=True)
    for i in range(d):
        incr = np.zeros_like(c)
        term = c                                   # Lap^k c
        k = 0
        while not _is_zero(term):
            incr = incr + weight_scale * _w(k, dt) * _kw(k, k, prob.kappa, dkappa) * _deriv(term, i, h[i], 1)
            term = _laplacian(term, h, d, 1)
            k += 1
        out[i] = out[i] - _truncate(incr, m, d, 1)
    return out


# ---------------------------------------------------------------------------
# Periodic gathers and half-steps
# ---------------------------------------------------------------------------
def _all_nodes(K) -> np.ndarray:
    grids = np.meshgrid(*[np.arange(k) for k in K], indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1)


def _gather(F: np.ndarray, nodes: np.ndarray, offset: int, d: int, K) -> np.ndarray:
    """Corner data F[node + offset + eps] for eps in {0,1}^d, shaped
    (2,)*d + (n,) + coefficient axes; indices taken mod K when K is given
    (periodic), else used as they are."""
    n = nodes.shape[0]
    out = np.empty((2,) * d + (n,) + F.shape[d:], dtype=F.dtype)
    for eps in itertools.product((0, 1), repeat=d):
        if K is None:
            idx = tuple(nodes[:, k] + offset + eps[k] for k in range(d))
        else:
            idx = tuple((nodes[:, k] + offset + eps[k]) % K[k] for k in range(d))
        out[eps] = F[idx]
    return out


def mirror_sign(i: int, k: int) -> float:
    """Mirror parity of velocity component i across a wall normal to x_k:
    +1 (even) for the normal component, -1 (odd) for tangential ones."""
    return 1.0 if i == k else -1.0


def ghost_pad(prob: Problem, U: np.ndarray) -> np.ndarray:
    """Velocity with one ghost layer of dual nodes on every wall (walls
    boundary): shape (d,) + (K+2,)*d + coefficient axes, the dual node q at
    index q + 1.  Ghost q = -1 mirrors q = 0 across x_k = 0, ghost q = K
    mirrors q = K-1 across x_k = L_k; a coefficient with index a_k is
    multiplied by mirror_sign * (-1)^{a_k}.  Dimensions are mirrored one after
    the other, so an edge or corner ghost is the mirror of a mirror."""
    d, m = prob.d, prob.m
    K = tuple(prob.K)
    out = np.zeros((d,) + tuple(k + 2 for k in K) + (m + 1,) * d)
    out[(slice(None),) + tuple(slice(1, k + 1) for k in K)] = U
    for i in range(d):
        for k in range(d):
            shape = [1] * (2 * d)
            shape[d + k] = m + 1
            flip = (mirror_sign(i, k) * (-1.0) ** np.arange(m + 1)).reshape(shape)
            lo = [slice(None)] * d
            src = [slice(None)] * d
            lo[k], src[k] = 0, 1
            out[(i,) + tuple(lo)] = flip[0] * out[(i,) + tuple(src)]
            lo[k], src[k] = K[k] + 1, K[k]
            out[(i,) + tuple(lo)] = flip[0] * out[(i,) + tuple(src)]
    return out


def p_half(prob: Problem, P: np.ndarray, U: np.ndarray, nodes=None, dt=None, dkappa: bool = False):
    """Pressure half-step.  P, U in natural layout.  Primal node j takes the
    dual corners q = j - 1 + eps (cell centred on x_j with ends x_{j-1/2},
    x_{j+1/2}); with walls, q = -1 and q = K are the ghost nodes.  With
    ``nodes`` (n, d) only those nodes are computed and an (n,)+coef array is
    returned; else the new P."""
    d = prob.d
    full = nodes is None
    nodes = _all_nodes(prob.p_nodes()) if full else np.asarray(nodes, dtype=np.int64).reshape(-1, d)
    if prob.walls:
        Ug, off, wrap = ghost_pad(prob, U), 0, None     # padded index q + 1
    else:
        Ug, off, wrap = U, -1, tuple(prob.K)
    res = np.empty((nodes.shape[0],) + P.shape[d:], dtype=np.float64)
    for a in range(0, nodes.shape[0], _CHUNK):
        nd = nodes[a:a + _CHUNK]
        uc = [_gather(Ug[i], nd, off, d, wrap) for i in range(d)]
        pv = P[tuple(nd[:, k] for k in range(d))]
        res[a:a + _CHUNK] = p_update_cells(prob, pv, uc, dt=dt, dkappa=dkappa)
    return res.reshape(P.shape) if full else res


def u_half(prob: Problem, U: np.ndarray, P: np.ndarray, nodes=None, dt=None,
           weight_scale: float = 1.0, dkappa: bool = False):
    """Velocity half-step.  Dual node q takes the primal corners j = q + eps
    (cell centred on x_{q+1/2} with ends x_q, x_{q+1})."""
    d = prob.d
    full = nodes is None
    nodes = _all_nodes(prob.u_nodes()) if full else np.asarray(nodes, dtype=np.int64).reshape(-1, d)
    wrap = None if prob.walls else tuple(prob.K)
    res = np.empty((d, nodes.shape[0]) + P.shape[d:], dtype=np.float64)
    for a in range(0, nodes.shape[0], _CHUNK):
        nd = nodes[a:a + _CHUNK]
        pc = _gather(P, nd, 0, d, wrap)
        uv = np.stack([U[i][tuple(nd[:, k] for k in range(d))] for i in range(d)])
        res[:, a:a + _CHUNK] = u_update_cells(prob, uv, pc, dt=dt, weight_scale=weight_scale, dkappa=dkappa)
    return res.reshape(U.shape) if full else res


def step(prob: Problem, P: np.ndarray, U: np.ndarray, nsteps: int = 1):
    """nsteps full steps: (P^n, U^{n+1/2}) -> (P^{n+N}, U^{n+N+1/2})."""
    P = np.array(P, dtype=np.float64, copy=True)
    U = np.array(U, dtype=np.float64, copy=True)
    for _ in range(int(nsteps)):
        P = p_half(prob, P, U)
        U = u_half(prob, U, P)
    return P, U


def startup(prob: Problem, P0: np.ndarray, U0: np.ndarray) -> np.ndarray:
    """U^{1/2} from (P^0, U^0): the Taylor series of u over dt/2 about t0.
    Odd terms are -(dt/2)^{2k+1}/(2k+1)! kappa^k grad Lap^k p, i.e. the u
    half-step with every w_k halved; even terms are those of U^0 alone and are
    dropped (exact when U^0 = 0, the start used here)."""
    return u_half(prob, U0, P0, weight_scale=0.5)


# ---------------------------------------------------------------------------
# Discrete adjoint (periodic grid)
# ---------------------------------------------------------------------------
# One step maps (P, U) to P' = P - A U, U' = U - B P'; A and B are the linear
# operators of the two half-steps (translation invariant on the periodic
# grid, one dense block per cell corner).  Its transpose maps (Pb', Ub') to
#     Pb = Pb' - B^T Ub',    Ub = Ub' - A^T Pb
# (substitute P' into U' and transpose the block matrix), i.e. the transposed
# half-steps in reverse order.  The blocks are read off the forward cell
# updates applied to unit data, so the adjoint is the forward oracle's own
# transpose.

def p_operator_blocks(prob: Problem) -> np.ndarray:
    """A[e][s][i][a]: the pressure half-step subtracts
    sum_e sum_{i,a} A[e][s][i][a] U_i[j - 1 + e][a] from P[j][s]."""
    d, nc = prob.d, prob.nc
    cshape = (prob.m + 1,) * d
    A = np.zeros((2,) * d + (nc, d, nc))
    for e in itertools.product((0, 1), repeat=d):
        for i in range(d):
            for a in range(nc):
                uc = [np.zeros((2,) * d + (1,) + cshape) for _ in range(d)]
                uc[i][e + (0,) + np.unravel_index(a, cshape)] = 1.0
                A[e + (slice(None), i, a)] = -p_update_cells(prob, np.zeros((1,) + cshape), uc)[0].ravel()
    return A


def u_operator_blocks(prob: Problem) -> np.ndarray:
    """B[e][i][s][a]: the velocity half-step subtracts
    sum_e sum_a B[e][i][s][a] P[q + e][a] from U_i[q][s]."""
    d, nc = prob.d, prob.nc
    cshape = (prob.m + 1,) * d
    B = np.zeros((2,) * d + (d, nc, nc))
    for e in itertools.product((0, 1), repeat=d):
        for a in range(nc):
            pc = np.zeros((2,) * d + (1,) + cshape)
            pc[e + (0,) + np.unravel_index(a, cshape)] = 1.0
            r = -u_update_cells(prob, np.zeros((d, 1) + cshape), pc)[:, 0]
            B[e + (slice(None), slice(None), a)] = r.reshape(d, nc)
    return B


def p_half_adjoint(prob: Problem, Pb: np.ndarray, Ub: np.ndarray, B=None) -> np.ndarray:
    """Pb - B^T Ub: P[j] receives sum_e B[e]^T Ub[j - e] (the dual nodes
    q = j - 1 + e' with e' = 1 - e, the pressure half-step's corners)."""
    d, K, nc = prob.d, tuple(prob.K), prob.nc
    B = u_operator_blocks(prob) if B is None else B
    Ubf = Ub.reshape((d,) + K + (nc,))
    out = Pb.reshape(K + (nc,)).copy()
    for e in itertools.product((0, 1), repeat=d):
        src = np.roll(Ubf, shift=tuple(e), axis=tuple(range(1, d + 1)))      # Ub[j - e]
        out -= np.einsum("isa,i...s->...a", B[e], src)
    return out.reshape(Pb.shape)


def u_half_adjoint(prob: Problem, Ub: np.ndarray, Pb: np.ndarray, A=None) -> np.ndarray:
    """Ub - A^T Pb: U[q] receives sum_e A[e]^T Pb[q + 1 - e] (the primal
    nodes j = q + e' with e' = 1 - e, the velocity half-step's corners)."""
    d, K, nc = prob.d, tuple(prob.K), prob.nc
    A = p_operator_blocks(prob) if A is None else A
    Pbf = Pb.reshape(K + (nc,))
    out = Ub.reshape((d,) + K + (nc,)).copy()
    for e in itertools.product((0, 1), repeat=d):
        src = np.roll(Pbf, shift=tuple(e[k] - 1 for k in range(d)), axis=tuple(range(d)))   # Pb[q + 1 - e]
        out -= np.einsum("sia,...s->i...a", A[e], src)
    return out.reshape(Ub.shape)


# Reflecting walls.  The walled step is P' = P - A G U, U' = U - B P', with G
# the ghost padding of U (ghost_pad, linear) and A, B the same per-corner
# blocks (the cell updates do not depend on position); its transpose is
#     Pb = Pb' - B^T Ub',    Ub = Ub' - G^T A^T Pb,
# where B^T only gathers from the K dual nodes, A^T is evaluated on the whole
# padded dual array (primal corners outside [0, K] contribute nothing) and
# G^T folds each ghost's value back into the node it mirrors.

def ghost_pad_adjoint(prob: Problem, W: np.ndarray) -> np.ndarray:
    """Transpose of ghost_pad: W on the padded dual array (d,) + (K+2,)*d +
    coef to the K dual nodes.  ghost_pad overwrites, for each component and
    each dimension k in turn, the two ghost slices of dimension k with flipped
    copies of their neighbouring slices; the transpose undoes these copies in
    reverse order, adding each ghost slice (flipped) into its source slice and
    clearing it, then keeps the interior."""
    d, m = prob.d, prob.m
    K = tuple(prob.K)
    W = np.array(W, dtype=np.float64, copy=True)
    for i in range(d):
        for k in reversed(range(d)):
            shape = [1] * (2 * d)
            shape[d + k] = m + 1
            flip = (mirror_sign(i, k) * (-1.0) ** np.arange(m + 1)).reshape(shape)
            for g, src in ((K[k] + 1, K[k]), (0, 1)):   # reverse of ghost_pad's (lo, hi) order
                gs = [slice(None)] * d
                ss = [slice(None)] * d
                gs[k], ss[k] = g, src
                W[(i,) + tuple(ss)] += flip[0] * W[(i,) + tuple(gs)]
                W[(i,) + tuple(gs)] = 0.0
    return W[(slice(None),) + tuple(slice(1, k + 1) for k in K)]


def p_half_adjoint_walls(prob: Problem, Pb: np.ndarray, Ub: np.ndarray, B=None) -> np.ndarray:
    """Pb - B^T Ub on the walled box: the primal node j (0..K per dimension)
    receives B[e]^T Ub[j - e] from the dual nodes j - e inside [0, K-1]."""
    d, nc = prob.d, prob.nc
    K = tuple(prob.K)
    B = u_operator_blocks(prob) if B is None else B
    Ubf = Ub.reshape((d,) + K + (nc,))
    pad = np.zeros((d,) + tuple(k + 1 for k in K) + (nc,))   # Ub at q = j - e, zero outside
    out = Pb.reshape(tuple(k + 1 for k in K) + (nc,)).copy()
    for e in itertools.product((0, 1), repeat=d):
        pad[...] = 0.0
        pad[(slice(None),) + tuple(slice(e[k], e[k] + K[k]) for k in range(d))] = Ubf
        out -= np.einsum("isa,i...s->...a", B[e], pad)
    return out.reshape(Pb.shape)


def u_half_adjoint_walls(prob: Problem, Ub: np.ndarray, Pb: np.ndarray, A=None) -> np.ndarray:
    """Ub - G^T A^T Pb on the walled box: A^T Pb at every padded dual node
    (q = -1..K per dimension, index q + 1) from the primal nodes q + 1 - e
    inside [0, K], then the ghost fold G^T."""
    d, nc = prob.d, prob.nc
    K = tuple(prob.K)
    A = p_operator_blocks(prob) if A is None else A
    Pbf = Pb.reshape(tuple(k + 1 for k in K) + (nc,))
    W = np.zeros((d,) + tuple(k + 2 for k in K) + (nc,))
    for e in itertools.product((0, 1), repeat=d):
        # padded index r = q + 1 takes Pb[q + 1 - e] = Pb[r - e], r - e in [0, K]
        src = np.zeros(tuple(k + 2 for k in K) + (nc,))
        src[tuple(slice(e[k], e[k] + K[k] + 1) for k in range(d))] = Pbf
        W += np.einsum("sia,...s->i...a", A[e], src)
    cshape = (prob.m + 1,) * d
    Wt = ghost_pad_adjoint(prob, W.reshape((d,) + tuple(k + 2 for k in K) + cshape))
    return (Ub.reshape((d,) + K + cshape) - Wt).reshape(Ub.shape)


def adjoint_step(prob: Problem, Pb: np.ndarray, Ub: np.ndarray, nsteps: int = 1):
    """Transpose of `step`: nsteps times Pb <- Pb - B^T Ub, then Ub <- Ub -
    A^T Pb (periodic), or Ub <- Ub - G^T A^T Pb (reflecting walls)."""
    A, B = p_operator_blocks(prob), u_operator_blocks(prob)
    Pb = np.array(Pb, dtype=np.float64, copy=True)
    Ub = np.array(Ub, dtype=np.float64, copy=True)
    for _ in range(int(nsteps)):
        if prob.walls:
            Pb = p_half_adjoint_walls(prob, Pb, Ub, B)
            Ub = u_half_adjoint_walls(prob, Ub, Pb, A)
        else:
            Pb = p_half_adjoint(prob, Pb, Ub, B)
            Ub = u_half_adjoint(prob, Ub, Pb, A)
    return Pb, Ub


def kappa_gradient(prob: Problem, P0: np.ndarray, U0: np.ndarray, Pbn: np.ndarray, Ubn: np.ndarray,
                   nsteps: int):
    """d/dkappa of <Pbn, P_n> + <Ubn, U_n> for n steps from (P0, U0), and the
    adjoint state (Pb_0, Ub_0) (periodic grid or reflecting walls; with walls
    A stands for A G, the ghost padding included in the pressure half-step).

    With P' = P - A U, U' = U - B P' and the adjoint lambda_{t+1} = (Pb', Ub')
    of the state after step t, the step's kappa-derivative contributes
        -<Pb' - B^T Ub', A_kappa U_t> - <Ub', B_kappa P'>
    (chain rule through both half-steps), where A_kappa, B_kappa are the
    half-step operators with every kappa power replaced by its derivative.
    The forward trajectory is stored (no recomputation)."""
    A, B = p_operator_blocks(prob), u_operator_blocks(prob)
    states = [(np.array(P0, dtype=np.float64), np.array(U0, dtype=np.float64))]
    for _ in range(int(nsteps)):
        P, U = states[-1]
        P1 = p_half(prob, P, U)
        states.append((P1, u_half(prob, U, P1)))
    padj, uadj = (p_half_adjoint_walls, u_half_adjoint_walls) if prob.walls else (p_half_adjoint, u_half_adjoint)
    Pb, Ub = np.array(Pbn, dtype=np.float64), np.array(Ubn, dtype=np.float64)
    g = 0.0
    for t in range(int(nsteps) - 1, -1, -1):
        P_t, U_t = states[t]
        P_1 = states[t + 1][0]
        BkP = -u_half(prob, np.zeros_like(U_t), P_1, dkappa=True)                  # B_kappa P'
        g -= np.sum(Ub * BkP)
        Pb = padj(prob, Pb, Ub, B)
        AkU = -p_half(prob, np.zeros_like(P_t), U_t, dkappa=True)                   # A_kappa U_t
        g -= np.sum(Pb * AkU)
        Ub = uadj(prob, Ub, Pb, A)
    return g, Pb, Ub


# ---------------------------------------------------------------------------
# Variable coefficient kappa(x) (periodic grid)
# ---------------------------------------------------------------------------
# The paper expands the coefficient about every grid node in a local Taylor
# polynomial of degree 2m+1 (Sec. 4, "Smoothly varying wave speed"):
#     kappa~_b = prod_k h_k^{b_k} / b_k!  d^b kappa (node),  b in {0..2m+1}^d,
# and runs the Cauchy-Kowalevsky recurrence with it.  From p_t = -kappa div u,
# u_t = -grad p:  d_t^{2k+1} p = -(kappa Lap)^k (kappa div u) and
# d_t^{2k+1} u = -grad (kappa Lap)^k p.  Reading taken (the printed formula
# is garbled): every product is a product of cell polynomials truncated to
# degree 2m+1 per variable, T[.]; kappa is expanded about the cell centre,
# i.e. about the primal node for the pressure half-step and the dual node for
# the velocity half-step.  With variable kappa the series does not terminate
# (every product with kappa refills the degrees a Laplacian removed), so its
# length is a choice; the one taken is k = 0..kmax with kmax = d m, the last k
# at which Lap^k of a cell polynomial of degree 2m+1 in each variable can be
# nonzero (Lap^k is a sum of D_1^{2 i_1} .. D_d^{2 i_d}, i_1 + .. + i_d = k,
# and D_l^{2 i} kills the polynomial once 2 i > 2m+1).  This is where the
# constant-coefficient series ends, so constant kappa data reproduce the
# constant step exactly, and in 1D it is the paper's sum over odd time
# derivatives up to order 2m+1.  The paper's variable-speed experiments are
# 1D only, so for d >= 2 the length is unpinned by the paper:
#     P <- P - sum_k w_k r_k,  r_0 = T[kappa div c],  r_k = T[kappa Lap r_{k-1}],
#     U_i <- U_i - sum_k w_k D_i g_k,  g_0 = c,  g_k = T[kappa Lap g_{k-1}].

def kmax_var(d: int, m: int) -> int:
    return d * m


def _tmul(a: np.ndarray, b: np.ndarray, d: int, ns: int) -> np.ndarray:
    """T[a b]: product of batched cell polynomials (ns batch axes, then d
    coefficient axes of length 2m+2), truncated to the same degrees."""
    n = a.shape[ns]
    out = np.zeros(np.broadcast_shapes(a.shape, b.shape), dtype=np.result_type(a, b))
    for s in itertools.product(range(n), repeat=d):
        bs = a[(slice(None),) * ns + s]
        dst = (slice(None),) * ns + tuple(slice(sk, n) for sk in s)
        src = (slice(None),) * ns + tuple(slice(0, n - sk) for sk in s)
        out[dst] += bs.reshape(bs.shape + (1,) * d) * b[src]
    return out


def p_update_cells_var(prob: Problem, p_vals, u_corners, kap, dt=None):
    """Pressure update with kappa Taylor data kap, (n,) + (2m+2,)*d, about
    each node (see the block comment above)."""
    d, m = prob.d, prob.m
    dt = prob.dt if dt is None else dt
    h = prob.h
    H = hermite_matrix(m)
    div = None
    for i in range(d):
        di = _deriv(_interpolate(np.asarray(u_corners[i], dtype=np.float64), H, d, 1), i, h[i], 1)
        div = di if div is None else div + di
    r = _tmul(kap, div, d, 1)
    incr = _w(0, dt) * r
    for k in range(1, kmax_var(d, m) + 1):
        r = _tmul(kap, _laplacian(r, h, d, 1), d, 1)
        incr = incr + _w(k, dt) * r
    return p_vals - _truncate(incr, m, d, 1)


def u_update_cells_var(prob: Problem, u_vals, p_corners, kap, dt=None, weight_scale: float = 1.0):
    """Velocity update with kappa Taylor data kap about each dual node."""
    d, m = prob.d, prob.m
    dt = prob.dt if dt is None else dt
    h = prob.h
    g = _interpolate(np.asarray(p_corners, dtype=np.float64), hermite_matrix(m), d, 1)
    q = _w(0, dt) * g
    for k in range(1, kmax_var(d, m) + 1):
        g = _tmul(kap, _laplacian(g, h, d, 1), d, 1)
        q = q + _w(k, dt) * g
    out = np.array(u_vals, dtype=np.result_type(u_vals, q), copy=True)
    for i in range(d):
        out[i] = out[i] - weight_scale * _truncate(_deriv(q, i, h[i], 1), m, d, 1)
    return out


def p_half_var(prob: Problem, P, U, Kp, nodes=None, dt=None):
    """Pressure half-step with kappa data Kp, p_nodes() + (2m+2,)*d on the
    primal nodes; with walls the dual corners include the ghost layer of U as
    in p_half (the mirror rule does not involve kappa)."""
    d = prob.d
    full = nodes is None
    nodes = _all_nodes(prob.p_nodes()) if full else np.asarray(nodes, dtype=np.int64).reshape(-1, d)
    if prob.walls:
        Ug, off, wrap = ghost_pad(prob, U), 0, None     # padded index q + 1
    else:
        Ug, off, wrap = U, -1, tuple(prob.K)
    res = np.empty((nodes.shape[0],) + P.shape[d:], dtype=np.float64)
    for a in range(0, nodes.shape[0], _CHUNK):
        nd = nodes[a:a + _CHUNK]
        idx = tuple(nd[:, k] for k in range(d))
        uc = [_gather(Ug[i], nd, off, d, wrap) for i in range(d)]
        res[a:a + _CHUNK] = p_update_cells_var(prob, P[idx], uc, Kp[idx], dt=dt)
    return res.reshape(P.shape) if full else res


def u_half_var(prob: Problem, U, P, Ku, nodes=None, dt=None, weight_scale: float = 1.0):
    """Velocity half-step with kappa data Ku, u_nodes() + (2m+2,)*d on the dual
    nodes (periodic, or walls: the primal corners are all real nodes)."""
    d = prob.d
    full = nodes is None
    nodes = _all_nodes(prob.u_nodes()) if full else np.asarray(nodes, dtype=np.int64).reshape(-1, d)
    wrap = None if prob.walls else tuple(prob.K)
    res = np.empty((d, nodes.shape[0]) + P.shape[d:], dtype=np.float64)
    for a in range(0, nodes.shape[0], _CHUNK):
        nd = nodes[a:a + _CHUNK]
        idx = tuple(nd[:, k] for k in range(d))
        pc = _gather(P, nd, 0, d, wrap)
        uv = np.stack([U[i][idx] for i in range(d)])
        res[:, a:a + _CHUNK] = u_update_cells_var(prob, uv, pc, Ku[idx], dt=dt, weight_scale=weight_scale)
    return res.reshape(U.shape) if full else res


def step_var(prob: Problem, P, U, Kp, Ku, nsteps: int = 1):
    P = np.array(P, dtype=np.float64, copy=True)
    U = np.array(U, dtype=np.float64, copy=True)
    for _ in range(int(nsteps)):
        P = p_half_var(prob, P, U, Kp)
        U = u_half_var(prob, U, P, Ku)
    return P, U


# ---------------------------------------------------------------------------
# Variable kappa: transposed step and gradient with respect to the kappa data
# ---------------------------------------------------------------------------
# With kappa data per node the half-step operators are no longer translation
# invariant: A_j (pressure half-step at primal node j) and B_q (velocity
# half-step at dual node q) are dense per-node blocks, read off the forward
# cell updates applied to unit corner data with that node's kappa.  The
# transpose of a step is again Pb <- Pb - B^T Ub, then Ub <- Ub - A^T Pb.
# The gradient of <Pb_n, P_n> + <Ub_n, U_n> with respect to the kappa data of
# node j collects, over the steps, the derivative of that node's cell update
# paired with the adjoint state at the node (the same chain rule as
# kappa_gradient, node by node).  The derivative of a cell update with respect
# to one kappa coefficient is taken by the complex-step method (Squire and
# Trapp, SIAM Review 40 (1998)): the update is a polynomial in the kappa data
# with real coefficients, so Im f(kappa + i eps e_b) / eps is its derivative
# up to rounding for a tiny eps (no difference of nearby values is formed).

_CSTEP = 1e-30


def _node_kappa(prob: Problem, Kap: np.ndarray) -> np.ndarray:
    """Kappa data flattened to (nodes,) + (2m+2,)*d in node order."""
    d = prob.d
    return np.asarray(Kap).reshape((-1,) + Kap.shape[d:])


def p_operator_blocks_var(prob: Problem, Kp: np.ndarray) -> np.ndarray:
    """A[j][e][s][i][a] (j the flat primal node): the pressure half-step with
    kappa data Kp subtracts sum_e sum_{i,a} A[j][e][s][i][a] U_i[j - 1 + e][a]
    from P[j][s]."""
    d, nc = prob.d, prob.nc
    cshape = (prob.m + 1,) * d
    kap = _node_kappa(prob, Kp)
    n = kap.shape[0]
    A = np.zeros((n,) + (2,) * d + (nc, d, nc))
    for e in itertools.product((0, 1), repeat=d):
        for i in range(d):
            for a in range(nc):
                uc = [np.zeros((2,) * d + (n,) + cshape) for _ in range(d)]
                uc[i][e + (slice(None),) + np.unravel_index(a, cshape)] = 1.0
                r = -p_update_cells_var(prob, np.zeros((n,) + cshape), uc, kap)
                A[(slice(None),) + e + (slice(None), i, a)] = r.reshape(n, nc)
    return A


def u_operator_blocks_var(prob: Problem, Ku: np.ndarray) -> np.ndarray:
    """B[q][e][i][s][a] (q the flat dual node): the velocity half-step with
    kappa data Ku subtracts sum_e sum_a B[q][e][i][s][a] P[q + e][a] from
    U_i[q][s]."""
    d, nc = prob.d, prob.nc
    cshape = (prob.m + 1,) * d
    kap = _node_kappa(prob, Ku)
    n = kap.shape[0]
    B = np.zeros((n,) + (2,) * d + (d, nc, nc))
    for e in itertools.product((0, 1), repeat=d):
        for a in range(nc):
            pc = np.zeros((2,) * d + (n,) + cshape)
            pc[e + (slice(None),) + np.unravel_index(a, cshape)] = 1.0
            r = -u_update_cells_var(prob, np.zeros((d, n) + cshape), pc, kap)
            B[(slice(None),) + e + (slice(None), slice(None), a)] = r.reshape(d, n, nc).transpose(1, 0, 2)
    return B


def p_half_var_adjoint(prob: Problem, Pb: np.ndarray, Ub: np.ndarray, Ku: np.ndarray, B=None) -> np.ndarray:
    """Pb - B(Ku)^T Ub: P[j] receives sum_e B[q]^T Ub[q] from the dual nodes
    q = j - e whose velocity cells have j as corner e."""
    d, K, nc = prob.d, tuple(prob.K), prob.nc
    B = u_operator_blocks_var(prob, Ku) if B is None else B
    Bn = B.reshape(K + B.shape[1:])
    Ubf = Ub.reshape((d,) + K + (nc,))
    out = Pb.reshape(K + (nc,)).copy()
    axes = tuple(range(d))
    for e in itertools.product((0, 1), repeat=d):
        blk = np.roll(Bn[(slice(None),) * d + e], shift=tuple(e), axis=axes)       # B[j - e][e]
        src = np.roll(Ubf, shift=tuple(e), axis=tuple(range(1, d + 1)))           # Ub[j - e]
        out -= np.einsum("...isa,i...s->...a", blk, src)
    return out.reshape(Pb.shape)


def u_half_var_adjoint(prob: Problem, Ub: np.ndarray, Pb: np.ndarray, Kp: np.ndarray, A=None) -> np.ndarray:
    """Ub - A(Kp)^T Pb: U_i[q] receives sum_e A[j]^T Pb[j] from the primal
    nodes j = q + 1 - e whose pressure cells have q as corner e."""
    d, K, nc = prob.d, tuple(prob.K), prob.nc
    A = p_operator_blocks_var(prob, Kp) if A is None else A
    An = A.reshape(K + A.shape[1:])
    Pbf = Pb.reshape(K + (nc,))
    out = Ub.reshape((d,) + K + (nc,)).copy()
    axes = tuple(range(d))
    for e in itertools.product((0, 1), repeat=d):
        sh = tuple(e[k] - 1 for k in range(d))
        blk = np.roll(An[(slice(None),) * d + e], shift=sh, axis=axes)           # A[q + 1 - e][e]
        src = np.roll(Pbf, shift=sh, axis=axes)                                   # Pb[q + 1 - e]
        out -= np.einsum("...sia,...s->i...a", blk, src)
    return out.reshape(Ub.shape)


def adjoint_step_var(prob: Problem, Pb, Ub, Kp, Ku, nsteps: int = 1):
    """Transpose of `step_var`: nsteps times Pb <- Pb - B^T Ub, then
    Ub <- Ub - A^T Pb (periodic grid)."""
    if prob.walls:
        raise NotImplementedError("the adjoint is built for the periodic grid")
    A, B = p_operator_blocks_var(prob, Kp), u_operator_blocks_var(prob, Ku)
    Pb = np.array(Pb, dtype=np.float64, copy=True)
    Ub = np.array(Ub, dtype=np.float64, copy=True)
    for _ in range(int(nsteps)):
        Pb = p_half_var_adjoint(prob, Pb, Ub, Ku, B)
        Ub = u_half_var_adjoint(prob, Ub, Pb, Kp, A)
    return Pb, Ub


def _cstep_p(prob: Problem, U, Kp, Pb) -> np.ndarray:
    """d/dKp[j][b] of <Pb[j], increment part of the pressure cell update at
    j> for the velocity U, per node j and kappa coefficient b."""
    d, K = prob.d, tuple(prob.K)
    nodes = _all_nodes(K)
    kap = _node_kappa(prob, Kp).astype(np.complex128)
    n, npc = kap.shape[0], kap[0].size
    uc = [_gather(U[i], nodes, -1, d, K) for i in range(d)]
    pb = Pb.reshape(n, -1)
    cshape = (prob.m + 1,) * d
    g = np.zeros((n, npc))
    for b in range(npc):
        kb = kap.copy()
        kb.reshape(n, npc)[:, b] += 1j * _CSTEP
        r = p_update_cells_var(prob, np.zeros((n,) + cshape, dtype=np.complex128), uc, kb)
        g[:, b] = np.sum(pb * r.reshape(n, -1).imag, axis=1) / _CSTEP
    return g.reshape(Kp.shape)


def _cstep_u(prob: Problem, P, Ku, Ub) -> np.ndarray:
    """d/dKu[q][b] of <Ub[:, q], increment part of the velocity cell update at
    q> for the pressure P."""
    d, K = prob.d, tuple(prob.K)
    nodes = _all_nodes(K)
    kap = _node_kappa(prob, Ku).astype(np.complex128)
    n, npc = kap.shape[0], kap[0].size
    pc = _gather(P, nodes, 0, d, K)
    ub = Ub.reshape(d, n, -1)
    cshape = (prob.m + 1,) * d
    g = np.zeros((n, npc))
    for b in range(npc):
        kb = kap.copy()
        kb.reshape(n, npc)[:, b] += 1j * _CSTEP
        r = u_update_cells_var(prob, np.zeros((d, n) + cshape, dtype=np.complex128), pc, kb)
        g[:, b] = np.sum(ub * r.reshape(d, n, -1).imag, axis=(0, 2)) / _CSTEP
    return g.reshape(Ku.shape)


def kappa_field_gradient(prob: Problem, P0, U0, Kp, Ku, Pbn, Ubn, nsteps: int, p_sources=None):
    """Gradient with respect to the kappa data Kp, Ku of
        <Pbn, P_n> + <Ubn, U_n> + sum_t <p_sources[t], P_{t+1}>
    for n steps of `step_var` from (P0, U0); returns (gKp, gKu, Pb_0, Ub_0),
    the last two being the gradient with respect to (P0, U0).  p_sources[t]
    (optional, one array per step) is the adjoint source of a loss on the
    pressure after step t (e.g. a seismogram misfit at receiver nodes).

    Reverse sweep over the stored trajectory: for step t with adjoint (Pb',
    Ub') of its result, the velocity half-step contributes d/dKu <Ub', -B P'>,
    then Pb = Pb' - B^T Ub', the pressure half-step contributes
    d/dKp <Pb, -A U_t>, then Ub = Ub' - A^T Pb."""
    if prob.walls:
        raise NotImplementedError("the adjoint is built for the periodic grid")
    A, B = p_operator_blocks_var(prob, Kp), u_operator_blocks_var(prob, Ku)
    states = [(np.array(P0, dtype=np.float64), np.array(U0, dtype=np.float64))]
    for _ in range(int(nsteps)):
        P, U = states[-1]
        P1 = p_half_var(prob, P, U, Kp)
        states.append((P1, u_half_var(prob, U, P1, Ku)))
    Pb, Ub = np.array(Pbn, dtype=np.float64), np.array(Ubn, dtype=np.float64)
    gKp = np.zeros(np.shape(Kp))
    gKu = np.zeros(np.shape(Ku))
    for t in range(int(nsteps) - 1, -1, -1):
        if p_sources is not None:
            Pb = Pb + p_sources[t]
        U_t = states[t][1]
        P_1 = states[t + 1][0]
        gKu += _cstep_u(prob, P_1, Ku, Ub)
        Pb = p_half_var_adjoint(prob, Pb, Ub, Ku, B)
        gKp += _cstep_p(prob, U_t, Kp, Pb)
        Ub = u_half_var_adjoint(prob, Ub, Pb, Kp, A)
    return gKp, gKu, Pb, Ub


# ---------------------------------------------------------------------------
# Variable kappa with reflecting walls: the transpose and the kappa gradient
# by their definitions (tiny grids).  For fixed kappa data the walled
# variable-kappa step is linear in the state (P, U), so its transpose is read
# off the unit responses: entry x of J^T y is <step(e_x), y>.  The gradient of
# L = <Pbn, P_n> + <Ubn, U_n> with respect to one kappa entry is taken by
# fourth-order central differences of the step (L is a polynomial in the
# kappa data).  Both work on the periodic grid too, where they check the
# structured adjoint above.
# ---------------------------------------------------------------------------

def step_matrix_var(prob: Problem, Kp, Ku) -> np.ndarray:
    """J with (P', U') = J (P, U), states flattened as the P entries then the U
    entries in their array order; one `step_var` per unit state entry."""
    ps, us = prob.p_shape(), prob.u_shape()
    npn, nun = int(np.prod(ps)), int(np.prod(us))
    J = np.zeros((npn + nun, npn + nun))
    for x in range(npn + nun):
        e = np.zeros(npn + nun)
        e[x] = 1.0
        P1, U1 = step_var(prob, e[:npn].reshape(ps), e[npn:].reshape(us), Kp, Ku, 1)
        J[:, x] = np.concatenate([P1.ravel(), U1.ravel()])
    return J


def adjoint_step_var_bruteforce(prob: Problem, Pb, Ub, Kp, Ku, nsteps: int = 1):
    """(J^T)^nsteps (Pb, Ub) for the step J of `step_var` (either boundary)."""
    J = step_matrix_var(prob, Kp, Ku)
    v = np.concatenate([np.ravel(Pb), np.ravel(Ub)]).astype(np.float64)
    for _ in range(int(nsteps)):
        v = J.T @ v
    npn = int(np.prod(prob.p_shape()))
    return v[:npn].reshape(prob.p_shape()), v[npn:].reshape(prob.u_shape())


def kappa_field_gradient_fd(prob: Problem, P0, U0, Kp, Ku, Pbn, Ubn, nsteps: int, entries, eps: float = 1e-3):
    """dL/dkappa at the listed entries (field, flat index) - field 0: Kp,
    field 1: Ku - of L = <Pbn, P_n> + <Ubn, U_n> after nsteps of `step_var`
    from (P0, U0), by fourth-order central differences with step eps."""
    def L(kp, ku):
        P, U = step_var(prob, P0, U0, kp, ku, nsteps)
        return float(np.sum(Pbn * P) + np.sum(Ubn * U))

    out = []
    for f, i in entries:
        def Ls(s):
            kp, ku = np.array(Kp, dtype=np.float64), np.array(Ku, dtype=np.float64)
            (kp if f == 0 else ku).reshape(-1)[int(i)] += s
            return L(kp, ku)
        out.append((-Ls(2 * eps) + 8 * Ls(eps) - 8 * Ls(-eps) + Ls(-2 * eps)) / (12 * eps))
    return np.array(out)

# ---------------------------------------------------------------------------
# Source term (periodic or walls)
# ---------------------------------------------------------------------------
# p_t = -kappa div u + z(x, t) with z = r(t) g(x) (Sec. 4, eq. (waveEq1D)
# forcing).  The paper does not say how z enters the step.  Reading taken:
# the midpoint rule over the step, P^{n+1} = [pressure half-step] + dt r(t_n +
# dt/2) G, before the velocity half-step (G: scaled Taylor data of g at the
# primal nodes).

def step_with_source(prob: Problem, P, U, G, r, t0: float, nsteps: int, Kp=None, Ku=None):
    """nsteps steps from time t0 with the source r(t) G (r a callable);
    variable kappa when Kp, Ku are given (periodic)."""
    P = np.array(P, dtype=np.float64, copy=True)
    U = np.array(U, dtype=np.float64, copy=True)
    for n in range(int(nsteps)):
        P = p_half(prob, P, U) if Kp is None else p_half_var(prob, P, U, Kp)
        P = P + prob.dt * r(t0 + (n + 0.5) * prob.dt) * G
        U = u_half(prob, U, P) if Ku is None else u_half_var(prob, U, P, Ku)
    return P, U
