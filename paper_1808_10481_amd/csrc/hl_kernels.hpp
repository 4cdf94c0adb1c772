// hl_kernels.hpp - Hermite-leapfrog half-step kernels for gfx950.
//
// One work-item per output node.  For the pressure half-step at primal node
// j the cell's corners are the dual nodes q = j - 1 + e, e in {0,1}^d; for the
// velocity half-step at dual node q they are the primal nodes j = q + e
// (Sec. 2, eqs. (pGrid), (dGrid); Sec. 5).  The interpolant of the corner
// data (Sec. 2, eq. (interp)) is built one dimension at a time (Sec. 5): the
// x pass runs explicitly with compile-time coefficients; the remaining
// dimensions' interpolation and the Cauchy-Kowalevsky weights (Sec. 2,
// eq. (final1); Sec. 3.1.2, eqs. (pdup), (vdup)) are applied together through
// a runtime merged table (hl_layout.hpp) acting on sums and differences of
// corners, so the (2m+2)^d interpolant never exists as a whole.
//
// Storage (hl_storage.hpp) is a template policy S: S::C is the arithmetic
// type, S::load / S::update / S::planes / S::bload the only memory accesses
// to the state.  Planes are coefficient-major: plane index
// comp * (m+1)^d + c, c = a_1 + (m+1)(a_2 + (m+1) a_3), node
// n = i_1 + E_1 (i_2 + E_2 i_3) in an array of extents E.
//
// Boundaries.  Periodic: both grids have K nodes per dimension, corner
// indices wrap.  Reflecting walls: the primal grid has K+1 nodes (the end
// nodes on the walls), the dual grid K nodes stored inside a (K+2)-node array
// whose outer shell holds ghost nodes (filled by ghost_fill before every
// pressure half-step); no index wraps.  A Grid describes one half-step: the
// nodes it updates (K, stored at index j + ooff of the output array) and the
// corner array (corner lo of node j at j + soff, hi at lo + 1, wrapped into
// [0, sext) for periodic grids).
//
// Launch: tiles of TileShape nodes, one workgroup per tile.  Workgroup i runs
// on XCD i mod 8 and takes tile number t = (i mod 8) * per_xcd + i / 8, so
// each XCD sweeps one contiguous band of tile numbers.  Tile numbers run x
// fastest, then y inside a group of `ygroup` tile rows, then z, then the
// groups; in 3D a small group keeps the z-neighbour planes of the tiles in
// flight inside the XCD's L2 (a whole z-plane of corner data does not fit).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "hl_layout.hpp"
#include "hl_storage.hpp"

// Scheduling barrier mask inside the merged-table loop: instruction classes
// allowed to move across (0 = none; 0x2 VALU, 0x4 SALU, 0x20 VMEM reads).
// Scalar table loads never cross, which bounds the table's live range in
// SGPRs; measured on the 2D m=3 workload, 0 is fastest (letting vector loads
// cross raised register pressure and cost 5-8%).
#ifndef HL_SCHED_MASK
#define HL_SCHED_MASK 0
#endif
// Minimum waves per SIMD requested from the register allocator (0 = none).
#ifndef HL_WAVES_PER_EU
#define HL_WAVES_PER_EU 0
#endif
// 3D velocity half-step for m <= 2 through the fully merged table (1) or the
// explicit x pass plus the (y, z) merged table (0).
#ifndef HL_U3_FULL
#define HL_U3_FULL 1
#endif
// 3D tile extent in x and y (x * y = 256 work-items).
#ifndef HL_TILE3_X
#define HL_TILE3_X 64
#endif

namespace hl {

constexpr int kXcds = 8;

struct Grid {
  int32_t K[3];       // nodes updated per dimension (1 for unused dimensions)
  int32_t nt[3];      // tiles per dimension
  int32_t tiles;      // nt[0] * nt[1] * nt[2]
  int32_t per_xcd;    // ceil(tiles / kXcds)
  int32_t ygroup;     // tile rows per group in the tile numbering, 1..nt[1]
  int32_t ooff;       // output node j is stored at index j + ooff (0, or 1 in a ghost-padded array)
  int32_t oext[3];    // output array extents
  int32_t soff;       // lower corner of node j at index j + soff (-1 or 0)
  int32_t sext[3];    // corner (source) array extents
  int32_t tx, ty;     // tile extents in x and y = the workgroup shape (tx * ty <= 256)
  int32_t pad;
  int64_t onodes;     // output array nodes (plane size)
  int64_t snodes;     // source array nodes (plane size)
};

template <int D>
struct TileShape {
  static constexpr int X = D == 1 ? 256 : D == 2 ? 64 : HL_TILE3_X;
  static constexpr int Y = 256 / X;
  static constexpr int Z = 1;
};

// out[b] = sum_l pass_coef<M,FLIP>(b, l) * (b + l + FLIP even ? R_l + L_l : R_l - L_l)
template <int M, int FLIP, typename T>
__device__ __forceinline__ void pass1d(const T* L, const T* R, T* out) {
  constexpr int MP = M + 1, N2 = 2 * M + 2;
  T sg[MP], df[MP];
#pragma unroll
  for (int l = 0; l < MP; ++l) {
    sg[l] = R[l] + L[l];
    df[l] = R[l] - L[l];
  }
#pragma unroll
  for (int b = 0; b < N2; ++b) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < MP; ++l) {
      const double c = pass_coef<M, FLIP>(b, l);
      if (c != 0.0) acc = fma(T(c), ((b + l + FLIP) & 1) ? df[l] : sg[l], acc);
    }
    out[b] = acc;
  }
}

// Node of this work-item in workgroup `blk` of the grid's launch; false when
// outside the grid.
template <int D>
__device__ __forceinline__ bool node_of_block(const Grid& g, int blk, int32_t* j) {
  const int i = blk;
  const int t = (i % kXcds) * g.per_xcd + i / kXcds;
  if (t >= g.tiles) return false;
  int tx = t % g.nt[0], ty = 0, tz = 0;
  if constexpr (D > 1) {
    const int r = t / g.nt[0];
    const int grp_rows = g.ygroup * g.nt[2];  // tile rows (y, z) per group
    const int grp = r / grp_rows;
    const int rem = r - grp * grp_rows;
    const int gy = min(g.ygroup, g.nt[1] - grp * g.ygroup);  // rows of y in this (possibly ragged) group
    ty = grp * g.ygroup + rem % gy;
    tz = rem / gy;
  }
  j[0] = tx * g.tx + threadIdx.x;
  j[1] = ty * g.ty + threadIdx.y;
  j[2] = tz;
  return j[0] < g.K[0] && j[1] < g.K[1] && j[2] < g.K[2];
}

template <int D>
__device__ __forceinline__ uint32_t node_index(int32_t x, int32_t y, int32_t z, const int32_t* E) {
  uint32_t n = (uint32_t)x;
  if (D > 1) n += (uint32_t)E[0] * (uint32_t)y;
  if (D > 2) n += (uint32_t)E[0] * (uint32_t)E[1] * (uint32_t)z;
  return n;
}

// Index of this work-item's output node in the output array.
template <int D>
__device__ __forceinline__ uint32_t out_index(const Grid& g, const int32_t* j) {
  return node_index<D>(j[0] + g.ooff, j[1] + g.ooff, j[2] + g.ooff, g.oext);
}

// Node indices of the 2^d cell corners e (bit k of e: upper side in
// dimension k): lo = j + soff and hi = lo + 1, wrapped into the source array.
template <int D>
__device__ __forceinline__ void corner_nodes(const Grid& g, const int32_t* j, uint32_t* cn) {
  int32_t lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < D) {
      lo[k] = j[k] + g.soff;
      hi[k] = lo[k] + 1;
      if (lo[k] < 0) lo[k] += g.sext[k];
      if (hi[k] == g.sext[k]) hi[k] = 0;
    } else {
      lo[k] = hi[k] = 0;
    }
  }
#pragma unroll
  for (int e = 0; e < (1 << D); ++e)
    cn[e] = node_index<D>((e & 1) ? hi[0] : lo[0], (e & 2) ? hi[1] : lo[1], (e & 4) ? hi[2] : lo[2], g.sext);
}

// entry <- f(entry) at node n0 of plane pl.  3D kernels address their planes
// through buffer descriptors (scalar plane base, 32-bit per-lane offset), the
// others through plain pointers.
template <int D, class S, class F>
__device__ __forceinline__ void update_entry(const typename S::View& v, int pl, uint32_t n0, F f) {
  if constexpr (D == 3) {
    const typename S::Planes pr = S::planes(v, pl);
    S::bstore(pr, n0, f(S::bload(pr, n0)));
  } else {
    S::update(v, pl, n0, f);
  }
}

// p -= acc at node n0.
template <int D, int M, class S>
__device__ __forceinline__ void finish_pressure(const typename S::View& p, uint32_t n0, const typename S::C* acc) {
  using T = typename S::C;
#pragma unroll
  for (int s = 0; s < Dims<D, M>::NC; ++s) update_entry<D, S>(p, s, n0, [&](T x) { return x - acc[s]; });
}

// u_i[s] -= wscale * (s_i + 1) / h_i * Q[s + e_i]   (Q on the set G)
template <int D, int M, class S>
__device__ __forceinline__ void finish_velocity(const typename S::View& u, uint32_t n0, const typename S::C* Q,
                                                typename S::C wscale, const typename S::C* ih) {
  using T = typename S::C;
  constexpr int MP = M + 1, NC = Dims<D, M>::NC;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T f = wscale * ih[i];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      const T a = -(T)(digit(s, MP, i) + 1) * f;
      const T q = Q[kGIndex<D, M>.g[i][s]];
      update_entry<D, S>(u, i * NC + s, n0, [&](T x) { return fma(a, q, x); });
    }
  }
}

// ---------------------------------------------------------------------------
// 1D and 2D kernels: the merged table covers the last dimension.
// ---------------------------------------------------------------------------

// Slice of the interpolant for last-dimension corner eL and last-dimension
// datum l: Y[b], b in {0..2m+1}^{d-1}, from the 2^{d-1} corners with that eL.
// FLIP0 = 1 makes the x pass the derivative pass (units of 1/h_x).  comp:
// field component; cn[e]: corner node indices.
template <int D, int M, int FLIP0, class S>
__device__ __forceinline__ void slice(const typename S::View& f, int comp, const uint32_t* cn, int eL, int l,
                                      typename S::C* Y) {
  using T = typename S::C;
  constexpr int MP = M + 1, NC = Dims<D, M>::NC;
  static_assert(D == 1 || D == 2, "3D uses the x-line kernels");
  if constexpr (D == 1) {
    Y[0] = S::load(f, comp * NC + l, cn[eL]);
  } else {
    T Lv[MP], Rv[MP];
#pragma unroll
    for (int a0 = 0; a0 < MP; ++a0) {
      const int pl = comp * NC + a0 + MP * l;
      Lv[a0] = S::load(f, pl, cn[0 + 2 * eL]);
      Rv[a0] = S::load(f, pl, cn[1 + 2 * eL]);
    }
    pass1d<M, FLIP0>(Lv, Rv, Y);
  }
}

// acc[o] += sum_b Mt[t] * (sigma or delta)[b] over the structurally nonzero
// (o, b) of one merged table row-block (datum l); the walk comes from the
// compile-time MergeSpec, so every index is a constant after unrolling.
template <int D, int M, bool VEL, int FLIPL, typename T, typename TP>
__device__ __forceinline__ void merge(TP Mt, int l, const T* Sg, const T* Df, T* acc) {
  using Sp = MergeSpec<D, M, VEL, FLIPL>;
  // Scalar table loads are consumed in chunks: without the barriers the
  // scheduler hoists every s_load of the table to the top of the kernel and
  // runs out of SGPRs (spilling them through VGPR lanes).
  constexpr int kChunk = sizeof(T) == 8 ? 16 : 32;
#pragma unroll
  for (int t = 0; t < Sp::NNZ; ++t) {
    if (t % kChunk == 0) __builtin_amdgcn_sched_barrier(HL_SCHED_MASK);
    const int o = kMerge<D, M, VEL, FLIPL>.o[t];
    const int b = kMerge<D, M, VEL, FLIPL>.b[t];
    const bool dl = kMerge<D, M, VEL, FLIPL>.base_delta[o] != ((l & 1) != 0);
    acc[o] = fma(Mt[t], dl ? Df[b] : Sg[b], acc[o]);
  }
}

// Sigma/delta of the two last-dimension slices, then the merged table.
template <int D, int M, bool VEL, int FLIP0, int FLIPL, class S, typename TP>
__device__ __forceinline__ void slice_pair_merge(const typename S::View& f, int comp, const uint32_t* cn, int l, TP Mt,
                                                 typename S::C* acc) {
  using T = typename S::C;
  constexpr int NB = Dims<D, M>::NB;
  T YL[NB], YR[NB], Sg[NB], Df[NB];
  slice<D, M, FLIP0, S>(f, comp, cn, 0, l, YL);
  slice<D, M, FLIP0, S>(f, comp, cn, 1, l, YR);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    Sg[b] = YR[b] + YL[b];
    Df[b] = YR[b] - YL[b];
  }
  merge<D, M, VEL, FLIPL>(Mt, l, Sg, Df, acc);
}

// Pressure half-step at every primal node (1D and 2D).
// tab: packed merged tables (hl_layout.hpp TableLayout), in S::C.
template <int D, int M, class S, typename TP>
__device__ __forceinline__ void p_half_body(typename S::View p, typename S::View u,
                                            TP tab,
                                            Grid g, int blk) {
  using T = typename S::C;
  using TL = TableLayout<D, M>;
  constexpr int MP = M + 1, NC = Dims<D, M>::NC;
  constexpr int NNZ = merged_nnz<D, M>(false);
  int32_t j[3];
  if (!node_of_block<D>(g, blk, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);  // dual q = j - 1 + e (p) or primal j = q + e (u)
  T acc[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) acc[s] = T(0);
#pragma unroll
  for (int l = 0; l < MP; ++l) {
    // x-component (2D): derivative pass in x, interpolation in the merged table
    if constexpr (D > 1) slice_pair_merge<D, M, false, 1, 0, S>(u, 0, cn, l, tab + TL::P_A_OFF + l * NNZ, acc);
    // last component: interpolation pass in x, derivative in the merged table
    slice_pair_merge<D, M, false, 0, 1, S>(u, D - 1, cn, l, tab + TL::P_B_OFF + l * NNZ, acc);
  }
  finish_pressure<D, M, S>(p, out_index<D>(g, j), acc);
}

template <int D, int M, class S>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) p_half_kernel(typename S::View p, typename S::View u,
                                                                       const typename S::C* __restrict__ tab,
                                                                       Grid g) {
  p_half_body<D, M, S, const typename S::C* __restrict__>(p, u, tab, g, blockIdx.x);
}

// Velocity half-step at every dual node (1D and 2D), weights scaled by wscale.
template <int D, int M, class S, typename TP>
__device__ __forceinline__ void u_half_body(typename S::View u, typename S::View p,
                                            TP tab,
                                            Grid g, typename S::C wscale,
                                            typename S::C ih0, typename S::C ih1,
                                            typename S::C ih2, int blk) {
  using T = typename S::C;
  using TL = TableLayout<D, M>;
  constexpr int MP = M + 1;
  constexpr int NG = GSet<D, M>::NG;
  constexpr int NNZ = merged_nnz<D, M>(true);
  int32_t j[3];
  if (!node_of_block<D>(g, blk, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);  // dual q = j - 1 + e (p) or primal j = q + e (u)
  T Q[NG];
#pragma unroll
  for (int o = 0; o < NG; ++o) Q[o] = T(0);
#pragma unroll
  for (int l = 0; l < MP; ++l) slice_pair_merge<D, M, true, 0, 0, S>(p, 0, cn, l, tab + TL::U_OFF + l * NNZ, Q);
  const T ih[3] = {ih0, ih1, ih2};
  finish_velocity<D, M, S>(u, out_index<D>(g, j), Q, wscale, ih);
}

template <int D, int M, class S>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) u_half_kernel(typename S::View u, typename S::View p,
                                                                       const typename S::C* __restrict__ tab,
                                                                       Grid g, typename S::C wscale,
                                                                       typename S::C ih0, typename S::C ih1,
                                                                       typename S::C ih2) {
  u_half_body<D, M, S, const typename S::C* __restrict__>(u, p, tab, g, wscale, ih0, ih1, ih2, blockIdx.x);
}

// ---------------------------------------------------------------------------
// 3D kernels.  A work-item interpolates explicitly only along x: for every
// y/z datum pair (a_y, a_z) it loads the 8 corners' x-lines, applies the x
// pass (derivative pass for the x-component of the pressure half-step), and
// combines the four (y, z) corners into sigma/delta in y and in z.  The y and
// z interpolation, the Cauchy-Kowalevsky weights and (for the y- and
// z-components) the divergence are all in the runtime table (Merge3Spec).
// Coefficient planes are read through buffer descriptors, one per plane, with
// a 32-bit per-lane offset: the kernels touch 4 (m+1)^3 planes, too many for
// a 64-bit scalar base each.
// ---------------------------------------------------------------------------

// X[k_y][k_z][b_x] for datum pair (a_y, a_z), whose m+1 coefficient planes
// (a_x = 0..m) start at plane pl0; cn[e], e = e_x + 2 e_y + 4 e_z, are the
// corners' node indices.
template <int M, int FLIPX, class S>
__device__ __forceinline__ void xlines(const typename S::View& f, int pl0, const uint32_t* cn,
                                       typename S::C (&X)[2][2][2 * M + 2]) {
  using T = typename S::C;
  constexpr int MP = M + 1, N2 = 2 * M + 2;
  // for large m keep the loads of different (a_y, a_z) blocks apart, or the
  // scheduler clusters them and runs out of registers
  if constexpr (M >= 3) __builtin_amdgcn_sched_barrier(0);
  typename S::Planes pr[MP];
#pragma unroll
  for (int ax = 0; ax < MP; ++ax) pr[ax] = S::planes(f, pl0 + ax);
  T Y[2][2][N2];  // [e_y][e_z][b_x]
#pragma unroll
  for (int ez = 0; ez < 2; ++ez)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
      T Lv[MP], Rv[MP];
#pragma unroll
      for (int ax = 0; ax < MP; ++ax) {
        Lv[ax] = S::bload(pr[ax], cn[0 + 2 * ey + 4 * ez]);
        Rv[ax] = S::bload(pr[ax], cn[1 + 2 * ey + 4 * ez]);
      }
      pass1d<M, FLIPX>(Lv, Rv, Y[ey][ez]);
    }
#pragma unroll
  for (int b = 0; b < N2; ++b) {
    const T s0 = Y[1][0][b] + Y[0][0][b], d0 = Y[1][0][b] - Y[0][0][b];  // z = lower
    const T s1 = Y[1][1][b] + Y[0][1][b], d1 = Y[1][1][b] - Y[0][1][b];  // z = upper
    X[0][0][b] = s1 + s0;
    X[0][1][b] = s1 - s0;
    X[1][0][b] = d1 + d0;
    X[1][1][b] = d1 - d0;
  }
}

template <int M, bool VEL, int FY, int FZ, typename T, typename TP>
__device__ __forceinline__ void merge3(TP Mt, int ay, int az, const T (&X)[2][2][2 * M + 2], T* acc) {
  constexpr int NNZ = Merge3Spec<M, VEL, FY, FZ>::NNZ;
  constexpr int kChunk = sizeof(T) == 8 ? 16 : 32;
#pragma unroll
  for (int t = 0; t < NNZ; ++t) {
    if (t % kChunk == 0) __builtin_amdgcn_sched_barrier(HL_SCHED_MASK);
    const int o = kMerge3<M, VEL, FY, FZ>.o[t];
    const int bx = kMerge3<M, VEL, FY, FZ>.bx[t];
    const int ky = kMerge3<M, VEL, FY, FZ>.ky[t][ay];
    const int kz = kMerge3<M, VEL, FY, FZ>.kz[t][az];
    acc[o] = fma(Mt[t], X[ky][kz][bx], acc[o]);
  }
}

// Pressure half-step, 3D, m <= 2: the x interpolation is merged into the
// table as well.  Per component i and datum a the 8 corners are combined into
// sigma/delta in x, y and z (X[k], k = k_x + 2 k_y + 4 k_z, 0 = sigma); output
// o takes the combination whose parity in each dimension is that of
// o_k + a_k (+1 in the divergence dimension k = i), times F[i][a][o].  Per
// node and component: 8 loads, 24 add/sub and 27 FMA per datum, against the
// explicit x pass's 72 VALU per datum (at m = 2 the x pass costs more than
// the table it saves).
template <int M, class S, typename TP>
__device__ __forceinline__ void p_half_3d_full_body(typename S::View p, typename S::View u, TP tab, Grid g,
                                                    int blk) {
  using T = typename S::C;
  using TL = TableLayout<3, M>;
  constexpr int MP = M + 1, NC = Dims<3, M>::NC;
  int32_t j[3];
  if (!node_of_block<3>(g, blk, j)) return;
  uint32_t cn[8];
  corner_nodes<3>(g, j, cn);  // dual q = j - 1 + e
  T acc[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) acc[s] = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      // keep the scalar table loads of one datum together (SGPR pressure)
      __builtin_amdgcn_sched_barrier(0);
      const typename S::Planes pr = S::planes(u, i * NC + a);
      T v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = S::bload(pr, cn[e]);
      T X[8];  // [k_x + 2 k_y + 4 k_z]
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // x: corners (2q, 2q+1)
        X[2 * q] = v[2 * q + 1] + v[2 * q];
        X[2 * q + 1] = v[2 * q + 1] - v[2 * q];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = X[q];
#pragma unroll
      for (int kz = 0; kz < 2; ++kz)  // y: pairs (kx + 4 kz, kx + 2 + 4 kz)
#pragma unroll
        for (int kx = 0; kx < 2; ++kx) {
          const T lo = v[kx + 4 * kz], hi = v[kx + 2 + 4 * kz];
          X[kx + 4 * kz] = hi + lo;
          X[kx + 2 + 4 * kz] = hi - lo;
        }
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // z: pairs (q, q + 4)
        const T lo = X[q], hi = X[q + 4];
        v[q] = hi + lo;
        v[q + 4] = hi - lo;
      }
      const int ax = a % MP, ay = (a / MP) % MP, az = a / (MP * MP);
#pragma unroll
      for (int o = 0; o < NC; ++o) {
        const int ox = o % MP, oy = (o / MP) % MP, oz = o / (MP * MP);
        const int k = ((ox + ax + (i == 0)) & 1) + 2 * ((oy + ay + (i == 1)) & 1) + 4 * ((oz + az + (i == 2)) & 1);
        acc[o] = fma(tab[TL::F_OFF + (i * NC + a) * NC + o], v[k], acc[o]);
      }
    }
  finish_pressure<3, M, S>(p, out_index<3>(g, j), acc);
}

template <int M, class S, typename TP>
__device__ __forceinline__ void p_half_3d_body(typename S::View p, typename S::View u,
                                               TP tab, Grid g, int blk) {
  using T = typename S::C;
  using TL = TableLayout<3, M>;
  constexpr int MP = M + 1, NC = Dims<3, M>::NC, N2 = 2 * M + 2;
  constexpr int NNZ = Merge3Spec<M, false, 0, 0>::NNZ;
  int32_t j[3];
  if (!node_of_block<3>(g, blk, j)) return;
  uint32_t cn[8];
  corner_nodes<3>(g, j, cn);  // dual q = j - 1 + e (p) or primal j = q + e (u)
  T acc[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) acc[s] = T(0);
#pragma unroll
  for (int az = 0; az < MP; ++az)
#pragma unroll
    for (int ay = 0; ay < MP; ++ay) {
      const int blk = ay + MP * az;
      {
        T X[2][2][N2];
        xlines<M, 1, S>(u, MP * blk, cn, X);
        merge3<M, false, 0, 0>(tab + TL::p_off(0) + blk * NNZ, ay, az, X, acc);
      }
      {
        T X[2][2][N2];
        xlines<M, 0, S>(u, NC + MP * blk, cn, X);
        merge3<M, false, 1, 0>(tab + TL::p_off(1) + blk * NNZ, ay, az, X, acc);
      }
      {
        T X[2][2][N2];
        xlines<M, 0, S>(u, 2 * NC + MP * blk, cn, X);
        merge3<M, false, 0, 1>(tab + TL::p_off(2) + blk * NNZ, ay, az, X, acc);
      }
    }
  finish_pressure<3, M, S>(p, out_index<3>(g, j), acc);
}

template <int M, class S>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) p_half_3d(typename S::View p, typename S::View u,
                                                                   const typename S::C* __restrict__ tab, Grid g) {
  if constexpr (TableLayout<3, M>::FULL_P)
    p_half_3d_full_body<M, S, const typename S::C* __restrict__>(p, u, tab, g, blockIdx.x);
  else
    p_half_3d_body<M, S, const typename S::C* __restrict__>(p, u, tab, g, blockIdx.x);
}

// Velocity half-step, 3D, m <= 2: the x interpolation merged into the table
// as well (as for the pressure half-step).  Per datum a of the primal corners
// the 8 corner values are combined into the sigma/delta products X[k] (x, y
// and z, k = k_x + 2 k_y + 4 k_z); member o of G takes the product whose
// parity in each dimension is that of o_k + a_k, times Fu[a][o].  Per node:
// 8 loads, 24 add/sub and |G| FMA per datum (27 x 77 VALU at m = 2) against
// the explicit x pass plus the (y, z) merged table (about 2700 VALU).
template <int M, class S, typename TP>
__device__ __forceinline__ void u3_full_Q(const typename S::View& p, const uint32_t* cn, TP tab,
                                          typename S::C* Q) {
  using T = typename S::C;
  using TL = TableLayout<3, M>;
  constexpr int MP = M + 1, NC = Dims<3, M>::NC, NG = GSet<3, M>::NG;
#pragma unroll
  for (int o = 0; o < NG; ++o) Q[o] = T(0);
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    // keep the scalar table loads of one datum together (SGPR pressure)
    __builtin_amdgcn_sched_barrier(0);
    const typename S::Planes pr = S::planes(p, a);
    T v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = S::bload(pr, cn[e]);
    T X[8];  // [k_x + 2 k_y + 4 k_z]
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // x: corners (2q, 2q+1)
      X[2 * q] = v[2 * q + 1] + v[2 * q];
      X[2 * q + 1] = v[2 * q + 1] - v[2 * q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = X[q];
#pragma unroll
    for (int kz = 0; kz < 2; ++kz)  // y: pairs (kx + 4 kz, kx + 2 + 4 kz)
#pragma unroll
      for (int kx = 0; kx < 2; ++kx) {
        const T lo = v[kx + 4 * kz], hi = v[kx + 2 + 4 * kz];
        X[kx + 4 * kz] = hi + lo;
        X[kx + 2 + 4 * kz] = hi - lo;
      }
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // z: pairs (q, q + 4)
      const T lo = X[q], hi = X[q + 4];
      v[q] = hi + lo;
      v[q + 4] = hi - lo;
    }
    const int ax = a % MP, ay = (a / MP) % MP, az = a / (MP * MP);
#pragma unroll
    for (int o = 0; o < NG; ++o) {
      if (o == NG / 2) __builtin_amdgcn_sched_barrier(0);  // two halves of the datum's table loads
      const int k = ((kGSet<3, M>.dig[o][0] + ax) & 1) + 2 * ((kGSet<3, M>.dig[o][1] + ay) & 1) +
                    4 * ((kGSet<3, M>.dig[o][2] + az) & 1);
      Q[o] = fma(tab[TL::FU_OFF + a * NG + o], v[k], Q[o]);
    }
  }
}

template <int M, class S, typename TP>
__device__ __forceinline__ void u_half_3d_body(typename S::View u, typename S::View p,
                                               TP tab, Grid g,
                                               typename S::C wscale, typename S::C ih0,
                                               typename S::C ih1, typename S::C ih2, int blk) {
  using T = typename S::C;
  using TL = TableLayout<3, M>;
  constexpr int MP = M + 1, N2 = 2 * M + 2;
  constexpr int NG = GSet<3, M>::NG;
  constexpr int NNZ = Merge3Spec<M, true, 0, 0>::NNZ;
  int32_t j[3];
  if (!node_of_block<3>(g, blk, j)) return;
  uint32_t cn[8];
  corner_nodes<3>(g, j, cn);  // dual q = j - 1 + e (p) or primal j = q + e (u)
  T Q[NG];
  if constexpr (TL::FULL_U && HL_U3_FULL) {
    u3_full_Q<M, S>(p, cn, tab, Q);
  } else {
#pragma unroll
    for (int o = 0; o < NG; ++o) Q[o] = T(0);
#pragma unroll
    for (int az = 0; az < MP; ++az)
#pragma unroll
      for (int ay = 0; ay < MP; ++ay) {
        const int blk = ay + MP * az;
        T X[2][2][N2];
        xlines<M, 0, S>(p, MP * blk, cn, X);
        merge3<M, true, 0, 0>(tab + TL::U_OFF + blk * NNZ, ay, az, X, Q);
      }
  }
  const T ih[3] = {ih0, ih1, ih2};
  finish_velocity<3, M, S>(u, out_index<3>(g, j), Q, wscale, ih);
}

template <int M, class S>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) u_half_3d(typename S::View u, typename S::View p,
                                                                   const typename S::C* __restrict__ tab, Grid g,
                                                                   typename S::C wscale, typename S::C ih0,
                                                                   typename S::C ih1, typename S::C ih2) {
  u_half_3d_body<M, S, const typename S::C* __restrict__>(u, p, tab, g, wscale, ih0, ih1, ih2, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Ghost dual nodes for reflecting walls (Sec. 5, "Imposing reflective boundary
// conditions"): p = 0 on the walls makes p odd across each wall, so by
// u_t = -grad p the normal velocity component is even and the tangential ones
// odd.  The velocity array is padded by one node per side (extents E_k =
// K_k + 2); each shell node is the mirror of the interior node reached by
// reflecting every ghost index across its wall (0 <- 1, E-1 <- E-2).  A scaled
// coefficient mirrored in dimension k gets (-1)^{a_k}, and -1 more for a
// tangential component (i != k).  Edge and corner ghosts are mirrors in
// several dimensions at once.
//
// Launch: grid (ceil(max face nodes / 256), D), block 256.  Face k (grid y)
// holds the shell nodes whose first ghost index is in dimension k: index k in
// {0, E_k - 1}, indices j < k interior, indices j > k anything; every shell
// node is written by exactly one work-item.
// ---------------------------------------------------------------------------
template <int D, int M, class S>
__global__ void __launch_bounds__(256) ghost_fill(typename S::View u, int32_t E0, int32_t E1, int32_t E2) {
  using T = typename S::C;
  constexpr int MP = M + 1, NC = Dims<D, M>::NC;
  const int32_t E[3] = {E0, E1, E2};
  const int k = blockIdx.y;
  int64_t cnt = 2;
  for (int j = 0; j < D; ++j)
    if (j != k) cnt *= (j < k) ? (E[j] - 2) : E[j];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  int32_t idx[3] = {0, 0, 0};
  int64_t r = t / 2;
  for (int j = 0; j < D; ++j) {
    if (j == k) {
      idx[j] = (t % 2) ? E[j] - 1 : 0;
    } else if (j < k) {
      idx[j] = 1 + (int32_t)(r % (E[j] - 2));
      r /= (E[j] - 2);
    } else {
      idx[j] = (int32_t)(r % E[j]);
      r /= E[j];
    }
  }
  int32_t src[3] = {0, 0, 0};
  bool mir[3] = {false, false, false};
  for (int j = 0; j < D; ++j) {
    mir[j] = idx[j] == 0 || idx[j] == E[j] - 1;
    src[j] = idx[j] == 0 ? 1 : (idx[j] == E[j] - 1 ? E[j] - 2 : idx[j]);
  }
  const uint32_t n_dst = node_index<D>(idx[0], idx[1], idx[2], E);
  const uint32_t n_src = node_index<D>(src[0], src[1], src[2], E);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      bool neg = false;
#pragma unroll
      for (int j = 0; j < D; ++j)
        if (mir[j]) neg ^= ((digit(c, MP, j) & 1) != 0) != (i != j);
      const T v = S::load(u, i * NC + c, n_src);
      S::store(u, i * NC + c, n_dst, neg ? -v : v);
    }
}

// ---------------------------------------------------------------------------
// Discrete adjoint (periodic grids).  A step maps (P, U) to P' = P - A U,
// U' = U - B P'; its transpose is Pb <- Pb - B^T Ub, then Ub <- Ub - A^T Pb:
// the transposed half-steps in reverse order.  On the periodic grid each
// transposed half-step is again a gather with the forward stencil: B^T Ub at
// primal node j reads the dual nodes q = j - 1 + e' (the pressure half-step's
// corners) and A^T Pb at dual node q reads the primal nodes j = q + e' (the
// velocity half-step's), so no atomics are needed.  The operators are dense
// per corner: T[e'][io][ii][r][c] (nc x nc blocks for output component io and
// input component ii), built on the host from the same interpolation and
// weight operators as the forward tables.
//   PTYPE = true:  out = Pb (1 component), in = Ub (D components)
//   PTYPE = false: out = Ub (D components), in = Pb (1 component)
// ---------------------------------------------------------------------------
constexpr int kAdjointMaxNC = 27;  // register budget: nc inputs + nc accumulators

template <int D, int M, class S, bool PTYPE>
__device__ __forceinline__ void adjoint_half_body(typename S::View out, typename S::View in,
                                                  const typename S::C* __restrict__ tab, Grid g, int blk) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC, NO = PTYPE ? 1 : D, NI = PTYPE ? D : 1;
  static_assert(NC <= kAdjointMaxNC, "adjoint kernels are built for nc <= 27");
  int32_t j[3];
  if (!node_of_block<D>(g, blk, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);
  const uint32_t n0 = out_index<D>(g, j);
#pragma unroll 1
  for (int io = 0; io < NO; ++io) {
    T acc[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) acc[r] = T(0);
#pragma unroll
    for (int e = 0; e < (1 << D); ++e) {
#pragma unroll 1
      for (int ii = 0; ii < NI; ++ii) {
        T src[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) src[c] = S::load(in, ii * NC + c, cn[e]);
        const T* __restrict__ Tb = tab + ((int64_t)((e * NO + io) * NI + ii) * NC) * NC;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
          // keep the scalar table loads of one row together (SGPR pressure)
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[r] = fma(Tb[r * NC + c], src[c], acc[r]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NC; ++r) S::update(out, io * NC + r, n0, [&](T x) { return x - acc[r]; });
  }
}

template <int D, int M, class S, bool PTYPE>
__global__ void __launch_bounds__(256) adjoint_half(typename S::View out, typename S::View in,
                                                    const typename S::C* __restrict__ tab, Grid g) {
  adjoint_half_body<D, M, S, PTYPE>(out, in, tab, g, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Variable coefficient kappa(x) (Sec. 4, "Smoothly varying wave speed"):
// kappa is given per node as a Taylor polynomial of degree 2m+1 per variable
// (scaled like the data), about the primal nodes for the pressure half-step
// and the dual nodes for the velocity half-step.  From p_t = -kappa div u and
// u_t = -grad p the odd time derivatives are
//   d_t^{2k+1} p = -(kappa Lap)^k (kappa div u),   d_t^{2k+1} u = -grad (kappa Lap)^k p,
// evaluated on the cell polynomials with every product truncated to degree
// 2m+1 per variable, k = 0..kmax, kmax = d m (the last k at which Lap^k of a
// polynomial of degree 2m+1 in each variable can be nonzero, i.e. where the
// constant-coefficient series ends; with variable kappa the series would go
// on, and this length is a reading for d >= 2):
//   P <- P - sum_k w_k r_k,   r_0 = T[kappa div c],  r_k = T[kappa Lap r_{k-1}]
//   U_i <- U_i - sum_k w_k D_i g_k,   g_0 = c,  g_k = T[kappa Lap g_{k-1}].
// No operator can be merged into a constant table here (kappa differs per
// cell), so the kernels build the full (2m+2)^d interpolant in registers;
// built for d = 1 (all m) and d = 2 (m <= 3).
// ---------------------------------------------------------------------------
template <int D, int M>
struct VK {
  static constexpr int N2 = 2 * M + 2, MP = M + 1;
  static constexpr int NP = ipow(N2, D);            // cell polynomial coefficients
  static constexpr int KMAX = D * M;
};

// The series is accumulated as t_k = w_k r_k with t_k = (w_k / w_{k-1})
// T[kappa Lap t_{k-1}]: the ratio (dt/2)^2 / (2k (2k+1)) cancels the 1/h^2 of
// each Laplacian, so every term stays O(1) (r_k alone grows like h^{-2k} and
// overflows FP32 for large m).
template <typename T>
struct VarArgs {
  T w0;        // w_0 = dt
  T ratio[9];  // w_k / w_{k-1} = (dt/2)^2 / (2k (2k+1)), k = 1..kmax (kmax <= 8)
  T ih[3];     // 1 / h_k
};

// Full interpolant c[b_x + N2 (b_y + N2 b_z)] of one component from its 2^D
// corner blocks.
template <int D, int M, class S>
__device__ __forceinline__ void interp_full(const typename S::View& f, int comp, const uint32_t* cn,
                                            typename S::C* c) {
  using T = typename S::C;
  constexpr int MP = M + 1, N2 = 2 * M + 2, NC = Dims<D, M>::NC;
  if constexpr (D == 3) {
    // x pass on the 8 corners' x-lines per (a_y, a_z), then y, then z
    T Xc[2][2][MP][MP][N2];  // [e_y][e_z][a_y][a_z][b_x]
#pragma unroll
    for (int ez = 0; ez < 2; ++ez)
#pragma unroll
      for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int az = 0; az < MP; ++az)
#pragma unroll
          for (int ay = 0; ay < MP; ++ay) {
            T L[MP], R[MP];
#pragma unroll
            for (int ax = 0; ax < MP; ++ax) {
              const int pl = comp * NC + ax + MP * (ay + MP * az);
              L[ax] = S::load(f, pl, cn[0 + 2 * ey + 4 * ez]);
              R[ax] = S::load(f, pl, cn[1 + 2 * ey + 4 * ez]);
            }
            pass1d<M, 0>(L, R, Xc[ey][ez][ay][az]);
          }
    T Yc[2][MP][N2][N2];  // [e_z][a_z][b_x][b_y]
#pragma unroll
    for (int ez = 0; ez < 2; ++ez)
#pragma unroll
      for (int az = 0; az < MP; ++az)
#pragma unroll
        for (int bx = 0; bx < N2; ++bx) {
          T L[MP], R[MP];
#pragma unroll
          for (int ay = 0; ay < MP; ++ay) {
            L[ay] = Xc[0][ez][ay][az][bx];
            R[ay] = Xc[1][ez][ay][az][bx];
          }
          pass1d<M, 0>(L, R, Yc[ez][az][bx]);
        }
#pragma unroll
    for (int by = 0; by < N2; ++by)
#pragma unroll
      for (int bx = 0; bx < N2; ++bx) {
        T L[MP], R[MP], out[N2];
#pragma unroll
        for (int az = 0; az < MP; ++az) {
          L[az] = Yc[0][az][bx][by];
          R[az] = Yc[1][az][bx][by];
        }
        pass1d<M, 0>(L, R, out);
#pragma unroll
        for (int bz = 0; bz < N2; ++bz) c[bx + N2 * (by + N2 * bz)] = out[bz];
      }
  } else if constexpr (D == 1) {
    T L[MP], R[MP];
#pragma unroll
    for (int a = 0; a < MP; ++a) {
      L[a] = S::load(f, comp * NC + a, cn[0]);
      R[a] = S::load(f, comp * NC + a, cn[1]);
    }
    pass1d<M, 0>(L, R, c);
  } else {
    T Yl[MP][N2], Yh[MP][N2];  // x pass at the lower / upper y corners, per a_y
#pragma unroll
    for (int ay = 0; ay < MP; ++ay) {
      T L[MP], R[MP];
#pragma unroll
      for (int ax = 0; ax < MP; ++ax) {
        L[ax] = S::load(f, comp * NC + ax + MP * ay, cn[0]);
        R[ax] = S::load(f, comp * NC + ax + MP * ay, cn[1]);
      }
      pass1d<M, 0>(L, R, Yl[ay]);
#pragma unroll
      for (int ax = 0; ax < MP; ++ax) {
        L[ax] = S::load(f, comp * NC + ax + MP * ay, cn[2]);
        R[ax] = S::load(f, comp * NC + ax + MP * ay, cn[3]);
      }
      pass1d<M, 0>(L, R, Yh[ay]);
    }
#pragma unroll
    for (int bx = 0; bx < N2; ++bx) {
      T L[MP], R[MP], out[N2];
#pragma unroll
      for (int ay = 0; ay < MP; ++ay) {
        L[ay] = Yl[ay][bx];
        R[ay] = Yh[ay][bx];
      }
      pass1d<M, 0>(L, R, out);
#pragma unroll
      for (int by = 0; by < N2; ++by) c[bx + N2 * by] = out[by];
    }
  }
}

// out += kappa_A f shifted by A (one term of the truncated product; A is a
// template argument so that every register index is a compile-time constant:
// as one 64 x 64 loop nest the compiler stopped unrolling and indexed f
// through scratch memory).
template <int D, int M, int A, class S>
__device__ __forceinline__ void tprod_term(const typename S::View& kv, uint32_t n0, const typename S::C* f,
                                           typename S::C* out) {
  constexpr int N2 = 2 * M + 2, AX = A % N2, AY = (A / N2) % N2, AZ = A / (N2 * N2);
  constexpr int NY = D > 1 ? N2 : 1, NZ = D > 2 ? N2 : 1;
  const typename S::C ka = S::load(kv, A, n0);
#pragma unroll
  for (int bz = AZ; bz < NZ; ++bz)
#pragma unroll
    for (int by = AY; by < NY; ++by)
#pragma unroll
      for (int bx = AX; bx < N2; ++bx) {
        const int o = bx + N2 * (by + N2 * bz);
        out[o] = fma(ka, f[(bx - AX) + N2 * ((by - AY) + N2 * (bz - AZ))], out[o]);
      }
}

template <int D, int M, class S, int... A>
__device__ __forceinline__ void tprod_terms(const typename S::View& kv, uint32_t n0, const typename S::C* f,
                                            typename S::C* out, std::integer_sequence<int, A...>) {
  (tprod_term<D, M, A, S>(kv, n0, f, out), ...);
}

// out = T[kappa f]: out_b = sum_{a <= b} kappa_a f_{b-a} (per variable),
// kappa_a read from plane a of the kappa array at node n0.
template <int D, int M, class S>
__device__ __forceinline__ void tprod(const typename S::View& kv, uint32_t n0, const typename S::C* f,
                                      typename S::C* out) {
  using T = typename S::C;
  constexpr int NP = VK<D, M>::NP;
#pragma unroll
  for (int b = 0; b < NP; ++b) out[b] = T(0);
  tprod_terms<D, M, S>(kv, n0, f, out, std::make_integer_sequence<int, NP>{});
}

// out = sc Lap f in coefficient space: sc sum_i (b_i + 1)(b_i + 2) / h_i^2 f_{b + 2 e_i}.
template <int D, int M, typename T>
__device__ __forceinline__ void lap_coef(const T* f, T* out, const T* ih, T sc) {
  constexpr int N2 = 2 * M + 2, NP = VK<D, M>::NP;
  const T ix2 = sc * ih[0] * ih[0], iy2 = sc * ih[1] * ih[1], iz2 = sc * ih[2] * ih[2];
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    const int bx = b % N2, by = (b / N2) % N2, bz = b / (N2 * N2);
    T v = T(0);
    if (bx + 2 < N2) v = fma(T((bx + 1) * (bx + 2)) * ix2, f[b + 2], v);
    if (D > 1 && by + 2 < N2) v = fma(T((by + 1) * (by + 2)) * iy2, f[b + 2 * N2], v);
    if (D > 2 && bz + 2 < N2) v = fma(T((bz + 1) * (bz + 2)) * iz2, f[b + 2 * N2 * N2], v);
    out[b] = v;
  }
}

// Index of the cell-polynomial coefficient s + delta (s in {0..m}^D in the
// data's order, delta a shift per dimension) in the (2m+2)^D layout.
template <int D, int M>
__host__ __device__ constexpr int poly_index(int s, int dx, int dy, int dz) {
  constexpr int MP = M + 1, N2 = 2 * M + 2;
  const int sx = s % MP, sy = D > 1 ? (s / MP) % MP : 0, sz = D > 2 ? s / (MP * MP) : 0;
  return (sx + dx) + N2 * ((sy + dy) + N2 * (sz + dz));
}

template <int D, int M, class S>
__device__ __forceinline__ void p_half_var_body(typename S::View p, typename S::View u, typename S::View kp,
                                                Grid g, VarArgs<typename S::C> va, int blk) {
  using T = typename S::C;
  constexpr int N2 = 2 * M + 2, MP = M + 1, NP = VK<D, M>::NP, NC = Dims<D, M>::NC;
  int32_t j[3];
  if (!node_of_block<D>(g, blk, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);  // dual q = j - 1 + e
  const uint32_t n0 = out_index<D>(g, j);
  T div[NP];  // w_0 div c
#pragma unroll
  for (int b = 0; b < NP; ++b) div[b] = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T c[NP];
    interp_full<D, M, S>(u, i, cn, c);
    const int st = i == 0 ? 1 : i == 1 ? N2 : N2 * N2;
    const T f = va.w0 * va.ih[i];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int bi = (b / st) % N2;
      if (bi + 1 < N2) div[b] = fma(T(bi + 1) * f, c[b + st], div[b]);
    }
  }
  T t[NP], acc[NC];
  tprod<D, M, S>(kp, n0, div, t);  // t_0 = w_0 r_0
#pragma unroll
  for (int s = 0; s < NC; ++s) acc[s] = t[poly_index<D, M>(s, 0, 0, 0)];
#pragma unroll 1
  for (int k = 1; k <= VK<D, M>::KMAX; ++k) {
    T l[NP];
    lap_coef<D, M>(t, l, va.ih, va.ratio[k]);
    tprod<D, M, S>(kp, n0, l, t);  // t_k = w_k r_k
#pragma unroll
    for (int s = 0; s < NC; ++s) acc[s] += t[poly_index<D, M>(s, 0, 0, 0)];
  }
  finish_pressure<D, M, S>(p, n0, acc);
}

template <int D, int M, class S>
__global__ void __launch_bounds__(256) p_half_var(typename S::View p, typename S::View u, typename S::View kp,
                                                  Grid g, VarArgs<typename S::C> va) {
  p_half_var_body<D, M, S>(p, u, kp, g, va, blockIdx.x);
}

template <int D, int M, class S>
__device__ __forceinline__ void u_half_var_body(typename S::View u, typename S::View p, typename S::View ku,
                                                Grid g, VarArgs<typename S::C> va, typename S::C wscale, int blk) {
  using T = typename S::C;
  constexpr int N2 = 2 * M + 2, MP = M + 1, NP = VK<D, M>::NP, NC = Dims<D, M>::NC;
  int32_t j[3];
  if (!node_of_block<D>(g, blk, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);  // primal j = q + e
  const uint32_t n0 = out_index<D>(g, j);
  T gk[NP], q[NP];  // gk: t_k = w_k g_k
  interp_full<D, M, S>(p, 0, cn, gk);
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    gk[b] *= va.w0;
    q[b] = gk[b];
  }
#pragma unroll 1
  for (int k = 1; k <= VK<D, M>::KMAX; ++k) {
    T l[NP];
    lap_coef<D, M>(gk, l, va.ih, va.ratio[k]);
    tprod<D, M, S>(ku, n0, l, gk);
#pragma unroll
    for (int b = 0; b < NP; ++b) q[b] += gk[b];
  }
  // u_i[s] -= wscale (s_i + 1) / h_i q[s + e_i]
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T f = wscale * va.ih[i];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      const int si = digit(s, MP, i);
      const T qv = q[poly_index<D, M>(s, i == 0, i == 1, i == 2)];
      const T a = -(T)(si + 1) * f;
      S::update(u, i * NC + s, n0, [&](T x) { return fma(a, qv, x); });
    }
  }
}

template <int D, int M, class S>
__global__ void __launch_bounds__(256) u_half_var(typename S::View u, typename S::View p, typename S::View ku,
                                                  Grid g, VarArgs<typename S::C> va, typename S::C wscale) {
  u_half_var_body<D, M, S>(u, p, ku, g, va, wscale, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Variable kappa: transposed half-steps and the gradient with respect to the
// kappa data.  The increment of a half-step at one node, paired with adjoint
// data y spread onto the cell polynomial, is
//   S = <y, sum_k t_k>,   t_0 = T[kappa f] (pressure) or f (velocity),
//   t_k = r_k T[kappa Lap t_{k-1}],   r_k = w_k / w_{k-1},
// with f = w_0 div c (pressure) or w_0 c (velocity).  With the adjoint series
//   lam_kmax = y,   lam_{k-1} = y + r_k Lap^T T^T[kappa] lam_k
// (T^T[kappa] g: b -> sum_a kappa_a g_{a+b}) one has S = <lam_0, t_0>, so
//   dS/df = T^T[kappa] lam_0 (pressure), lam_0 (velocity), and
//   dS/dkappa_a = sum_k sum_b lam_k[a + b] g_k[b],
//   g_k = r_k Lap t_{k-1} (k >= 1), g_0 = f (pressure side only).
// The transposed interpolation then spreads dS/dc onto the 2^d corner blocks
// (a gather over the neighbouring cells, second kernel).  t_{k-1} is
// recomputed from t_0 for each k: no per-node stack of kmax polynomials.
// ---------------------------------------------------------------------------

// out_b += kappa_A g_{A+b} (one term of the transposed truncated product).
template <int D, int M, int A, class S>
__device__ __forceinline__ void tprodT_term(const typename S::View& kv, uint32_t n0, const typename S::C* g,
                                            typename S::C* out) {
  constexpr int N2 = 2 * M + 2, AX = A % N2, AY = A / N2, NY = D > 1 ? N2 : 1;
  const typename S::C ka = S::load(kv, A, n0);
#pragma unroll
  for (int by = 0; by + AY < NY; ++by)
#pragma unroll
    for (int bx = 0; bx + AX < N2; ++bx) out[bx + N2 * by] = fma(ka, g[(bx + AX) + N2 * (by + AY)], out[bx + N2 * by]);
}

template <int D, int M, class S, int... A>
__device__ __forceinline__ void tprodT_terms(const typename S::View& kv, uint32_t n0, const typename S::C* g,
                                             typename S::C* out, std::integer_sequence<int, A...>) {
  (tprodT_term<D, M, A, S>(kv, n0, g, out), ...);
}

// out = T^T[kappa] g.
template <int D, int M, class S>
__device__ __forceinline__ void tprodT(const typename S::View& kv, uint32_t n0, const typename S::C* g,
                                       typename S::C* out) {
  using T = typename S::C;
  constexpr int NP = VK<D, M>::NP;
#pragma unroll
  for (int b = 0; b < NP; ++b) out[b] = T(0);
  tprodT_terms<D, M, S>(kv, n0, g, out, std::make_integer_sequence<int, NP>{});
}

// grad_A += sum_b lam_{A+b} g_b (the kappa_A derivative of <lam, T[kappa g]>).
template <int D, int M, int A, typename T>
__device__ __forceinline__ void corr_term(const T* lam, const T* g, T* grad) {
  constexpr int N2 = 2 * M + 2, AX = A % N2, AY = A / N2, NY = D > 1 ? N2 : 1;
  T acc = grad[A];
#pragma unroll
  for (int by = 0; by + AY < NY; ++by)
#pragma unroll
    for (int bx = 0; bx + AX < N2; ++bx) acc = fma(lam[(bx + AX) + N2 * (by + AY)], g[bx + N2 * by], acc);
  grad[A] = acc;
}

template <int D, int M, typename T, int... A>
__device__ __forceinline__ void corr_terms(const T* lam, const T* g, T* grad, std::integer_sequence<int, A...>) {
  (corr_term<D, M, A>(lam, g, grad), ...);
}

template <int D, int M, typename T>
__device__ __forceinline__ void corr(const T* lam, const T* g, T* grad) {
  corr_terms<D, M>(lam, g, grad, std::make_integer_sequence<int, VK<D, M>::NP>{});
}

// out = sc Lap^T f: sc sum_i (b_i - 1) b_i / h_i^2 f_{b - 2 e_i}.
template <int D, int M, typename T>
__device__ __forceinline__ void lapT_coef(const T* f, T* out, const T* ih, T sc) {
  constexpr int N2 = 2 * M + 2, NP = VK<D, M>::NP;
  const T ix2 = sc * ih[0] * ih[0], iy2 = sc * ih[1] * ih[1];
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    const int bx = b % N2, by = b / N2;
    T v = T(0);
    if (bx >= 2) v = fma(T((bx - 1) * bx) * ix2, f[b - 2], v);
    if (D > 1 && by >= 2) v = fma(T((by - 1) * by) * iy2, f[b - 2 * N2], v);
    out[b] = v;
  }
}

// The series part shared by both sides: given t_0 and y, returns lam_0 in lam
// and adds sum_{k >= 1} sum_b lam_k[a + b] g_k[b] to grad.
template <int D, int M, class S>
__device__ __forceinline__ void adjoint_series(const typename S::View& kv, uint32_t n0, const typename S::C* t0,
                                               const typename S::C* y, const VarArgs<typename S::C>& va,
                                               typename S::C* lam, typename S::C* grad) {
  using T = typename S::C;
  constexpr int NP = VK<D, M>::NP;
#pragma unroll
  for (int b = 0; b < NP; ++b) lam[b] = y[b];
#pragma unroll 1
  for (int k = VK<D, M>::KMAX; k >= 1; --k) {
    T t[NP], l[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) t[b] = t0[b];
#pragma unroll 1
    for (int q = 1; q < k; ++q) {  // t = t_{k-1}
      lap_coef<D, M>(t, l, va.ih, va.ratio[q]);
      tprod<D, M, S>(kv, n0, l, t);
    }
    lap_coef<D, M>(t, l, va.ih, va.ratio[k]);  // g_k
    corr<D, M>(lam, l, grad);
    tprodT<D, M, S>(kv, n0, lam, t);
    lapT_coef<D, M>(t, l, va.ih, va.ratio[k]);
#pragma unroll
    for (int b = 0; b < NP; ++b) lam[b] = y[b] + l[b];
  }
}

// Pressure side at primal node j: with Pb the adjoint pressure and U_t the
// velocity before the step, gk -= dS/dkappa (FP64 accumulators, one plane per
// kappa coefficient) and rho_i = d S / d c^(i) (D NP planes of scratch).
template <int D, int M, class S>
__global__ void __launch_bounds__(256) grad_p_var(typename S::View pb, typename S::View u, typename S::View kp,
                                                  double* __restrict__ gk, typename S::View rho, Grid g,
                                                  VarArgs<typename S::C> va) {
  using T = typename S::C;
  constexpr int N2 = 2 * M + 2, MP = M + 1, NP = VK<D, M>::NP, NC = Dims<D, M>::NC;
  int32_t j[3];
  if (!node_of_block<D>(g, blockIdx.x, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);  // dual q = j - 1 + e
  const uint32_t n0 = out_index<D>(g, j);
  T f[NP];  // f = w_0 div c
#pragma unroll
  for (int b = 0; b < NP; ++b) f[b] = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T c[NP];
    interp_full<D, M, S>(u, i, cn, c);
    const int st = i == 0 ? 1 : N2;
    const T w = va.w0 * va.ih[i];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int bi = i == 0 ? b % N2 : b / N2;
      if (bi + 1 < N2) f[b] = fma(T(bi + 1) * w, c[b + st], f[b]);
    }
  }
  T y[NP], t0[NP], lam[NP], grad[NP];
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    y[b] = T(0);
    grad[b] = T(0);
  }
#pragma unroll
  for (int s = 0; s < NC; ++s) y[(s % MP) + N2 * (s / MP)] = S::load(pb, s, n0);
  tprod<D, M, S>(kp, n0, f, t0);
  adjoint_series<D, M, S>(kp, n0, t0, y, va, lam, grad);
  corr<D, M>(lam, f, grad);  // k = 0: t_0 = T[kappa f]
#pragma unroll
  for (int b = 0; b < NP; ++b) gk[(size_t)b * g.onodes + n0] -= (double)grad[b];
  T phi[NP];  // dS/df
  tprodT<D, M, S>(kp, n0, lam, phi);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T w = va.w0 * va.ih[i];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int bi = i == 0 ? b % N2 : b / N2;
      const T v = bi >= 1 ? T(bi) * w * phi[b - (i == 0 ? 1 : N2)] : T(0);
      S::store(rho, i * NP + b, n0, v);
    }
  }
}

// Velocity side at dual node q: with Ub the adjoint velocity and P' the
// pressure after the step's pressure half-step, gk -= dS/dkappa and
// z = dS/dc (NP planes of scratch).
template <int D, int M, class S>
__global__ void __launch_bounds__(256) grad_u_var(typename S::View ub, typename S::View p, typename S::View ku,
                                                  double* __restrict__ gk, typename S::View z, Grid g,
                                                  VarArgs<typename S::C> va) {
  using T = typename S::C;
  constexpr int N2 = 2 * M + 2, MP = M + 1, NP = VK<D, M>::NP, NC = Dims<D, M>::NC;
  int32_t j[3];
  if (!node_of_block<D>(g, blockIdx.x, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);  // primal j = q + e
  const uint32_t n0 = out_index<D>(g, j);
  T t0[NP], y[NP], lam[NP], grad[NP];
  interp_full<D, M, S>(p, 0, cn, t0);
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    t0[b] *= va.w0;
    y[b] = T(0);
    grad[b] = T(0);
  }
  // S = sum_i sum_s Ub_i[s] (s_i + 1) / h_i Q[s + e_i]
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      const int sx = s % MP, sy = s / MP;
      const int si = i == 0 ? sx : sy;
      y[(sx + (i == 0)) + N2 * (sy + (i == 1))] += T(si + 1) * va.ih[i] * S::load(ub, i * NC + s, n0);
    }
  adjoint_series<D, M, S>(ku, n0, t0, y, va, lam, grad);
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    gk[(size_t)b * g.onodes + n0] -= (double)grad[b];
    S::store(z, b, n0, va.w0 * lam[b]);
  }
}

// acc[a] += sum_b H_e(b, a) z[b]: the transposed interpolation onto corner e
// (bit k: upper side in dimension k) of a cell.  H_e(b, a) is the weight of
// corner datum a in coefficient b of the interpolant: pass_coef for the upper
// corner, with the sign of the delta combination for the lower one.
template <int M, int SIDE>
constexpr double hcol(int b, int a) {
  return pass_coef<M, 0>(b, a) * ((SIDE == 0 && ((b + a) & 1)) ? -1.0 : 1.0);
}

template <int D, int M, int E, typename T>
__device__ __forceinline__ void interp_T(const T* z, T* acc) {
  constexpr int N2 = 2 * M + 2, MP = M + 1;
  if constexpr (D == 1) {
#pragma unroll
    for (int a = 0; a < MP; ++a)
#pragma unroll
      for (int b = 0; b < N2; ++b) {
        const double h = hcol<M, E & 1>(b, a);
        if (h != 0.0) acc[a] = fma(T(h), z[b], acc[a]);
      }
  } else {
    T zy[N2][MP];
#pragma unroll
    for (int bx = 0; bx < N2; ++bx)
#pragma unroll
      for (int ay = 0; ay < MP; ++ay) {
        T v = T(0);
#pragma unroll
        for (int by = 0; by < N2; ++by) {
          const double h = hcol<M, (E >> 1) & 1>(by, ay);
          if (h != 0.0) v = fma(T(h), z[bx + N2 * by], v);
        }
        zy[bx][ay] = v;
      }
#pragma unroll
    for (int ay = 0; ay < MP; ++ay)
#pragma unroll
      for (int ax = 0; ax < MP; ++ax)
#pragma unroll
        for (int bx = 0; bx < N2; ++bx) {
          const double h = hcol<M, E & 1>(bx, ax);
          if (h != 0.0) acc[ax + MP * ay] = fma(T(h), zy[bx][ay], acc[ax + MP * ay]);
        }
  }
}

template <int D, int M, class S, int EP>
__device__ __forceinline__ void gather_corner(const typename S::View& scr, int comp, uint32_t node,
                                              typename S::C* acc) {
  constexpr int NP = VK<D, M>::NP;
  typename S::C z[NP];
#pragma unroll
  for (int b = 0; b < NP; ++b) z[b] = S::load(scr, comp * NP + b, node);
  // slot EP of the output node's stencil is corner E = EP ^ (2^D - 1) of the
  // source node's cell
  interp_T<D, M, EP ^ ((1 << D) - 1)>(z, acc);
}

template <int D, int M, class S, int... EP>
__device__ __forceinline__ void gather_corners(const typename S::View& scr, int comp, const uint32_t* cn,
                                               typename S::C* acc, std::integer_sequence<int, EP...>) {
  (gather_corner<D, M, S, EP>(scr, comp, cn[EP], acc), ...);
}

// Second stage of a transposed variable-kappa half-step: out -= the
// transposed interpolation of the per-cell dS/dc held in scr over the
// output node's stencil (the source node's cell has the output node as
// corner 1 - e where the output's stencil has the source as slot e).
//   PTYPE = true:  out = Pb (primal), scr = z over the dual nodes (NP planes)
//   PTYPE = false: out = Ub (dual, D components), scr = rho over the primal
//                  nodes (D NP planes)
template <int D, int M, class S, bool PTYPE>
__global__ void __launch_bounds__(256) var_adjoint_gather(typename S::View out, typename S::View scr, Grid g) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC, NO = PTYPE ? 1 : D;
  int32_t j[3];
  if (!node_of_block<D>(g, blockIdx.x, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);
  const uint32_t n0 = out_index<D>(g, j);
#pragma unroll 1
  for (int io = 0; io < NO; ++io) {
    T acc[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) acc[a] = T(0);
    gather_corners<D, M, S>(scr, io, cn, acc, std::make_integer_sequence<int, (1 << D)>{});
#pragma unroll
    for (int a = 0; a < NC; ++a) S::update(out, io * NC + a, n0, [&](T x) { return x - acc[a]; });
  }
}

// ---------------------------------------------------------------------------
// Batched shots: one launch per half-step advances many independent problems
// ("shots": the paper's experiments repeated over sources and grids) of the
// same (d, m, storage), each with its own grid, time step, coefficient and
// buffers.  Shot s owns the workgroups [first_block, first_block + 8 per_xcd)
// of the launch; first_block is a multiple of 8, so every shot keeps its own
// XCD band mapping.  A workgroup finds its shot by binary search over the
// descriptor array (uniform, read through the scalar cache).
// ---------------------------------------------------------------------------
template <class S>
struct ShotHalf {
  typename S::View out, in, kap;   // kap: variable-kappa data (unused for constant kappa)
  const typename S::C* tab;        // merged tables (constant kappa)
  Grid g;
  VarArgs<typename S::C> va;       // variable kappa
  typename S::C wscale, ih[3];     // velocity half-step
  int32_t first_block, pad;
};

// A table pointer read from memory, recast to the constant address space so
// that uniform table reads become scalar loads (a pointer loaded from memory
// is generic, and generic loads are per-lane flat loads).
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ ConstPtr<T> const_ptr(const T* p) {
  return (ConstPtr<T>)(uintptr_t)p;
}

template <class S>
__device__ __forceinline__ int shot_of(const ShotHalf<S>* __restrict__ sh, int n, int blk) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (__builtin_amdgcn_readfirstlane(sh[mid].first_block) <= blk)
      lo = mid;
    else
      hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// The descriptor of this workgroup's shot, every word passed through
// readfirstlane: the values are uniform, and saying so keeps pointers, grid
// and table addresses in scalar registers (otherwise the merged tables are
// read with vector loads, as in a kernel whose table pointer may vary by lane).
template <class S>
__device__ __forceinline__ ShotHalf<S> shot_desc(const ShotHalf<S>* __restrict__ shots, int s) {
  static_assert(sizeof(ShotHalf<S>) % 4 == 0, "descriptor must be whole words");
  ShotHalf<S> d;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(shots + s);
  uint32_t w[sizeof(ShotHalf<S>) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(ShotHalf<S>) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
  __builtin_memcpy(&d, w, sizeof d);
  return d;
}

template <int D, int M, class S, bool VAR>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) p_half_batch(const ShotHalf<S>* __restrict__ shots, int n) {
  const ShotHalf<S> sh = shot_desc(shots, shot_of(shots, n, blockIdx.x));
  const int blk = (int)blockIdx.x - sh.first_block;
  const ConstPtr<typename S::C> tab = const_ptr(sh.tab);
  using G = typename S::Global;
  const typename G::View out = S::global(sh.out), in = S::global(sh.in), kap = S::global(sh.kap);
  if constexpr (VAR)
    p_half_var_body<D, M, G>(out, in, kap, sh.g, sh.va, blk);
  else if constexpr (D == 3 && TableLayout<3, M>::FULL_P)
    p_half_3d_full_body<M, G>(out, in, tab, sh.g, blk);
  else if constexpr (D == 3)
    p_half_3d_body<M, G>(out, in, tab, sh.g, blk);
  else
    p_half_body<D, M, G>(out, in, tab, sh.g, blk);
}

template <int D, int M, class S, bool VAR>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) u_half_batch(const ShotHalf<S>* __restrict__ shots, int n) {
  const ShotHalf<S> sh = shot_desc(shots, shot_of(shots, n, blockIdx.x));
  const int blk = (int)blockIdx.x - sh.first_block;
  const ConstPtr<typename S::C> tab = const_ptr(sh.tab);
  using G = typename S::Global;
  const typename G::View out = S::global(sh.out), in = S::global(sh.in), kap = S::global(sh.kap);
  if constexpr (VAR)
    u_half_var_body<D, M, G>(out, in, kap, sh.g, sh.va, sh.wscale, blk);
  else if constexpr (D == 3)
    u_half_3d_body<M, G>(out, in, tab, sh.g, sh.wscale, sh.ih[0], sh.ih[1], sh.ih[2], blk);
  else
    u_half_body<D, M, G>(out, in, tab, sh.g, sh.wscale, sh.ih[0], sh.ih[1], sh.ih[2], blk);
}

// Sources inside a batch (the source term z = r(t) g(x) of Sec. 4, added by
// the midpoint rule after each pressure half-step): entry i adds
// amps[shot][n] * val[i] to word `word` of its shot's pressure array, n the
// batch's step counter (no source from step namps on).  The entries are the
// nodes of each shot's (compactly supported) g, so the launch is small.
struct BatchSource {
  int32_t shot;
  uint32_t word;  // plane * nodes + node in the shot's pressure array
};

template <typename W>
__global__ void __launch_bounds__(256) batch_source_add(W* const* __restrict__ pbase,
                                                        const BatchSource* __restrict__ ent,
                                                        const W* __restrict__ val, const W* __restrict__ amps,
                                                        int64_t namps, const int64_t* __restrict__ counter,
                                                        int64_t nent) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nent) return;
  const int64_t n = counter[0];
  if (n < 0 || n >= namps) return;
  const BatchSource e = ent[i];
  W* q = pbase[e.shot] + e.word;
  *q = fma(amps[(int64_t)e.shot * namps + n], val[i], *q);
}

}  // namespace hl
