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
// 3D half-steps (fully merged tables): load the next datum's 8 corners before the current
// datum's arithmetic (HL_PREFETCH3: 0 never, 1 for FP64 storage, 2 always).
// With FP64 words the half-steps wait on memory at 3-5 resident waves per
// SIMD, and a second datum in flight per wave pays (256^3 u half-step 7.57 ->
// 7.05 ms, p half-step 7.70 -> 7.61); FP32 (VALU-bound p half-step 2.97 ->
// 3.14 ms) and the split FP32+BF16 storage (16 loads per datum: u half-step
// 7.01 -> 15.3 ms) run slower with it.
#ifndef HL_PREFETCH3
#define HL_PREFETCH3 1
#endif
// Cache policy of the 3D half-steps' read-modify-write of their outputs: 2,
// the non-temporal bit.  Each output word is read and written once per
// half-step, while the corner words are read by up to 8 neighbouring nodes;
// streaming the outputs leaves the L2 to the corners (256^3 m = 2 step: FP64
// 14.68 -> 14.27 ms, FP32 6.20 -> 6.06 ms).
#ifndef HL_STREAM_AUX
#define HL_STREAM_AUX 2
#endif
// 1D and 2D: the same streaming of the outputs for FP64 and FP32_COMP words
// (2D m = 3 1024^2 step: FP64 0.295 -> 0.267 ms, FP32_COMP 0.220 -> 0.202 ms);
// not for FP32, whose 1024^2 state (201 MB) stays in the 256 MB MALL between
// half-steps when its outputs are cached (0.098 -> 0.125 ms streamed).
#ifndef HL_STREAM2D
#define HL_STREAM2D 1
#endif
template <class S>
constexpr bool kPrefetch3 = HL_PREFETCH3 == 2 || (HL_PREFETCH3 == 1 && S::kBytes == 8);

// Minimum waves per SIMD requested from the register allocator (0 = none).
#ifndef HL_WAVES_PER_EU
#define HL_WAVES_PER_EU 0
#endif
// 3D velocity half-step through the fully merged table (1) or the explicit x
// pass plus the (y, z) merged table (0).
#ifndef HL_U3_FULL
#define HL_U3_FULL 1
#endif
// 3D tile extent in x and y (x * y = 256 work-items).
#ifndef HL_TILE3_X
#define HL_TILE3_X 64
#endif

namespace hl {

constexpr int kXcds = 8;

// Constant-address-space view of a table: uniform reads become scalar loads
// (a pointer read from memory, or made opaque, is otherwise generic).
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ ConstPtr<T> const_ptr(const T* p) {
  return (ConstPtr<T>)(uintptr_t)p;
}

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
    S::template bstore<HL_STREAM_AUX>(pr, n0, f(S::template bload<HL_STREAM_AUX>(pr, n0)));
  } else if constexpr (HL_STREAM2D && S::kBytes >= 6) {
    S::update_nt(v, pl, n0, f);
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

// Pressure half-step, 3D: the x interpolation is merged into the
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
  T vn[8];  // the next datum's corners, loaded one datum ahead
  if constexpr (kPrefetch3<S>) {
    const typename S::Planes pr = S::planes(u, 0);
#pragma unroll
    for (int e = 0; e < 8; ++e) vn[e] = S::bload(pr, cn[e]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      // keep the scalar table loads of one datum together (SGPR pressure)
      __builtin_amdgcn_sched_barrier(0);
      T v[8];
      if constexpr (kPrefetch3<S>) {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = vn[e];
        if (i * NC + a + 1 < 3 * NC) {
          int zero;  // opaque: the plane base is formed here, not hoisted to the kernel start
          asm volatile("s_mov_b32 %0, 0" : "=s"(zero));
          const typename S::Planes pn = S::planes(u, i * NC + a + 1 + zero);
#pragma unroll
          for (int e = 0; e < 8; ++e) vn[e] = S::bload(pn, cn[e]);
        }
      } else {
        const typename S::Planes pr = S::planes(u, i * NC + a);
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = S::bload(pr, cn[e]);
      }
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

// Velocity half-step, 3D: the x interpolation merged into the table
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
  T vn[8];  // the next datum's corners, loaded one datum ahead
  if constexpr (kPrefetch3<S>) {
    const typename S::Planes pr = S::planes(p, 0);
#pragma unroll
    for (int e = 0; e < 8; ++e) vn[e] = S::bload(pr, cn[e]);
  }
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    // keep the scalar table loads of one datum together (SGPR pressure)
    __builtin_amdgcn_sched_barrier(0);
    T v[8];
    if constexpr (kPrefetch3<S>) {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = vn[e];
      if (a + 1 < NC) {
        int zero;  // opaque: the plane base is formed here, not hoisted to the kernel start
        asm volatile("s_mov_b32 %0, 0" : "=s"(zero));
        const typename S::Planes pn = S::planes(p, a + 1 + zero);
#pragma unroll
        for (int e = 0; e < 8; ++e) vn[e] = S::bload(pn, cn[e]);
      }
    } else {
      const typename S::Planes pr = S::planes(p, a);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = S::bload(pr, cn[e]);
    }
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

}  // namespace hl
