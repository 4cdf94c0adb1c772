// hl_kernels.hpp - Hermite-leapfrog half-step kernels for gfx950.
//
// One work-item per output node.  For the pressure half-step at primal node
// j the cell's corners are the dual nodes q = j - 1 + e, e in {0,1}^d; for the
// velocity half-step at dual node q they are the primal nodes j = q + e
// (Sec. 2, eqs. (pGrid), (dGrid); Sec. 5).  The interpolant of the corner
// data (Sec. 2, eq. (interp)) is built one dimension at a time (Sec. 5) for
// every dimension but the last, with compile-time coefficients; the last
// dimension's interpolation and the Cauchy-Kowalevsky weights (Sec. 2,
// eq. (final1); Sec. 3.1.2, eqs. (pdup), (vdup)) are applied together through
// a runtime merged table (hl_layout.hpp) acting on the sum and difference of
// the two last-dimension corners.  Only a (2m+2)^{d-1} slice of the
// interpolant is live at a time.
//
// Device layout: coefficient-major planes, field[c * nodes + n],
// n = j_1 + K_1 (j_2 + K_2 j_3), c = a_1 + (m+1)(a_2 + (m+1) a_3).
//
// Launch: tiles of 64 x 4 x 1 nodes (256 x 1 x 1 in 1D), one workgroup per
// tile.  Workgroup i runs on XCD i mod 8; tile t = (i mod 8) * per + i / 8,
// so each XCD sweeps one contiguous band of tiles in row-major order and the
// corners shared between neighbouring tiles are re-read from that XCD's L2
// instead of from HBM.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hl_layout.hpp"

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

namespace hl {

constexpr int kXcds = 8;

struct Grid {
  int32_t K[3];       // nodes per dimension (1 for unused dimensions)
  int32_t nt[3];      // tiles per dimension
  int32_t tiles;      // nt[0] * nt[1] * nt[2]
  int32_t per_xcd;    // ceil(tiles / kXcds)
  int64_t nodes;      // K[0] * K[1] * K[2]
};

template <int D>
struct TileShape {
  static constexpr int X = D == 1 ? 256 : 64;
  static constexpr int Y = D == 1 ? 1 : 4;
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

// Load field[c][node] with a uniform plane base and a 32-bit byte offset
// (the address mode with a scalar base; planes are < 4 GiB by plan check).
template <typename T>
__device__ __forceinline__ T ld(const T* __restrict__ f, int64_t plane_words, int c, uint32_t off) {
  const char* base = reinterpret_cast<const char*>(f + (int64_t)c * plane_words);
  return *reinterpret_cast<const T*>(base + off);
}

// Slice of the interpolant for last-dimension corner eL and last-dimension
// datum l (1D and 2D kernels): Y[b], b in {0..2m+1}^{d-1}, from the 2^{d-1}
// corners with that eL.  FLIP0 = 1 makes the x pass the derivative pass
// (units of 1/h_x).  cb[e]: byte offset of corner e inside a coefficient plane.
template <int D, int M, int FLIP0, int FLIP1, typename T>
__device__ __forceinline__ void slice(const T* __restrict__ f, int64_t nodes, const uint32_t* cb, int eL, int l,
                                      T* Y) {
  constexpr int MP = M + 1;
  static_assert(D == 1 || D == 2, "3D uses the x-line kernels");
  if constexpr (D == 1) {
    Y[0] = ld(f, nodes, l, cb[eL]);
  } else if constexpr (D == 2) {
    T Lv[MP], Rv[MP];
#pragma unroll
    for (int a0 = 0; a0 < MP; ++a0) {
      const int c = a0 + MP * l;
      Lv[a0] = ld(f, nodes, c, cb[0 + 2 * eL]);
      Rv[a0] = ld(f, nodes, c, cb[1 + 2 * eL]);
    }
    pass1d<M, FLIP0>(Lv, Rv, Y);
  }
}

// acc[o] += sum_b Mt[t] * (sigma or delta)[b] over the structurally nonzero
// (o, b) of one merged table row-block (datum l); the walk comes from the
// compile-time MergeSpec, so every index is a constant after unrolling.
template <int D, int M, bool VEL, int FLIPL, typename T>
__device__ __forceinline__ void merge(const T* __restrict__ Mt, int l, const T* S, const T* Df, T* acc) {
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
    acc[o] = fma(Mt[t], dl ? Df[b] : S[b], acc[o]);
  }
}

// Plane form of the merge (z-march kernels): t_o = sum_b Mt * Y[b] is the
// plane's contribution through the table; it adds to the cell for which the
// plane is the upper corner (accR, + t) and to the cell for which it is the
// lower corner (accL, + t for sigma entries, - t for delta entries).  The
// table walk is ordered by output, so t_o is complete when o changes.
template <int D, int M, bool VEL, int FLIPL, bool DO_R, bool DO_L, typename T, typename TP>
__device__ __forceinline__ void merge_plane(TP Mt, int l, const T* Y, T* accR, T* accL) {
  using Sp = MergeSpec<D, M, VEL, FLIPL>;
  constexpr int kChunk = sizeof(T) == 8 ? 16 : 32;
  T acc = T(0);
#pragma unroll
  for (int t = 0; t < Sp::NNZ; ++t) {
    if (t % kChunk == 0) __builtin_amdgcn_sched_barrier(HL_SCHED_MASK);
    const int o = kMerge<D, M, VEL, FLIPL>.o[t];
    acc = fma(Mt[t], Y[kMerge<D, M, VEL, FLIPL>.b[t]], acc);
    if (t + 1 == Sp::NNZ || kMerge<D, M, VEL, FLIPL>.o[t + 1] != o) {
      const bool dl = kMerge<D, M, VEL, FLIPL>.base_delta[o] != ((l & 1) != 0);
      if (DO_R) accR[o] += acc;
      if (DO_L) accL[o] += dl ? -acc : acc;
      acc = T(0);
    }
  }
}

// Node of this work-item (XCD band mapping); false when outside the grid.
template <int D>
__device__ __forceinline__ bool node_of_thread(const Grid& g, int32_t* j) {
  const int i = blockIdx.x;
  const int t = (i % kXcds) * g.per_xcd + i / kXcds;
  if (t >= g.tiles) return false;
  const int tx = t % g.nt[0];
  const int ty = (t / g.nt[0]) % g.nt[1];
  const int tz = t / (g.nt[0] * g.nt[1]);
  j[0] = tx * TileShape<D>::X + threadIdx.x;
  j[1] = ty * TileShape<D>::Y + threadIdx.y;
  j[2] = tz;
  return j[0] < g.K[0] && j[1] < g.K[1] && j[2] < g.K[2];
}

template <int D>
__device__ __forceinline__ uint32_t node_index(int32_t x, int32_t y, int32_t z, const Grid& g) {
  uint32_t n = (uint32_t)x;
  if (D > 1) n += (uint32_t)g.K[0] * (uint32_t)y;
  if (D > 2) n += (uint32_t)g.K[0] * (uint32_t)g.K[1] * (uint32_t)z;
  return n;
}

// Pressure half-step at every primal node (1D and 2D).
// tab: packed merged tables (hl_layout.hpp TableLayout).
template <int D, int M, typename T>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) p_half_kernel(T* __restrict__ p, const T* __restrict__ u,
                                                                       const T* __restrict__ tab, Grid g) {
  using Dm = Dims<D, M>;
  using TL = TableLayout<D, M>;
  constexpr int MP = Dm::MP, NC = Dm::NC, NB = Dm::NB;
  constexpr int NNZ = merged_nnz<D, M>(false);
  int32_t j[3];
  if (!node_of_thread<D>(g, j)) return;
  int32_t lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = (j[k] == 0 ? g.K[k] : j[k]) - 1;  // dual q = j - 1 (wrapped)
    hi[k] = j[k];                              // dual q = j
  }
  uint32_t cb[1 << D];
#pragma unroll
  for (int e = 0; e < (1 << D); ++e)
    cb[e] = (uint32_t)sizeof(T) *
            node_index<D>((e & 1) ? hi[0] : lo[0], (e & 2) ? hi[1] : lo[1], (e & 4) ? hi[2] : lo[2], g);

  T acc[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) acc[s] = T(0);
  const int64_t nodes = g.nodes;
  const int64_t field = (int64_t)NC * nodes;

#pragma unroll
  for (int l = 0; l < MP; ++l) {
    if constexpr (D > 1) {
      // x-component: derivative pass in x; last pass H
      T YL[NB], YR[NB];
      slice<D, M, 1, 0>(u, nodes, cb, 0, l, YL);
      slice<D, M, 1, 0>(u, nodes, cb, 1, l, YR);
      T S[NB], Df[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        S[b] = YR[b] + YL[b];
        Df[b] = YR[b] - YL[b];
      }
      merge<D, M, false, 0>(tab + TL::P_A_OFF + l * NNZ, l, S, Df, acc);
    }
    {
      // last component: interpolation pass in x, derivative in the last pass
      T YL[NB], YR[NB], S[NB], Df[NB];
      slice<D, M, 0, 0>(u + (D - 1) * field, nodes, cb, 0, l, YL);
      slice<D, M, 0, 0>(u + (D - 1) * field, nodes, cb, 1, l, YR);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        S[b] = YR[b] + YL[b];
        Df[b] = YR[b] - YL[b];
      }
      merge<D, M, false, 1>(tab + TL::P_B_OFF + l * NNZ, l, S, Df, acc);
    }
  }
  const uint32_t o0 = (uint32_t)sizeof(T) * node_index<D>(j[0], j[1], j[2], g);
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    T* q = reinterpret_cast<T*>(reinterpret_cast<char*>(p + (int64_t)s * nodes) + o0);
    *q = *q - acc[s];
  }
}

// u_i[s] -= wscale * (s_i + 1) / h_i * Q[s + e_i]   (Q on the set G)
template <int D, int M, typename T>
__device__ __forceinline__ void finish_velocity(T* __restrict__ u, int64_t field, int64_t nodes, uint32_t o0,
                                                const T* Q, T wscale, const T* ih) {
  constexpr int MP = M + 1;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T f = wscale * ih[i];
#pragma unroll
    for (int s = 0; s < Dims<D, M>::NC; ++s) {
      const int si1 = digit(s, MP, i) + 1;
      T* q = reinterpret_cast<T*>(reinterpret_cast<char*>(u + (int64_t)i * field + (int64_t)s * nodes) + o0);
      *q = fma(-(T)si1 * f, Q[kGIndex<D, M>.g[i][s]], *q);
    }
  }
}

// Velocity half-step at every dual node, weights scaled by wscale.
template <int D, int M, typename T>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) u_half_kernel(T* __restrict__ u, const T* __restrict__ p,
                                                                       const T* __restrict__ tab, Grid g, T wscale,
                                                                       T ih0, T ih1, T ih2) {
  using Dm = Dims<D, M>;
  using TL = TableLayout<D, M>;
  constexpr int MP = Dm::MP, NB = Dm::NB;
  constexpr int NG = GSet<D, M>::NG;
  int32_t j[3];
  if (!node_of_thread<D>(g, j)) return;
  int32_t lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = j[k];                                  // primal j = q
    hi[k] = (j[k] + 1 == g.K[k]) ? 0 : j[k] + 1;   // primal j = q + 1 (wrapped)
  }
  uint32_t cb[1 << D];
#pragma unroll
  for (int e = 0; e < (1 << D); ++e)
    cb[e] = (uint32_t)sizeof(T) *
            node_index<D>((e & 1) ? hi[0] : lo[0], (e & 2) ? hi[1] : lo[1], (e & 4) ? hi[2] : lo[2], g);

  T Q[NG];
#pragma unroll
  for (int o = 0; o < NG; ++o) Q[o] = T(0);
  const int64_t nodes = g.nodes;
  const int64_t field = (int64_t)Dm::NC * nodes;
  constexpr int NNZ = merged_nnz<D, M>(true);

#pragma unroll
  for (int l = 0; l < MP; ++l) {
    T YL[NB], YR[NB], S[NB], Df[NB];
    slice<D, M, 0, 0>(p, nodes, cb, 0, l, YL);
    slice<D, M, 0, 0>(p, nodes, cb, 1, l, YR);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      S[b] = YR[b] + YL[b];
      Df[b] = YR[b] - YL[b];
    }
    merge<D, M, true, 0>(tab + TL::U_OFF + l * NNZ, l, S, Df, Q);
  }
  const T ih[3] = {ih0, ih1, ih2};
  finish_velocity<D, M>(u, field, nodes, (uint32_t)sizeof(T) * node_index<D>(j[0], j[1], j[2], g), Q, wscale, ih);
}

// ---------------------------------------------------------------------------
// 3D kernels.  A work-item interpolates explicitly only along x: for every
// y/z datum pair (a_y, a_z) it loads the 8 corners' x-lines, applies the x
// pass (derivative pass for the x-component of the pressure half-step), and
// combines the four (y, z) corners into sigma/delta in y and in z.  The y and
// z interpolation, the Cauchy-Kowalevsky weights and (for the y- and
// z-components) the divergence are all in the runtime table (Merge3Spec).
// Coefficient planes are read through buffer descriptors: one per field and
// (a_y, a_z), a 32-bit per-lane corner offset and a scalar plane offset.
// ---------------------------------------------------------------------------

// Buffer resource over n consecutive coefficient planes starting at plane c0
// (raw dword addressing, gfx9 descriptor word 3).  Offsets past num_records
// read as zero.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t planes_rsrc(const T* f, int64_t nodes, int c0, int n) {
  const T* base = f + (int64_t)c0 * nodes;
  const uint32_t bytes = (uint32_t)((int64_t)n * nodes * (int64_t)sizeof(T));
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// X[k_y][k_z][b_x] for datum pair (a_y, a_z), whose m+1 coefficient planes
// (a_x = 0..m) start at plane c0 of field f; cb[e], e = e_x + 2 e_y + 4 e_z,
// are the corners' byte offsets inside a plane.  One buffer descriptor per
// plane keeps every offset below 4 GiB for any plane below 4 GiB.
template <int M, int FLIPX, typename T>
__device__ __forceinline__ void xlines(const T* f, int64_t nodes, int c0, const uint32_t* cb,
                                       T (&X)[2][2][2 * M + 2]) {
  constexpr int MP = M + 1, N2 = 2 * M + 2;
  // for large m keep the loads of different (a_y, a_z) blocks apart, or the
  // scheduler clusters them and runs out of registers
  if constexpr (M >= 3) __builtin_amdgcn_sched_barrier(0);
  __amdgpu_buffer_rsrc_t rs[MP];
#pragma unroll
  for (int ax = 0; ax < MP; ++ax) rs[ax] = planes_rsrc(f, nodes, c0 + ax, 1);
  T Y[2][2][N2];  // [e_y][e_z][b_x]
#pragma unroll
  for (int ez = 0; ez < 2; ++ez)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
      T Lv[MP], Rv[MP];
#pragma unroll
      for (int ax = 0; ax < MP; ++ax) {
        Lv[ax] = bload<T>(rs[ax], cb[0 + 2 * ey + 4 * ez], 0u);
        Rv[ax] = bload<T>(rs[ax], cb[1 + 2 * ey + 4 * ez], 0u);
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

template <typename T>
__device__ __forceinline__ void corners3(const Grid& g, const int32_t* lo, const int32_t* hi, uint32_t* cb) {
#pragma unroll
  for (int e = 0; e < 8; ++e)
    cb[e] = (uint32_t)sizeof(T) *
            node_index<3>((e & 1) ? hi[0] : lo[0], (e & 2) ? hi[1] : lo[1], (e & 4) ? hi[2] : lo[2], g);
}

template <int M, typename T>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) p_half_3d(T* __restrict__ p, const T* __restrict__ u,
                                                                   const T* __restrict__ tab, Grid g) {
  using TL = TableLayout<3, M>;
  constexpr int MP = M + 1, NC = Dims<3, M>::NC, N2 = 2 * M + 2;
  constexpr int NNZ = Merge3Spec<M, false, 0, 0>::NNZ;
  int32_t j[3];
  if (!node_of_thread<3>(g, j)) return;
  int32_t lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = (j[k] == 0 ? g.K[k] : j[k]) - 1;  // dual q = j - 1 (wrapped)
    hi[k] = j[k];                              // dual q = j
  }
  uint32_t cb[8];
  corners3<T>(g, lo, hi, cb);
  const int64_t nodes = g.nodes;
  const int64_t field = (int64_t)NC * nodes;
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
        xlines<M, 1>(u, nodes, MP * blk, cb, X);
        merge3<M, false, 0, 0>(tab + TL::p_off(0) + blk * NNZ, ay, az, X, acc);
      }
      {
        T X[2][2][N2];
        xlines<M, 0>(u + field, nodes, MP * blk, cb, X);
        merge3<M, false, 1, 0>(tab + TL::p_off(1) + blk * NNZ, ay, az, X, acc);
      }
      {
        T X[2][2][N2];
        xlines<M, 0>(u + 2 * field, nodes, MP * blk, cb, X);
        merge3<M, false, 0, 1>(tab + TL::p_off(2) + blk * NNZ, ay, az, X, acc);
      }
    }
  const uint32_t o0 = (uint32_t)sizeof(T) * node_index<3>(j[0], j[1], j[2], g);
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    T* q = reinterpret_cast<T*>(reinterpret_cast<char*>(p + (int64_t)s * nodes) + o0);
    *q = *q - acc[s];
  }
}

template <int M, typename T>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) u_half_3d(T* __restrict__ u, const T* __restrict__ p,
                                                                   const T* __restrict__ tab, Grid g, T wscale,
                                                                   T ih0, T ih1, T ih2) {
  using TL = TableLayout<3, M>;
  constexpr int MP = M + 1, NC = Dims<3, M>::NC, N2 = 2 * M + 2;
  constexpr int NG = GSet<3, M>::NG;
  constexpr int NNZ = Merge3Spec<M, true, 0, 0>::NNZ;
  int32_t j[3];
  if (!node_of_thread<3>(g, j)) return;
  int32_t lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = j[k];                                  // primal j = q
    hi[k] = (j[k] + 1 == g.K[k]) ? 0 : j[k] + 1;   // primal j = q + 1 (wrapped)
  }
  uint32_t cb[8];
  corners3<T>(g, lo, hi, cb);
  const int64_t nodes = g.nodes;
  const int64_t field = (int64_t)NC * nodes;
  T Q[NG];
#pragma unroll
  for (int o = 0; o < NG; ++o) Q[o] = T(0);
#pragma unroll
  for (int az = 0; az < MP; ++az)
#pragma unroll
    for (int ay = 0; ay < MP; ++ay) {
      const int blk = ay + MP * az;
      T X[2][2][N2];
      xlines<M, 0>(p, nodes, MP * blk, cb, X);
      merge3<M, true, 0, 0>(tab + TL::U_OFF + blk * NNZ, ay, az, X, Q);
    }
  const T ih[3] = {ih0, ih1, ih2};
  finish_velocity<3, M>(u, field, nodes, (uint32_t)sizeof(T) * node_index<3>(j[0], j[1], j[2], g), Q, wscale, ih);
}

}  // namespace hl
