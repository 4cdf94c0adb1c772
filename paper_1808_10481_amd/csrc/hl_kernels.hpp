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
// datum l: Y[b], b in {0..2m+1}^{d-1}, from the 2^{d-1} corners with that eL.
// FLIPk = 1 makes transverse pass k the derivative pass (units of 1/h_k).
// cb[e]: byte offset of corner e inside a coefficient plane.
template <int D, int M, int FLIP0, int FLIP1, typename T>
__device__ __forceinline__ void slice(const T* __restrict__ f, int64_t nodes, const uint32_t* cb, int eL, int l,
                                      T* Y) {
  constexpr int MP = M + 1, N2 = 2 * M + 2;
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
  } else {
    T Z[2][MP][N2];  // [e1][a1][b0]
#pragma unroll
    for (int e1 = 0; e1 < 2; ++e1)
#pragma unroll
      for (int a1 = 0; a1 < MP; ++a1) {
        T Lv[MP], Rv[MP];
#pragma unroll
        for (int a0 = 0; a0 < MP; ++a0) {
          const int c = a0 + MP * (a1 + MP * l);
          Lv[a0] = ld(f, nodes, c, cb[0 + 2 * e1 + 4 * eL]);
          Rv[a0] = ld(f, nodes, c, cb[1 + 2 * e1 + 4 * eL]);
        }
        pass1d<M, FLIP0>(Lv, Rv, Z[e1][a1]);
      }
#pragma unroll
    for (int b0 = 0; b0 < N2; ++b0) {
      T Lv[MP], Rv[MP], out[N2];
#pragma unroll
      for (int a1 = 0; a1 < MP; ++a1) {
        Lv[a1] = Z[0][a1][b0];
        Rv[a1] = Z[1][a1][b0];
      }
      pass1d<M, FLIP1>(Lv, Rv, out);
#pragma unroll
      for (int b1 = 0; b1 < N2; ++b1) Y[b0 + N2 * b1] = out[b1];
    }
  }
}

// acc[s] += sum_b Mt[t] * (sigma or delta)[b] over the structurally nonzero
// (s, b) of one merged table row-block (datum l).  t is a compile-time
// constant once the loops are unrolled.
template <int D, int M, int DD, int FLIPL, typename T>
__device__ __forceinline__ void merge(const T* __restrict__ Mt, int l, const T* S, const T* Df, T* acc) {
  using Dm = Dims<D, M>;
  // Scalar table loads are consumed in chunks: without the barriers the
  // scheduler hoists every s_load of the table to the top of the kernel and
  // runs out of SGPRs (spilling them through VGPR lanes).
  constexpr int kChunk = sizeof(T) == 8 ? 16 : 32;
  int t = 0;
#pragma unroll
  for (int s = 0; s < Dm::NC; ++s) {
    const bool dl = merged_uses_delta<D, M>(DD, FLIPL, s, l);
#pragma unroll
    for (int b = 0; b < Dm::NB; ++b)
      if (merged_valid<D, M>(DD, s, b)) {
        if (t % kChunk == 0) __builtin_amdgcn_sched_barrier(HL_SCHED_MASK);
        acc[s] = fma(Mt[t], dl ? Df[b] : S[b], acc[s]);
        ++t;
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

// Pressure half-step at every primal node.
// tab: packed merged tables (hl_layout.hpp TableLayout).  r01 = h_x / h_y
// scales the y-component's slice into the units of group A, whose table
// carries 1/h_x (3D only).
template <int D, int M, typename T>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) p_half_kernel(T* __restrict__ p, const T* __restrict__ u,
                                                      const T* __restrict__ tab, Grid g, T r01) {
  using Dm = Dims<D, M>;
  using TL = TableLayout<D, M>;
  constexpr int MP = Dm::MP, NC = Dm::NC, NB = Dm::NB;
  constexpr int NNZ = merged_nnz<D, M>(-1);
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
      // group A: components 0..d-2 with the derivative pass in their own
      // dimension; last pass H
      T YL[NB], YR[NB];
      slice<D, M, 1, 0>(u, nodes, cb, 0, l, YL);
      slice<D, M, 1, 0>(u, nodes, cb, 1, l, YR);
      if constexpr (D == 3) {
        T ZL[NB], ZR[NB];
        slice<D, M, 0, 1>(u + field, nodes, cb, 0, l, ZL);
        slice<D, M, 0, 1>(u + field, nodes, cb, 1, l, ZR);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          YL[b] = fma(r01, ZL[b], YL[b]);
          YR[b] = fma(r01, ZR[b], YR[b]);
        }
      }
      T S[NB], Df[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        S[b] = YR[b] + YL[b];
        Df[b] = YR[b] - YL[b];
      }
      merge<D, M, -1, 0>(tab + TL::P_A_OFF + l * NNZ, l, S, Df, acc);
    }
    {
      // group B: component d-1, transverse passes H, last pass D_d H
      T YL[NB], YR[NB], S[NB], Df[NB];
      slice<D, M, 0, 0>(u + (D - 1) * field, nodes, cb, 0, l, YL);
      slice<D, M, 0, 0>(u + (D - 1) * field, nodes, cb, 1, l, YR);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        S[b] = YR[b] + YL[b];
        Df[b] = YR[b] - YL[b];
      }
      merge<D, M, -1, 1>(tab + TL::P_B_OFF + l * NNZ, l, S, Df, acc);
    }
  }
  const uint32_t o0 = (uint32_t)sizeof(T) * node_index<D>(j[0], j[1], j[2], g);
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    T* q = reinterpret_cast<T*>(reinterpret_cast<char*>(p + (int64_t)s * nodes) + o0);
    *q = *q - acc[s];
  }
}

// Velocity half-step at every dual node, weights scaled by wscale.
template <int D, int M, typename T>
__global__ void __launch_bounds__(256, HL_WAVES_PER_EU) u_half_kernel(T* __restrict__ u, const T* __restrict__ p,
                                                      const T* __restrict__ tab, Grid g, T wscale) {
  using Dm = Dims<D, M>;
  using TL = TableLayout<D, M>;
  constexpr int MP = Dm::MP, NC = Dm::NC, NB = Dm::NB;
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

  T acc[D][NC];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int s = 0; s < NC; ++s) acc[i][s] = T(0);
  const int64_t nodes = g.nodes;
  const int64_t field = (int64_t)NC * nodes;

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
    merge<D, M, 0, 0>(tab + TL::u_off(0) + l * merged_nnz<D, M>(0), l, S, Df, acc[0]);
    if constexpr (D > 1) merge<D, M, 1, 0>(tab + TL::u_off(1) + l * merged_nnz<D, M>(1), l, S, Df, acc[1]);
    if constexpr (D > 2) merge<D, M, 2, 0>(tab + TL::u_off(2) + l * merged_nnz<D, M>(2), l, S, Df, acc[2]);
  }
  const uint32_t o0 = (uint32_t)sizeof(T) * node_index<D>(j[0], j[1], j[2], g);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      T* q = reinterpret_cast<T*>(reinterpret_cast<char*>(u + (int64_t)i * field + (int64_t)s * nodes) + o0);
      *q = fma(-wscale, acc[i][s], *q);
    }
}

}  // namespace hl
