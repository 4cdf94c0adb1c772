// hl_kernels.hpp - generic Hermite-leapfrog half-step kernels for gfx950.
//
// One work-item per output node.  For the pressure half-step at primal node
// j the cell's corners are the dual nodes q = j - 1 + e, e in {0,1}^d; for the
// velocity half-step at dual node q they are the primal nodes j = q + e
// (Sec. 2, eqs. (pGrid), (dGrid); Sec. 5).  The interpolant of the corner
// data (Sec. 2, eq. (interp)) is built one dimension at a time (Sec. 5) for
// every dimension but the last; the last dimension's interpolation and the
// Cauchy-Kowalevsky weights (Sec. 2, eq. (final1); Sec. 3.1.2, eqs. (pdup),
// (vdup)) are applied together through a merged table (hl_layout.hpp), so
// only a (2m+2)^{d-1} slice of the interpolant is live at a time.
//
// Device layout: coefficient-major planes, field[c * nodes + n],
// n = j_1 + K_1 (j_2 + K_2 j_3), c = a_1 + (m+1)(a_2 + (m+1) a_3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hl_layout.hpp"

namespace hl {

struct Grid {
  int32_t K[3];     // nodes per dimension (1 for unused dimensions)
  int64_t nodes;    // K[0] * K[1] * K[2]
};

// out[b] = sum_l G[b][l] * (b + l + FLIP even ? R_l + L_l : R_l - L_l),
// b = 0..2M+1 (the last row of a derivative table, FLIP = 1, is zero).
template <int M, int FLIP, typename T>
__device__ __forceinline__ void pass1d(const T* __restrict__ G, const T* L, const T* R, T* out) {
  constexpr int MP = M + 1, N2 = 2 * M + 2;
  T sg[MP], df[MP];
#pragma unroll
  for (int l = 0; l < MP; ++l) {
    sg[l] = R[l] + L[l];
    df[l] = R[l] - L[l];
  }
#pragma unroll
  for (int b = 0; b < N2; ++b) {
    if (FLIP && b == N2 - 1) {
      out[b] = T(0);
      continue;
    }
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < MP; ++l) acc = fma(G[b * MP + l], ((b + l + FLIP) & 1) ? df[l] : sg[l], acc);
    out[b] = acc;
  }
}

// Corner node indices of a cell.  base[k] is the low corner index in dim k
// (already wrapped); the high corner is base + 1 (wrapped).  Returns the
// linear node index of corner e (bit k of e = high in dim k).
template <int D>
__device__ __forceinline__ int64_t corner_node(const int32_t* lo, const int32_t* hi, int e, const Grid& g) {
  int64_t n = (e & 1) ? hi[0] : lo[0];
  if (D > 1) n += (int64_t)g.K[0] * ((e & 2) ? hi[1] : lo[1]);
  if (D > 2) n += (int64_t)g.K[0] * g.K[1] * ((e & 4) ? hi[2] : lo[2]);
  return n;
}

// Slice of the interpolant for last-dimension corner eL and last-dimension
// datum l: Y[b], b in {0..2m+1}^{d-1}, from the 2^{d-1} corners with that eL.
// FLIPk selects D_k H (1) or H (0) for transverse pass k; Gk its table.
template <int D, int M, int FLIP0, int FLIP1, typename T>
__device__ __forceinline__ void slice(const T* __restrict__ f, int64_t nodes, const int64_t* cn, int eL, int l,
                                      const T* __restrict__ G0, const T* __restrict__ G1, T* Y) {
  using Dm = Dims<D, M>;
  constexpr int MP = Dm::MP, N2 = Dm::N2;
  if constexpr (D == 1) {
    Y[0] = f[(int64_t)l * nodes + cn[eL]];
  } else if constexpr (D == 2) {
    T Lv[MP], Rv[MP];
#pragma unroll
    for (int a0 = 0; a0 < MP; ++a0) {
      const int64_t c = (int64_t)(a0 + MP * l) * nodes;
      Lv[a0] = f[c + cn[0 + 2 * eL]];
      Rv[a0] = f[c + cn[1 + 2 * eL]];
    }
    pass1d<M, FLIP0>(G0, Lv, Rv, Y);
  } else {
    T Z[2][MP][N2];  // [e1][a1][b0]
#pragma unroll
    for (int e1 = 0; e1 < 2; ++e1)
#pragma unroll
      for (int a1 = 0; a1 < MP; ++a1) {
        T Lv[MP], Rv[MP];
#pragma unroll
        for (int a0 = 0; a0 < MP; ++a0) {
          const int64_t c = (int64_t)(a0 + MP * (a1 + MP * l)) * nodes;
          Lv[a0] = f[c + cn[0 + 2 * e1 + 4 * eL]];
          Rv[a0] = f[c + cn[1 + 2 * e1 + 4 * eL]];
        }
        pass1d<M, FLIP0>(G0, Lv, Rv, Z[e1][a1]);
      }
#pragma unroll
    for (int b0 = 0; b0 < N2; ++b0) {
      T Lv[MP], Rv[MP], out[N2];
#pragma unroll
      for (int a1 = 0; a1 < MP; ++a1) {
        Lv[a1] = Z[0][a1][b0];
        Rv[a1] = Z[1][a1][b0];
      }
      pass1d<M, FLIP1>(G1, Lv, Rv, out);
#pragma unroll
      for (int b1 = 0; b1 < N2; ++b1) Y[b0 + N2 * b1] = out[b1];
    }
  }
}

// acc[s] += sum_b Mtab[..] * Y[b] over the structurally nonzero (s, b) of a
// merged table (running packed index t, a compile-time constant once the
// loops are unrolled).
template <int D, int M, int DD, typename T>
__device__ __forceinline__ void merge(const T* __restrict__ Mt, const T* Y, T* acc) {
  using Dm = Dims<D, M>;
  int t = 0;
#pragma unroll
  for (int s = 0; s < Dm::NC; ++s)
#pragma unroll
    for (int b = 0; b < Dm::NB; ++b)
      if (merged_valid<D, M>(DD, s, b)) {
        acc[s] = fma(Mt[t], Y[b], acc[s]);
        ++t;
      }
}

template <int D>
__device__ __forceinline__ bool node_of_thread(const Grid& g, int32_t* j) {
  j[0] = blockIdx.x * blockDim.x + threadIdx.x;
  j[1] = (D > 1) ? (int32_t)(blockIdx.y * blockDim.y + threadIdx.y) : 0;
  j[2] = (D > 2) ? (int32_t)blockIdx.z : 0;
  return j[0] < g.K[0] && (D < 2 || j[1] < g.K[1]) && (D < 3 || j[2] < g.K[2]);
}

// Pressure half-step at every primal node.
// tab: packed tables (hl_layout.hpp TableLayout), u: velocity (d planes sets).
template <int D, int M, typename T>
__global__ void __launch_bounds__(256) p_half_kernel(T* __restrict__ p, const T* __restrict__ u,
                                                      const T* __restrict__ tab, Grid g) {
  using Dm = Dims<D, M>;
  using TL = TableLayout<D, M>;
  constexpr int MP = Dm::MP, NC = Dm::NC, NB = Dm::NB;
  int32_t j[3];
  if (!node_of_thread<D>(g, j)) return;
  int32_t lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = (j[k] == 0 ? g.K[k] : j[k]) - 1;  // dual q = j - 1 (wrapped)
    hi[k] = j[k];                              // dual q = j
  }
  int64_t cn[1 << D];
#pragma unroll
  for (int e = 0; e < (1 << D); ++e) cn[e] = corner_node<D>(lo, hi, e, g);

  const T* H = tab + TL::PASS_OFF;
  T acc[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) acc[s] = T(0);
  const int64_t nodes = g.nodes;
  const int64_t field = (int64_t)NC * nodes;

#pragma unroll
  for (int eL = 0; eL < 2; ++eL)
#pragma unroll
    for (int l = 0; l < MP; ++l) {
      const int slot = eL * MP + l;
      if constexpr (D > 1) {
        // group A: components 0..d-2, last pass H, derivative in transverse pass i
        T Y[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) Y[b] = T(0);
#pragma unroll
        for (int i = 0; i < D - 1; ++i) {
          T Yi[NB];
          const T* G0 = H + (i == 0 ? 1 : 0) * TL::PASS;  // D_1 H for component 0
          const T* G1 = H + (i == 1 ? 2 : 0) * TL::PASS;  // D_2 H for component 1
          if (i == 0)
            slice<D, M, 1, 0>(u + i * field, nodes, cn, eL, l, G0, G1, Yi);
          else
            slice<D, M, 0, 1>(u + i * field, nodes, cn, eL, l, G0, G1, Yi);
#pragma unroll
          for (int b = 0; b < NB; ++b) Y[b] += Yi[b];
        }
        merge<D, M, -1>(tab + TL::P_A_OFF + slot * merged_nnz<D, M>(-1), Y, acc);
      }
      {
        // group B: component d-1, transverse passes H, last pass D_d H
        T Y[NB];
        slice<D, M, 0, 0>(u + (D - 1) * field, nodes, cn, eL, l, H, H, Y);
        merge<D, M, -1>(tab + TL::P_B_OFF + slot * merged_nnz<D, M>(-1), Y, acc);
      }
    }
  const int64_t n0 = corner_node<D>(hi, hi, 0, g);  // the node itself
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const int64_t a = (int64_t)s * nodes + n0;
    p[a] = p[a] - acc[s];
  }
}

// Velocity half-step at every dual node, weights scaled by wscale.
template <int D, int M, typename T>
__global__ void __launch_bounds__(256) u_half_kernel(T* __restrict__ u, const T* __restrict__ p,
                                                      const T* __restrict__ tab, Grid g, T wscale) {
  using Dm = Dims<D, M>;
  using TL = TableLayout<D, M>;
  constexpr int MP = Dm::MP, NC = Dm::NC, NB = Dm::NB;
  int32_t j[3];
  if (!node_of_thread<D>(g, j)) return;
  int32_t lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = j[k];                               // primal j = q
    hi[k] = (j[k] + 1 == g.K[k]) ? 0 : j[k] + 1;  // primal j = q + 1 (wrapped)
  }
  int64_t cn[1 << D];
#pragma unroll
  for (int e = 0; e < (1 << D); ++e) cn[e] = corner_node<D>(lo, hi, e, g);

  const T* H = tab + TL::PASS_OFF;
  T acc[D][NC];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int s = 0; s < NC; ++s) acc[i][s] = T(0);
  const int64_t nodes = g.nodes;
  const int64_t field = (int64_t)NC * nodes;

#pragma unroll
  for (int eL = 0; eL < 2; ++eL)
#pragma unroll
    for (int l = 0; l < MP; ++l) {
      const int slot = eL * MP + l;
      T Y[NB];
      slice<D, M, 0, 0>(p, nodes, cn, eL, l, H, H, Y);
      merge<D, M, 0>(tab + TL::u_off(0) + slot * merged_nnz<D, M>(0), Y, acc[0]);
      if constexpr (D > 1) merge<D, M, 1>(tab + TL::u_off(1) + slot * merged_nnz<D, M>(1), Y, acc[1]);
      if constexpr (D > 2) merge<D, M, 2>(tab + TL::u_off(2) + slot * merged_nnz<D, M>(2), Y, acc[2]);
    }
  const int64_t n0 = corner_node<D>(lo, lo, 0, g);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      const int64_t a = (int64_t)i * field + (int64_t)s * nodes + n0;
      u[a] = fma(-wscale, acc[i][s], u[a]);
    }
}

}  // namespace hl
