// hl_kernels_ext.hpp - kernels beyond the constant-coefficient step: the
// discrete adjoint (periodic and walled), the variable-coefficient half-steps
// and their adjoint, the batched-shot launches and their sources.  They reuse
// the half-step bodies and helpers of hl_kernels.hpp.
#pragma once

#include "hl_kernels.hpp"

namespace hl {

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
// Output rows per pass: all nc at once up to nc = 27 (nc inputs plus nc
// accumulators in registers); beyond that (2D m >= 5, 3D m = 3) passes of 16
// rows, each re-reading the corner data (L1/L2 hits) so that the registers
// and the unrolled code stay bounded.
constexpr int kAdjointMaxNC = 27;
template <int NC>
constexpr int kAdjRows = NC <= kAdjointMaxNC ? NC : 16;

// acc[r] += sum_c Tb[r][c] src[c] for the rows r0 + r < NC of one pass.
template <int NC, int RB, typename T>
__device__ __forceinline__ void dense_rows(const T* __restrict__ Tb, int r0, const T* src, T* acc) {
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (r0 + r >= NC) break;
    // keep the scalar table loads of one row together (SGPR pressure)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[r] = fma(Tb[r * NC + c], src[c], acc[r]);
  }
}

template <int D, int M, class S, bool PTYPE>
__device__ __forceinline__ void adjoint_half_body(typename S::View out, typename S::View in,
                                                  const typename S::C* __restrict__ tab, Grid g, int blk) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC, NO = PTYPE ? 1 : D, NI = PTYPE ? D : 1;
  constexpr int RB = kAdjRows<NC>, NRB = (NC + RB - 1) / RB;
  int32_t j[3];
  if (!node_of_block<D>(g, blk, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);
  const uint32_t n0 = out_index<D>(g, j);
#pragma unroll 1
  for (int io = 0; io < NO; ++io) {
#pragma unroll 1
    for (int rb = 0; rb < NRB; ++rb) {
      T acc[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) acc[r] = T(0);
#pragma unroll
      for (int e = 0; e < (1 << D); ++e) {
#pragma unroll 1
        for (int ii = 0; ii < NI; ++ii) {
          T src[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) src[c] = S::load(in, ii * NC + c, cn[e]);
          dense_rows<NC, RB>(tab + ((int64_t)((e * NO + io) * NI + ii) * NC + rb * RB) * NC, rb * RB, src, acc);
        }
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (rb * RB + r >= NC) break;
        S::update(out, io * NC + rb * RB + r, n0, [&](T x) { return x - acc[r]; });
      }
    }
  }
}

template <int D, int M, class S, bool PTYPE>
__global__ void __launch_bounds__(256) adjoint_half(typename S::View out, typename S::View in,
                                                    const typename S::C* __restrict__ tab, Grid g) {
  adjoint_half_body<D, M, S, PTYPE>(out, in, tab, g, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Discrete adjoint with reflecting walls.  The walled step is P' = P - A G U,
// U' = U - B P' with G the ghost refresh (each ghost the signed mirror of an
// interior node); its transpose is Pb <- Pb - B^T Ub (adjoint_half with the
// pressure grid, the ghost slots of Ub held at zero: B writes no ghost), then
// Ub <- Ub - G^T A^T Pb: A^T Pb on every slot of the padded velocity array
// (adjoint_walls_at below; primal corners beyond the walls contribute
// nothing) into a scratch array, then the fold G^T (ghost_fold) that adds
// each ghost slot, with its mirror sign, into the node it mirrors.
// ---------------------------------------------------------------------------

// scr[r] -= sum_e' T[e'] Pb[r - 1 + e'] at padded dual slot r (0..K+1 per
// dimension) over the primal corners inside [0, K]: the grid's K are the
// padded extents, soff = -1, sext the primal extents.
template <int D, int M, class S>
__global__ void __launch_bounds__(256) adjoint_walls_at(typename S::View scr, typename S::View pb,
                                                        const typename S::C* __restrict__ tab, Grid g) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC, RB = kAdjRows<NC>, NRB = (NC + RB - 1) / RB;
  int32_t j[3];
  if (!node_of_block<D>(g, blockIdx.x, j)) return;
  int32_t lo[3] = {0, 0, 0};
  bool vlo[3] = {true, true, true}, vhi[3] = {true, true, true};
#pragma unroll
  for (int k = 0; k < D; ++k) {
    lo[k] = j[k] - 1;
    vlo[k] = lo[k] >= 0;
    vhi[k] = lo[k] + 1 < g.sext[k];
  }
  const uint32_t n0 = node_index<D>(j[0], j[1], j[2], g.oext);
#pragma unroll 1
  for (int io = 0; io < D; ++io) {
#pragma unroll 1
    for (int rb = 0; rb < NRB; ++rb) {
      T acc[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) acc[r] = T(0);
#pragma unroll
      for (int e = 0; e < (1 << D); ++e) {
        bool valid = true;
        int32_t c3[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const bool up = (e >> k) & 1;
          valid = valid && (up ? vhi[k] : vlo[k]);
          c3[k] = lo[k] + (up ? 1 : 0);
        }
        if (!valid) continue;
        const uint32_t cn = node_index<D>(c3[0], c3[1], c3[2], g.sext);
        T src[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) src[c] = S::load(pb, c, cn);
        dense_rows<NC, RB>(tab + ((int64_t)(e * D + io) * NC + rb * RB) * NC, rb * RB, src, acc);
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (rb * RB + r >= NC) break;
        S::update(scr, io * NC + rb * RB + r, n0, [&](T x) { return x - acc[r]; });
      }
    }
  }
}

// G^T: ub[q] += scr[q] + sum over the ghost slots mirroring q of the signed
// ghost value, and every scratch slot read is cleared (each ghost mirrors
// exactly one interior node, so each slot is read once).  One work-item per
// interior dual node; E the padded extents.
template <int D, int M, class S>
__global__ void __launch_bounds__(256) ghost_fold(typename S::View ub, typename S::View scr, int32_t E0, int32_t E1,
                                                  int32_t E2) {
  using T = typename S::C;
  constexpr int MP = M + 1, NC = Dims<D, M>::NC;
  const int32_t E[3] = {E0, E1, E2};
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t q[3] = {1, 1, 1};  // padded index of the interior node
  int64_t total = 1;
  for (int k = 0; k < D; ++k) total *= E[k] - 2;
  if (t >= total) return;
  for (int k = 0; k < D; ++k) {
    q[k] = 1 + (int32_t)(t % (E[k] - 2));
    t /= (E[k] - 2);
  }
  // dimensions where q touches a wall and the ghost index across it
  int32_t gidx[3] = {0, 0, 0};
  bool at[3] = {false, false, false};
  for (int k = 0; k < D; ++k) {
    if (q[k] == 1) {
      at[k] = true;
      gidx[k] = 0;
    } else if (q[k] == E[k] - 2) {
      at[k] = true;
      gidx[k] = E[k] - 1;
    }
  }
  const uint32_t n_q = node_index<D>(q[0], q[1], q[2], E);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T v = S::load(scr, i * NC + c, n_q);
      S::store(scr, i * NC + c, n_q, T(0));
      // every nonempty subset R of the wall dimensions: the ghost reflected in R
#pragma unroll
      for (int R = 1; R < (1 << D); ++R) {
        bool ok = true, neg = false;
        int32_t gq[3] = {q[0], q[1], q[2]};
#pragma unroll
        for (int k = 0; k < D; ++k)
          if ((R >> k) & 1) {
            ok = ok && at[k];
            gq[k] = gidx[k];
            neg ^= ((digit(c, MP, k) & 1) != 0) != (i != k);
          }
        if (!ok) continue;
        const uint32_t n_g = node_index<D>(gq[0], gq[1], gq[2], E);
        const T w = S::load(scr, i * NC + c, n_g);
        S::store(scr, i * NC + c, n_g, T(0));
        v += neg ? -w : w;
      }
      S::update(ub, i * NC + c, n_q, [&](T x) { return x + v; });
    }
}

// Zero the ghost shell of a padded velocity array (E the padded extents).
template <int D, int M, class S>
__global__ void __launch_bounds__(256) ghost_zero(typename S::View u, int32_t E0, int32_t E1, int32_t E2) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC;
  const int32_t E[3] = {E0, E1, E2};
  int64_t total = 1;
  for (int k = 0; k < D; ++k) total *= E[k];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  int32_t idx[3] = {0, 0, 0};
  bool shell = false;
  for (int k = 0; k < D; ++k) {
    idx[k] = (int32_t)(t % E[k]);
    t /= E[k];
    shell = shell || idx[k] == 0 || idx[k] == E[k] - 1;
  }
  if (!shell) return;
  const uint32_t n = node_index<D>(idx[0], idx[1], idx[2], E);
  for (int pl = 0; pl < D * NC; ++pl) S::store(u, pl, n, T(0));
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
// cell), so the kernels build the full (2m+2)^d interpolant in registers, one
// work-item per node (d = 1, d = 2, and d = 3 with m <= 1); 3D m >= 2 uses
// one wavefront per node (below).
// ---------------------------------------------------------------------------
template <int D, int M>
struct VK {
  static constexpr int N2 = 2 * M + 2, MP = M + 1;
  static constexpr int NP = ipow(N2, D);            // cell polynomial coefficients
  static constexpr int KMAX = D * M;
};

// w_k / w_{k-1} for k = 1..kVarMaxK (kmax = d m <= 10 for every built (d, m):
// 2D m = 5 reaches 10).
constexpr int kVarMaxK = 10;

// The series is accumulated as t_k = w_k r_k with t_k = (w_k / w_{k-1})
// T[kappa Lap t_{k-1}]: the ratio (dt/2)^2 / (2k (2k+1)) cancels the 1/h^2 of
// each Laplacian, so every term stays O(1) (r_k alone grows like h^{-2k} and
// overflows FP32 for large m).
template <typename T>
struct VarArgs {
  T w0;        // w_0 = dt
  T ratio[kVarMaxK + 1];  // w_k / w_{k-1} = (dt/2)^2 / (2k (2k+1)), k = 1..kmax
  T ih[3];     // 1 / h_k
};

// The truncated products of the adjoint kernels load their kappa terms in
// groups of kKappaGroup, each group issued while the previous one is applied.
// The plane base of every load is formed from an opaque scalar zero taken
// once per group: otherwise the compiler keeps one 64-bit address per kappa
// plane for the whole kernel (2 VGPRs per term: 128 at 2D m = 3), and with
// the scheduling barrier after each group it cannot hoist every load of a
// product to its start either.
constexpr int kKappaGroup = 4;

// out_b += kappa_A f_{b-A} (TR = false: T[kappa f]) or out_b += kappa_A f_{A+b}
// (TR = true: T^T[kappa] f), for one term A.
template <int D, int M, bool TR, int A, typename T>
__device__ __forceinline__ void kterm_apply(T ka, const T* f, T* out) {
  constexpr int N2 = 2 * M + 2, AX = A % N2, AY = (A / N2) % N2, AZ = A / (N2 * N2);
  constexpr int NY = D > 1 ? N2 : 1, NZ = D > 2 ? N2 : 1;
#pragma unroll
  for (int bz = 0; bz + AZ < NZ; ++bz)
#pragma unroll
    for (int by = 0; by + AY < NY; ++by)
#pragma unroll
      for (int bx = 0; bx + AX < N2; ++bx) {
        const int lo = bx + N2 * (by + N2 * bz), hi = (bx + AX) + N2 * ((by + AY) + N2 * (bz + AZ));
        if constexpr (TR)
          out[lo] = fma(ka, f[hi], out[lo]);
        else
          out[hi] = fma(ka, f[lo], out[hi]);
      }
}

template <int D, int M, bool TR, int BASE, typename T, int... I>
__device__ __forceinline__ void kgroup_apply(const T* kc, const T* f, T* out, std::integer_sequence<int, I...>) {
  (kterm_apply<D, M, TR, BASE + I>(kc[I], f, out), ...);
}

// kb[i] = kappa_{BASE + i} for the terms BASE + i < NP.
template <class S, int BASE, int NP>
__device__ __forceinline__ void kgroup_load(const typename S::View& kv, uint32_t n0, typename S::C* kb) {
  int zero;
  asm volatile("s_mov_b32 %0, 0" : "=s"(zero));
#pragma unroll
  for (int i = 0; i < kKappaGroup; ++i)
    if (BASE + i < NP) kb[i] = S::load(kv, BASE + i + zero, n0);
}

template <int D, int M, bool TR, class S, int GRP>
__device__ __forceinline__ void kgroup_step(const typename S::View& kv, uint32_t n0, const typename S::C* f,
                                            typename S::C* out, typename S::C (*kb)[kKappaGroup]) {
  constexpr int G = kKappaGroup, NP = VK<D, M>::NP, NG = (NP + G - 1) / G;
  constexpr int CNT = NP - GRP * G < G ? NP - GRP * G : G;
  if constexpr (GRP + 1 < NG) kgroup_load<S, (GRP + 1) * G, NP>(kv, n0, kb[(GRP + 1) & 1]);
  kgroup_apply<D, M, TR, GRP * G>(kb[GRP & 1], f, out, std::make_integer_sequence<int, CNT>{});
  __builtin_amdgcn_sched_barrier(0);
}

template <int D, int M, bool TR, class S, int... GRP>
__device__ __forceinline__ void kgroup_steps(const typename S::View& kv, uint32_t n0, const typename S::C* f,
                                             typename S::C* out, std::integer_sequence<int, GRP...>) {
  typename S::C kb[2][kKappaGroup];
  kgroup_load<S, 0, VK<D, M>::NP>(kv, n0, kb[0]);
  (kgroup_step<D, M, TR, S, GRP>(kv, n0, f, out, kb), ...);
}

// out = T[kappa f] (TR = false) or T^T[kappa] f (TR = true), kappa_a read
// from plane a of the kappa array at node n0.  The same terms in the same
// order as tprod.
template <int D, int M, bool TR, class S>
__device__ __forceinline__ void tprod_grouped(const typename S::View& kv, uint32_t n0, const typename S::C* f,
                                              typename S::C* out) {
  using T = typename S::C;
  constexpr int NP = VK<D, M>::NP, NG = (NP + kKappaGroup - 1) / kKappaGroup;
#pragma unroll
  for (int b = 0; b < NP; ++b) out[b] = T(0);
  kgroup_steps<D, M, TR, S>(kv, n0, f, out, std::make_integer_sequence<int, NG>{});
}

// The forward variable-kappa half-steps take the grouped kappa loads from
// m = 4 on, where the per-term loads' addresses spill (2D m = 4 FP64: 788 ->
// 124 bytes of scratch per lane, m = 5 FP32: 507 -> 359 VGPRs); below, the
// per-term loads measured faster (2D m = 3 1024^2 FP32 0.86 against 0.91 ms).
template <int D, int M, class S>
__device__ __forceinline__ void tprod_fwd(const typename S::View& kv, uint32_t n0, const typename S::C* f,
                                          typename S::C* out) {
  if constexpr (M >= 4)
    tprod_grouped<D, M, false, S>(kv, n0, f, out);
  else
    tprod<D, M, S>(kv, n0, f, out);
}

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
  static_assert(VK<D, M>::KMAX <= kVarMaxK, "series longer than the ratio table");
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
  tprod_fwd<D, M, S>(kp, n0, div, t);  // t_0 = w_0 r_0
#pragma unroll
  for (int s = 0; s < NC; ++s) acc[s] = t[poly_index<D, M>(s, 0, 0, 0)];
#pragma unroll 1
  for (int k = 1; k <= VK<D, M>::KMAX; ++k) {
    T l[NP];
    lap_coef<D, M>(t, l, va.ih, va.ratio[k]);
    tprod_fwd<D, M, S>(kp, n0, l, t);  // t_k = w_k r_k
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
    tprod_fwd<D, M, S>(ku, n0, l, gk);
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
// Variable kappa, 3D m = 2 and 3: one wavefront per node.  The cell
// polynomial has (2m+2)^3 coefficients per field (216 at m = 2, 512 at
// m = 3): two of them (the current term and its Laplacian) no longer fit in
// one work-item's registers, so the 64 work-items of a workgroup share one
// node.  Its polynomials live in LDS, and in the products and Laplacians
// lane l < (2m+2)^2 owns the x-pencil b_y = l mod (2m+2), b_z = l div (2m+2)
// (2m+2 coefficients along x, held in registers).  The arithmetic is that of
// the per-node kernels above (the same tensor-product passes, and the same
// products kappa_a f_{b-a}), except that at m = 2 a pencil's sum is formed
// from partial sums over chunks of its terms (below).
// ---------------------------------------------------------------------------
template <int M>
struct VW {
  static constexpr int MP = M + 1, N2 = 2 * M + 2, NP = N2 * N2 * N2, NPEN = N2 * N2, NC = MP * MP * MP;
  static_assert(NPEN <= 64 && 8 * NC == NP && 4 * MP * MP == NPEN, "one pencil and one line per lane");
};

// Node of workgroup blk when every workgroup updates one node: consecutive
// node numbers (x fastest) go to one XCD, so neighbours share its L2.
__device__ __forceinline__ bool wave_node(const Grid& g, int blk, int32_t per_xcd, int32_t* j) {
  const int64_t t = (int64_t)(blk % kXcds) * per_xcd + blk / kXcds;
  if (t >= (int64_t)g.K[0] * g.K[1] * g.K[2]) return false;
  j[0] = (int32_t)(t % g.K[0]);
  j[1] = (int32_t)((t / g.K[0]) % g.K[1]);
  j[2] = (int32_t)(t / ((int64_t)g.K[0] * g.K[1]));
  return true;
}

// Corner e of the node's cell (bit k of e: upper side in dimension k), wrapped
// as corner_nodes wraps it.
__device__ __forceinline__ uint32_t corner_node_of(const Grid& g, const int32_t* j, int e) {
  int32_t c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int32_t lo = j[k] + g.soff, hi = lo + 1;
    if (lo < 0) lo += g.sext[k];
    if (hi == g.sext[k]) hi = 0;
    c[k] = ((e >> k) & 1) ? hi : lo;
  }
  return node_index<3>(c[0], c[1], c[2], g.sext);
}

// Full interpolant of component comp into B[b_x + N2 (b_y + N2 b_z)], through
// A: the raw corner data A[e + 8 a], the x pass into B (line ey + 2 ez + 4
// (ay + MP az), entries b_x), the y pass into A (line ez + 2 (az + MP b_x),
// entries b_y), the z pass into B.  Every line is one lane's.
template <int M, class S>
__device__ __forceinline__ void interp_wave(const typename S::View& f, int comp, uint32_t cnl, int lane,
                                            typename S::C* A, typename S::C* B) {
  using T = typename S::C;
  constexpr int MP = VW<M>::MP, N2 = VW<M>::N2, NC = VW<M>::NC, NL = VW<M>::NPEN;
  for (int a = lane >> 3; a < NC; a += 8) A[(lane & 7) + 8 * a] = S::load(f, comp * NC + a, cnl);
  __syncthreads();
  if (lane < NL) {
    const int ey = lane & 1, ez = (lane >> 1) & 1, ay = (lane >> 2) % MP, az = (lane >> 2) / MP;
    T L[MP], R[MP], o[N2];
#pragma unroll
    for (int ax = 0; ax < MP; ++ax) {
      const int a = ax + MP * (ay + MP * az);
      L[ax] = A[2 * ey + 4 * ez + 8 * a];
      R[ax] = A[1 + 2 * ey + 4 * ez + 8 * a];
    }
    pass1d<M, 0>(L, R, o);
#pragma unroll
    for (int b = 0; b < N2; ++b) B[lane * N2 + b] = o[b];
  }
  __syncthreads();
  if (lane < NL) {
    const int ez = lane & 1, az = (lane >> 1) % MP, bx = (lane >> 1) / MP;
    T L[MP], R[MP], o[N2];
#pragma unroll
    for (int ay = 0; ay < MP; ++ay) {
      L[ay] = B[(2 * ez + 4 * (ay + MP * az)) * N2 + bx];
      R[ay] = B[(1 + 2 * ez + 4 * (ay + MP * az)) * N2 + bx];
    }
    pass1d<M, 0>(L, R, o);
#pragma unroll
    for (int b = 0; b < N2; ++b) A[lane * N2 + b] = o[b];
  }
  __syncthreads();
  if (lane < NL) {
    const int bx = lane % N2, by = lane / N2;
    T L[MP], R[MP], o[N2];
#pragma unroll
    for (int az = 0; az < MP; ++az) {
      L[az] = A[(2 * (az + MP * bx)) * N2 + by];
      R[az] = A[(1 + 2 * (az + MP * bx)) * N2 + by];
    }
    pass1d<M, 0>(L, R, o);
#pragma unroll
    for (int b = 0; b < N2; ++b) B[bx + N2 * (by + N2 * b)] = o[b];
  }
  __syncthreads();
}

// Work split of one truncated product over the 64 lanes.  Pencil (by, bz)
// sums over the (by+1)(bz+1) pairs (a_y, a_z) <= (by, bz) (a_z outer), 2m+2
// to 36 of them at m = 2; one lane per pencil would leave 28 lanes idle and
// wait on the longest pencil.  Instead every pencil's pairs are cut into
// chunks of at most C consecutive pairs, one chunk per lane, C the smallest
// length that needs at most 64 chunks (m = 2: C = 10, 60 chunks; m = 3: no
// cut, the 64 pencils take the 64 lanes), and each pencil then adds its
// chunks' partial sums in chunk order.
template <int M>
struct WaveSched {
  int C, n;
  int8_t by[64], bz[64], i0[64], cnt[64];  // chunk (lane) -> pencil, first pair, pairs
  int8_t first[64], nch[64];               // pencil -> its first chunk, chunks
};

template <int M>
constexpr WaveSched<M> wave_sched() {
  constexpr int N2 = 2 * M + 2;
  WaveSched<M> s{};
  int C = 1;
  for (;; ++C) {
    int n = 0;
    for (int q = 0; q < N2 * N2; ++q) n += ((q % N2 + 1) * (q / N2 + 1) + C - 1) / C;
    if (n <= 64) break;
  }
  s.C = C;
  int c = 0;
  for (int q = 0; q < N2 * N2; ++q) {
    const int w = (q % N2 + 1) * (q / N2 + 1);
    s.first[q] = (int8_t)c;
    s.nch[q] = (int8_t)((w + C - 1) / C);
    for (int i = 0; i < w; i += C, ++c) {
      s.by[c] = (int8_t)(q % N2);
      s.bz[c] = (int8_t)(q / N2);
      s.i0[c] = (int8_t)i;
      s.cnt[c] = (int8_t)(w - i < C ? w - i : C);
    }
  }
  s.n = c;
  return s;
}

// Every pencil's pairs covered once, in order, by its chunks.
template <int M>
constexpr bool wave_sched_ok(const WaveSched<M>& s) {
  constexpr int N2 = 2 * M + 2;
  if (s.n > 64) return false;
  for (int q = 0; q < N2 * N2; ++q) {
    int next = 0;
    for (int c = s.first[q]; c < s.first[q] + s.nch[q]; ++c) {
      if (s.by[c] != q % N2 || s.bz[c] != q / N2 || s.i0[c] != next || s.cnt[c] < 1 || s.cnt[c] > s.C) return false;
      next += s.cnt[c];
    }
    if (next != (q % N2 + 1) * (q / N2 + 1)) return false;
  }
  return true;
}

template <int M>
constexpr WaveSched<M> kWaveSched = wave_sched<M>();
static_assert(wave_sched_ok<2>(kWaveSched<2>) && kWaveSched<2>.C == 10 && kWaveSched<2>.n == 60, "m = 2 split");
static_assert(wave_sched_ok<3>(kWaveSched<3>) && kWaveSched<3>.n == 64, "m = 3: one chunk per pencil");
// LDS words for the chunks' partial sums (1 when no pencil is cut)
template <int M>
constexpr int kWaveRed = kWaveSched<M>.n > VW<M>::NPEN ? 64 * VW<M>::N2 : 1;

// Partial sum of pencil (by, bz) of T[kappa f] over the pairs i0 .. i0+cnt-1:
// out[b_x] = sum of kappa_a f_{b-a}, a_x <= b_x, K and F in LDS.
template <int M, typename T>
__device__ __forceinline__ void tprod_chunk(const T* KA, const T* F, int by, int bz, int i0, int cnt, T* out) {
  constexpr int N2 = VW<M>::N2;
#pragma unroll
  for (int b = 0; b < N2; ++b) out[b] = T(0);
  int ay = i0 % (by + 1), az = i0 / (by + 1);
  for (int i = 0; i < cnt; ++i) {
    T kp[N2], fp[N2];
    const T* kr = KA + N2 * (ay + N2 * az);
    const T* fr = F + N2 * ((by - ay) + N2 * (bz - az));
#pragma unroll
    for (int b = 0; b < N2; ++b) {
      kp[b] = kr[b];
      fp[b] = fr[b];
    }
#pragma unroll
    for (int bx = 0; bx < N2; ++bx)
#pragma unroll
      for (int ax = 0; ax <= bx; ++ax) out[bx] = fma(kp[ax], fp[bx - ax], out[bx]);
    if (++ay > by) {
      ay = 0;
      ++az;
    }
  }
}

// Pencil (by, bz) of T[kappa f] in one lane (no cut): a_z outer, a_y inner.
template <int M, typename T>
__device__ __forceinline__ void tprod_pencil(const T* KA, const T* F, int by, int bz, T* out) {
  constexpr int N2 = VW<M>::N2;
#pragma unroll
  for (int b = 0; b < N2; ++b) out[b] = T(0);
  for (int az = 0; az <= bz; ++az)
    for (int ay = 0; ay <= by; ++ay) {
      T kp[N2], fp[N2];
      const T* kr = KA + N2 * (ay + N2 * az);
      const T* fr = F + N2 * ((by - ay) + N2 * (bz - az));
#pragma unroll
      for (int b = 0; b < N2; ++b) {
        kp[b] = kr[b];
        fp[b] = fr[b];
      }
#pragma unroll
      for (int bx = 0; bx < N2; ++bx)
#pragma unroll
        for (int ax = 0; ax <= bx; ++ax) out[bx] = fma(kp[ax], fp[bx - ax], out[bx]);
    }
}

// This lane's chunk of a truncated product, and the pencil totals.
template <int M>
struct WaveLane {
  int lane, cby, cbz, ci0, ccnt;  // the lane's chunk
  bool pen;                       // lane < (2m+2)^2 owns pencil (by, bz) = (lane mod N2, lane div N2)
  int by, bz, first, nch;
  __device__ __forceinline__ explicit WaveLane(int l) : lane(l) {
    constexpr int N2 = VW<M>::N2;
    const WaveSched<M>& s = kWaveSched<M>;
    const bool has = l < s.n;
    cby = has ? s.by[l] : 0;
    cbz = has ? s.bz[l] : 0;
    ci0 = has ? s.i0[l] : 0;
    ccnt = has ? s.cnt[l] : 0;
    pen = l < VW<M>::NPEN;
    by = pen ? l % N2 : 0;
    bz = pen ? l / N2 : 0;
    first = pen ? s.first[l] : 0;
    nch = pen ? s.nch[l] : 0;
  }
};

// t = pencil (by, bz) of T[kappa F] on the owning lanes; RED: 64 (2m+2)
// partial sums.  Begins and ends with LDS reads only; callers separate it
// from the next writes of F and RED by a barrier.
template <int M, typename T>
__device__ __forceinline__ void tprod_wave(const T* KA, const T* F, T* RED, const WaveLane<M>& w, T* t) {
  constexpr int N2 = VW<M>::N2;
  constexpr bool kSplit = kWaveSched<M>.n > VW<M>::NPEN;
  T part[N2];
  if constexpr (kSplit)
    tprod_chunk<M>(KA, F, w.cby, w.cbz, w.ci0, w.ccnt, part);
  else
    tprod_pencil<M>(KA, F, w.cby, w.cbz, part);
  if constexpr (kSplit) {
#pragma unroll
    for (int b = 0; b < N2; ++b) RED[w.lane * N2 + b] = part[b];
    __syncthreads();
#pragma unroll
    for (int b = 0; b < N2; ++b) t[b] = T(0);
    for (int q = 0; q < w.nch; ++q) {
#pragma unroll
      for (int b = 0; b < N2; ++b) t[b] += RED[(w.first + q) * N2 + b];
    }
  } else {  // chunk c is pencil c
#pragma unroll
    for (int b = 0; b < N2; ++b) t[b] = part[b];
  }
}

// Pencil (by, bz) of sc Lap t (coefficient space), t in LDS.
template <int M, typename T>
__device__ __forceinline__ void lap_pencil(const T* t, int by, int bz, const T* ih, T sc, T* out) {
  constexpr int N2 = VW<M>::N2;
  const T ix2 = sc * ih[0] * ih[0], iy2 = sc * ih[1] * ih[1], iz2 = sc * ih[2] * ih[2];
  const T* r0 = t + N2 * (by + N2 * bz);
#pragma unroll
  for (int bx = 0; bx < N2; ++bx) {
    T v = T(0);
    if (bx + 2 < N2) v = fma(T((bx + 1) * (bx + 2)) * ix2, r0[bx + 2], v);
    if (by + 2 < N2) v = fma(T((by + 1) * (by + 2)) * iy2, r0[bx + 2 * N2], v);
    if (bz + 2 < N2) v = fma(T((bz + 1) * (bz + 2)) * iz2, r0[bx + 2 * N2 * N2], v);
    out[bx] = v;
  }
}

template <int M, class S>
__device__ __forceinline__ void p_half_var_wave_body(typename S::View p, typename S::View u, typename S::View kp,
                                                     Grid g, VarArgs<typename S::C> va, int32_t per_xcd, int blk) {
  using T = typename S::C;
  constexpr int MP = VW<M>::MP, N2 = VW<M>::N2, NP = VW<M>::NP;
  static_assert(VK<3, M>::KMAX <= kVarMaxK, "series longer than the ratio table");
  __shared__ T A[NP], B[NP], KA[NP], RED[kWaveRed<M>];
  int32_t j[3];
  if (!wave_node(g, blk, per_xcd, j)) return;  // uniform over the workgroup
  const int lane = threadIdx.x;
  const WaveLane<M> w(lane);
  const uint32_t n0 = out_index<3>(g, j);
  const uint32_t cnl = corner_node_of(g, j, lane & 7);  // dual q = j - 1 + e
  for (int a = lane; a < NP; a += 64) KA[a] = S::load(kp, a, n0);
  const bool pen = w.pen;
  const int by = w.by, bz = w.bz;
  T dv[N2];  // w_0 div c on the lane's pencil
#pragma unroll
  for (int b = 0; b < N2; ++b) dv[b] = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    interp_wave<M, S>(u, i, cnl, lane, A, B);
    if (pen) {
      const T f = va.w0 * va.ih[i];
      const T* r = B + N2 * (by + N2 * bz);
#pragma unroll
      for (int bx = 0; bx < N2; ++bx) {
        if (i == 0 && bx + 1 < N2) dv[bx] = fma(T(bx + 1) * f, r[bx + 1], dv[bx]);
        if (i == 1 && by + 1 < N2) dv[bx] = fma(T(by + 1) * f, r[bx + N2], dv[bx]);
        if (i == 2 && bz + 1 < N2) dv[bx] = fma(T(bz + 1) * f, r[bx + N2 * N2], dv[bx]);
      }
    }
    __syncthreads();
  }
  T* F = A;  // Laplacian of the current term (input of the product)
  T* Tc = B;  // current term t_k
  if (pen) {
#pragma unroll
    for (int b = 0; b < N2; ++b) F[N2 * (by + N2 * bz) + b] = dv[b];
  }
  __syncthreads();
  const bool own = pen && by < MP && bz < MP;  // pencil holds data entries (b_x < MP)
  T acc[MP], t[N2];
#pragma unroll
  for (int b = 0; b < N2; ++b) t[b] = T(0);
  tprod_wave<M>(KA, F, RED, w, t);  // t_0 = w_0 r_0
#pragma unroll
  for (int b = 0; b < MP; ++b) acc[b] = t[b];
#pragma unroll 1
  for (int k = 1; k <= VK<3, M>::KMAX; ++k) {
    if (pen) {
#pragma unroll
      for (int b = 0; b < N2; ++b) Tc[N2 * (by + N2 * bz) + b] = t[b];
    }
    __syncthreads();
    if (pen) {
      T l[N2];
      lap_pencil<M>(Tc, by, bz, va.ih, va.ratio[k], l);
#pragma unroll
      for (int b = 0; b < N2; ++b) F[N2 * (by + N2 * bz) + b] = l[b];
    }
    __syncthreads();
    tprod_wave<M>(KA, F, RED, w, t);  // t_k = w_k r_k
#pragma unroll
    for (int b = 0; b < MP; ++b) acc[b] += t[b];
  }
  if (own) {
#pragma unroll
    for (int bx = 0; bx < MP; ++bx)
      S::update(p, bx + MP * (by + MP * bz), n0, [&](T x) { return x - acc[bx]; });
  }
}

template <int M, class S>
__device__ __forceinline__ void u_half_var_wave_body(typename S::View u, typename S::View p, typename S::View ku,
                                                     Grid g, VarArgs<typename S::C> va, typename S::C wscale,
                                                     int32_t per_xcd, int blk) {
  using T = typename S::C;
  constexpr int MP = VW<M>::MP, N2 = VW<M>::N2, NP = VW<M>::NP, NC = VW<M>::NC;
  __shared__ T A[NP], B[NP], KA[NP], RED[kWaveRed<M>];
  int32_t j[3];
  if (!wave_node(g, blk, per_xcd, j)) return;  // uniform over the workgroup
  const int lane = threadIdx.x;
  const WaveLane<M> w(lane);
  const uint32_t n0 = out_index<3>(g, j);
  const uint32_t cnl = corner_node_of(g, j, lane & 7);  // primal j = q + e
  for (int a = lane; a < NP; a += 64) KA[a] = S::load(ku, a, n0);
  const bool pen = w.pen;
  const int by = w.by, bz = w.bz;
  interp_wave<M, S>(p, 0, cnl, lane, A, B);
  T* F = A;  // Laplacian of the current term (input of the product)
  T* Tc = B;  // current term g_k
  T gk[N2], q[N2];
#pragma unroll
  for (int b = 0; b < N2; ++b) gk[b] = T(0);
  if (pen) {
#pragma unroll
    for (int b = 0; b < N2; ++b) gk[b] = Tc[N2 * (by + N2 * bz) + b] * va.w0;
  }
#pragma unroll
  for (int b = 0; b < N2; ++b) q[b] = gk[b];
  __syncthreads();
#pragma unroll 1
  for (int k = 1; k <= VK<3, M>::KMAX; ++k) {
    if (pen) {
#pragma unroll
      for (int b = 0; b < N2; ++b) Tc[N2 * (by + N2 * bz) + b] = gk[b];
    }
    __syncthreads();
    if (pen) {
      T l[N2];
      lap_pencil<M>(Tc, by, bz, va.ih, va.ratio[k], l);
#pragma unroll
      for (int b = 0; b < N2; ++b) F[N2 * (by + N2 * bz) + b] = l[b];
    }
    __syncthreads();
    tprod_wave<M>(KA, F, RED, w, gk);
#pragma unroll
    for (int b = 0; b < N2; ++b) q[b] += gk[b];
  }
  // u_i[s] -= wscale (s_i + 1) / h_i q[s + e_i]: the pencil holding q[s + e_i]
  // updates u_i[s]
  if (pen) {
    if (by < MP && bz < MP) {
      const T f = wscale * va.ih[0];
#pragma unroll
      for (int sx = 0; sx < MP; ++sx) {
        const T a = -(T)(sx + 1) * f, qv = q[sx + 1];
        S::update(u, sx + MP * (by + MP * bz), n0, [&](T x) { return fma(a, qv, x); });
      }
    }
    if (by >= 1 && by <= MP && bz < MP) {
      const T a = -(T)by * (wscale * va.ih[1]);
#pragma unroll
      for (int sx = 0; sx < MP; ++sx) {
        const T qv = q[sx];
        S::update(u, NC + sx + MP * ((by - 1) + MP * bz), n0, [&](T x) { return fma(a, qv, x); });
      }
    }
    if (by < MP && bz >= 1 && bz <= MP) {
      const T a = -(T)bz * (wscale * va.ih[2]);
#pragma unroll
      for (int sx = 0; sx < MP; ++sx) {
        const T qv = q[sx];
        S::update(u, 2 * NC + sx + MP * (by + MP * (bz - 1)), n0, [&](T x) { return fma(a, qv, x); });
      }
    }
  }
}

template <int M, class S>
__global__ void __launch_bounds__(64) p_half_var_wave(typename S::View p, typename S::View u, typename S::View kp,
                                                      Grid g, VarArgs<typename S::C> va, int32_t per_xcd) {
  p_half_var_wave_body<M, S>(p, u, kp, g, va, per_xcd, blockIdx.x);
}

template <int M, class S>
__global__ void __launch_bounds__(64) u_half_var_wave(typename S::View u, typename S::View p, typename S::View ku,
                                                      Grid g, VarArgs<typename S::C> va, typename S::C wscale,
                                                      int32_t per_xcd) {
  u_half_var_wave_body<M, S>(u, p, ku, g, va, wscale, per_xcd, blockIdx.x);
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

// Cell-polynomial slots on which the adjoint data y of a node can be nonzero:
// b in {0..m}^D (pressure side: the node's data block) or b = s + e_i with s
// in {0..m}^D (velocity side: the derivatives of Q that the velocity takes).
// y is held compactly on these slots.
template <int D, int M, bool PSIDE>
struct YSupport {
  static constexpr int N2 = 2 * M + 2, NP = VK<D, M>::NP;
  static constexpr bool in(int b) {
    const int dg[3] = {b % N2, D > 1 ? (b / N2) % N2 : 0, D > 2 ? b / (N2 * N2) : 0};
    int over = 0, top = 0, sum = 0;
    for (int k = 0; k < D; ++k) {
      if (dg[k] > M + 1) return false;
      top += dg[k] == M + 1;
      over += dg[k] > M;
      sum += dg[k];
    }
    return PSIDE ? over == 0 : top <= 1 && sum > 0;
  }
  static constexpr int count() {
    int c = 0;
    for (int b = 0; b < NP; ++b) c += in(b);
    return c;
  }
  static constexpr int idx(int b) {  // compact slot of b, -1 off the support
    int c = 0;
    for (int x = 0; x < b; ++x) c += in(x);
    return in(b) ? c : -1;
  }
  static constexpr int NY = count();
};

// Per-work-item arrays in LDS, slot (a, b) of lane l at [(a NP + b) 64 + l]:
// the adjoint kernels run 64 work-items per workgroup, consecutive lanes in
// consecutive banks.
template <typename T>
struct LaneLds {
  T* base;
  int lane;
  __device__ __forceinline__ T& operator()(int a, int b, int np) const { return base[(a * np + b) * 64 + lane]; }
};

// The gradient accumulators live in LDS (slot GS); t_0 and, on the pressure
// side, f as well when a cell polynomial takes 512 bytes or more (FP64 at
// 2D m = 3), where registers would spill to scratch.
template <int D, int M, typename T>
constexpr bool kGradStage = sizeof(T) * VK<D, M>::NP >= 512;

// grad_A += sum_b lam_{A+b} g_b (the kappa_A derivative of <lam, T[kappa g]>).
template <int D, int M, int A, typename T>
__device__ __forceinline__ void corr_term(const T* lam, const T* g, const LaneLds<T>& L, int gs) {
  constexpr int N2 = 2 * M + 2, AX = A % N2, AY = (A / N2) % N2, AZ = A / (N2 * N2);
  constexpr int NY = D > 1 ? N2 : 1, NZ = D > 2 ? N2 : 1, NP = VK<D, M>::NP;
  T acc = L(gs, A, NP);
#pragma unroll
  for (int bz = 0; bz + AZ < NZ; ++bz)
#pragma unroll
    for (int by = 0; by + AY < NY; ++by)
#pragma unroll
      for (int bx = 0; bx + AX < N2; ++bx)
        acc = fma(lam[(bx + AX) + N2 * ((by + AY) + N2 * (bz + AZ))], g[bx + N2 * (by + N2 * bz)], acc);
  L(gs, A, NP) = acc;
}

template <int D, int M, typename T, int... A>
__device__ __forceinline__ void corr_terms(const T* lam, const T* g, const LaneLds<T>& L, int gs,
                                           std::integer_sequence<int, A...>) {
  (corr_term<D, M, A>(lam, g, L, gs), ...);
}

template <int D, int M, typename T>
__device__ __forceinline__ void corr(const T* lam, const T* g, const LaneLds<T>& L, int gs) {
  corr_terms<D, M>(lam, g, L, gs, std::make_integer_sequence<int, VK<D, M>::NP>{});
}

// out = sc Lap^T f: sc sum_i (b_i - 1) b_i / h_i^2 f_{b - 2 e_i}.
template <int D, int M, typename T>
__device__ __forceinline__ void lapT_coef(const T* f, T* out, const T* ih, T sc) {
  constexpr int N2 = 2 * M + 2, NP = VK<D, M>::NP;
  const T ix2 = sc * ih[0] * ih[0], iy2 = sc * ih[1] * ih[1], iz2 = sc * ih[2] * ih[2];
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    const int bx = b % N2, by = (b / N2) % N2, bz = b / (N2 * N2);
    T v = T(0);
    if (bx >= 2) v = fma(T((bx - 1) * bx) * ix2, f[b - 2], v);
    if (D > 1 && by >= 2) v = fma(T((by - 1) * by) * iy2, f[b - 2 * N2], v);
    if (D > 2 && bz >= 2) v = fma(T((bz - 1) * bz) * iz2, f[b - 2 * N2 * N2], v);
    out[b] = v;
  }
}

// The series part shared by both sides: given t_0 (registers t0r, or LDS
// slot t0s when staged) and y (compact on its support), returns lam_0 in lam
// and adds sum_{k >= 1} sum_b lam_k[a + b] g_k[b] to the gradient (LDS slot gs).
template <int D, int M, bool PSIDE, class S>
__device__ __forceinline__ void adjoint_series(const typename S::View& kv, uint32_t n0,
                                               const LaneLds<typename S::C>& L, const typename S::C* t0r, int t0s,
                                               int gs, const typename S::C* yc, const VarArgs<typename S::C>& va,
                                               typename S::C* lam) {
  using T = typename S::C;
  using Y = YSupport<D, M, PSIDE>;
  constexpr int NP = VK<D, M>::NP;
  constexpr bool STAGE = kGradStage<D, M, T>;
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    const int yi = Y::idx(b);
    lam[b] = yi >= 0 ? yc[yi < 0 ? 0 : yi] : T(0);
  }
#pragma unroll 1
  for (int k = VK<D, M>::KMAX; k >= 1; --k) {
    T t[NP], l[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) t[b] = STAGE ? L(t0s, b, NP) : t0r[b];
#pragma unroll 1
    for (int q = 1; q < k; ++q) {  // t = t_{k-1}
      lap_coef<D, M>(t, l, va.ih, va.ratio[q]);
      tprod_grouped<D, M, false, S>(kv, n0, l, t);
    }
    lap_coef<D, M>(t, l, va.ih, va.ratio[k]);  // g_k
    corr<D, M>(lam, l, L, gs);
    tprod_grouped<D, M, true, S>(kv, n0, lam, t);
    lapT_coef<D, M>(t, l, va.ih, va.ratio[k]);
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int yi = Y::idx(b);
      lam[b] = (yi >= 0 ? yc[yi < 0 ? 0 : yi] : T(0)) + l[b];
    }
  }
}

// Pressure side at primal node j: with Pb the adjoint pressure and U_t the
// velocity before the step, gk -= dS/dkappa (FP64 accumulators, one plane per
// kappa coefficient) and rho_i = d S / d c^(i) (D NP planes of scratch).
// 64 work-items per workgroup (a 64 x 1 tile).
template <int D, int M, class S>
__global__ void __launch_bounds__(64) grad_p_var(typename S::View pb, typename S::View u, typename S::View kp,
                                                 double* __restrict__ gk, typename S::View rho, Grid g,
                                                 VarArgs<typename S::C> va) {
  static_assert(D <= 2 || M <= 1, "the adjoint of the variable-kappa half-steps: d <= 2, or d = 3 with m <= 1");
  using T = typename S::C;
  using Y = YSupport<D, M, true>;
  constexpr int N2 = 2 * M + 2, MP = M + 1, NP = VK<D, M>::NP, NC = Dims<D, M>::NC;
  constexpr bool STAGE = kGradStage<D, M, T>;
  constexpr int FS = 0, T0S = 1, GS = STAGE ? 2 : 0;  // LDS slots
  __shared__ T lds[(STAGE ? 3 : 1) * NP * 64];
  const LaneLds<T> L{lds, (int)threadIdx.x};
  int32_t j[3];
  if (!node_of_block<D>(g, blockIdx.x, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);  // dual q = j - 1 + e
  const uint32_t n0 = out_index<D>(g, j);
  T f[NP], t0[NP];  // f = w_0 div c, t_0 = T[kappa f]
#pragma unroll
  for (int b = 0; b < NP; ++b) f[b] = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T c[NP];
    interp_full<D, M, S>(u, i, cn, c);
    const int st = i == 0 ? 1 : i == 1 ? N2 : N2 * N2;
    const T w = va.w0 * va.ih[i];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int bi = digit(b, N2, i);
      if (bi + 1 < N2) f[b] = fma(T(bi + 1) * w, c[b + st], f[b]);
    }
  }
  tprod_grouped<D, M, false, S>(kp, n0, f, t0);
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    if (STAGE) {
      L(FS, b, NP) = f[b];
      L(T0S, b, NP) = t0[b];
    }
    L(GS, b, NP) = T(0);
  }
  T yc[Y::NY];
#pragma unroll
  for (int s = 0; s < NC; ++s) yc[Y::idx(poly_index<D, M>(s, 0, 0, 0))] = S::load(pb, s, n0);
  T lam[NP];
  adjoint_series<D, M, true, S>(kp, n0, L, t0, T0S, GS, yc, va, lam);
  if (STAGE) {
#pragma unroll
    for (int b = 0; b < NP; ++b) f[b] = L(FS, b, NP);
  }
  corr<D, M>(lam, f, L, GS);  // k = 0: t_0 = T[kappa f]
#pragma unroll
  for (int b = 0; b < NP; ++b) gk[(size_t)b * g.onodes + n0] -= (double)L(GS, b, NP);
  T phi[NP];  // dS/df
  tprod_grouped<D, M, true, S>(kp, n0, lam, phi);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T w = va.w0 * va.ih[i];
    const int st = i == 0 ? 1 : i == 1 ? N2 : N2 * N2;
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int bi = digit(b, N2, i);
      const T v = bi >= 1 ? T(bi) * w * phi[b - st] : T(0);
      S::store(rho, i * NP + b, n0, v);
    }
  }
}

// Velocity side at dual node q: with Ub the adjoint velocity and P' the
// pressure after the step's pressure half-step, gk -= dS/dkappa and
// z = dS/dc (NP planes of scratch).  64 work-items per workgroup.
template <int D, int M, class S>
__global__ void __launch_bounds__(64) grad_u_var(typename S::View ub, typename S::View p, typename S::View ku,
                                                 double* __restrict__ gk, typename S::View z, Grid g,
                                                 VarArgs<typename S::C> va) {
  static_assert(D <= 2 || M <= 1, "the adjoint of the variable-kappa half-steps: d <= 2, or d = 3 with m <= 1");
  using T = typename S::C;
  using Y = YSupport<D, M, false>;
  constexpr int N2 = 2 * M + 2, MP = M + 1, NP = VK<D, M>::NP, NC = Dims<D, M>::NC;
  constexpr bool STAGE = kGradStage<D, M, T>;
  constexpr int T0S = 0, GS = STAGE ? 1 : 0;  // LDS slots
  __shared__ T lds[(STAGE ? 2 : 1) * NP * 64];
  const LaneLds<T> L{lds, (int)threadIdx.x};
  int32_t j[3];
  if (!node_of_block<D>(g, blockIdx.x, j)) return;
  uint32_t cn[1 << D];
  corner_nodes<D>(g, j, cn);  // primal j = q + e
  const uint32_t n0 = out_index<D>(g, j);
  T t0[NP];
  interp_full<D, M, S>(p, 0, cn, t0);
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    t0[b] *= va.w0;
    if (STAGE) L(T0S, b, NP) = t0[b];
    L(GS, b, NP) = T(0);
  }
  // S = sum_i sum_s Ub_i[s] (s_i + 1) / h_i Q[s + e_i]
  T yc[Y::NY];
#pragma unroll
  for (int a = 0; a < Y::NY; ++a) yc[a] = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      const int si = digit(s, MP, i);
      yc[Y::idx(poly_index<D, M>(s, i == 0, i == 1, i == 2))] += T(si + 1) * va.ih[i] * S::load(ub, i * NC + s, n0);
    }
  T lam[NP];
  adjoint_series<D, M, false, S>(ku, n0, L, t0, T0S, GS, yc, va, lam);
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    gk[(size_t)b * g.onodes + n0] -= (double)L(GS, b, NP);
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
  } else if constexpr (D == 3) {
    T zz[N2][N2][MP];  // [b_x][b_y][a_z]
#pragma unroll
    for (int bx = 0; bx < N2; ++bx)
#pragma unroll
      for (int by = 0; by < N2; ++by)
#pragma unroll
        for (int az = 0; az < MP; ++az) {
          T v = T(0);
#pragma unroll
          for (int bz = 0; bz < N2; ++bz) {
            const double h = hcol<M, (E >> 2) & 1>(bz, az);
            if (h != 0.0) v = fma(T(h), z[bx + N2 * (by + N2 * bz)], v);
          }
          zz[bx][by][az] = v;
        }
    T zy[N2][MP][MP];  // [b_x][a_y][a_z]
#pragma unroll
    for (int bx = 0; bx < N2; ++bx)
#pragma unroll
      for (int ay = 0; ay < MP; ++ay)
#pragma unroll
        for (int az = 0; az < MP; ++az) {
          T v = T(0);
#pragma unroll
          for (int by = 0; by < N2; ++by) {
            const double h = hcol<M, (E >> 1) & 1>(by, ay);
            if (h != 0.0) v = fma(T(h), zz[bx][by][az], v);
          }
          zy[bx][ay][az] = v;
        }
#pragma unroll
    for (int az = 0; az < MP; ++az)
#pragma unroll
      for (int ay = 0; ay < MP; ++ay)
#pragma unroll
        for (int ax = 0; ax < MP; ++ax)
#pragma unroll
          for (int bx = 0; bx < N2; ++bx) {
            const double h = hcol<M, E & 1>(bx, ax);
            if (h != 0.0) acc[ax + MP * (ay + MP * az)] = fma(T(h), zy[bx][ay][az], acc[ax + MP * (ay + MP * az)]);
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

// In 3D a scheduling barrier after each corner keeps the compiler from
// issuing all 8 corners' (2m+2)^3 loads up front (2 KB of scratch per lane at
// m = 1 in FP64).
template <int D, int M, class S, int EP>
__device__ __forceinline__ void gather_corner_fenced(const typename S::View& scr, int comp, uint32_t node,
                                                     typename S::C* acc) {
  gather_corner<D, M, S, EP>(scr, comp, node, acc);
  if constexpr (D == 3) __builtin_amdgcn_sched_barrier(0);
}

template <int D, int M, class S, int... EP>
__device__ __forceinline__ void gather_corners(const typename S::View& scr, int comp, const uint32_t* cn,
                                               typename S::C* acc, std::integer_sequence<int, EP...>) {
  (gather_corner_fenced<D, M, S, EP>(scr, comp, cn[EP], acc), ...);
}

template <int D, int M, class S, int... EP>
__device__ __forceinline__ void gather_corners_masked(const typename S::View& scr, int comp, const uint32_t* cn,
                                                      const bool* valid, typename S::C* acc,
                                                      std::integer_sequence<int, EP...>) {
  ((valid[EP] ? gather_corner<D, M, S, EP>(scr, comp, cn[EP], acc) : void()), ...);
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
  // The output loop stays a loop even for one output (an opaque bound): in 3D,
  // straight-line code let the compiler issue every corner's loads at once.
  int zero = 0;
  if constexpr (D == 3) asm volatile("s_mov_b32 %0, 0" : "=s"(zero));
#pragma unroll 1
  for (int io = 0; io < NO + zero; ++io) {
    T acc[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) acc[a] = T(0);
    gather_corners<D, M, S>(scr, io, cn, acc, std::make_integer_sequence<int, (1 << D)>{});
#pragma unroll
    for (int a = 0; a < NC; ++a) S::update(out, io * NC + a, n0, [&](T x) { return x - acc[a]; });
  }
}

// Walls, velocity side: scr[s] -= the transposed interpolation of rho over the
// primal corners of padded dual slot s (0..K+1 per dimension, dual node
// q = s - 1) that lie inside [0, K] (corners past a wall are not nodes of the
// walled step and contribute nothing).  The fold G^T (ghost_fold) then adds
// each ghost slot, with its mirror sign, into the node it mirrors.  The grid's
// K are the padded extents, sext the primal extents.
template <int D, int M, class S>
__global__ void __launch_bounds__(256) var_adjoint_gather_walls(typename S::View scr, typename S::View rho, Grid g) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC;
  int32_t j[3];
  if (!node_of_block<D>(g, blockIdx.x, j)) return;
  uint32_t cn[1 << D];
  bool valid[1 << D];
#pragma unroll
  for (int e = 0; e < (1 << D); ++e) {
    int32_t c3[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      c3[k] = j[k] - 1 + ((e >> k) & 1);
      ok = ok && c3[k] >= 0 && c3[k] < g.sext[k];
    }
    valid[e] = ok;
    cn[e] = ok ? node_index<D>(c3[0], c3[1], c3[2], g.sext) : 0u;
  }
  const uint32_t n0 = node_index<D>(j[0], j[1], j[2], g.oext);
#pragma unroll 1
  for (int io = 0; io < D; ++io) {
    T acc[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) acc[a] = T(0);
    gather_corners_masked<D, M, S>(rho, io, cn, valid, acc, std::make_integer_sequence<int, (1 << D)>{});
#pragma unroll
    for (int a = 0; a < NC; ++a) S::update(scr, io * NC + a, n0, [&](T x) { return x - acc[a]; });
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
  int32_t first_block;
  int32_t wave_per_xcd;            // variable kappa, 3D m >= 2: nodes per XCD run (one workgroup per node)
};

// A table pointer read from memory, recast to the constant address space so
// that uniform table reads become scalar loads (a pointer loaded from memory
// is generic, and generic loads are per-lane flat loads).

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

// Variable kappa, 3D m >= 2, batched: one 64-wide workgroup per node of each
// shot, as in the single-shot launch.
template <int M, class S>
__global__ void __launch_bounds__(64) p_half_batch_wave(const ShotHalf<S>* __restrict__ shots, int n) {
  const ShotHalf<S> sh = shot_desc(shots, shot_of(shots, n, blockIdx.x));
  using G = typename S::Global;
  p_half_var_wave_body<M, G>(S::global(sh.out), S::global(sh.in), S::global(sh.kap), sh.g, sh.va, sh.wave_per_xcd,
                             (int)blockIdx.x - sh.first_block);
}

template <int M, class S>
__global__ void __launch_bounds__(64) u_half_batch_wave(const ShotHalf<S>* __restrict__ shots, int n) {
  const ShotHalf<S> sh = shot_desc(shots, shot_of(shots, n, blockIdx.x));
  using G = typename S::Global;
  u_half_var_wave_body<M, G>(S::global(sh.out), S::global(sh.in), S::global(sh.kap), sh.g, sh.va, sh.wscale,
                             sh.wave_per_xcd, (int)blockIdx.x - sh.first_block);
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

// The same in FP32_COMP storage: pbase holds each shot's hi base and lo base
// (entries 2s and 2s + 1); values and amplitudes are FP64 (the values as the
// split storage holds them), and the update rounds to hi + lo as every write
// of that storage does.
template <class S>
__global__ void __launch_bounds__(256) batch_source_add_split(void* const* __restrict__ pbase,
                                                              const BatchSource* __restrict__ ent,
                                                              const double* __restrict__ val,
                                                              const double* __restrict__ amps, int64_t namps,
                                                              const int64_t* __restrict__ counter, int64_t nent) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nent) return;
  const int64_t n = counter[0];
  if (n < 0 || n >= namps) return;
  const BatchSource e = ent[i];
  const typename S::View v{static_cast<float*>(pbase[2 * e.shot]), static_cast<uint16_t*>(pbase[2 * e.shot + 1]), 0};
  const double a = amps[(int64_t)e.shot * namps + n], g = val[i];
  S::update(v, 0, e.word, [&](double x) { return fma(a, g, x); });
}

}  // namespace hl
