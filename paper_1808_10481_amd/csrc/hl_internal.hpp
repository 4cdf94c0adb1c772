// hl_internal.hpp - plan object and kernel registry shared by the C ABI
// (hl_api.hip) and the per-dimension kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <vector>

#include "hl.h"
#include "hl_kernels_ext.hpp"

namespace hl {

// What a launcher needs from a plan.
struct PlanView {
  Grid gp, gu;          // pressure / velocity half-step grids
  const void* adj_tab;  // transposed half-step blocks (periodic plans with an adjoint), or NULL
  const void* kap_p;    // variable kappa: Taylor data on the primal / dual nodes, or NULL
  const void* kap_u;
  double dt;            // time step (variable-kappa kernels)
  int32_t uext[3];      // velocity array extents (ghost fill, walls only)
  const void* tab;      // packed operator tables in the plan's arithmetic type
  int d, m, precision;
  double ih[3];         // 1 / h_k (velocity half-step)
};

typedef hipError_t (*PHalfFn)(const PlanView&, void* p, const void* u, hipStream_t);
typedef hipError_t (*UHalfFn)(const PlanView&, void* u, const void* p, double wscale, hipStream_t);
typedef hipError_t (*GhostFn)(const PlanView&, void* u, hipStream_t);
// Transposed half-steps: pb -= B^T ub (AdjFn p), ub -= A^T pb (AdjFn u).
typedef hipError_t (*AdjFn)(const PlanView&, void* out, const void* in, hipStream_t);
// Walls: ub -= G^T A^T pb through a zeroed scratch array shaped like u (left
// zeroed), and the ghost-shell clear of an adjoint velocity.
typedef hipError_t (*AdjWallFn)(const PlanView&, const Grid& gfull, void* ub, const void* pb, void* scr,
                                hipStream_t);
typedef hipError_t (*GhostZeroFn)(const PlanView&, void* u, hipStream_t);
// Batched shots: descriptor images of the p and u half-steps of every shot
// (built where the storage type is known) and the two batched launches.
struct BatchShot {
  const PlanView* v;
  void* p;
  void* u;
};
typedef void (*BatchDescFn)(const BatchShot* shots, int n, bool var, std::vector<unsigned char>* pdesc,
                            std::vector<unsigned char>* udesc, int* pblocks, int* ublocks);
typedef hipError_t (*BatchHalfFn)(const void* desc, int n, int blocks, bool var, dim3 block, hipStream_t);
// Variable-kappa adjoint: the per-node gradient kernels (bar: adjoint field of
// the half-step's output, fwd: the forward field it reads, gk: FP64 kappa
// gradient accumulators, scr: scratch of d (2m+2)^d planes) and the gathers
// that finish the transposed half-steps from that scratch.
typedef hipError_t (*VarGradFn)(const PlanView&, const void* bar, const void* fwd, double* gk, void* scr,
                                hipStream_t);
typedef hipError_t (*VarGatherFn)(const PlanView&, void* bar, const void* scr, hipStream_t);
// Batched sources: pbase (device array of the shots' pressure buffers), the
// entries, their values and the amplitude table in the storage word type.
typedef hipError_t (*BatchSrcFn)(const void* pbase, const void* ent, const void* val, const void* amps,
                                 int64_t namps, const int64_t* counter, int64_t nent, hipStream_t);

struct KernelSet {
  PHalfFn p_half;
  UHalfFn u_half;
  GhostFn ghost;         // ghost-shell refresh of a wall-bounded velocity array
  AdjFn adj_p, adj_u;    // transposed half-steps, NULL where not built
  AdjWallFn adj_u_walls; // walls: ub -= G^T A^T pb, NULL where not built
  AdjWallFn gather_u_var_walls;  // walls, variable kappa: ub -= G^T (A^T pb from rho), NULL where not built
  GhostZeroFn ghost_zero;
  PHalfFn p_half_var;    // variable-kappa half-steps, NULL where not built
  UHalfFn u_half_var;
  bool batch_var;        // variable kappa in batched steps
  VarGradFn grad_p_var, grad_u_var;      // variable-kappa adjoint, NULL where not built
  VarGatherFn gather_p_var, gather_u_var;
  BatchDescFn batch_desc;
  BatchHalfFn p_batch, u_batch;
  BatchSrcFn batch_src;
  int table_words;       // TableLayout<D, M>::TOTAL
  int p_off[3];          // offsets of the pressure merged tables, per component
  int u_off;             // offset of the velocity (Q) merged table
  int f_off;             // offset of the fully merged 3D pressure table, or -1
  int fu_off;            // offset of the fully merged 3D velocity table, or -1
  int ng;                // size of the velocity output set G
  int tile[3];           // tile extent in x, y and z
};

// Registries, one translation unit per (dimension, storage) so the build
// compiles them in parallel (hl_kernels_d<d>_<storage>.hip); each returns false
// when m is not built for that dimension.
bool kernels_d1_fp64(int m, KernelSet* out);
bool kernels_d1_fp32(int m, KernelSet* out);
bool kernels_d1_comp(int m, KernelSet* out);
bool kernels_d2_fp64(int m, KernelSet* out);
bool kernels_d2_fp32(int m, KernelSet* out);
bool kernels_d2_comp(int m, KernelSet* out);
bool kernels_d3_fp64(int m, KernelSet* out);
bool kernels_d3_fp32(int m, KernelSet* out);
bool kernels_d3_comp(int m, KernelSet* out);

inline bool kernels_for(int d, int m, int precision, KernelSet* out) {
  typedef bool (*Reg)(int, KernelSet*);
  static const Reg reg[3][3] = {{kernels_d1_fp64, kernels_d1_fp32, kernels_d1_comp},
                                {kernels_d2_fp64, kernels_d2_fp32, kernels_d2_comp},
                                {kernels_d3_fp64, kernels_d3_fp32, kernels_d3_comp}};
  if (d < 1 || d > 3 || precision < HL_FP64 || precision > HL_FP32_COMP) return false;
  return reg[d - 1][precision](m, out);
}

// Table layout queries for a (d, m) the registry supports.
template <int D, int M>
inline void fill_layout(KernelSet* ks) {
  using TL = TableLayout<D, M>;
  ks->table_words = TL::TOTAL;
  for (int i = 0; i < 3; ++i) ks->p_off[i] = i < D ? TL::p_off(i) : -1;
  ks->u_off = TL::U_OFF;
  if constexpr (D == 3) {
    ks->f_off = TL::FULL_P ? TL::F_OFF : -1;
    ks->fu_off = TL::FULL_U ? TL::FU_OFF : -1;
  } else {
    ks->f_off = -1;
    ks->fu_off = -1;
  }
  ks->ng = GSet<D, M>::NG;
  ks->tile[0] = TileShape<D>::X;
  ks->tile[1] = TileShape<D>::Y;
  ks->tile[2] = TileShape<D>::Z;
}

template <int D>
inline dim3 block_shape() {
  return dim3(TileShape<D>::X, TileShape<D>::Y, 1);
}

// Workgroup shape of a grid (its tile).
inline dim3 block_shape(const Grid& g) { return dim3((unsigned)g.tx, (unsigned)g.ty, 1); }

inline dim3 grid_shape(const Grid& g) { return dim3((unsigned)(g.per_xcd * kXcds), 1, 1); }

template <int D, int M, class S>
hipError_t launch_p(const PlanView& pv, void* p, const void* u, hipStream_t s) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC;
  const Grid& g = pv.gp;
  const typename S::View vp = S::make(p, 1, NC, g.onodes);
  const typename S::View vu = S::make(u, D, NC, g.snodes);
  if constexpr (D == 3)
    hipLaunchKernelGGL((p_half_3d<M, S>), grid_shape(g), block_shape(g), 0, s, vp, vu, (const T*)pv.tab, g);
  else
    hipLaunchKernelGGL((p_half_kernel<D, M, S>), grid_shape(g), block_shape(g), 0, s, vp, vu, (const T*)pv.tab,
                       g);
  return hipGetLastError();
}

template <int D, int M, class S>
hipError_t launch_u(const PlanView& pv, void* u, const void* p, double wscale, hipStream_t s) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC;
  const Grid& g = pv.gu;
  const typename S::View vu = S::make(u, D, NC, g.onodes);
  const typename S::View vp = S::make(p, 1, NC, g.snodes);
  if constexpr (D == 3)
    hipLaunchKernelGGL((u_half_3d<M, S>), grid_shape(g), block_shape(g), 0, s, vu, vp, (const T*)pv.tab, g,
                       (T)wscale, (T)pv.ih[0], (T)pv.ih[1], (T)pv.ih[2]);
  else
    hipLaunchKernelGGL((u_half_kernel<D, M, S>), grid_shape(g), block_shape(g), 0, s, vu, vp, (const T*)pv.tab,
                       g, (T)wscale, (T)pv.ih[0], (T)pv.ih[1], (T)pv.ih[2]);
  return hipGetLastError();
}

template <int D, int M, class S>
hipError_t launch_ghost(const PlanView& pv, void* u, hipStream_t s) {
  constexpr int NC = Dims<D, M>::NC;
  int64_t nodes = 1, face = 0;
  for (int k = 0; k < D; ++k) nodes *= pv.uext[k];
  for (int k = 0; k < D; ++k) {
    int64_t f = 2;
    for (int j = 0; j < D; ++j)
      if (j != k) f *= (j < k) ? (pv.uext[j] - 2) : pv.uext[j];
    face = f > face ? f : face;
  }
  const typename S::View vu = S::make(u, D, NC, nodes);
  hipLaunchKernelGGL((ghost_fill<D, M, S>), dim3((unsigned)((face + 255) / 256), D, 1), dim3(256, 1, 1), 0, s, vu,
                     pv.uext[0], pv.uext[1], pv.uext[2]);
  return hipGetLastError();
}

template <int D, int M, class S, bool PTYPE>
hipError_t launch_adjoint(const PlanView& pv, void* out, const void* in, hipStream_t s) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC;
  const Grid& g = PTYPE ? pv.gp : pv.gu;
  const typename S::View vo = S::make(out, PTYPE ? 1 : D, NC, g.onodes);
  const typename S::View vi = S::make(in, PTYPE ? D : 1, NC, g.snodes);
  hipLaunchKernelGGL((adjoint_half<D, M, S, PTYPE>), grid_shape(g), block_shape(g), 0, s, vo, vi,
                     (const T*)pv.adj_tab, g);
  return hipGetLastError();
}

template <int D, int M, class S>
hipError_t launch_adj_u_walls(const PlanView& pv, const Grid& gf, void* ub, const void* pb, void* scr,
                              hipStream_t s) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC;
  const typename S::View vs = S::make(scr, D, NC, gf.onodes);
  hipLaunchKernelGGL((adjoint_walls_at<D, M, S>), grid_shape(gf), block_shape(gf), 0, s, vs,
                     S::make(pb, 1, NC, gf.snodes), (const T*)pv.adj_tab, gf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t interior = 1;
  for (int k = 0; k < D; ++k) interior *= pv.uext[k] - 2;
  hipLaunchKernelGGL((ghost_fold<D, M, S>), dim3((unsigned)((interior + 255) / 256)), dim3(256), 0, s,
                     S::make(ub, D, NC, gf.onodes), vs, pv.uext[0], pv.uext[1], pv.uext[2]);
  return hipGetLastError();
}

template <int D, int M, class S>
hipError_t launch_ghost_zero(const PlanView& pv, void* u, hipStream_t s) {
  constexpr int NC = Dims<D, M>::NC;
  int64_t nodes = 1;
  for (int k = 0; k < D; ++k) nodes *= pv.uext[k];
  hipLaunchKernelGGL((ghost_zero<D, M, S>), dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, s,
                     S::make(u, D, NC, nodes), pv.uext[0], pv.uext[1], pv.uext[2]);
  return hipGetLastError();
}

template <class S>
VarArgs<typename S::C> var_args(const PlanView& pv) {
  VarArgs<typename S::C> va;
  va.w0 = (typename S::C)pv.dt;
  va.ratio[0] = 0;
  for (int k = 1; k <= kVarMaxK; ++k)
    va.ratio[k] = (typename S::C)(0.25 * pv.dt * pv.dt / ((2.0 * k) * (2.0 * k + 1.0)));
  for (int k = 0; k < 3; ++k) va.ih[k] = (typename S::C)pv.ih[k];
  return va;
}

template <int D, int M, class S>
hipError_t launch_p_var(const PlanView& pv, void* p, const void* u, hipStream_t s) {
  constexpr int NC = Dims<D, M>::NC, NP = VK<D, M>::NP;
  const Grid& g = pv.gp;
  hipLaunchKernelGGL((p_half_var<D, M, S>), grid_shape(g), block_shape(g), 0, s, S::make(p, 1, NC, g.onodes),
                     S::make(u, D, NC, g.snodes), S::make(pv.kap_p, 1, NP, g.onodes), g, var_args<S>(pv));
  return hipGetLastError();
}

template <int D, int M, class S>
hipError_t launch_u_var(const PlanView& pv, void* u, const void* p, double wscale, hipStream_t s) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC, NP = VK<D, M>::NP;
  const Grid& g = pv.gu;
  hipLaunchKernelGGL((u_half_var<D, M, S>), grid_shape(g), block_shape(g), 0, s, S::make(u, D, NC, g.onodes),
                     S::make(p, 1, NC, g.snodes), S::make(pv.kap_u, 1, NP, g.onodes), g, var_args<S>(pv),
                     (T)wscale);
  return hipGetLastError();
}

// 3D m >= 2: one workgroup (one wavefront) per node, nodes in XCD-contiguous runs.
template <int M, class S>
hipError_t launch_p_var_wave(const PlanView& pv, void* p, const void* u, hipStream_t s) {
  constexpr int NC = Dims<3, M>::NC, NP = VK<3, M>::NP;
  const Grid& g = pv.gp;
  const int64_t per = ((int64_t)g.K[0] * g.K[1] * g.K[2] + kXcds - 1) / kXcds;
  if (per * kXcds > INT32_MAX) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((p_half_var_wave<M, S>), dim3((unsigned)(per * kXcds)), dim3(64), 0, s,
                     S::make(p, 1, NC, g.onodes), S::make(u, 3, NC, g.snodes), S::make(pv.kap_p, 1, NP, g.onodes), g,
                     var_args<S>(pv), (int32_t)per);
  return hipGetLastError();
}

template <int M, class S>
hipError_t launch_u_var_wave(const PlanView& pv, void* u, const void* p, double wscale, hipStream_t s) {
  using T = typename S::C;
  constexpr int NC = Dims<3, M>::NC, NP = VK<3, M>::NP;
  const Grid& g = pv.gu;
  const int64_t per = ((int64_t)g.K[0] * g.K[1] * g.K[2] + kXcds - 1) / kXcds;
  if (per * kXcds > INT32_MAX) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((u_half_var_wave<M, S>), dim3((unsigned)(per * kXcds)), dim3(64), 0, s,
                     S::make(u, 3, NC, g.onodes), S::make(p, 1, NC, g.snodes), S::make(pv.kap_u, 1, NP, g.onodes), g,
                     var_args<S>(pv), (T)wscale, (int32_t)per);
  return hipGetLastError();
}

template <int D, int M, class S>
hipError_t launch_grad_p_var(const PlanView& pv, const void* pb, const void* u, double* gk, void* scr,
                             hipStream_t s) {
  constexpr int NC = Dims<D, M>::NC, NP = VK<D, M>::NP;
  const Grid& g = pv.gp;
  if (g.tx != 64 || g.ty != 1) return hipErrorInvalidConfiguration;  // per-lane LDS arrays of 64 lanes
  hipLaunchKernelGGL((grad_p_var<D, M, S>), grid_shape(g), block_shape(g), 0, s, S::make(pb, 1, NC, g.onodes),
                     S::make(u, D, NC, g.snodes), S::make(pv.kap_p, 1, NP, g.onodes), gk,
                     S::make(scr, D, NP, g.onodes), g, var_args<S>(pv));
  return hipGetLastError();
}

template <int D, int M, class S>
hipError_t launch_grad_u_var(const PlanView& pv, const void* ub, const void* p, double* gk, void* scr,
                             hipStream_t s) {
  constexpr int NC = Dims<D, M>::NC, NP = VK<D, M>::NP;
  const Grid& g = pv.gu;
  if (g.tx != 64 || g.ty != 1) return hipErrorInvalidConfiguration;  // per-lane LDS arrays of 64 lanes
  hipLaunchKernelGGL((grad_u_var<D, M, S>), grid_shape(g), block_shape(g), 0, s, S::make(ub, D, NC, g.onodes),
                     S::make(p, 1, NC, g.snodes), S::make(pv.kap_u, 1, NP, g.onodes), gk,
                     S::make(scr, 1, NP, g.onodes), g, var_args<S>(pv));
  return hipGetLastError();
}

// Pb -= sum over the dual nodes q = j - e of the transposed interpolation of z[q]
template <int D, int M, class S>
hipError_t launch_gather_p_var(const PlanView& pv, void* pb, const void* scr, hipStream_t s) {
  constexpr int NC = Dims<D, M>::NC, NP = VK<D, M>::NP;
  const Grid& g = pv.gp;
  hipLaunchKernelGGL((var_adjoint_gather<D, M, S, true>), grid_shape(g), block_shape(g), 0, s,
                     S::make(pb, 1, NC, g.onodes), S::make(scr, 1, NP, g.snodes), g);
  return hipGetLastError();
}

// Ub -= sum over the primal nodes j = q + 1 - e of the transposed interpolation of rho[j]
template <int D, int M, class S>
hipError_t launch_gather_u_var(const PlanView& pv, void* ub, const void* scr, hipStream_t s) {
  constexpr int NC = Dims<D, M>::NC, NP = VK<D, M>::NP;
  const Grid& g = pv.gu;
  hipLaunchKernelGGL((var_adjoint_gather<D, M, S, false>), grid_shape(g), block_shape(g), 0, s,
                     S::make(ub, D, NC, g.onodes), S::make(scr, D, NP, g.snodes), g);
  return hipGetLastError();
}

// Walls, variable kappa: scr -= the transposed interpolation of rho on every
// slot of the padded velocity array (gf: the padded extents, primal corners
// inside [0, K]), then ub += G^T scr (scratch left zeroed).
template <int D, int M, class S>
hipError_t launch_gather_u_var_walls(const PlanView& pv, const Grid& gf, void* ub, const void* rho, void* scr,
                                     hipStream_t s) {
  constexpr int NC = Dims<D, M>::NC, NP = VK<D, M>::NP;
  const typename S::View vs = S::make(scr, D, NC, gf.onodes);
  hipLaunchKernelGGL((var_adjoint_gather_walls<D, M, S>), grid_shape(gf), block_shape(gf), 0, s, vs,
                     S::make(rho, D, NP, gf.snodes), gf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t interior = 1;
  for (int k = 0; k < D; ++k) interior *= pv.uext[k] - 2;
  hipLaunchKernelGGL((ghost_fold<D, M, S>), dim3((unsigned)((interior + 255) / 256)), dim3(256), 0, s,
                     S::make(ub, D, NC, gf.onodes), vs, pv.uext[0], pv.uext[1], pv.uext[2]);
  return hipGetLastError();
}

template <class S>
constexpr bool kPlain = false;
template <typename W>
constexpr bool kPlain<PlainStore<W>> = true;

template <int D, int M, class S>
constexpr bool kVarBuilt = D <= 2 || (D == 3 && M <= 1);
template <int D, int M, class S>
constexpr bool kVarWaveBuilt = D == 3 && M >= 2 && M <= 3;
template <int D, int M, class S>
constexpr bool kVarGradBuilt = D == 1 || (D == 2 && M <= 3) || (D == 3 && M <= 1);

template <int D, int M, class S>
void batch_desc(const BatchShot* shots, int n, bool var, std::vector<unsigned char>* pdesc,
                std::vector<unsigned char>* udesc, int* pblocks, int* ublocks) {
  using T = typename S::C;
  constexpr int NC = Dims<D, M>::NC, NP = VK<D, M>::NP;
  std::vector<ShotHalf<S>> P((size_t)n), U((size_t)n);
  int fp = 0, fu = 0;
  for (int i = 0; i < n; ++i) {
    const PlanView& v = *shots[i].v;
    ShotHalf<S>& a = P[i];
    a = ShotHalf<S>{};
    a.out = S::make(shots[i].p, 1, NC, v.gp.onodes);
    a.in = S::make(shots[i].u, D, NC, v.gp.snodes);
    a.kap = var ? S::make(v.kap_p, 1, NP, v.gp.onodes) : a.out;
    a.tab = (const T*)v.tab;
    a.g = v.gp;
    a.va = var_args<S>(v);
    a.wscale = T(1);
    for (int k = 0; k < 3; ++k) a.ih[k] = (T)v.ih[k];
    a.first_block = fp;
    if (var && kVarWaveBuilt<D, M, S>) {  // one workgroup per node
      a.wave_per_xcd = (int32_t)(((int64_t)v.gp.K[0] * v.gp.K[1] * v.gp.K[2] + kXcds - 1) / kXcds);
      fp += a.wave_per_xcd * kXcds;
    } else {
      fp += v.gp.per_xcd * kXcds;
    }
    ShotHalf<S>& b = U[i];
    b = ShotHalf<S>{};
    b.out = S::make(shots[i].u, D, NC, v.gu.onodes);
    b.in = S::make(shots[i].p, 1, NC, v.gu.snodes);
    b.kap = var ? S::make(v.kap_u, 1, NP, v.gu.onodes) : b.out;
    b.tab = (const T*)v.tab;
    b.g = v.gu;
    b.va = a.va;
    b.wscale = T(1);
    for (int k = 0; k < 3; ++k) b.ih[k] = (T)v.ih[k];
    b.first_block = fu;
    if (var && kVarWaveBuilt<D, M, S>) {
      b.wave_per_xcd = (int32_t)(((int64_t)v.gu.K[0] * v.gu.K[1] * v.gu.K[2] + kXcds - 1) / kXcds);
      fu += b.wave_per_xcd * kXcds;
    } else {
      fu += v.gu.per_xcd * kXcds;
    }
  }
  const size_t bytes = (size_t)n * sizeof(ShotHalf<S>);
  pdesc->resize(bytes);
  udesc->resize(bytes);
  std::memcpy(pdesc->data(), P.data(), bytes);
  std::memcpy(udesc->data(), U.data(), bytes);
  *pblocks = fp;
  *ublocks = fu;
}

template <int D, int M, class S, bool P>
hipError_t launch_batch(const void* desc, int n, int blocks, bool var, dim3 block, hipStream_t s) {
  const ShotHalf<S>* d = static_cast<const ShotHalf<S>*>(desc);
  if (var) {
    if constexpr (kVarBuilt<D, M, S>) {
      if (P)
        hipLaunchKernelGGL((p_half_batch<D, M, S, true>), dim3((unsigned)blocks), block, 0, s, d, n);
      else
        hipLaunchKernelGGL((u_half_batch<D, M, S, true>), dim3((unsigned)blocks), block, 0, s, d, n);
    } else if constexpr (kVarWaveBuilt<D, M, S>) {
      if (P)
        hipLaunchKernelGGL((p_half_batch_wave<M, S>), dim3((unsigned)blocks), dim3(64), 0, s, d, n);
      else
        hipLaunchKernelGGL((u_half_batch_wave<M, S>), dim3((unsigned)blocks), dim3(64), 0, s, d, n);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    if (P)
      hipLaunchKernelGGL((p_half_batch<D, M, S, false>), dim3((unsigned)blocks), block, 0, s, d, n);
    else
      hipLaunchKernelGGL((u_half_batch<D, M, S, false>), dim3((unsigned)blocks), block, 0, s, d, n);
  }
  return hipGetLastError();
}
template <typename W>
hipError_t launch_batch_src(const void* pbase, const void* ent, const void* val, const void* amps, int64_t namps,
                            const int64_t* counter, int64_t nent, hipStream_t s) {
  if (nent <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_source_add<W>, dim3((unsigned)((nent + 255) / 256)), dim3(256), 0, s,
                     static_cast<W* const*>(pbase), static_cast<const BatchSource*>(ent),
                     static_cast<const W*>(val), static_cast<const W*>(amps), namps, counter, nent);
  return hipGetLastError();
}

inline hipError_t launch_batch_src_split(const void* pbase, const void* ent, const void* val, const void* amps,
                                         int64_t namps, const int64_t* counter, int64_t nent, hipStream_t s) {
  if (nent <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_source_add_split<SplitStore>, dim3((unsigned)((nent + 255) / 256)), dim3(256), 0, s,
                     static_cast<void* const*>(pbase), static_cast<const BatchSource*>(ent),
                     static_cast<const double*>(val), static_cast<const double*>(amps), namps, counter, nent);
  return hipGetLastError();
}

template <class S>
struct SrcLauncher {
  static constexpr BatchSrcFn fn = &launch_batch_src_split;  // FP32_COMP
};
template <typename W>
struct SrcLauncher<PlainStore<W>> {
  static constexpr BatchSrcFn fn = &launch_batch_src<W>;
};

template <int D, class S, int M>
inline bool make_set(KernelSet* out) {
  fill_layout<D, M>(out);
  out->p_half = &launch_p<D, M, S>;
  out->u_half = &launch_u<D, M, S>;
  out->ghost = &launch_ghost<D, M, S>;
  out->adj_p = nullptr;
  out->adj_u = nullptr;
  out->adj_u_walls = nullptr;
  out->ghost_zero = nullptr;
  // adjoint: every storage and (d, m)
  out->adj_p = &launch_adjoint<D, M, S, true>;
  out->adj_u = &launch_adjoint<D, M, S, false>;
  out->adj_u_walls = &launch_adj_u_walls<D, M, S>;
  out->ghost_zero = &launch_ghost_zero<D, M, S>;
  out->p_half_var = nullptr;
  out->u_half_var = nullptr;
  out->batch_desc = &batch_desc<D, M, S>;
  out->p_batch = &launch_batch<D, M, S, true>;
  out->u_batch = &launch_batch<D, M, S, false>;
  out->batch_src = SrcLauncher<S>::fn;
  // variable kappa: every storage and (d, m), batched too
  out->batch_var = false;
  if constexpr (kVarBuilt<D, M, S>) {
    out->p_half_var = &launch_p_var<D, M, S>;
    out->u_half_var = &launch_u_var<D, M, S>;
    out->batch_var = true;
  } else if constexpr (kVarWaveBuilt<D, M, S>) {
    out->p_half_var = &launch_p_var_wave<M, S>;
    out->u_half_var = &launch_u_var_wave<M, S>;
    out->batch_var = true;
  }
  // variable-kappa adjoint and kappa gradient: d = 1 (all m), d = 2 (m <= 3), d = 3 (m <= 1)
  out->grad_p_var = nullptr;
  out->grad_u_var = nullptr;
  out->gather_p_var = nullptr;
  out->gather_u_var = nullptr;
  out->gather_u_var_walls = nullptr;
  if constexpr (kVarGradBuilt<D, M, S>) {
    out->grad_p_var = &launch_grad_p_var<D, M, S>;
    out->grad_u_var = &launch_grad_u_var<D, M, S>;
    out->gather_p_var = &launch_gather_p_var<D, M, S>;
    out->gather_u_var_walls = &launch_gather_u_var_walls<D, M, S>;
    out->gather_u_var = &launch_gather_u_var<D, M, S>;
  }
  return true;
}

// Registry body: the kernel set for m, one of the compile-time orders Ms.
template <int D, class S, int... Ms>
inline bool make_set_for(int m, KernelSet* out) {
  return ((m == Ms && make_set<D, S, Ms>(out)) || ...);
}

}  // namespace hl
