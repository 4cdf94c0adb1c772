// hl_internal.hpp - plan object and kernel registry shared by the C ABI
// (hl_api.cpp) and the per-dimension kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hl.h"
#include "hl_kernels.hpp"

namespace hl {

// What a launcher needs from a plan.
struct PlanView {
  Grid grid;
  const void* tab;      // packed operator tables in the plan precision
  int d, m, precision;
  double ih[3];         // 1 / h_k (velocity half-step)
};

typedef hipError_t (*PHalfFn)(const PlanView&, void* p, const void* u, hipStream_t);
typedef hipError_t (*UHalfFn)(const PlanView&, void* u, const void* p, double wscale, hipStream_t);

struct KernelSet {
  PHalfFn p_half;
  UHalfFn u_half;
  int table_words;       // TableLayout<D, M>::TOTAL
  int p_off[3];          // offsets of the pressure merged tables, per component
  int u_off;             // offset of the velocity (Q) merged table
  int ng;                // size of the velocity output set G
  int tile[3];           // tile extent in x, y and z
};

// Registries implemented by hl_kernels_d{1,2,3}.hip; return false when
// (m, precision) is not built for that dimension.
bool kernels_d1(int m, int precision, KernelSet* out);
bool kernels_d2(int m, int precision, KernelSet* out);
bool kernels_d3(int m, int precision, KernelSet* out);

// Table layout queries for a (d, m) the registry supports.
template <int D, int M>
inline void fill_layout(KernelSet* ks) {
  using TL = TableLayout<D, M>;
  ks->table_words = TL::TOTAL;
  for (int i = 0; i < 3; ++i) ks->p_off[i] = i < D ? TL::p_off(i) : -1;
  ks->u_off = TL::U_OFF;
  ks->ng = GSet<D, M>::NG;
  ks->tile[0] = TileShape<D>::X;
  ks->tile[1] = TileShape<D>::Y;
  ks->tile[2] = TileShape<D>::Z;
}

template <int D>
inline dim3 block_shape() {
  return dim3(TileShape<D>::X, TileShape<D>::Y, 1);
}

inline dim3 grid_shape(const Grid& g) { return dim3((unsigned)(g.per_xcd * kXcds), 1, 1); }

template <int D, int M, typename T>
hipError_t launch_p_generic(const PlanView& pv, void* p, const void* u, hipStream_t s) {
  if constexpr (D == 3)
    hipLaunchKernelGGL((p_half_3d<M, T>), grid_shape(pv.grid), block_shape<D>(), 0, s, (T*)p, (const T*)u,
                       (const T*)pv.tab, pv.grid);
  else
    hipLaunchKernelGGL((p_half_kernel<D, M, T>), grid_shape(pv.grid), block_shape<D>(), 0, s, (T*)p,
                       (const T*)u, (const T*)pv.tab, pv.grid);
  return hipGetLastError();
}

template <int D, int M, typename T>
hipError_t launch_u_generic(const PlanView& pv, void* u, const void* p, double wscale, hipStream_t s) {
  if constexpr (D == 3)
    hipLaunchKernelGGL((u_half_3d<M, T>), grid_shape(pv.grid), block_shape<D>(), 0, s, (T*)u, (const T*)p,
                       (const T*)pv.tab, pv.grid, (T)wscale, (T)pv.ih[0], (T)pv.ih[1], (T)pv.ih[2]);
  else
    hipLaunchKernelGGL((u_half_kernel<D, M, T>), grid_shape(pv.grid), block_shape<D>(), 0, s, (T*)u,
                       (const T*)p, (const T*)pv.tab, pv.grid, (T)wscale, (T)pv.ih[0], (T)pv.ih[1],
                       (T)pv.ih[2]);
  return hipGetLastError();
}

template <int D, int M>
inline bool make_set(int precision, KernelSet* out) {
  fill_layout<D, M>(out);
  if (precision == HL_FP64) {
    out->p_half = &launch_p_generic<D, M, double>;
    out->u_half = &launch_u_generic<D, M, double>;
  } else {
    out->p_half = &launch_p_generic<D, M, float>;
    out->u_half = &launch_u_generic<D, M, float>;
  }
  return true;
}

}  // namespace hl
