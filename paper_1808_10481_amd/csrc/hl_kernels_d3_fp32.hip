// hl_kernels_d3_fp32.hip - 3-dimensional half-step kernels, FP32 words, m <= 2
// (m = 3, the slowest to compile, has a translation unit of its own).
#include "hl_internal.hpp"

namespace hl {

bool kernels_d3m3_fp32(KernelSet* out);

bool kernels_d3_fp32(int m, KernelSet* out) {
  return m == 3 ? kernels_d3m3_fp32(out) : make_set_for<3, PlainStore<float>, 0, 1, 2>(m, out);
}

}  // namespace hl
