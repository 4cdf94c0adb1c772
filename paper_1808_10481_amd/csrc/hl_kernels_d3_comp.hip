// hl_kernels_d3_comp.hip - 3-dimensional half-step kernels, FP32 + BF16 split words, FP64 arithmetic, m <= 2
// (m = 3, the slowest to compile, has a translation unit of its own).
#include "hl_internal.hpp"

namespace hl {

bool kernels_d3m3_comp(KernelSet* out);

bool kernels_d3_comp(int m, KernelSet* out) {
  return m == 3 ? kernels_d3m3_comp(out) : make_set_for<3, SplitStore, 0, 1, 2>(m, out);
}

}  // namespace hl
