// hl_kernels_d2_comp.hip - 2-dimensional half-step kernels, FP32 + BF16 split words, FP64 arithmetic.
#include "hl_internal.hpp"

namespace hl {

bool kernels_d2_comp(int m, KernelSet* out) { return make_set_for<2, SplitStore, 0, 1, 2, 3, 4, 5>(m, out); }

}  // namespace hl
