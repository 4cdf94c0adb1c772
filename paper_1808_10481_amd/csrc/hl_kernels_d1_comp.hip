// hl_kernels_d1_comp.hip - 1-dimensional half-step kernels, FP32 + BF16 split words, FP64 arithmetic.
#include "hl_internal.hpp"

namespace hl {

bool kernels_d1_comp(int m, KernelSet* out) { return make_set_for<1, SplitStore, 0, 1, 2, 3, 4, 5, 6, 7>(m, out); }

}  // namespace hl
