// hl_kernels_d3m3_comp.hip - 3-dimensional half-step kernels for m = 3, FP32 + BF16 split words, FP64 arithmetic.
#include "hl_internal.hpp"

namespace hl {

bool kernels_d3m3_comp(KernelSet* out) { return make_set<3, SplitStore, 3>(out); }

}  // namespace hl
