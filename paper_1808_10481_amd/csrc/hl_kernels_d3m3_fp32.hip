// hl_kernels_d3m3_fp32.hip - 3-dimensional half-step kernels for m = 3, FP32 words.
#include "hl_internal.hpp"

namespace hl {

bool kernels_d3m3_fp32(KernelSet* out) { return make_set<3, PlainStore<float>, 3>(out); }

}  // namespace hl
