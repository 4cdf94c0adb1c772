// hl_kernels_d3m3_fp64.hip - 3-dimensional half-step kernels for m = 3, FP64 words.
#include "hl_internal.hpp"

namespace hl {

bool kernels_d3m3_fp64(KernelSet* out) { return make_set<3, PlainStore<double>, 3>(out); }

}  // namespace hl
