// hl_kernels_d1_fp32.hip - 1-dimensional half-step kernels, FP32 words.
#include "hl_internal.hpp"

namespace hl {

bool kernels_d1_fp32(int m, KernelSet* out) { return make_set_for<1, PlainStore<float>, 0, 1, 2, 3, 4, 5, 6, 7>(m, out); }

}  // namespace hl
