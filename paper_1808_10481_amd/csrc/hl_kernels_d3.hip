// hl_kernels_d3.hip - instantiations of the 3-dimensional half-step kernels.
#include "hl_internal.hpp"

namespace hl {

bool kernels_d3(int m, int precision, KernelSet* out) {
  switch (m) {
    case 0: return make_set<3, 0>(precision, out);
    case 1: return make_set<3, 1>(precision, out);
    case 2: return make_set<3, 2>(precision, out);
    case 3: return make_set<3, 3>(precision, out);
    default: return false;
  }
}

}  // namespace hl
