// hl_kernels_d2.hip - instantiations of the 2-dimensional half-step kernels.
#include "hl_internal.hpp"

namespace hl {

bool kernels_d2(int m, int precision, KernelSet* out) {
  switch (m) {
    case 0: return make_set<2, 0>(precision, out);
    case 1: return make_set<2, 1>(precision, out);
    case 2: return make_set<2, 2>(precision, out);
    case 3: return make_set<2, 3>(precision, out);
    case 4: return make_set<2, 4>(precision, out);
    case 5: return make_set<2, 5>(precision, out);
    default: return false;
  }
}

}  // namespace hl
