// hl_kernels_d1.hip - instantiations of the 1-dimensional half-step kernels.
#include "hl_internal.hpp"

namespace hl {

bool kernels_d1(int m, int precision, KernelSet* out) {
  switch (m) {
    case 0: return make_set<1, 0>(precision, out);
    case 1: return make_set<1, 1>(precision, out);
    case 2: return make_set<1, 2>(precision, out);
    case 3: return make_set<1, 3>(precision, out);
    case 4: return make_set<1, 4>(precision, out);
    case 5: return make_set<1, 5>(precision, out);
    case 6: return make_set<1, 6>(precision, out);
    case 7: return make_set<1, 7>(precision, out);
    default: return false;
  }
}

}  // namespace hl
