// CPU check of the host <-> device layout conversion (hl_host_layout.hpp),
// built by tests/test_host_layout.py with AddressSanitizer and UBSan.
// For every (d, m, storage, boundary, field): the map visits every host entry
// once and every device node it targets once, inside the device image; ghost
// nodes stay untouched; a host -> device -> host round trip is exact in FP64,
// within 2^-24 relative in FP32 and 2^-33 in FP32_COMP.
#include <cmath>
#include <cstdio>
#include <vector>

#include "hl_host_layout.hpp"

int main() {
  int bad = 0;
  const int32_t Ks[3] = {7, 5, 3};
  for (int d = 1; d <= 3; ++d)
    for (int m = 0; m <= (d == 1 ? 7 : d == 2 ? 5 : 3); ++m)
      for (int prec = HL_FP64; prec <= HL_FP32_COMP; ++prec)
        for (int walls = 0; walls < 2; ++walls)
          for (int field = 0; field < 2; ++field) {
            const hl_host::LayoutMap L = hl_host::field_layout(d, m, Ks, walls, field);
            const int64_t host_n = (int64_t)L.nc * L.K[0] * L.K[1] * L.K[2];
            const int64_t dev_n = (int64_t)L.nc * L.nodes;
            std::vector<double> src(host_n), back(host_n, NAN);
            for (int64_t i = 0; i < host_n; ++i) src[i] = std::sin(1.0 + 0.37 * i) * (1 + i % 7);
            std::vector<int> hits_h(host_n, 0), hits_d(dev_n, 0);
            L.for_each([&](int64_t h, int64_t dv) {
              if (h < 0 || h >= host_n || dv < 0 || dv >= dev_n) {
                ++bad;
                return;
              }
              ++hits_h[h];
              ++hits_d[dv];
            });
            int64_t touched = 0;
            for (int64_t i = 0; i < host_n; ++i) bad += hits_h[i] != 1;
            for (int64_t i = 0; i < dev_n; ++i) {
              bad += hits_d[i] > 1;
              touched += hits_d[i];
            }
            bad += touched != host_n;
            hl_host::FieldImage im{prec, dev_n, {}, {}};
            if (!im.alloc()) return 2;
            std::fill(im.hi.begin(), im.hi.end(), (unsigned char)0);
            std::fill(im.lo.begin(), im.lo.end(), (unsigned char)0);
            L.for_each([&](int64_t h, int64_t dv) { im.put(dv, src[h]); });
            L.for_each([&](int64_t h, int64_t dv) { back[h] = im.get(dv); });
            for (int64_t i = 0; i < dev_n; ++i)
              if (!hits_d[i]) bad += im.get(i) != 0.0;  // ghosts / unused stay zero
            const double tol = prec == HL_FP64 ? 0.0 : (prec == HL_FP32 ? std::ldexp(1.0, -24) : std::ldexp(1.0, -33));
            for (int64_t i = 0; i < host_n; ++i)
              if (!(std::fabs(back[i] - src[i]) <= tol * std::fabs(src[i]))) ++bad;
            if (bad) {
              std::printf("FAIL d=%d m=%d prec=%d walls=%d field=%d\n", d, m, prec, walls, field);
              return 1;
            }
          }
  std::printf("ok\n");
  return 0;
}
