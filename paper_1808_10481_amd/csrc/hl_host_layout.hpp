// hl_host_layout.hpp - host-side conversion between the host layout of the
// C ABI (FP64, C order, nodes then coefficients) and a device image of one
// field component (coefficient-major planes in the plan's storage format).
// Plain C++ (no HIP), so the CPU tests compile it under the sanitizers.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "hl.h"

namespace hl_host {

// host layout offset of (node j, coefficient a) -> device offset
struct LayoutMap {
  int d, MP, nc;
  int64_t K[3];      // host nodes per dimension
  int64_t E[3];      // device array extents
  int64_t off;       // device index of host node j is j + off per dimension
  int64_t nodes;     // device plane size
  template <typename F>
  void for_each(F&& f) const {
    // host: ((j1 K2 + j2) K3 + j3) * nc + ((a1 MP + a2) MP + a3)
    // device: c * nodes + n, n = i1 + E1 (i2 + E2 i3), i = j + off, c = a1 + MP (a2 + MP a3)
    const int64_t K1 = K[0], K2 = d > 1 ? K[1] : 1, K3 = d > 2 ? K[2] : 1;
    const int64_t o2 = d > 1 ? off : 0, o3 = d > 2 ? off : 0;
    const int nthreads = (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int w = 0; w < nthreads; ++w)
      th.emplace_back([&, w]() {
        for (int64_t j1 = w; j1 < K1; j1 += nthreads)
          for (int64_t j2 = 0; j2 < K2; ++j2)
            for (int64_t j3 = 0; j3 < K3; ++j3) {
              const int64_t hbase = ((j1 * K2 + j2) * K3 + j3) * nc;
              const int64_t n = (j1 + off) + E[0] * ((j2 + o2) + E[1] * (j3 + o3));
              for (int ha = 0; ha < nc; ++ha) {
                // host coefficient index ha = (a1 MP + a2) MP + a3 (a1 slowest)
                int a[3] = {0, 0, 0}, r = ha;
                for (int k = d - 1; k >= 0; --k) {
                  a[k] = r % MP;
                  r /= MP;
                }
                const int c = a[0] + MP * (a[1] + MP * a[2]);
                f(hbase + ha, (int64_t)c * nodes + n);
              }
            }
      });
    for (auto& t : th) t.join();
  }
};

// Layout of field 0 (p: K nodes per dimension, K+1 with walls, the end nodes
// on the walls) or field 1 (u: K dual nodes per dimension, stored inside an
// array padded by one ghost node per side with walls).  K[k] for k >= d is
// ignored.
inline LayoutMap field_layout(int d, int m, const int32_t* K, bool walls, int field) {
  LayoutMap L;
  L.d = d;
  L.MP = m + 1;
  L.nc = 1;
  for (int k = 0; k < d; ++k) L.nc *= m + 1;
  L.nodes = 1;
  for (int k = 0; k < 3; ++k) {
    const bool in = k < d;
    L.K[k] = in ? K[k] + (field == 0 && walls ? 1 : 0) : 1;
    L.E[k] = in ? K[k] + (walls ? (field == 0 ? 1 : 2) : 0) : 1;
    L.nodes *= L.E[k];
  }
  L.off = field == 1 && walls ? 1 : 0;
  return L;
}

// BF16 bits of x rounded to nearest even (x finite); the device side of the
// FP32_COMP format rounds the same way.
uint16_t bf16_rne(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
float bf16_value(uint16_t h) {
  const uint32_t b = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}

// Device image of one field component: the hi (or only) word plane set and,
// for FP32_COMP, the lo plane set; component i of ncomp sits at
// i * hi_bytes (hi) and ncomp * hi_bytes + i * lo_bytes (lo).
struct FieldImage {
  int precision;
  int64_t fw;  // coefficients per component
  std::vector<unsigned char> hi, lo;
  size_t hi_bytes() const { return (size_t)fw * (precision == HL_FP64 ? 8 : 4); }
  size_t lo_bytes() const { return precision == HL_FP32_COMP ? (size_t)fw * 2 : 0; }
  bool alloc() {
    try {
      hi.resize(hi_bytes());
      lo.resize(lo_bytes());
    } catch (const std::bad_alloc&) {
      return false;
    }
    return true;
  }
  void put(int64_t i, double x) {
    switch (precision) {
      case HL_FP64: reinterpret_cast<double*>(hi.data())[i] = x; break;
      case HL_FP32: reinterpret_cast<float*>(hi.data())[i] = (float)x; break;
      default: {
        const float h = (float)x;
        reinterpret_cast<float*>(hi.data())[i] = h;
        reinterpret_cast<uint16_t*>(lo.data())[i] = bf16_rne((float)(x - (double)h));
      }
    }
  }
  double get(int64_t i) const {
    switch (precision) {
      case HL_FP64: return reinterpret_cast<const double*>(hi.data())[i];
      case HL_FP32: return (double)reinterpret_cast<const float*>(hi.data())[i];
      default:
        return (double)reinterpret_cast<const float*>(hi.data())[i] +
               (double)bf16_value(reinterpret_cast<const uint16_t*>(lo.data())[i]);
    }
  }
};

}  // namespace hl_host
