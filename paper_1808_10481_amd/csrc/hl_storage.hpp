// hl_storage.hpp - how the state is stored in device memory, separately from
// the type the kernels compute in.
//
// A state buffer holds `ncomp` fields (p: 1, u: d) of (m+1)^d coefficient
// planes of `nodes` entries each, coefficient-major; kernels address an entry
// by its global plane index (component * (m+1)^d + coefficient) and node
// index and never form the byte address themselves.
//
//  * PlainStore<double>, PlainStore<float>: one word per coefficient, computed
//    in the same type.
//  * SplitStore: value = hi + lo, hi the FP32 rounding of the value and lo the
//    BF16 rounding of the residual, stored as two plane sets in one buffer
//    (every hi plane, then every lo plane): 6 bytes per coefficient and a
//    relative storage error near 2^-33 instead of FP32's 2^-24.  It computes
//    in FP64: on MI355X an FP64 FMA issues at the rate of an unpacked FP32 FMA,
//    so against FP64 only the bytes moved differ, and they are 3/4.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hl {

// Pointer to T in address space AS: 0 = generic (flat), 1 = global.  Kernel
// arguments are known to be global; a pointer read from memory (the batched
// shots' descriptors) is generic unless recast, and generic loads are flat
// loads with a 64-bit address per lane.
template <typename T, int AS>
struct AsPtr {
  using type = T*;
};
template <typename T>
struct AsPtr<T, 1> {
  using type = __attribute__((address_space(1))) T*;
};

// Raw buffer descriptor over `bytes` bytes at `base` (gfx9 word 3: 32-bit
// untyped data); loads at offsets past the end return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename W, int AS = 0>
struct PlainStore {
  using C = W;
  static constexpr int kBytes = (int)sizeof(W);
  using WP = typename AsPtr<W, AS>::type;
  using CP = typename AsPtr<char, AS>::type;
  struct View {
    WP base;
    int64_t nodes;
  };
  // The same storage addressed through global pointers (batched shots).
  using Global = PlainStore<W, 1>;
  template <int A = 1>  // (a template, so that PlainStore<W, 1> is not needed inside itself)
  __device__ static __forceinline__ typename PlainStore<W, A>::View global(const View& v) {
    return typename PlainStore<W, A>::View{(typename PlainStore<W, A>::WP)(uintptr_t)v.base, v.nodes};
  }
  // View of a buffer of ncomp fields of nc planes.
  __host__ static View make(const void* ptr, int ncomp, int nc, int64_t nodes) {
    (void)ncomp, (void)nc;
    return View{static_cast<W*>(const_cast<void*>(ptr)), nodes};
  }
  __device__ static __forceinline__ CP plane(const View& v, int pl) {
    return reinterpret_cast<CP>(v.base + (int64_t)pl * v.nodes);
  }
  // Uniform plane base plus a 32-bit per-lane byte offset (planes < 4 GiB).
  __device__ static __forceinline__ C load(const View& v, int pl, uint32_t node) {
    return *reinterpret_cast<WP>(plane(v, pl) + node * (uint32_t)sizeof(W));
  }
  // entry <- f(entry)
  template <class F>
  __device__ static __forceinline__ void update(const View& v, int pl, uint32_t node, F f) {
    WP q = reinterpret_cast<WP>(plane(v, pl) + node * (uint32_t)sizeof(W));
    *q = f(*q);
  }
  // the same with non-temporal accesses
  template <class F>
  __device__ static __forceinline__ void update_nt(const View& v, int pl, uint32_t node, F f) {
    WP q = reinterpret_cast<WP>(plane(v, pl) + node * (uint32_t)sizeof(W));
    __builtin_nontemporal_store(f(__builtin_nontemporal_load(q)), q);
  }
  __device__ static __forceinline__ void store(const View& v, int pl, uint32_t node, C x) {
    *reinterpret_cast<WP>(plane(v, pl) + node * (uint32_t)sizeof(W)) = x;
  }

  // Buffer-descriptor loads (3D kernels): one descriptor per plane.
  struct Planes {
    __amdgpu_buffer_rsrc_t r;
  };
  __device__ static __forceinline__ Planes planes(const View& v, int pl) {
    return Planes{raw_rsrc((const void*)(uintptr_t)plane(v, pl), (uint32_t)(v.nodes * (int64_t)sizeof(W)))};
  }
  // AUX: the cache-policy operand of the buffer instruction (0: default).
  template <int AUX = 0>
  __device__ static __forceinline__ C bload(const Planes& p, uint32_t node) {
    const uint32_t off = node * (uint32_t)sizeof(W);
    if constexpr (sizeof(W) == 4)
      return __builtin_bit_cast(W, __builtin_amdgcn_raw_buffer_load_b32(p.r, off, 0u, AUX));
    else
      return __builtin_bit_cast(W, __builtin_amdgcn_raw_buffer_load_b64(p.r, off, 0u, AUX));
  }
  template <int AUX = 0>
  __device__ static __forceinline__ void bstore(const Planes& p, uint32_t node, C x) {
    const uint32_t off = node * (uint32_t)sizeof(W);
    if constexpr (sizeof(W) == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), p.r, off, 0u, AUX);
    } else {
      typedef uint32_t u2 __attribute__((ext_vector_type(2)));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), p.r, off, 0u, AUX);
    }
  }
};

template <int AS = 0>
struct SplitStoreT {
  using C = double;
  static constexpr int kBytes = 6;
  using FP = typename AsPtr<float, AS>::type;
  using HP = typename AsPtr<uint16_t, AS>::type;
  using CP = typename AsPtr<char, AS>::type;
  struct View {
    FP hi;  // hi planes
    HP lo;  // lo planes (BF16 bit patterns), same plane numbering
    int64_t nodes;
  };
  using Global = SplitStoreT<1>;
  template <int A = 1>
  __device__ static __forceinline__ typename SplitStoreT<A>::View global(const View& v) {
    return typename SplitStoreT<A>::View{(typename SplitStoreT<A>::FP)(uintptr_t)v.hi,
                                         (typename SplitStoreT<A>::HP)(uintptr_t)v.lo, v.nodes};
  }
  __host__ static View make(const void* ptr, int ncomp, int nc, int64_t nodes) {
    float* hi = static_cast<float*>(const_cast<void*>(ptr));
    return View{hi, reinterpret_cast<uint16_t*>(hi + (int64_t)ncomp * nc * nodes), nodes};
  }
  __device__ static __forceinline__ double widen(float hi, uint16_t lo) {
    return (double)hi + (double)__builtin_bit_cast(float, (uint32_t)lo << 16);
  }
  // BF16 bits of x rounded to nearest even (x finite).
  __device__ static __forceinline__ uint16_t to_bf16(float x) {
    uint32_t b = __builtin_bit_cast(uint32_t, x);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
  }
  __device__ static __forceinline__ FP hi_plane(const View& v, int pl) { return v.hi + (int64_t)pl * v.nodes; }
  __device__ static __forceinline__ HP lo_plane(const View& v, int pl) { return v.lo + (int64_t)pl * v.nodes; }
  __device__ static __forceinline__ C load(const View& v, int pl, uint32_t node) {
    const float hi = *reinterpret_cast<FP>(reinterpret_cast<CP>(hi_plane(v, pl)) + node * 4u);
    const uint16_t lo = *reinterpret_cast<HP>(reinterpret_cast<CP>(lo_plane(v, pl)) + node * 2u);
    return widen(hi, lo);
  }
  template <class F>
  __device__ static __forceinline__ void update(const View& v, int pl, uint32_t node, F f) {
    FP qh = reinterpret_cast<FP>(reinterpret_cast<CP>(hi_plane(v, pl)) + node * 4u);
    HP ql = reinterpret_cast<HP>(reinterpret_cast<CP>(lo_plane(v, pl)) + node * 2u);
    const double val = f(widen(*qh, *ql));
    const float hi = (float)val;
    *qh = hi;
    *ql = to_bf16((float)(val - (double)hi));
  }
  __device__ static __forceinline__ void store(const View& v, int pl, uint32_t node, C x) {
    update(v, pl, node, [&](C) { return x; });
  }
  template <class F>
  __device__ static __forceinline__ void update_nt(const View& v, int pl, uint32_t node, F f) {
    FP qh = reinterpret_cast<FP>(reinterpret_cast<CP>(hi_plane(v, pl)) + node * 4u);
    HP ql = reinterpret_cast<HP>(reinterpret_cast<CP>(lo_plane(v, pl)) + node * 2u);
    const double val = f(widen(__builtin_nontemporal_load(qh), __builtin_nontemporal_load(ql)));
    const float hi = (float)val;
    __builtin_nontemporal_store(hi, qh);
    __builtin_nontemporal_store(to_bf16((float)(val - (double)hi)), ql);
  }

  struct Planes {
    __amdgpu_buffer_rsrc_t hi, lo;
  };
  __device__ static __forceinline__ Planes planes(const View& v, int pl) {
    const uint32_t n = (uint32_t)v.nodes;
    return Planes{raw_rsrc((const void*)(uintptr_t)hi_plane(v, pl), 4u * n),
                  raw_rsrc((const void*)(uintptr_t)lo_plane(v, pl), 2u * n)};
  }
  template <int AUX = 0>
  __device__ static __forceinline__ C bload(const Planes& p, uint32_t node) {
    const float hi = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(p.hi, node * 4u, 0u, AUX));
    const uint16_t lo = (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(p.lo, node * 2u, 0u, AUX);
    return widen(hi, lo);
  }
  // The same rounding as update / store: hi = FP32 of x, lo = BF16 of x - hi.
  template <int AUX = 0>
  __device__ static __forceinline__ void bstore(const Planes& p, uint32_t node, C x) {
    const float hi = (float)x;
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, hi), p.hi, node * 4u, 0u, AUX);
    __builtin_amdgcn_raw_buffer_store_b16(to_bf16((float)(x - (double)hi)), p.lo, node * 2u, 0u, AUX);
  }
};

using SplitStore = SplitStoreT<0>;

}  // namespace hl
