// Element-type traits shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mpx {

struct alignas(32) Double4 {
  double x, y, z, w;
};

template <typename F>
struct FTraits;

template <>
struct FTraits<float> {
  using V4 = float4;
  static __device__ __forceinline__ V4 zero4() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  // padding record: a = g = s = 0 and a huge finite u (see k_stats); finite,
  // so that writing a code into its low mantissa bits cannot make a NaN
  static __device__ __forceinline__ V4 pad4() { return make_float4(0.f, 0.f, 0.f, 3.0e38f); }
  static __device__ __forceinline__ V4 make4(double a, double b, double c, double d) {
    return make_float4((float)a, (float)b, (float)c, (float)d);
  }
};

template <>
struct FTraits<double> {
  using V4 = Double4;
  static __device__ __forceinline__ V4 zero4() { return Double4{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ V4 pad4() { return Double4{0.0, 0.0, 0.0, 1.0e300}; }
  static __device__ __forceinline__ V4 make4(double a, double b, double c, double d) {
    return Double4{a, b, c, d};
  }
};

// Packed (key, index) for the global minimum: the key is a non-negative
// double whose low `bits` bits are replaced by the index, so an unsigned
// 64-bit minimum is the minimum key with the smallest index on ties.
__device__ __forceinline__ uint64_t pack_global(double key, int64_t idx, int bits) {
  key = key > 0.0 ? key : 0.0;
  const uint64_t mask = (bits >= 64) ? ~0ull : ((1ull << bits) - 1ull);
  return ((uint64_t)__double_as_longlong(key) & ~mask) | ((uint64_t)idx & mask);
}

__device__ __forceinline__ double unpack_key(uint64_t k, int bits) {
  const uint64_t mask = (1ull << bits) - 1ull;
  return __longlong_as_double((long long)(k & ~mask));
}

__device__ __forceinline__ int64_t unpack_idx(uint64_t k, int bits) {
  return (int64_t)(k & ((1ull << bits) - 1ull));
}

}  // namespace mpx
