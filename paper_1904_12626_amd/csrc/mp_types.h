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

// Sixteen bytes of consecutive samples, aligned only to the element size.
template <typename T>
struct __attribute__((aligned(sizeof(T)))) Chunk16 {
  T v[16 / sizeof(T)];
};

// f(u, (double)x[u]) for u = 0 .. m-1, in that order.  Meant for a window at
// an arbitrary offset per lane (a neighbour picked by the profile index):
// it is read as 16-byte chunks, D in flight, so a wave touches a quarter
// of the cache lines per load instruction and never waits on the load it is
// about to use.  Reads stay inside x[0 .. m-1].
template <typename Tin, int D = 4, typename Fn>
__device__ __forceinline__ void for_each_sample(const Tin *__restrict__ x, int m, Fn &&f) {
  constexpr int E = 16 / sizeof(Tin);
  using C = Chunk16<Tin>;
  const int nch = m / E;
  auto chunk = [&](int q) { return *reinterpret_cast<const C *>(x + (int64_t)min(q, nch - 1) * E); };
  int q = 0;
  if (nch > 0) {
    C ring[D];
#pragma unroll
    for (int r = 0; r < D; ++r) ring[r] = chunk(r);
    for (; q + D <= nch; q += D) {
#pragma unroll
      for (int r = 0; r < D; ++r) {
        const C c = ring[r];
        ring[r] = chunk(q + r + D);  // clamped to the last chunk
#pragma unroll
        for (int e = 0; e < E; ++e) f((q + r) * E + e, (double)c.v[e]);
      }
    }
#pragma unroll
    for (int r = 0; r < D; ++r)
      if (q + r < nch) {
#pragma unroll
        for (int e = 0; e < E; ++e) f((q + r) * E + e, (double)ring[r].v[e]);
      }
  }
  for (int u = nch * E; u < m; ++u) f(u, (double)x[u]);
}

}  // namespace mpx
