// Data-mining passes over a profile index (Section 3.4): the arc counts of
// semantic segmentation (3.4.2) and time series chains (3.4.3).  Both are
// O(l) integer work: arcs are counted with integer atomics and a prefix
// sum, chain lengths by pointer jumping; every reduction is over integers or
// picks the smallest index on ties, so results are deterministic.
#include <cmath>

#include "mp_internal.h"

namespace mpx {

namespace {

__global__ void __launch_bounds__(256) k_fill_i64(int64_t *p, int64_t n, int64_t v) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    p[x] = v;
}

unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 16); }

// Arc of window i: from min(i, I[i]) (+1) to max(i, I[i]) (-1), so that the
// prefix sum at x counts the arcs with min <= x < max.
__global__ void __launch_bounds__(256) k_arc_marks(const int64_t *__restrict__ I, int64_t l, int64_t *marks) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const int64_t j = I[i];
  if (j < 0 || j >= l || j == i) return;
  const int64_t a = i < j ? i : j, b = i < j ? j : i;
  atomicAdd(reinterpret_cast<unsigned long long *>(marks + a), 1ull);
  atomicAdd(reinterpret_cast<unsigned long long *>(marks + b), ~0ull);  // -1 in two's complement
}

// Corrected arc curve: arc count over the count 2x(l - x)/l that arcs to
// uniformly random positions would give, capped at 1; 1 within `zone` of
// either end.  excl[x + 1] is the arc count at x.
__global__ void __launch_bounds__(256) k_cac(const int64_t *__restrict__ excl, int64_t l, int64_t zone,
                                             double *cac) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= l) return;
  double v = 1.0;
  if (x >= zone && x < l - zone) {
    const double ideal = 2.0 * (double)x * (double)(l - x) / (double)l;
    if (ideal > 0.0) v = fmin((double)excl[x + 1] / ideal, 1.0);
  }
  cac[x] = v;
}

// k segment boundaries: repeatedly the smallest CAC (smallest index on ties)
// outside the edge zones and farther than `zone` from every earlier pick.
// One workgroup; k is small.
constexpr int kMaxSegments = 64;
__global__ void __launch_bounds__(1024) k_fluss_pick(const double *__restrict__ cac, int64_t l, int64_t zone,
                                                     int k, int64_t *segments) {
  __shared__ double bv[1024];
  __shared__ int64_t bi[1024];
  __shared__ int64_t picks[kMaxSegments];
  const int tid = threadIdx.x;
  for (int q = 0; q < k; ++q) {
    double best = INFINITY;
    int64_t arg = -1;
    for (int64_t x = zone + tid; x < l - zone; x += blockDim.x) {
      bool masked = false;
      for (int p = 0; p < q; ++p) {
        const int64_t c = picks[p];
        if (c >= 0 && x >= c - zone && x <= c + zone) masked = true;
      }
      if (!masked && cac[x] < best) {  // x increases per thread: first minimum kept
        best = cac[x];
        arg = x;
      }
    }
    bv[tid] = best;
    bi[tid] = arg;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
      if (tid < h) {
        const double v2 = bv[tid + h];
        const int64_t i2 = bi[tid + h];
        if (i2 >= 0 && (bi[tid] < 0 || v2 < bv[tid] || (v2 == bv[tid] && i2 < bi[tid]))) {
          bv[tid] = v2;
          bi[tid] = i2;
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      picks[q] = bi[0];
      segments[q] = bi[0];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ chains
// next[i] = IR[i] when the link is confirmed from the other side
// (IL[IR[i]] == i), else -1; d = 1 per link for the pointer jumping.
__global__ void __launch_bounds__(256) k_chain_links(const int64_t *__restrict__ IL, const int64_t *__restrict__ IR,
                                                     int64_t l, int64_t *next, int64_t *d, int64_t *nx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const int64_t j = IR[i];
  const int64_t s = (j > i && j < l && IL[j] == i) ? j : -1;
  next[i] = s;
  d[i] = s >= 0 ? 1 : 0;
  nx[i] = s;
}

// One round of pointer jumping: distance to the chain's end and the node
// 2^r links ahead.
__global__ void __launch_bounds__(256) k_chain_jump(const int64_t *__restrict__ d0, const int64_t *__restrict__ n0,
                                                    int64_t *d1, int64_t *n1, int64_t l) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const int64_t s = n0[i];
  if (s >= 0) {
    d1[i] = d0[i] + d0[s];
    n1[i] = n0[s];
  } else {
    d1[i] = d0[i];
    n1[i] = -1;
  }
}

// Chain length from every node, and per chain head (a node that no
// confirmed link enters) the count of chains with >= min_len elements and
// the longest chain (smallest head on equal lengths) as one packed maximum:
// length in the high half, the complement of the head in the low half.
__global__ void __launch_bounds__(256) k_chain_summary(const int64_t *__restrict__ IL, const int64_t *__restrict__ next,
                                                       const int64_t *__restrict__ d, int64_t l, int64_t min_len,
                                                       int64_t *length, unsigned long long *acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const int64_t len = d[i] + 1;
  length[i] = len;
  const int64_t p = IL[i];
  const bool head = !(p >= 0 && p < i && next[p] == i);
  if (!head) return;
  if (len >= min_len) atomicAdd(&acc[0], 1ull);
  const unsigned long long key = ((unsigned long long)len << 32) | (0xFFFFFFFFull - (unsigned long long)i);
  atomicMax(&acc[1], key);
}

__global__ void k_chain_best(const int64_t *__restrict__ next, const unsigned long long *__restrict__ acc,
                             int64_t *summary, int64_t *best) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const unsigned long long key = acc[1];
  const int64_t len = (int64_t)(key >> 32);
  const int64_t head = len > 0 ? (int64_t)(0xFFFFFFFFull - (key & 0xFFFFFFFFull)) : -1;
  summary[0] = (int64_t)acc[0];
  summary[1] = head;
  summary[2] = len;
  int64_t v = head;
  for (int64_t t = 0; t < len && v >= 0; ++t) {
    best[t] = v;
    v = next[v];
  }
}

}  // namespace

size_t fluss_scratch_words(int64_t l) { return (size_t)(l + 1) * 2 + (size_t)((l + 1023) / 1024 + 1); }

hipError_t launch_fluss(const int64_t *I, int64_t l, int64_t zone, int k, double *cac, int64_t *segments,
                        int64_t *ws, hipStream_t st) {
  int64_t *marks = ws, *excl = ws + (l + 1), *partial = ws + 2 * (l + 1);
  hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(l + 1)), dim3(256), 0, st, marks, l + 1, (int64_t)0);
  hipLaunchKernelGGL(k_arc_marks, dim3((unsigned)((l + 255) / 256)), dim3(256), 0, st, I, l, marks);
  hipError_t e = launch_exclusive_scan(marks, excl, partial, l, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cac, dim3((unsigned)((l + 255) / 256)), dim3(256), 0, st, (const int64_t *)excl, l, zone,
                     cac);
  if (k > 0)
    hipLaunchKernelGGL(k_fluss_pick, dim3(1), dim3(1024), 0, st, (const double *)cac, l, zone, k, segments);
  return hipGetLastError();
}

size_t chains_scratch_words(int64_t l) { return (size_t)l * 4 + 2; }

hipError_t launch_chains(const int64_t *IL, const int64_t *IR, int64_t l, int64_t min_len, int64_t *next,
                         int64_t *length, int64_t *summary, int64_t *best, int64_t *ws, hipStream_t st) {
  int64_t *d0 = ws, *n0 = ws + l, *d1 = ws + 2 * l, *n1 = ws + 3 * l;
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(ws + 4 * l);
  const dim3 blk(256), grd((unsigned)((l + 255) / 256));
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(256), 0, st, reinterpret_cast<int64_t *>(acc), (int64_t)2,
                     (int64_t)0);
  hipLaunchKernelGGL(k_chain_links, grd, blk, 0, st, IL, IR, l, next, d0, n0);
  int rounds = 1;
  while (((int64_t)1 << rounds) < l) ++rounds;
  for (int r = 0; r < rounds; ++r) {
    hipLaunchKernelGGL(k_chain_jump, grd, blk, 0, st, (const int64_t *)d0, (const int64_t *)n0, d1, n1, l);
    std::swap(d0, d1);
    std::swap(n0, n1);
  }
  hipLaunchKernelGGL(k_chain_summary, grd, blk, 0, st, IL, (const int64_t *)next, (const int64_t *)d0, l, min_len,
                     length, acc);
  hipLaunchKernelGGL(k_chain_best, dim3(1), dim3(64), 0, st, (const int64_t *)next,
                     (const unsigned long long *)acc, summary, best);
  return hipGetLastError();
}

}  // namespace mpx
