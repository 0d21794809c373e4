// Exclusive prefix sum of int64 values (device), in three launches: one
// workgroup per chunk of 1024 entries (Hillis-Steele in LDS), one workgroup
// over the chunk totals, then the chunk offsets are added back.  The sums of
// integers do not depend on the order, so the result is exact and
// deterministic.
#include "mp_internal.h"

namespace mpx {

namespace {

__global__ void __launch_bounds__(1024) k_scan_chunks(const int64_t *__restrict__ in, int64_t *out,
                                                      int64_t *chunk_tot, int64_t n) {
  __shared__ int64_t sh[1024];
  const int64_t x = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int64_t v = x < n ? in[x] : 0;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t add = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  if (x < n) out[x] = sh[threadIdx.x] - v;
  if (threadIdx.x == 1023) chunk_tot[blockIdx.x] = sh[1023];
}

__global__ void __launch_bounds__(1024) k_scan_totals(int64_t *chunk_tot, int64_t nchunks, int64_t *out,
                                                      int64_t n) {
  __shared__ int64_t part[1024];
  const int tid = threadIdx.x;
  const int64_t per = (nchunks + 1023) / 1024;
  const int64_t a = min(nchunks, (int64_t)tid * per), e = min(nchunks, a + per);
  int64_t s = 0;
  for (int64_t c = a; c < e; ++c) s += chunk_tot[c];
  // inclusive log-step scan of the per-thread sums, then exclusive
  part[tid] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t add = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  if (tid == 1023) out[n] = part[tid];
  int64_t run = part[tid] - s;
  for (int64_t c = a; c < e; ++c) {
    const int64_t v = chunk_tot[c];
    chunk_tot[c] = run;
    run += v;
  }
}

__global__ void __launch_bounds__(1024) k_scan_add(int64_t *out, const int64_t *__restrict__ chunk_tot,
                                                   int64_t n) {
  const int64_t x = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (x < n) out[x] += chunk_tot[blockIdx.x];
}

}  // namespace

hipError_t launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t *partial, int64_t n,
                                 hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nchunks = (n + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nchunks), dim3(1024), 0, st, in, out, partial, n);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, st, partial, nchunks, out, n);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nchunks), dim3(1024), 0, st, out,
                     (const int64_t *)partial, n);
  return hipGetLastError();
}

}  // namespace mpx
