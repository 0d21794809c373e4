// Incremental self-join (Section 2 lists it as a property of the matrix
// profile; the paper gives no algorithm).  The stream keeps, in FP64, the
// profile of the windows seen so far, the statistics of every window and
// the centred cross products C(w, j) of the newest window w with every
// earlier window.  A new window w + 1 continues each diagonal:
//   C(w+1, j+1) = C(w, j) + a_j g_w + a_w g_j
// (C(w+1, 0) and, every `reseed` windows, all of them by direct dot
// products), scores its admissible earlier partners, takes the nearest as
// its own neighbour and offers itself to every one of them.
#include <cmath>

#include "mp_internal.h"
#include "mp_types.h"

namespace mpx {

namespace {

constexpr int kStreamBlock = 256;

template <typename Tin>
__device__ __forceinline__ double smp(const Tin *p) {
  const double v = (double)*p;
  return isfinite(v) ? v : 0.0;
}

}  // namespace

// Statistics of windows [w_lo, w_hi) and the a/g terms of every window whose
// successor sample is known (a_w needs x[w+m], so windows up to n - m - 1).
template <typename Tin>
__global__ void __launch_bounds__(256) k_stream_stats(StreamWork s, const Tin *__restrict__ T, int64_t n,
                                                      int m, int64_t w_lo, int64_t w_hi) {
  const int64_t w = w_lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= w_hi) return;
  const Tin *x = T + w;
  bool ok = true;
  double sum = 0.0, lo = 0.0, hi = 0.0;
  for (int u = 0; u < m; ++u) {
    const double v = (double)x[u];
    if (!isfinite(v)) ok = false;
    const double c = isfinite(v) ? v : 0.0;
    if (u == 0) { lo = c; hi = c; }
    lo = fmin(lo, c);
    hi = fmax(hi, c);
    sum += c;
  }
  const double mu = sum / m;
  double q = 0.0;
  for (int u = 0; u < m; ++u) {
    const double dv = smp(x + u) - mu;
    q = fma(dv, dv, q);
  }
  const bool cst = ok && (lo == hi || !(q > 0.0));
  s.mu[w] = mu;
  s.isd[w] = (ok && !cst) ? 1.0 / (sqrt((double)m) * sqrt(q / m)) : 0.0;
  s.flags[w] = (uint8_t)((ok ? 1 : 0) | (cst ? 2 : 0));
  const double a = (w + m < n) ? smp(x + m) - smp(x) : 0.0;
  s.a[w] = a;
  s.g[w] = smp(x) - mu + a * (double)(m - 1) / (2.0 * m);
}

// FP64 distance from the z-normalised form of two windows' statistics and
// their centred cross product; constant windows normalise to zero.
__device__ __forceinline__ double stream_dist(const StreamWork &s, int64_t i, int64_t j, double C, int m) {
  const uint8_t fi = s.flags[i], fj = s.flags[j];
  double key;
  if ((fi & 2) && (fj & 2)) key = 0.0;
  else if ((fi & 2) || (fj & 2)) key = 0.5;
  else key = 1.0 - C * s.isd[i] * s.isd[j];
  return sqrt(2.0 * m * fmax(key, 0.0));
}

template <typename Tin>
__device__ double direct_c(const Tin *T, int64_t i, int64_t j, const StreamWork &s, int m) {
  double acc = 0.0;
  const double mi = s.mu[i], mj = s.mu[j];
  for (int u = 0; u < m; ++u) acc = fma(smp(T + i + u) - mi, smp(T + j + u) - mj, acc);
  return acc;
}

// Cross products C(w, j) of window w with every j <= w - ez - 1, directly.
template <typename Tin>
__global__ void __launch_bounds__(256) k_stream_seed(StreamWork s, const Tin *__restrict__ T, int m,
                                                     int64_t w, int64_t jmax, double *C) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > jmax) return;
  C[j] = direct_c(T, w, j, s, m);
}

// Row w: continue (or seed) the cross products, score every admissible
// earlier partner j, offer w to j (strict improvement: ties keep the older,
// smaller partner), and reduce this block's best (d, j) for row w.
template <typename Tin>
__global__ void __launch_bounds__(kStreamBlock) k_stream_row(StreamWork s, const Tin *__restrict__ T, int m,
                                                             int64_t w, int64_t jmax, int seed,
                                                             const double *__restrict__ Cprev, double *Cnew,
                                                             int64_t *I) {
  __shared__ double bd[kStreamBlock];
  __shared__ int64_t bj[kStreamBlock];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double best = INFINITY;
  int64_t arg = -1;
  if (j <= jmax) {
    double C;
    if (seed || j == 0) C = direct_c(T, w, j, s, m);
    else C = Cprev[j - 1] + s.a[j - 1] * s.g[w - 1] + s.a[w - 1] * s.g[j - 1];
    Cnew[j] = C;
    if ((s.flags[w] & 1) && (s.flags[j] & 1)) {
      const double d = stream_dist(s, w, j, C, m);
      best = d;
      arg = j;
      if (d < s.Pd[j]) {
        s.Pd[j] = d;
        I[j] = w;
      }
    }
  }
  bd[threadIdx.x] = best;
  bj[threadIdx.x] = arg;
  __syncthreads();
  for (int h = kStreamBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double d2 = bd[threadIdx.x + h];
      const int64_t j2 = bj[threadIdx.x + h];
      if (j2 >= 0 && (bj[threadIdx.x] < 0 || d2 < bd[threadIdx.x] ||
                      (d2 == bd[threadIdx.x] && j2 < bj[threadIdx.x]))) {
        bd[threadIdx.x] = d2;
        bj[threadIdx.x] = j2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    s.part_d[blockIdx.x] = bd[0];
    s.part_j[blockIdx.x] = bj[0];
  }
}

// Row w's own neighbour from the per-block partial results (one workgroup;
// strict '<' in block order keeps the smallest index on ties).
__global__ void __launch_bounds__(256) k_stream_rowfin(StreamWork s, int64_t w, int64_t nblocks, int64_t *I) {
  __shared__ double bd[256];
  __shared__ int64_t bj[256];
  double best = INFINITY;
  int64_t arg = -1;
  for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) {
    const int64_t j2 = s.part_j[b];
    const double d2 = s.part_d[b];
    if (j2 >= 0 && (arg < 0 || d2 < best)) {
      best = d2;
      arg = j2;
    }
  }
  bd[threadIdx.x] = best;
  bj[threadIdx.x] = arg;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double d2 = bd[threadIdx.x + h];
      const int64_t j2 = bj[threadIdx.x + h];
      if (j2 >= 0 && (bj[threadIdx.x] < 0 || d2 < bd[threadIdx.x] ||
                      (d2 == bd[threadIdx.x] && j2 < bj[threadIdx.x]))) {
        bd[threadIdx.x] = d2;
        bj[threadIdx.x] = j2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const bool valid = s.flags[w] & 1;
    s.Pd[w] = (valid && bj[0] >= 0) ? bd[0] : INFINITY;
    I[w] = (valid && bj[0] >= 0) ? bj[0] : -1;
  }
}

// FP64 profile of the initial windows from their indices (exact distances
// of the chosen pairs), and the output copy of the profile.
template <typename Tin>
__global__ void __launch_bounds__(256) k_stream_pd(StreamWork s, const Tin *__restrict__ T, int m, int64_t l,
                                                   const int64_t *__restrict__ I) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= l) return;
  const int64_t j = I[w];
  double d = INFINITY;
  if (j >= 0 && (s.flags[w] & 1) && (s.flags[j] & 1)) d = stream_dist(s, w, j, direct_c(T, w, j, s, m), m);
  s.Pd[w] = d;
}

template <typename Tout>
__global__ void __launch_bounds__(256) k_stream_out(StreamWork s, int64_t l, Tout *P) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < l) P[w] = (Tout)s.Pd[w];
}

int64_t stream_partials(int64_t l_max) { return (l_max + kStreamBlock - 1) / kStreamBlock; }

template <typename Tin>
hipError_t stream_init_t(const StreamWork &s, const Tin *T, int64_t n, int m, int ez, const int64_t *I,
                         hipStream_t st) {
  const int64_t l = n - m + 1;
  const dim3 b(256), g((unsigned)((l + 255) / 256));
  hipLaunchKernelGGL((k_stream_stats<Tin>), g, b, 0, st, s, T, n, m, (int64_t)0, l);
  hipLaunchKernelGGL((k_stream_pd<Tin>), g, b, 0, st, s, T, m, l, I);
  // cross products of the newest window with its admissible partners
  const int64_t w = l - 1, jmax = w - ez - 1;
  if (jmax >= 0)
    hipLaunchKernelGGL((k_stream_seed<Tin>), dim3((unsigned)((jmax + 256) / 256)), b, 0, st, s, T, m, w, jmax,
                       s.C[w & 1]);
  return hipGetLastError();
}

// The cross products of window w live in C[w % 2].
template <typename Tin>
hipError_t stream_append_t(const StreamWork &s, const Tin *T, int64_t n_old, int64_t n_new, int m, int ez,
                           int reseed, int64_t *I, hipStream_t st) {
  const int64_t l_old = n_old - m + 1, l_new = n_new - m + 1;
  const dim3 b(256);
  // statistics of the new windows, and the a/g terms of the last old window
  // (its successor sample has arrived)
  hipLaunchKernelGGL((k_stream_stats<Tin>), dim3((unsigned)((l_new - l_old + 1 + 255) / 256)), b, 0, st, s, T,
                     n_new, m, l_old - 1, l_new);
  for (int64_t w = l_old; w < l_new; ++w) {
    const int64_t jmax = w - ez - 1;
    if (jmax < 0) {
      hipLaunchKernelGGL(k_stream_rowfin, dim3(1), dim3(256), 0, st, s, w, (int64_t)0, I);
      continue;
    }
    const int64_t nb = (jmax + kStreamBlock) / kStreamBlock;
    const int seed = (w % reseed) == 0 ? 1 : 0;
    hipLaunchKernelGGL((k_stream_row<Tin>), dim3((unsigned)nb), dim3(kStreamBlock), 0, st, s, T, m, w, jmax, seed,
                       (const double *)s.C[(w - 1) & 1], s.C[w & 1], I);
    hipLaunchKernelGGL(k_stream_rowfin, dim3(1), dim3(256), 0, st, s, w, nb, I);
  }
  return hipGetLastError();
}

hipError_t launch_stream_init(const StreamWork &s, const void *T, bool t_f64, int64_t n, int m, int ez,
                              const int64_t *I, hipStream_t st) {
  return t_f64 ? stream_init_t(s, (const double *)T, n, m, ez, I, st)
               : stream_init_t(s, (const float *)T, n, m, ez, I, st);
}

hipError_t launch_stream_append(const StreamWork &s, const void *T, bool t_f64, int64_t n_old, int64_t n_new,
                                int m, int ez, int reseed, int64_t *I, hipStream_t st) {
  return t_f64 ? stream_append_t(s, (const double *)T, n_old, n_new, m, ez, reseed, I, st)
               : stream_append_t(s, (const float *)T, n_old, n_new, m, ez, reseed, I, st);
}

hipError_t launch_stream_out(const StreamWork &s, int64_t l, void *P, bool out_f64, hipStream_t st) {
  const dim3 b(256), g((unsigned)((l + 255) / 256));
  if (out_f64) hipLaunchKernelGGL((k_stream_out<double>), g, b, 0, st, s, l, (double *)P);
  else hipLaunchKernelGGL((k_stream_out<float>), g, b, 0, st, s, l, (float *)P);
  return hipGetLastError();
}

}  // namespace mpx
