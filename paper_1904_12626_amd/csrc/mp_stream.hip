// Incremental self-join (Section 2 lists it as a property of the matrix
// profile; the paper gives no algorithm).  The stream keeps, in FP64, the
// profile of the windows seen so far, the statistics of every window and
// the centred cross products C(w, j) of the newest window w with every
// earlier window.  A new window w + 1 continues each diagonal:
//   C(w+1, j+1) = C(w, j) + a_j g_w + a_w g_j
// (C(w+1, 0) and, every `reseed` windows, all of them by direct dot
// products), scores its admissible earlier partners, takes the nearest as
// its own neighbour and offers itself to every one of them.
//
// New windows are processed B at a time (B <= ez + 1, so no new window is a
// candidate of another in the same batch): a workgroup owns 256 - (B-1)
// consecutive columns and also recomputes the B-1 columns to their left,
// whose cross products it needs (a trapezoid: after step b the leftmost b
// threads hold stale values, and none of them is owned).  Each thread
// keeps its column's terms in registers for all B rows and passes its cross
// product to the right neighbour through LDS, so a column's data is read
// once per batch instead of once per row.
#include <cmath>

#include "mp_internal.h"
#include "mp_types.h"

namespace mpx {

namespace {

constexpr int kStreamBlock = 256;

// Minimum of a double over the wave, returned wave-uniform: DPP row shifts
// of both halves inside each row of 16 lanes, then the four row minima.
template <int CTRL>
__device__ __forceinline__ double dpp_shr(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_value(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_min_f64(double v) {
  v = fmin(v, dpp_shr<0x111>(v));  // row_shr:1
  v = fmin(v, dpp_shr<0x112>(v));  // row_shr:2
  v = fmin(v, dpp_shr<0x114>(v));  // row_shr:4
  v = fmin(v, dpp_shr<0x118>(v));  // row_shr:8
  return fmin(fmin(lane_value(v, 15), lane_value(v, 31)), fmin(lane_value(v, 47), lane_value(v, 63)));
}

// Scalar load of a wave-uniform address (constant address space): the
// per-row terms are read-only in the batch kernel.
template <typename T>
__device__ __forceinline__ T ldu_s(const T *p) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef const uint32_t __attribute__((address_space(4))) *cptr;
  const cptr q = (cptr)(p);
  T out;
  uint32_t *o = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = q[i];
  return out;
#else
  return *p;
#endif
}

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

// Key d^2 / (2m) (= 1 - Pearson rho for varying windows) from two windows'
// statistics and their centred cross product; constant windows normalise to
// zero.  The state holds keys; distances are taken at the output.
__device__ __forceinline__ double stream_key(const StreamWork &s, int64_t i, int64_t j, double C) {
  const uint8_t fi = s.flags[i], fj = s.flags[j];
  if ((fi & 2) && (fj & 2)) return 0.0;
  if ((fi & 2) || (fj & 2)) return 0.5;
  return fmax(1.0 - C * s.isd[i] * s.isd[j], 0.0);
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

// C(w0 + b, 0) for the B windows of a batch: column 0 has no left
// neighbour to continue from, so its cross products are direct dot
// products, one wave per window.
template <typename Tin>
__global__ void __launch_bounds__(64) k_stream_col0(StreamWork s, const Tin *__restrict__ T, int m, int64_t w0) {
  const int64_t w = w0 + blockIdx.x;
  const double mw = s.mu[w], m0 = s.mu[0];
  double acc = 0.0;
  for (int u = threadIdx.x; u < m; u += 64) acc = fma(smp(T + w + u) - mw, smp(T + u) - m0, acc);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (threadIdx.x == 0) s.col0[blockIdx.x] = acc;
}

// One batch of B new windows w0 .. w0+B-1 (see the file comment).  Row
// minima of each step go to per-wave partials (reduced by
// k_stream_rowfin); owned columns update their own profile entries.  One
// barrier per step: the cross products move right through LDS.
template <typename Tin>
__global__ void __launch_bounds__(kStreamBlock) k_stream_batch(StreamWork s, const Tin *__restrict__ T, int m,
                                                               int ez, int64_t w0, int B, int seed_step,
                                                               const double *__restrict__ Cprev, double *Cnew,
                                                               int64_t *I, int64_t nparts) {
  __shared__ double xfer[2][kStreamBlock];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int H = B - 1;
  const int64_t c0 = (int64_t)blockIdx.x * (kStreamBlock - H);
  const int64_t j = c0 - H + tid;
  const bool owned = tid >= H;
  const int64_t jlast = w0 + B - 1 - ez - 1;  // last column any row of the batch scores
  double aj1 = 0.0, gj1 = 0.0, isdj = 0.0, Pdj = INFINITY;
  uint8_t fj = 0;
  int64_t Ij = -1;
  bool changed = false;
  if (j >= 0 && j <= jlast) {
    if (j >= 1) {
      aj1 = s.a[j - 1];
      gj1 = s.g[j - 1];
    }
    fj = s.flags[j];
    isdj = s.isd[j];
    if (owned) {
      Pdj = s.Pd[j];
      Ij = I[j];
    }
  }
  // C(w0 - 1, j - 1), available for j - 1 <= w0 - 1 - ez - 1
  double Cin = (j >= 1 && j - 1 <= w0 - ez - 2) ? Cprev[j - 1] : 0.0;
  double C = 0.0;
  const int64_t part = (int64_t)blockIdx.x * (kStreamBlock / 64) + wave;
  for (int b = 0; b < B; ++b) {
    const int64_t w = w0 + b, jmax = w - ez - 1;
    if (b > 0) Cin = tid > 0 ? xfer[(b - 1) & 1][tid - 1] : 0.0;
    double best = INFINITY;
    bool cand = false;
    if (j >= 0 && j <= jmax) {
      if (j == 0) C = s.col0[b];
      else if (b == seed_step) C = direct_c(T, w, j, s, m);
      else C = Cin + aj1 * ldu_s(s.g + w - 1) + ldu_s(s.a + w - 1) * gj1;
      const uint8_t fw = (uint8_t)(ldu_s(reinterpret_cast<const uint32_t *>(s.flags + (w & ~3ll))) >> (8 * (w & 3)));
      if ((fw & 1) && (fj & 1) && owned) {
        double key;
        if ((fw & 2) && (fj & 2)) key = 0.0;
        else if ((fw & 2) || (fj & 2)) key = 0.5;
        else key = fmax(1.0 - C * ldu_s(s.isd + w) * isdj, 0.0);
        const double d = key;
        best = d;
        cand = true;
        if (d < Pdj) {
          Pdj = d;
          Ij = w;
          changed = true;
        }
      }
    }
    xfer[b & 1][tid] = C;
    // this wave's best candidate for row w: the smallest distance, at its
    // first lane (lanes hold increasing columns)
    const double mn = wave_min_f64(best);
    const unsigned long long hit = __ballot(cand && best == mn);
    if (lane == 0) {
      int64_t jj = -1;
      if (hit) jj = c0 - H + wave * 64 + (__ffsll((long long)hit) - 1);
      s.part_d[(int64_t)b * nparts + part] = hit ? mn : INFINITY;
      s.part_j[(int64_t)b * nparts + part] = jj;
    }
    __syncthreads();
  }
  if (owned && j >= 0 && j <= jlast) {
    Cnew[j] = C;  // C(w0 + B - 1, j)
    if (changed) {
      s.Pd[j] = Pdj;
      I[j] = Ij;
    }
  }
}

// Row w0 + blockIdx.x: its own neighbour from the per-wave partials (strict
// '<' in partial order, which is column order, keeps the smallest index on
// ties).
__global__ void __launch_bounds__(256) k_stream_rowfin(StreamWork s, int64_t w0, int64_t nblocks, int64_t *I) {
  __shared__ double bd[256];
  __shared__ int64_t bj[256];
  const int64_t w = w0 + blockIdx.x;
  const double *pd = s.part_d + (int64_t)blockIdx.x * nblocks;
  const int64_t *pj = s.part_j + (int64_t)blockIdx.x * nblocks;
  double best = INFINITY;
  int64_t arg = -1;
  for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) {
    const int64_t j2 = pj[b];
    const double d2 = pd[b];
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
  if (j >= 0 && (s.flags[w] & 1) && (s.flags[j] & 1)) d = stream_key(s, w, j, direct_c(T, w, j, s, m));
  s.Pd[w] = d;
}

template <typename Tout>
__global__ void __launch_bounds__(256) k_stream_out(StreamWork s, int64_t l, int m, Tout *P) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < l) P[w] = (Tout)sqrt(2.0 * m * s.Pd[w]);
}

constexpr int kStreamMaxBatch = 63;
// partial row minima: up to kStreamMaxBatch rows x 4 waves per workgroup of
// >= 194 owned columns
int64_t stream_partials(int64_t l_max) {
  return (int64_t)kStreamMaxBatch * (kStreamBlock / 64) *
         ((l_max + (kStreamBlock - kStreamMaxBatch + 1) - 1) / (kStreamBlock - kStreamMaxBatch + 1) + 1);
}

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

// The cross products of window w live in C[w % 2]; batches have an odd
// number of windows, so a batch reads one buffer and writes the other.
template <typename Tin>
hipError_t stream_append_t(const StreamWork &s, const Tin *T, int64_t n_old, int64_t n_new, int m, int ez,
                           int reseed, int64_t *I, hipStream_t st) {
  const int64_t l_old = n_old - m + 1, l_new = n_new - m + 1;
  const dim3 b(256);
  // statistics of the new windows, and the a/g terms of the last old window
  // (its successor sample has arrived)
  hipLaunchKernelGGL((k_stream_stats<Tin>), dim3((unsigned)((l_new - l_old + 1 + 255) / 256)), b, 0, st, s, T,
                     n_new, m, l_old - 1, l_new);
  const int bmax = (int)std::min<int64_t>(kStreamMaxBatch, (int64_t)ez + 1);
  for (int64_t w0 = l_old; w0 < l_new;) {
    int B = (int)std::min<int64_t>(bmax, l_new - w0);
    if ((B & 1) == 0) --B;
    const int64_t jlast = w0 + B - 1 - ez - 1;
    if (jlast < 0) {  // no candidates yet: one window at a time
      hipLaunchKernelGGL(k_stream_rowfin, dim3(1), dim3(256), 0, st, s, w0, (int64_t)0, I);
      ++w0;
      continue;
    }
    const int owned = kStreamBlock - (B - 1);
    const int64_t nblocks = (jlast + 1 + owned - 1) / owned;
    const int64_t nparts = nblocks * (kStreamBlock / 64);
    int seed_step = -1;  // the step of this batch (if any) whose window is re-seeded
    for (int b2 = 0; b2 < B; ++b2)
      if ((w0 + b2) % reseed == 0) seed_step = b2;
    hipLaunchKernelGGL((k_stream_col0<Tin>), dim3((unsigned)B), dim3(64), 0, st, s, T, m, w0);
    hipLaunchKernelGGL((k_stream_batch<Tin>), dim3((unsigned)nblocks), dim3(kStreamBlock), 0, st, s, T, m, ez, w0,
                       B, seed_step, (const double *)s.C[(w0 - 1) & 1], s.C[(w0 + B - 1) & 1], I, nparts);
    hipLaunchKernelGGL(k_stream_rowfin, dim3((unsigned)B), dim3(256), 0, st, s, w0, nparts, I);
    w0 += B;
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

hipError_t launch_stream_out(const StreamWork &s, int64_t l, int m, void *P, bool out_f64, hipStream_t st) {
  const dim3 b(256), g((unsigned)((l + 255) / 256));
  if (out_f64) hipLaunchKernelGGL((k_stream_out<double>), g, b, 0, st, s, l, m, (double *)P);
  else hipLaunchKernelGGL((k_stream_out<float>), g, b, 0, st, s, l, m, (float *)P);
  return hipGetLastError();
}

}  // namespace mpx
