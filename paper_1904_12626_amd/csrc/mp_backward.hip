// Backward pass of a loss through the matrix profile, holding the index
// fixed: for every row i with neighbour j = I[i] and upstream gradient g,
//   d P_i / d T[i+u] = (rho z_i[u] - z_j[u]) / (sigma_i d),
//   d P_i / d T[j+u] = (rho z_j[u] - z_i[u]) / (sigma_j d),
// with z the z-normalised windows, d = ||z_i - z_j|| and rho = z_i.z_j / m
// (differentiating d through z = (x - mean)/sigma, whose Jacobian is
// (Id - 11^T/m - z z^T/m)/sigma).
//
// Deterministic gather: each row's contribution is four coefficients
//   on window i:  alpha z_i + beta z_j,   alpha = g rho/(sigma_i d), beta = -g/(sigma_i d)
//   on window j:  gamma z_j + delta z_i,  gamma = g rho/(sigma_j d), delta = -g/(sigma_j d)
// Rows are bucketed by their neighbour j (counting sort, each bucket then
// ordered by row index), and every output sample sums, in a fixed order, the rows
// whose own window covers it and the rows whose neighbour window covers it.
// No floating-point atomics: reruns are bitwise identical.
#include <cmath>

#include "mp_internal.h"
#include "mp_types.h"

namespace mpx {

namespace {

__device__ __forceinline__ int find_series_by_w(const Plan &plan, int64_t wi) {
  if (plan.s_ext) {
    int lo = 0, hi = plan.nseries - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (plan.s_ext[mid].w_off <= wi) lo = mid; else hi = mid - 1;
    }
    return lo;
  }
  return (plan.nseries > 1 && wi >= plan.s_inl[1].w_off) ? 1 : 0;
}

__device__ __forceinline__ int find_series_by_t(const Plan &plan, int64_t x) {
  if (plan.s_ext) {
    int lo = 0, hi = plan.nseries - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (plan.s_ext[mid].t_off <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
  }
  return (plan.nseries > 1 && x >= plan.s_inl[1].t_off) ? 1 : 0;
}

}  // namespace

// Window statistics for the gradient: mean and 1/sigma (0 for constant or
// non-finite windows, whose rows and neighbours contribute nothing).
template <typename Tin>
__global__ void __launch_bounds__(256) k_bwd_stats(Plan plan, BwdWork b, const Tin *__restrict__ Tb,
                                                   int64_t total_l) {
  const int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= total_l) return;
  const SeriesDesc S = plan.series(find_series_by_w(plan, wi));
  const Tin *x = Tb + S.t_off + (wi - S.w_off);
  const int m = S.m;
  double s = 0.0, lo = 0.0, hi = 0.0;
  bool ok = true;
  for (int u = 0; u < m; ++u) {
    const double v = (double)x[u];
    if (!isfinite(v)) ok = false;
    if (u == 0) { lo = v; hi = v; }
    lo = fmin(lo, v);
    hi = fmax(hi, v);
    s += v;
  }
  const double mu = s / m;
  double q = 0.0;
  for (int u = 0; u < m; ++u) {
    const double dv = (double)x[u] - mu;
    q = fma(dv, dv, q);
  }
  const double sg = sqrt(q / m);
  b.mu[wi] = ok ? mu : 0.0;
  b.isig[wi] = (ok && lo != hi && sg > 0.0) ? 1.0 / sg : 0.0;
  b.count[wi] = 0;
  b.fill[wi] = 0;
}

// Per-row coefficients; counts rows per neighbour window.
template <typename Tin, typename Tg>
__global__ void __launch_bounds__(256) k_bwd_coef(Plan plan, BwdWork b, const Tin *__restrict__ Tb,
                                                  const int64_t *__restrict__ I,
                                                  const Tg *__restrict__ gP, int64_t total_l) {
  // z_i - z_j must be exactly 0 for identical windows (d == 0 takes the
  // subgradient 0): no contraction of the products into the subtraction.
#pragma clang fp contract(off)
  const int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= total_l) return;
  const SeriesDesc S = plan.series(find_series_by_w(plan, wi));
  const int64_t i = wi - S.w_off;
  const int64_t j = I[wi];
  const double g = (double)gP[wi];
  Double4 c{0.0, 0.0, 0.0, 0.0};
  int64_t jw = -1;
  if (j >= 0 && j < S.l && j != i && g != 0.0 && isfinite(g)) {
    jw = S.w_off + j;
    const double isi = b.isig[wi], isj = b.isig[jw];
    if (isi > 0.0 && isj > 0.0) {
      const Tin *xi = Tb + S.t_off + i;
      const Tin *xj = Tb + S.t_off + j;
      const double mi = b.mu[wi], mj = b.mu[jw];
      double d2 = 0.0, dot = 0.0;
      for (int u = 0; u < S.m; ++u) {
        const double zi = ((double)xi[u] - mi) * isi, zj = ((double)xj[u] - mj) * isj;
        d2 = fma(zi - zj, zi - zj, d2);
        dot = fma(zi, zj, dot);
      }
      const double d = sqrt(d2);
      if (d > 0.0) {
        const double rho = dot / S.m;
        c = Double4{g * rho * isi / d, -g * isi / d, g * rho * isj / d, -g * isj / d};
      }
    }
  }
  reinterpret_cast<Double4 *>(b.coef)[wi] = c;
  const bool live = (c.x != 0.0 || c.y != 0.0 || c.z != 0.0 || c.w != 0.0);
  b.nbr[wi] = live ? jw : -1;
  if (live) atomicAdd(&b.count[jw], 1);
}

// Exclusive prefix sum of count[0..n) into off[0..n]: one workgroup per
// chunk of 1024 entries, then a single workgroup over the chunk totals, then
// the chunk offsets are added back.
__global__ void __launch_bounds__(1024) k_scan_chunks(const int32_t *__restrict__ cnt, int64_t *off,
                                                      int64_t *chunk_tot, int64_t n) {
  __shared__ int64_t sh[1024];
  const int64_t x = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int64_t v = x < n ? cnt[x] : 0;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t add = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  if (x < n) off[x] = sh[threadIdx.x] - v;
  if (threadIdx.x == 1023) chunk_tot[blockIdx.x] = sh[1023];
}

__global__ void __launch_bounds__(1024) k_scan_totals(int64_t *chunk_tot, int64_t nchunks, int64_t *off,
                                                      int64_t n) {
  __shared__ int64_t part[1024];
  const int tid = threadIdx.x;
  const int64_t per = (nchunks + 1023) / 1024;
  const int64_t a = min(nchunks, (int64_t)tid * per), e = min(nchunks, a + per);
  int64_t s = 0;
  for (int64_t c = a; c < e; ++c) s += chunk_tot[c];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    int64_t run = 0;
    for (int q = 0; q < 1024; ++q) {
      const int64_t v = part[q];
      part[q] = run;
      run += v;
    }
    off[n] = run;
  }
  __syncthreads();
  int64_t run = part[tid];
  for (int64_t c = a; c < e; ++c) {
    const int64_t v = chunk_tot[c];
    chunk_tot[c] = run;
    run += v;
  }
}

__global__ void __launch_bounds__(1024) k_scan_add(int64_t *off, const int64_t *__restrict__ chunk_tot,
                                                   int64_t n) {
  const int64_t x = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (x < n) off[x] += chunk_tot[blockIdx.x];
}

// Bucket the live rows by neighbour window (arbitrary order within a bucket).
__global__ void __launch_bounds__(256) k_bwd_place(BwdWork b, int64_t total_l) {
  const int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= total_l) return;
  const int64_t jw = b.nbr[wi];
  if (jw < 0) return;
  const int pos = atomicAdd(&b.fill[jw], 1);
  b.tmp[b.off[jw] + pos] = wi;
}

// Deterministic order within each bucket: a row's slot is the number of rows
// of its bucket with a smaller index.
__global__ void __launch_bounds__(256) k_bwd_rank(BwdWork b, int64_t total_l) {
  const int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= total_l) return;
  const int64_t jw = b.nbr[wi];
  if (jw < 0) return;
  const int64_t a = b.off[jw], e = b.off[jw + 1];
  int64_t r = 0;
  for (int64_t p = a; p < e; ++p) r += b.tmp[p] < wi;
  b.rows[a + r] = wi;
}

// One output sample: contributions of the rows whose window covers it and of
// the rows whose neighbour window covers it, in increasing window order.
template <typename Tin, typename Tg>
__global__ void __launch_bounds__(256) k_bwd_gather(Plan plan, BwdWork b, const Tin *__restrict__ Tb,
                                                    Tg *gT, int64_t total_n) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= total_n) return;
  const SeriesDesc S = plan.series(find_series_by_t(plan, x));
  const int64_t t = x - S.t_off;
  const int m = S.m;
  const double xt = (double)Tb[x];
  const int64_t w_lo = max((int64_t)0, t - m + 1), w_hi = min(t, S.l - 1);
  double acc = 0.0;
  for (int64_t w = w_lo; w <= w_hi; ++w) {
    const int64_t wi = S.w_off + w;
    // row w's own window covers t
    const int64_t jw = b.nbr[wi];
    if (jw >= 0) {
      const Double4 c = reinterpret_cast<const Double4 *>(b.coef)[wi];
      const int64_t u = t - w;
      const double zi = (xt - b.mu[wi]) * b.isig[wi];
      const double zj = ((double)Tb[S.t_off + (jw - S.w_off) + u] - b.mu[jw]) * b.isig[jw];
      acc = fma(c.x, zi, acc);
      acc = fma(c.y, zj, acc);
    }
    // rows whose neighbour is window w
    const int64_t a = b.off[wi], e = b.off[wi + 1];
    if (a < e) {
      const double zw = (xt - b.mu[wi]) * b.isig[wi];
      const int64_t u = t - w;
      for (int64_t p = a; p < e; ++p) {
        const int64_t ri = b.rows[p];
        const Double4 c = reinterpret_cast<const Double4 *>(b.coef)[ri];
        const double zr = ((double)Tb[S.t_off + (ri - S.w_off) + u] - b.mu[ri]) * b.isig[ri];
        acc = fma(c.z, zw, acc);
        acc = fma(c.w, zr, acc);
      }
    }
  }
  gT[x] = (Tg)acc;
}

hipError_t launch_backward(const Plan &plan, const BwdWork &b, const void *T, bool t_f64,
                           const int64_t *I, const void *gP, void *gT, int64_t total_l,
                           int64_t total_n, hipStream_t st) {
  const dim3 blk(256);
  const dim3 gl((unsigned)((total_l + 255) / 256)), gn((unsigned)((total_n + 255) / 256));
  const int64_t nchunks = (total_l + 1023) / 1024;
  if (t_f64) {
    hipLaunchKernelGGL((k_bwd_stats<double>), gl, blk, 0, st, plan, b, (const double *)T, total_l);
    hipLaunchKernelGGL((k_bwd_coef<double, double>), gl, blk, 0, st, plan, b, (const double *)T, I,
                       (const double *)gP, total_l);
  } else {
    hipLaunchKernelGGL((k_bwd_stats<float>), gl, blk, 0, st, plan, b, (const float *)T, total_l);
    hipLaunchKernelGGL((k_bwd_coef<float, float>), gl, blk, 0, st, plan, b, (const float *)T, I,
                       (const float *)gP, total_l);
  }
  hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nchunks), dim3(1024), 0, st, (const int32_t *)b.count,
                     b.off, b.chunk, total_l);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, st, b.chunk, nchunks, b.off, total_l);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nchunks), dim3(1024), 0, st, b.off, (const int64_t *)b.chunk,
                     total_l);
  hipLaunchKernelGGL(k_bwd_place, gl, blk, 0, st, b, total_l);
  hipLaunchKernelGGL(k_bwd_rank, gl, blk, 0, st, b, total_l);
  if (t_f64)
    hipLaunchKernelGGL((k_bwd_gather<double, double>), gn, blk, 0, st, plan, b, (const double *)T,
                       (double *)gT, total_n);
  else
    hipLaunchKernelGGL((k_bwd_gather<float, float>), gn, blk, 0, st, plan, b, (const float *)T, (float *)gT,
                       total_n);
  return hipGetLastError();
}

}  // namespace mpx
