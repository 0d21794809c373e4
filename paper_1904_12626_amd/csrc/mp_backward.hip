// Backward pass of a loss through the matrix profile, holding the index
// fixed: for every row i with neighbour j = I[i] and upstream gradient g,
//   d P_i / d T[i+u] = (rho z_i[u] - z_j[u]) / (sigma_i d),
//   d P_i / d T[j+u] = (rho z_j[u] - z_i[u]) / (sigma_j d),
// with z the z-normalised windows, d = ||z_i - z_j|| and rho = z_i.z_j / m
// (differentiating d through z = (x - mean)/sigma, whose Jacobian is
// (Id - 11^T/m - z z^T/m)/sigma).  Contributions are accumulated in FP64
// with atomics and converted to the output type at the end.
#include <cmath>

#include "mp_internal.h"
#include "mp_types.h"

namespace mpx {

namespace {

template <typename Tin>
__device__ __forceinline__ double sample_b(const Tin *p) {
  const double v = (double)*p;
  return isfinite(v) ? v : 0.0;
}

__device__ __forceinline__ int find_series_b(const Plan &plan, int64_t wi) {
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

template <typename Tin>
__device__ bool win_stats(const Tin *x, int m, double &mu, double &sg) {
  double s = 0.0, lo = 0.0, hi = 0.0;
  for (int u = 0; u < m; ++u) {
    const double v = (double)x[u];
    if (!isfinite(v)) return false;
    if (u == 0) { lo = v; hi = v; }
    lo = fmin(lo, v);
    hi = fmax(hi, v);
    s += v;
  }
  if (lo == hi) return false;  // constant window: subgradient 0
  mu = s / m;
  double q = 0.0;
  for (int u = 0; u < m; ++u) {
    const double dv = (double)x[u] - mu;
    q = fma(dv, dv, q);
  }
  sg = sqrt(q / m);
  return sg > 0.0;
}

}  // namespace

__global__ void __launch_bounds__(256) k_zero64(double *p, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    p[x] = 0.0;
}

template <typename Tin, typename Tg>
__global__ void __launch_bounds__(256) k_grad_rows(Plan plan, Work wk, const Tin *__restrict__ Tb,
                                                   const int64_t *__restrict__ I,
                                                   const Tg *__restrict__ gP, int64_t total_l) {
  const int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= total_l) return;
  const SeriesDesc S = plan.series(find_series_b(plan, wi));
  const int64_t i = wi - S.w_off;
  const int64_t j = I[wi];
  const double g = (double)gP[wi];
  if (j < 0 || j >= S.l || g == 0.0 || !isfinite(g)) return;
  const Tin *xi = Tb + S.t_off + i;
  const Tin *xj = Tb + S.t_off + j;
  const int m = S.m;
  double mi, si, mj, sj;
  if (!win_stats(xi, m, mi, si) || !win_stats(xj, m, mj, sj)) return;
  double d2 = 0.0, c = 0.0;
  for (int u = 0; u < m; ++u) {
    const double zi = ((double)xi[u] - mi) / si, zj = ((double)xj[u] - mj) / sj;
    d2 = fma(zi - zj, zi - zj, d2);
    c = fma(zi, zj, c);
  }
  const double d = sqrt(d2);
  if (!(d > 0.0)) return;
  const double rho = c / m;
  const double ci = g / (si * d), cj = g / (sj * d);
  double *gi = wk.grad + S.t_off + i, *gj = wk.grad + S.t_off + j;
  for (int u = 0; u < m; ++u) {
    const double zi = ((double)xi[u] - mi) / si, zj = ((double)xj[u] - mj) / sj;
    atomicAdd(gi + u, ci * (rho * zi - zj));
    atomicAdd(gj + u, cj * (rho * zj - zi));
  }
}

template <typename Tg>
__global__ void __launch_bounds__(256) k_grad_out(const double *__restrict__ acc, Tg *out, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    out[x] = (Tg)acc[x];
}

hipError_t launch_backward(const Plan &plan, const Work &w, const void *T, bool t_f64,
                           const int64_t *I, const void *gP, void *gT, int64_t total_l,
                           int64_t total_n, hipStream_t st) {
  const dim3 blk(256);
  const unsigned gz = (unsigned)std::min<int64_t>((total_n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_zero64, dim3(gz), blk, 0, st, w.grad, total_n);
  const dim3 grd((unsigned)((total_l + 255) / 256));
  if (t_f64)
    hipLaunchKernelGGL((k_grad_rows<double, double>), grd, blk, 0, st, plan, w, (const double *)T, I, (const double *)gP, total_l);
  else
    hipLaunchKernelGGL((k_grad_rows<float, float>), grd, blk, 0, st, plan, w, (const float *)T, I, (const float *)gP, total_l);
  if (t_f64)
    hipLaunchKernelGGL((k_grad_out<double>), dim3(gz), blk, 0, st, w.grad, (double *)gT, total_n);
  else
    hipLaunchKernelGGL((k_grad_out<float>), dim3(gz), blk, 0, st, w.grad, (float *)gT, total_n);
  return hipGetLastError();
}

}  // namespace mpx
