// Preparation kernels: the tile table of the diagonal sweep, per-window
// statistics (z-normalisation terms) and the suffix tables used to resolve
// constant and invalid windows.
#include <cmath>

#include "mp_internal.h"
#include "mp_types.h"

namespace mpx {

// The exponent e of the power of two 2^e that brings the spread of 32
// evenly spaced samples of a series (their largest distance from the first
// finite one) into [2^48, 2^49); 0 when they do not spread.  A window's
// spread is at most about that, so the sweep's cross products (m sigma^2)
// stay a thousand times below FP32's maximum for windows up to 2^20
// samples, while windows up to 10^33 times smaller still keep their
// increments above FP32's smallest normal number.  Clamped to [-500, 500],
// so that a scale, its inverse and the product of two stay finite.
template <typename Tin>
__device__ __forceinline__ void scale_samples(const Tin *x, int64_t n, Tin (&v)[32]) {
#pragma unroll
  for (int k = 0; k < 32; ++k) v[k] = x[(n - 1) * k / 31];  // all in flight at once
}
template <typename Tin>
__device__ int scale_exp_of(const Tin (&v)[32]) {
  double ref = 0.0, spread = 0.0;
  bool have = false;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const double d = (double)v[k];
    if (!isfinite(d)) continue;
    if (!have) {
      ref = d;
      have = true;
    }
    spread = fmax(spread, fabs(d - ref));
  }
  return (spread > 0.0 && isfinite(spread)) ? max(-500, min(500, 48 - ilogb(spread))) : 0;
}

// ------------------------------------------------------------------ plan
// Strip g of sweep s covers diagonals [k_lo + (g - seg_base) * W, +W); its
// longest diagonal has min(l_rows, l_cols - k0) cells, cut into tiles of R
// rows.  One workgroup writes the tile table (exclusive prefix sums) and
// clears the per-call counters.  Without seg_part the tiles are numbered
// strip by strip; with it, every full-height tile comes first (strip by
// strip) and the shorter last tiles of the strips after them, so that the
// persistent grid ends on short tiles (longest first).
// It also sets each series' scale for the sweep's records (when the job has
// them: w.scale); a thread's first series has its samples loaded before the
// table is built and its scale set after it, so that the loads' latency
// overlaps the table.
template <typename Tin>
__global__ void __launch_bounds__(1024) k_plan(Plan plan, Work w, const Tin *__restrict__ Tb, int W, int R,
                                               int64_t nseg) {
  __shared__ int64_t wpart[16], wpart2[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid < 4) w.counters[tid] = 0;
  const bool first = w.scale != nullptr && tid < plan.nseries;
  Tin smp[32];
  if (first) {
    const SeriesDesc S = plan.series(tid);
    scale_samples(series_samples(plan, Tb, S), S.n, smp);
  }
  for (int s = tid; s < plan.nseries; s += blockDim.x) {
    w.special[s] = 0;
    if (w.scale && s != tid) {
      const SeriesDesc S = plan.series(s);
      Tin v[32];
      scale_samples(series_samples(plan, Tb, S), S.n, v);
      w.scale[s] = ldexp(1.0, scale_exp_of(v));
    }
  }
  const bool lpt = w.seg_part != nullptr;

  const int64_t per = (nseg + blockDim.x - 1) / blockDim.x;
  const int64_t a = min(nseg, (int64_t)tid * per), b = min(nseg, a + per);
  // sweep holding strip a: the last one whose first strip is <= a
  int sw0 = 0;
  {
    int lo = 0, hi = plan.nsweeps - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (plan.sweep(mid).seg_base <= a) lo = mid; else hi = mid - 1;
    }
    sw0 = lo;
  }
  // The fields of the current sweep that a strip needs, reloaded only when
  // the strip is in the next sweep (a thread's strips are consecutive, so
  // mostly in one sweep): no chain of descriptor loads per strip.
  int sw;
  int64_t next_base, k_lo, seg_base, rl, cl;
  auto enter = [&](int s) {
    sw = s;
    const SweepDesc d = plan.sweep(s);
    next_base = s + 1 < plan.nsweeps ? plan.sweep(s + 1).seg_base : INT64_MAX;
    k_lo = d.k_lo;
    seg_base = d.seg_base;
    rl = plan.series(d.rs).l;
    cl = plan.series(d.cs).l;
  };
  // (full-height tiles, shorter last tile) of strip g, or (all tiles, 0);
  // a 32-bit division when the strip's length allows (64-bit division is a
  // long software sequence)
  auto tiles_of = [&](int64_t g, int64_t &t2) -> int64_t {
    while (next_base <= g) enter(sw + 1);
    const int64_t k0 = k_lo + (g - seg_base) * (int64_t)W;
    const int64_t L = min(rl, cl - k0);
    int64_t q;
    if (L >= 0 && L <= 0x7fffffff) {
      q = (int64_t)((uint32_t)L / (uint32_t)R);
    } else {
      q = L / R;
    }
    const bool part_tile = L - q * R != 0;
    if (!lpt) {
      t2 = 0;
      return q + (part_tile ? 1 : 0);
    }
    t2 = part_tile ? 1 : 0;
    return q;
  };
  int64_t sum = 0, sum2 = 0;
  if (a < b) enter(sw0);
  for (int64_t g = a; g < b; ++g) {
    int64_t t2;
    sum += tiles_of(g, t2);
    sum2 += t2;
  }
  // inclusive scan over the threads: within each wave by shuffles, then
  // the totals of the waves before it (16 waves of 64), then exclusive
  int64_t x = sum, x2 = sum2;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = __shfl_up(x, d, 64), y2 = __shfl_up(x2, d, 64);
    if (lane >= d) {
      x += y;
      x2 += y2;
    }
  }
  if (lane == 63) {
    wpart[wv] = x;
    wpart2[wv] = x2;
  }
  __syncthreads();
  for (int k = 0; k < wv; ++k) {
    x += wpart[k];
    x2 += wpart2[k];
  }
  if (tid == (int)blockDim.x - 1) {
    w.seg_prefix[nseg] = x;
    if (lpt) w.seg_part[nseg] = x2;
  }
  int64_t run = x - sum, run2 = x2 - sum2;
  if (a < b) enter(sw0);
  for (int64_t g = a; g < b; ++g) {
    int64_t t2;
    const int64_t t = tiles_of(g, t2);
    w.seg_prefix[g] = run;
    w.seg_sweep[g] = sw;
    if (lpt) w.seg_part[g] = run2;
    run += t;
    run2 += t2;
  }
  if (first) w.scale[tid] = ldexp(1.0, scale_exp_of(smp));
}

hipError_t launch_plan(const Plan &plan, const Work &w, const void *T, bool t_f64, int W, int R, int64_t nseg,
                       hipStream_t st) {
  if (t_f64)
    hipLaunchKernelGGL((k_plan<double>), dim3(1), dim3(1024), 0, st, plan, w, (const double *)T, W, R, nseg);
  else
    hipLaunchKernelGGL((k_plan<float>), dim3(1), dim3(1024), 0, st, plan, w, (const float *)T, W, R, nseg);
  return hipGetLastError();
}

// ---------------------------------------------------------------- stats
// Window i of a series, with x = T where finite and 0 elsewhere:
//   mu_i, sigma_i  two-pass FP64 mean and population std of x[i:i+m]
//   a_i = x[i+m] - x[i]                       (0 for the last window)
//   g_i = x[i] - mu_i + a_i (m-1)/(2m)
//   s_i = 1 / (sqrt(m) sigma_i)   (0 for constant or invalid windows)
//   u_i = 1 (valid), 1/2 (constant), 4 (invalid)
// The centred cross product C(i,j) = sum_t (x[i+t]-mu_i)(x[j+t]-mu_j) then
// obeys C(i+1,j+1) = C(i,j) + a_j g_i + a_i g_j exactly (expand
// x[i+m] = x[i] + a_i and mu_{i+1} = mu_i + a_i/m), and the sweep's key
// u_i - C s_i s_j equals 1 - rho(i,j) for valid windows.
// The records store a and g times the series' power of two k (set by k_plan)
// and s divided by it (the sweep multiplies its seeds of C by the k of both
// series): no key changes, since power-of-two factors commute with rounding,
// but the cross products of series with very large or very small values stay
// well inside FP32's range.

// Series owning padded row/column entry r.
__device__ __forceinline__ int series_of_rc(const Plan &plan, int64_t r) {
  if (plan.s_ext) {
    int lo = 0, hi = plan.nseries - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (plan.s_ext[mid].rc_off <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
  }
  return (plan.nseries > 1 && r >= plan.s_inl[1].rc_off) ? 1 : 0;
}

// A workgroup's 256 entries usually lie in one series: their samples (and
// the one after each window, for a_i) are then staged once in LDS.
constexpr int kStatsTile = 256;
constexpr int kStatsTileM = 2048;

template <typename F, typename Tin>
__global__ void __launch_bounds__(256) k_stats(Plan plan, Work w, const Tin *__restrict__ Tb,
                                               int64_t total_rc) {
  __shared__ Tin xs[kStatsTile + kStatsTileM + 1];
  const int64_t r0 = (int64_t)blockIdx.x * kStatsTile;
  const int64_t r = r0 + threadIdx.x;
  const int s0 = series_of_rc(plan, r0);
  const SeriesDesc S0 = plan.series(s0);
  const int64_t i0 = r0 - S0.rc_off;
  const bool tiled = S0.m <= kStatsTileM && s0 == series_of_rc(plan, min(r0 + kStatsTile, total_rc) - 1);
  if (tiled && i0 < S0.l) {
    const Tin *base = series_samples(plan, Tb, S0) + i0;
    const int cnt = (int)min((int64_t)(kStatsTile + S0.m), S0.n - i0);
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) xs[t] = base[t];
  }
  __syncthreads();
  if (r >= total_rc) return;
  const int si = tiled ? s0 : series_of_rc(plan, r);
  const SeriesDesc S = tiled ? S0 : plan.series(si);
  const int64_t i = r - S.rc_off;
  using V4 = typename FTraits<F>::V4;
  V4 *rc = reinterpret_cast<V4 *>(w.rc);
  if (i >= S.l) {
    // padding past the last window: as a row its huge u makes every key
    // huge (never a minimum); as a column its s = 0 scores like rho = 0, and
    // a row whose minimum lands there is rescanned exactly (k_finalize)
    rc[r] = FTraits<F>::pad4();
    return;
  }
  const Tin *x = series_samples(plan, Tb, S) + i;
  const int m = S.m;
  // Common case: every sample finite (then the sum is finite unless finite
  // samples overflow).  Otherwise the careful pass below zeroes non-finite
  // samples; both give the same mean and spread for finite windows.  The
  // body is instantiated once for the LDS tile and once for global memory.
  bool fin = true, cst;
  double mu, q = 0.0, x0, xm = 0.0;
  auto body = [&](auto at) {
    const Tin v0 = at(0);
    double s = 0.0;
    bool same = true;
#pragma unroll 4
    for (int u = 0; u < m; ++u) {
      const Tin v = at(u);
      same &= (v == v0);
      s += (double)v;
    }
    cst = same;
    if (isfinite(s)) {
      mu = s / m;
#pragma unroll 4
      for (int u = 0; u < m; ++u) {
        const double dv = (double)at(u) - mu;
        q = fma(dv, dv, q);
      }
    } else {
      double lo = 0.0, hi = 0.0;
      s = 0.0;
      for (int u = 0; u < m; ++u) {
        double v = (double)at(u);
        if (!isfinite(v)) { fin = false; v = 0.0; }
        if (u == 0) { lo = v; hi = v; }
        lo = fmin(lo, v);
        hi = fmax(hi, v);
        s += v;
      }
      mu = s / m;
      for (int u = 0; u < m; ++u) {
        double v = (double)at(u);
        if (!isfinite(v)) v = 0.0;
        const double dv = v - mu;
        q = fma(dv, dv, q);
      }
      cst = fin && (lo == hi);
    }
    x0 = (double)v0;
    if (i + m < S.n) xm = (double)at(m);
  };
  if (tiled) {
    const Tin *xl = xs + (i - i0);
    body([&](int u) { return xl[u]; });
  } else {
    body([&](int u) { return x[u]; });
  }
  const double sig = sqrt(q / m);
  if (!isfinite(x0)) x0 = 0.0;
  double a = 0.0;
  if (i + m < S.n) {
    if (!isfinite(xm)) xm = 0.0;
    a = xm - x0;
  }
  const double g = (x0 - mu) + a * ((double)(m - 1) / (2.0 * m));
  const double sc = (fin && !cst && sig > 0.0) ? 1.0 / (sqrt((double)m) * sig) : 0.0;
  const double uu = fin ? (cst ? 0.5 : 1.0) : 4.0;
  const double k = w.scale[si], kinv = ldexp(1.0, -ilogb(k));  // the series' power of two (k_plan)
  const int64_t wi = S.w_off + i;
  w.mu[wi] = mu;
  w.sig[wi] = sig;
  w.flags[wi] = (uint8_t)((fin ? 1 : 0) | (cst ? 2 : 0));
  w.keys[wi] = ~0ull;
  rc[r] = FTraits<F>::make4(a * k, g * k, sc * kinv, uu);
  const int bits = (fin ? 0 : 1) | (cst ? 2 : 0);
  if (bits) atomicOr(&w.special[si], bits);
}

hipError_t launch_stats(const Plan &plan, const Work &w, const void *T, bool t_f64, bool f64_sweep,
                        int64_t total_rc, hipStream_t st) {
  const dim3 blk(kStatsTile), grd((unsigned)((total_rc + kStatsTile - 1) / kStatsTile));
  if (t_f64) {
    if (f64_sweep)
      hipLaunchKernelGGL((k_stats<double, double>), grd, blk, 0, st, plan, w, (const double *)T, total_rc);
    else
      hipLaunchKernelGGL((k_stats<float, double>), grd, blk, 0, st, plan, w, (const double *)T, total_rc);
  } else {
    if (f64_sweep)
      hipLaunchKernelGGL((k_stats<double, float>), grd, blk, 0, st, plan, w, (const float *)T, total_rc);
    else
      hipLaunchKernelGGL((k_stats<float, float>), grd, blk, 0, st, plan, w, (const float *)T, total_rc);
  }
  return hipGetLastError();
}

// -------------------------------------------------------------- special
// For a series with constant or invalid windows: next_const[x] / next_valid[x]
// = smallest constant / valid window index >= x, or l if none (x in [0, l]).
// One workgroup per series; it exits at once when the series has neither.
__global__ void __launch_bounds__(1024) k_special(Plan plan, Work w) {
  const int si = blockIdx.x;
  if (w.special[si] == 0) return;
  const SeriesDesc S = plan.series(si);
  __shared__ int32_t cmin[1024], vmin[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t l = S.l;
  const int64_t per = (l + nt - 1) / nt;
  const int64_t a = min(l, (int64_t)tid * per), b = min(l, a + per);
  int32_t fc = (int32_t)l, fv = (int32_t)l;
  for (int64_t x = b - 1; x >= a; --x) {
    const uint8_t f = w.flags[S.w_off + x];
    if (f & 1) fv = (int32_t)x;
    if (f & 2) fc = (int32_t)x;
  }
  cmin[tid] = fc;
  vmin[tid] = fv;
  __syncthreads();
  if (tid == 0) {  // suffix minimum over the chunks, shifted by one chunk
    int32_t rc = (int32_t)l, rv = (int32_t)l;
    for (int q = nt - 1; q >= 0; --q) {
      const int32_t c = cmin[q], v = vmin[q];
      cmin[q] = rc;
      vmin[q] = rv;
      rc = min(rc, c);
      rv = min(rv, v);
    }
  }
  __syncthreads();
  int32_t nc = cmin[tid], nv = vmin[tid];
  for (int64_t x = b - 1; x >= a; --x) {
    const uint8_t f = w.flags[S.w_off + x];
    if (f & 1) nv = (int32_t)x;
    if (f & 2) nc = (int32_t)x;
    w.next_const[S.x_off + x] = nc;
    w.next_valid[S.x_off + x] = nv;
  }
  if (tid == 0) {
    w.next_const[S.x_off + l] = (int32_t)l;
    w.next_valid[S.x_off + l] = (int32_t)l;
  }
}

hipError_t launch_special(const Plan &plan, const Work &w, hipStream_t st) {
  hipLaunchKernelGGL(k_special, dim3(plan.nseries), dim3(1024), 0, st, plan, w);
  return hipGetLastError();
}

}  // namespace mpx
