// Backward pass of a loss through the matrix profile, holding the index
// fixed: for every row i with neighbour j = I[i] (a window of the same
// series for a self-join, of the other series for an AB-join) and upstream
// gradient g,
//   d P_i / d T[i+u] = (rho z_i[u] - z_j[u]) / (sigma_i d),
//   d P_i / d T[j+u] = (rho z_j[u] - z_i[u]) / (sigma_j d),
// with z the z-normalised windows, d = ||z_i - z_j|| and rho = z_i.z_j / m
// (differentiating d through z = (x - mean)/sigma, whose Jacobian is
// (Id - 11^T/m - z z^T/m)/sigma).
//
// Deterministic gather: each row's contribution is four coefficients
//   on window i:  alpha z_i + beta z_j,   alpha = g rho/(sigma_i d), beta = -g/(sigma_i d)
//   on window j:  gamma z_j + delta z_i,  gamma = g rho/(sigma_j d), delta = -g/(sigma_j d)
// Per destination window w, the multiples of z_w (its own alpha and the
// gammas of the rows whose neighbour is w) are summed in a fixed order; its
// row's beta term is the window's own edge, and the delta terms of the rows
// naming w are its bucket edges, in increasing row order.  A wave then
// produces 64 consecutive gradient samples by walking the windows that cover
// them in order, with the window and edge records uniform across the wave
// and the source samples loaded contiguously.  No floating-point atomics:
// reruns are bitwise identical.
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

// The samples of a workgroup's 256 consecutive windows, staged once in LDS
// (256 + m - 1 values) when the windows lie in one series and m <= kTileM;
// otherwise the kernels read the series directly.  Either way every window
// sees the same values, so results do not depend on the staging.
constexpr int kTileW = 256;
constexpr int kTileM = 2048;

// Returns whether the tile was staged; s0 = the series of the first window.
template <typename Tin>
__device__ __forceinline__ bool stage_tile(const Plan &plan, const Tin *__restrict__ Tb, int64_t total_l,
                                           double *xs, int &s0) {
  const int64_t w0 = (int64_t)blockIdx.x * kTileW;
  const int64_t wl = min(w0 + kTileW - 1, total_l - 1);
  s0 = find_series_by_w(plan, w0);
  const SeriesDesc S = plan.series(s0);
  if (s0 != find_series_by_w(plan, wl) || S.m > kTileM) return false;
  const Tin *base = series_samples(plan, Tb, S) + (w0 - S.w_off);
  const int cnt = (int)(wl - w0) + S.m;
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) xs[t] = (double)base[t];
  __syncthreads();
  return true;
}

// Window statistics for the gradient: mean and 1/sigma (0 for constant or
// non-finite windows, whose rows and neighbours contribute nothing).
template <typename Tin>
__global__ void __launch_bounds__(256) k_bwd_stats(Plan plan, BwdWork b, const Tin *__restrict__ Tb,
                                                   int64_t total_l) {
  __shared__ double xs[kTileW + kTileM];
  int s0;
  const bool tiled = stage_tile(plan, Tb, total_l, xs, s0);
  const int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wi == 0) *b.nbig = 0ull;
  if (wi >= total_l) return;
  const SeriesDesc S = plan.series(tiled ? s0 : find_series_by_w(plan, wi));
  const Tin *x = series_samples(plan, Tb, S) + (wi - S.w_off);
  const int m = S.m;
  double mu, sg;
  bool same = true, ok;
  // instantiated once for the LDS tile and once for global memory
  auto body = [&](auto at) {
    const double v0 = at(0);
    double s = 0.0;
#pragma unroll 4
    for (int u = 0; u < m; ++u) {
      const double v = at(u);
      same &= (v == v0);  // every sample equal to the first: a constant window
      s += v;
    }
    // A non-finite sample makes the sum non-finite; a sum that is not finite
    // only because finite samples overflowed is told apart sample by sample.
    ok = isfinite(s);
    if (!ok) {
      ok = true;
      for (int u = 0; u < m; ++u) ok &= (bool)isfinite(at(u));
    }
    mu = s / m;
    double q = 0.0;
#pragma unroll 4
    for (int u = 0; u < m; ++u) {
      const double dv = at(u) - mu;
      q = fma(dv, dv, q);
    }
    sg = sqrt(q / m);
  };
  if (tiled) {
    const double *xl = xs + threadIdx.x;
    body([&](int u) { return xl[u]; });
  } else {
    body([&](int u) { return (double)x[u]; });
  }
  b.mu[wi] = ok ? mu : 0.0;
  b.isig[wi] = (ok && !same && sg > 0.0) ? 1.0 / sg : 0.0;
  b.count[wi] = 0ull;
}

// Per-row coefficients: row i's alpha and window record (its mean, its own
// edge) and, for a contributing row, its bucket edge and gamma on the
// neighbour window, and its arrival position in that window's bucket.
template <typename Tin, typename Tg>
__global__ void __launch_bounds__(256, sizeof(Tin) == 4 ? 7 : 6) k_bwd_coef(Plan plan, BwdWork b, const Tin *__restrict__ Tb,
                                                  const int64_t *__restrict__ I,
                                                  const Tg *__restrict__ gP, int64_t total_l) {
  // z_i - z_j must be exactly 0 for identical windows (d == 0 takes the
  // subgradient 0): no contraction of the products into the subtraction.
#pragma clang fp contract(off)
  __shared__ double xs[kTileW + kTileM];
  int s0;
  const bool tiled = stage_tile(plan, Tb, total_l, xs, s0);
  const int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= total_l) return;
  const int si = tiled ? s0 : find_series_by_w(plan, wi);
  const SeriesDesc S = plan.series(si);
  const SeriesDesc Q = plan.series(S.partner);  // the series I indexes into
  const int64_t i = wi - S.w_off;
  const int64_t j = I[wi];
  const double g = (double)gP[wi];
  const double mi = b.mu[wi];
  Double4 c{0.0, 0.0, 0.0, 0.0};
  int64_t jw = -1;
  double isi = 0.0, isj = 0.0, mj = 0.0;
  if (j >= 0 && j < Q.l && !(S.partner == si && j == i) && g != 0.0 && isfinite(g)) {
    jw = Q.w_off + j;
    isi = b.isig[wi];
    isj = b.isig[jw];
    if (isi > 0.0 && isj > 0.0) {
      const Tin *xi = series_samples(plan, Tb, S) + i;
      const Tin *xj = series_samples(plan, Tb, Q) + j;
      mj = b.mu[jw];
      double d2 = 0.0, dot = 0.0;
      const int m = S.m;
      // terms summed in sample order; the neighbour's window is read in
      // 16-byte chunks, two in flight (with seven waves per SIMD for float
      // input, six for double, to hide the rest of the latency)
      auto row = [&](auto xi_at) {
        for_each_sample<Tin, 2>(xj, m, [&](int u, double vj) {
          const double zi = (xi_at(u) - mi) * isi, zj = (vj - mj) * isj;
          d2 = fma(zi - zj, zi - zj, d2);
          dot = fma(zi, zj, dot);
        });
      };
      if (tiled) {
        const double *xl = xs + threadIdx.x;
        row([&](int u) { return xl[u]; });
      } else {
        row([&](int u) { return (double)xi[u]; });
      }
      const double d = sqrt(d2);
      if (d > 0.0) {
        const double rho = dot / S.m;
        c = Double4{g * rho * isi / d, -g * isi / d, g * rho * isj / d, -g * isj / d};
      }
    }
  }
  const bool live = (c.x != 0.0 || c.y != 0.0 || c.z != 0.0 || c.w != 0.0);
  b.nbr[wi] = live ? jw : -1;
  // source offset of the own edge: neighbour start - window start
  const int64_t delta = live ? (Q.t_off + j) - (S.t_off + i) : 0;
  b.wrec[wi] = BwdWin{mi, live ? c.y * isj : 0.0, live ? mj : 0.0, delta};
  b.alpha[wi] = c.x;
  if (live) {
    b.bedge[wi] = BwdEdge{c.w * isi, mi, -delta, jw};
    b.bgam[wi] = c.z;
    b.bpos[wi] = (uint32_t)atomicAdd(&b.count[jw], 1ull);
  }
}

// ------------------------------------------- backward after the forward
// k_bwd_stats from the forward's window statistics (the same two-pass FP64
// arithmetic, so the same values): each window's mean (0 for a non-finite
// window) and 1/sigma (0 for constant or non-finite windows) into the
// backward's arrays; the bucket counts and the large-bucket list cleared.
__global__ void __launch_bounds__(256) k_bwd_stats_fwd(BwdWork b, int64_t total_l) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w == 0) *b.nbig = 0ull;
  if (w >= total_l) return;
  const uint8_t f = b.fflags[w];
  const double sg = b.fsig[w];
  const bool ok = (f & 1) != 0;
  b.mu[w] = ok ? b.fmu[w] : 0.0;
  b.isig[w] = (ok && !(f & 2) && sg > 0.0) ? 1.0 / sg : 0.0;
  b.count[w] = 0ull;
}

// k_bwd_coef without reading any sample: the row's distance d is its entry
// of the forward's FP64-finalized profile (the direct-difference sum that
// k_bwd_coef forms itself), and rho = 1 - d^2/(2m) (d^2 = 2m(1 - rho) for
// z-normalised windows).
template <typename Tp, typename Tg>
__global__ void __launch_bounds__(256) k_bwd_coef_fwd(Plan plan, BwdWork b, const int64_t *__restrict__ I,
                                                      const Tp *__restrict__ P, const Tg *__restrict__ gP,
                                                      int64_t total_l) {
  const int64_t w0 = (int64_t)blockIdx.x * blockDim.x;
  const int s0 = find_series_by_w(plan, w0);
  const bool one = s0 == find_series_by_w(plan, min(w0 + (int64_t)blockDim.x, total_l) - 1);
  const int64_t wi = w0 + threadIdx.x;
  if (wi >= total_l) return;
  const int si = one ? s0 : find_series_by_w(plan, wi);
  const SeriesDesc S = plan.series(si);
  const SeriesDesc Q = plan.series(S.partner);
  const int64_t i = wi - S.w_off;
  const int64_t j = I[wi];
  const double g = (double)gP[wi];
  const double mi = b.mu[wi], isi = b.isig[wi];
  Double4 c{0.0, 0.0, 0.0, 0.0};
  int64_t jw = -1;
  double isj = 0.0, mj = 0.0;
  if (j >= 0 && j < Q.l && !(S.partner == si && j == i) && g != 0.0 && isfinite(g)) {
    jw = Q.w_off + j;
    mj = b.mu[jw];
    isj = b.isig[jw];
    const double d = (double)P[wi];
    if (isi > 0.0 && isj > 0.0 && d > 0.0 && isfinite(d)) {
      const double rho = 1.0 - d * d / (2.0 * S.m);
      c = Double4{g * rho * isi / d, -g * isi / d, g * rho * isj / d, -g * isj / d};
    }
  }
  const bool live = (c.x != 0.0 || c.y != 0.0 || c.z != 0.0 || c.w != 0.0);
  b.nbr[wi] = live ? jw : -1;
  const int64_t delta = live ? (Q.t_off + j) - (S.t_off + i) : 0;
  b.wrec[wi] = BwdWin{mi, live ? c.y * isj : 0.0, live ? mj : 0.0, delta};
  b.alpha[wi] = c.x;
  if (live) {
    b.bedge[wi] = BwdEdge{c.w * isi, mi, -delta, jw};
    b.bgam[wi] = c.z;
    b.bpos[wi] = (uint32_t)atomicAdd(&b.count[jw], 1ull);
  }
}

// Bucket entry of each contributing row on its neighbour window, at its
// arrival position (arbitrary order; k_bwd_rank and k_bwd_bigsort order it).
__global__ void __launch_bounds__(256) k_bwd_place(BwdWork b, int64_t total_l) {
  const int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= total_l) return;
  const int64_t jw = b.nbr[wi];
  if (jw < 0) return;
  const int64_t base = b.off[jw];
  const uint32_t pos = b.bpos[wi];
  b.tmp[base + (int64_t)pos] = wi;
  // the first row placed in a large bucket lists it for the workgroup sort
  if (pos == 0 && b.off[jw + 1] - base > kBwdSmallBucket) b.big[atomicAdd(b.nbig, 1ull)] = jw;
}

// Edge slot p holds the bucket edge of row wi.
__device__ __forceinline__ void put_bucket_edge(const BwdWork &b, int64_t p, int64_t wi) {
  b.erec[p] = b.bedge[wi];
  b.egam[p] = b.bgam[wi];
}

// Bucket edges in increasing row order.  In a bucket of at most
// kBwdSmallBucket rows a row's slot is the number of rows of the bucket with
// a smaller index; larger buckets are left to k_bwd_bigsort.
__global__ void __launch_bounds__(256) k_bwd_rank(BwdWork b, int64_t total_l) {
  const int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= total_l) return;
  const int64_t jw = b.nbr[wi];
  if (jw < 0) return;
  const int64_t a = b.off[jw], e = b.off[jw + 1];
  if (e - a > kBwdSmallBucket) return;
  int64_t r = 0;
  for (int64_t p = a; p < e; ++p) r += b.tmp[p] < wi;
  put_bucket_edge(b, a + r, wi);
}

// Large buckets: one workgroup sorts a bucket's row indices (a bitonic
// network whose comparators all point the same way, so any length works:
// the missing elements past the end count as +infinity and never move) in
// LDS, or in place in global memory when longer than the LDS buffer; then
// writes the bucket's edges in that order.  O(h log^2 h) for h rows.
constexpr int kSortLds = 4096;
__device__ __forceinline__ void cmpx(int64_t *v, int64_t i, int64_t p) {
  const int64_t x = v[i], y = v[p];
  if (x > y) {
    v[i] = y;
    v[p] = x;
  }
}
__device__ void sort_rows(int64_t *v, int64_t n) {
  int64_t N = 1;
  while (N < n) N <<= 1;
  for (int64_t k = 2; k <= N; k <<= 1) {
    const int64_t hk = k >> 1;
    for (int64_t t = threadIdx.x; t < N / 2; t += blockDim.x) {
      const int64_t i = (t / hk) * k + (t % hk), p = i ^ (k - 1);
      if (p < n) cmpx(v, i, p);
    }
    __syncthreads();
    for (int64_t j = k >> 2; j >= 1; j >>= 1) {
      for (int64_t t = threadIdx.x; t < N / 2; t += blockDim.x) {
        const int64_t i = (t / j) * 2 * j + (t % j), p = i | j;
        if (p < n) cmpx(v, i, p);
      }
      __syncthreads();
    }
  }
}
__global__ void __launch_bounds__(256) k_bwd_bigsort(BwdWork b) {
  __shared__ int64_t ks[kSortLds];
  const unsigned long long nb = *b.nbig;
  for (unsigned long long q = blockIdx.x; q < nb; q += gridDim.x) {
    const int64_t jw = b.big[q];
    const int64_t a = b.off[jw], h = b.off[jw + 1] - a;
    int64_t *v = b.tmp + a;
    if (h <= kSortLds) {
      for (int64_t t = threadIdx.x; t < h; t += blockDim.x) ks[t] = v[t];
      __syncthreads();
      sort_rows(ks, h);
      v = ks;
    } else {
      sort_rows(v, h);
    }
    for (int64_t t = threadIdx.x; t < h; t += blockDim.x) put_bucket_edge(b, a + t, v[t]);
    __syncthreads();
  }
}

// Per window: its own alpha plus the gammas of its bucket, in edge order,
// times 1/sigma.
__global__ void __launch_bounds__(256) k_bwd_window(BwdWork b, int64_t total_l) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= total_l) return;
  double s = b.alpha[w];
  const int64_t e = b.off[w + 1];
  for (int64_t p = b.off[w]; p < e; ++p) s += b.egam[p];
  b.wsc[w] = s * b.isig[w];
}

// A wave-uniform 64-bit value in scalar registers.
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Windows covering global sample x: [lo, hi] (global window indices).
__device__ __forceinline__ void covering(const Plan &plan, int64_t x, int64_t &lo, int64_t &hi) {
  const SeriesDesc S = plan.series(find_series_by_t(plan, x));
  const int64_t t = x - S.t_off;
  lo = S.w_off + max((int64_t)0, t - S.m + 1);
  hi = S.w_off + min(t, S.l - 1);
}

// Source-sample loads of the gather.  kBuf: buffer loads against the whole
// sample array with 32-bit byte offsets (arrays under 2 GiB).  An offset
// outside the array reads 0 and does not fault, so a lane outside an edge's
// window may load at any offset; its term is discarded.  Otherwise flat loads
// with the offset replaced by 0 (the lane's own sample) outside the window.
template <typename Tin, bool kBuf>
struct GatherSrc;
template <typename Tin>
struct GatherSrc<Tin, true> {
  __amdgpu_buffer_rsrc_t r;
  uint32_t own;  // the lane's sample, in bytes
  __device__ GatherSrc(const Tin *Tb, int64_t total_n, int64_t x)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<Tin *>(Tb), (short)0, (int)(total_n * (int64_t)sizeof(Tin)),
                                            0x00020000)),
        own((uint32_t)(x * (int64_t)sizeof(Tin))) {}
  __device__ __forceinline__ double load(int32_t dbytes, int64_t, bool) const {
    const uint32_t o = own + (uint32_t)dbytes;
    if constexpr (sizeof(Tin) == 4)
      return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0));
    else
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0));
  }
};
template <typename Tin>
struct GatherSrc<Tin, false> {
  const Tin *xp;
  __device__ GatherSrc(const Tin *Tb, int64_t, int64_t x) : xp(Tb + x) {}
  __device__ __forceinline__ double load(int32_t, int64_t delta, bool in) const {
    return (double)xp[in ? delta : 0];
  }
};

// Staged records.  A window: sc and mu, then its own edge's c and mu (one
// 16-byte read each) and source offset in bytes (buffer loads) and in
// samples (flat loads).  A bucket edge: c and mu, then its destination
// window relative to the wave's first covering window and the source offset.
struct GatherWin {
  double sc, mu, oc, omu;
  int64_t odelta;
  int32_t dbytes, pad_;
};
struct GatherEdge {
  double c, mu;
  int32_t rel, dbytes;
  int64_t delta;
};

// One wave = 64 consecutive samples.  Every sample of a series is covered by
// at least one window and the covering ranges are non-decreasing in the
// sample index, so the wave walks [lo(first sample), hi(last sample)].
// Records are fetched 64 at a time, one per lane (coalesced, all in flight
// together), staged in the wave's own LDS slots and read back by the whole
// wave as broadcasts.  Window ranges are tested in 32 bits relative to the
// wave's first covering window: lane-local (rel - lt) <= span, unsigned.  A
// lane outside a term's window adds c * 0 (its sample, which may be any
// value, is replaced before the product).
template <typename Tin, typename Tg, bool kBuf>
__global__ void __launch_bounds__(256) k_bwd_gather(Plan plan, BwdWork b, const Tin *__restrict__ Tb,
                                                    Tg *gT, int64_t total_n) {
  __shared__ GatherWin stage_w[4][64];   // per wave: 64 window records
  __shared__ GatherEdge stage_e[4][64];  // per wave: 64 bucket edges
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t x0 = uni64(x - (int64_t)(threadIdx.x & 63));
  if (x0 >= total_n) return;
  const int64_t xl = min(x0 + 63, total_n - 1);
  const bool act = x < total_n;
  const int64_t xs = act ? x : xl;
  int64_t lo_t, hi_t, lo_w, hi_w, dummy;
  covering(plan, xs, lo_t, hi_t);
  covering(plan, x0, lo_w, dummy);
  covering(plan, xl, dummy, hi_w);
  lo_w = uni64(lo_w);
  hi_w = uni64(hi_w);
  const uint32_t lt = (uint32_t)(lo_t - lo_w), span = (uint32_t)(hi_t - lo_t);
  const GatherSrc<Tin, kBuf> src(Tb, total_n, xs);
  // a non-finite sample lies only in windows with sc = 0 and mu = 0: read
  // as 0 it adds exact zeros there
  double xt = (double)Tb[xs];
  xt = isfinite(xt) ? xt : 0.0;
  const BwdWin *__restrict__ wrec = b.wrec;
  const double *__restrict__ wsc = b.wsc;
  const BwdEdge *__restrict__ erec = b.erec;
  const int64_t *__restrict__ off = b.off;
  const int lane = threadIdx.x & 63;
  GatherWin *const sw = stage_w[threadIdx.x >> 6];
  GatherEdge *const se = stage_e[threadIdx.x >> 6];
  double acc = 0.0;
  // First each covering window's multiple of its own z and its own edge
  // (four windows per step: their source loads are issued together).  A
  // window without an own edge (oc = 0) keeps its source sample out: that
  // sample may lie in a non-finite window.  Slots past the last window are
  // zero and lie beyond every lane's range.
  for (int64_t c = lo_w; c <= hi_w; c += 64) {
    GatherWin q{0.0, 0.0, 0.0, 0.0, 0, 0, 0};
    if (c + lane <= hi_w) {
      const BwdWin w = wrec[c + lane];
      q = GatherWin{wsc[c + lane], w.mu, w.oc, w.omu, w.odelta, (int32_t)(w.odelta * (int64_t)sizeof(Tin)), 0};
    }
    sw[lane] = q;
    __builtin_amdgcn_wave_barrier();
    const int cnt = ((int)min((int64_t)64, hi_w - c + 1) + 3) & ~3;
    const uint32_t base = (uint32_t)(c - lo_w) - lt;
    for (int k = 0; k < cnt; k += 4) {
      double v[4];
      bool in[4], io[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const GatherWin &g = sw[k + u];
        const double oc = g.oc;
        in[u] = base + (uint32_t)(k + u) <= span;
        io[u] = in[u] & (oc != 0.0);
        v[u] = src.load(g.dbytes, g.odelta, io[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 sm = *reinterpret_cast<const double2 *>(&sw[k + u].sc);
        const double2 om = *reinterpret_cast<const double2 *>(&sw[k + u].oc);
        const double dt = xt - sm.y, dv = v[u] - om.y;
        acc = fma(sm.x, in[u] ? dt : 0.0, acc);
        acc = fma(om.x, io[u] ? dv : 0.0, acc);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  // ... then the bucket edges of the covering windows, one flat run of the
  // edge array (each edge carries its destination window).  Eight edges per
  // step.  Fetch slots past the run get a destination no lane covers.
  const int64_t eb = uni64(off[lo_w]), ee = uni64(off[hi_w + 1]);
  for (int64_t c = eb; c < ee; c += 64) {
    GatherEdge q{0.0, 0.0, INT32_MIN, 0, 0};
    if (c + lane < ee) {
      const BwdEdge e = erec[c + lane];
      q = GatherEdge{e.c, e.mu, (int32_t)(e.dest - lo_w), (int32_t)(e.delta * (int64_t)sizeof(Tin)), e.delta};
    }
    se[lane] = q;
    __builtin_amdgcn_wave_barrier();
    const int cnt = ((int)min((int64_t)64, ee - c) + 7) & ~7;
    for (int k = 0; k < cnt; k += 8) {
      double v[8];
      bool in[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const GatherEdge &g = se[k + u];
        in[u] = (uint32_t)g.rel - lt <= span;
        v[u] = src.load(g.dbytes, g.delta, in[u]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double2 cm = *reinterpret_cast<const double2 *>(&se[k + u]);
        const double dv = v[u] - cm.y;
        acc = fma(cm.x, in[u] ? dv : 0.0, acc);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (act) gT[x] = (Tg)acc;
}

namespace {

// Everything after the per-row coefficients: bucket offsets, placement,
// ordering, per-window sums and the gather.
hipError_t launch_backward_tail(const Plan &plan, const BwdWork &b, const void *T, bool t_f64, void *gT,
                                int64_t total_l, int64_t total_n, bool flat_loads, hipStream_t st) {
  const dim3 blk(256);
  const dim3 gl((unsigned)((total_l + 255) / 256)), gn((unsigned)((total_n + 255) / 256));
  const hipError_t e = launch_exclusive_scan(reinterpret_cast<const int64_t *>(b.count), b.off, b.chunk,
                                             total_l, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bwd_place, gl, blk, 0, st, b, total_l);
  hipLaunchKernelGGL(k_bwd_rank, gl, blk, 0, st, b, total_l);
  hipLaunchKernelGGL(k_bwd_bigsort, dim3(256), blk, 0, st, b);
  hipLaunchKernelGGL(k_bwd_window, gl, blk, 0, st, b, total_l);
  // buffer loads while the sample array's byte offsets fit in 31 bits
  const bool buf = !flat_loads && total_n * (int64_t)(t_f64 ? sizeof(double) : sizeof(float)) < ((int64_t)1 << 31);
  if (t_f64) {
    if (buf)
      hipLaunchKernelGGL((k_bwd_gather<double, double, true>), gn, blk, 0, st, plan, b, (const double *)T,
                         (double *)gT, total_n);
    else
      hipLaunchKernelGGL((k_bwd_gather<double, double, false>), gn, blk, 0, st, plan, b, (const double *)T,
                         (double *)gT, total_n);
  } else {
    if (buf)
      hipLaunchKernelGGL((k_bwd_gather<float, float, true>), gn, blk, 0, st, plan, b, (const float *)T,
                         (float *)gT, total_n);
    else
      hipLaunchKernelGGL((k_bwd_gather<float, float, false>), gn, blk, 0, st, plan, b, (const float *)T,
                         (float *)gT, total_n);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(const Plan &plan, const BwdWork &b, const void *T, bool t_f64,
                           const int64_t *I, const void *gP, void *gT, int64_t total_l,
                           int64_t total_n, bool flat_loads, hipStream_t st) {
  const dim3 blk(256);
  const dim3 gl((unsigned)((total_l + 255) / 256));
  if (t_f64) {
    hipLaunchKernelGGL((k_bwd_stats<double>), gl, blk, 0, st, plan, b, (const double *)T, total_l);
    hipLaunchKernelGGL((k_bwd_coef<double, double>), gl, blk, 0, st, plan, b, (const double *)T, I,
                       (const double *)gP, total_l);
  } else {
    hipLaunchKernelGGL((k_bwd_stats<float>), gl, blk, 0, st, plan, b, (const float *)T, total_l);
    hipLaunchKernelGGL((k_bwd_coef<float, float>), gl, blk, 0, st, plan, b, (const float *)T, I,
                       (const float *)gP, total_l);
  }
  return launch_backward_tail(plan, b, T, t_f64, gT, total_l, total_n, flat_loads, st);
}

hipError_t launch_backward_after_forward(const Plan &plan, const BwdWork &b, const void *T, bool t_f64,
                                         const int64_t *I, const void *P, const void *gP, void *gT,
                                         int64_t total_l, int64_t total_n, bool flat_loads, hipStream_t st) {
  const dim3 blk(256);
  const dim3 gl((unsigned)((total_l + 255) / 256));
  hipLaunchKernelGGL(k_bwd_stats_fwd, gl, blk, 0, st, b, total_l);
  if (t_f64)
    hipLaunchKernelGGL((k_bwd_coef_fwd<double, double>), gl, blk, 0, st, plan, b, I, (const double *)P,
                       (const double *)gP, total_l);
  else
    hipLaunchKernelGGL((k_bwd_coef_fwd<float, float>), gl, blk, 0, st, plan, b, I, (const float *)P,
                       (const float *)gP, total_l);
  return launch_backward_tail(plan, b, T, t_f64, gT, total_l, total_n, flat_loads, st);
}

}  // namespace mpx
