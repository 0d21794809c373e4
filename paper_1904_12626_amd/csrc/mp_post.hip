// After the sweep: decode the packed minima into (P, I), resolve windows the
// sweep cannot express exactly (constant and invalid windows), optionally
// recompute P in FP64 from the chosen pair, and the FP64 recheck of the best
// motif pairs and discords.
#include <algorithm>
#include <cmath>

#include "mp_internal.h"
#include "mp_types.h"

namespace mpx {

namespace {

__device__ __forceinline__ int find_series_w(const Plan &plan, int64_t wi) {
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
__device__ __forceinline__ double sample(const Tin *p) {
  const double v = (double)*p;
  return isfinite(v) ? v : 0.0;
}

// FP64 z-normalised Euclidean distance between window i of series A and
// window j of series B, in the direct difference form (constant windows
// normalise to zero).  Callers pass valid windows only.
template <typename Tin>
__device__ double pair_dist64(const Tin *TA, double muA, double sgA, bool cA, const Tin *TB,
                              double muB, double sgB, bool cB, int m) {
  // z_a - z_b must be exactly 0 for windows that are offset copies: each z is
  // rounded before the subtraction (no contraction into a fused multiply-add)
#pragma clang fp contract(off)
  const double ia = cA ? 0.0 : 1.0 / sgA, ib = cB ? 0.0 : 1.0 / sgB;
  double s = 0.0;
  for (int u = 0; u < m; ++u) {
    const double za = (sample(TA + u) - muA) * ia;
    const double zb = (sample(TB + u) - muB) * ib;
    const double d = za - zb;
    s = fma(d, d, s);
  }
  return sqrt(s);
}

// Is window j of the partner series a candidate of window w of series S?
// AB sides: always.  Self-joins: |j - w| > ez, on S's side(s), and with the
// offset |j - w| in the plan's chunk set when there is one.
__device__ __forceinline__ bool candidate(const Plan &plan, const SeriesDesc &S, int64_t w,
                                          int64_t j) {
  if (S.ez < 0) return true;
  const int64_t k = j - w;
  const int64_t a = k < 0 ? -k : k;
  if (a <= S.ez) return false;
  if (S.side == kSideRight && k < 0) return false;
  if (S.side == kSideLeft && k > 0) return false;
  if (plan.kmask) {
    const int64_t c = (a - S.ez - 1) / plan.kchunk;
    if (!((plan.kmask[c >> 5] >> (c & 31)) & 1u)) return false;
  }
  return true;
}

// Smallest candidate j of window w (see `candidate`) in a partner series of
// l windows that is a member of the set tabulated by `next` (next[x] =
// smallest member >= x, l if none; null: every window is a member), or -1.
// The candidates form at most a few intervals of j (one per side, or one per
// chunk of offsets); each interval costs one table lookup.
__device__ int64_t first_candidate(const Plan &plan, const SeriesDesc &S, const int32_t *next,
                                   int64_t l, int64_t w) {
  auto first_in = [&](int64_t lo, int64_t hi) -> int64_t {
    lo = lo < 0 ? 0 : lo;
    hi = hi > l - 1 ? l - 1 : hi;
    if (lo > hi) return -1;
    const int64_t g = next ? (int64_t)next[lo] : lo;
    return g <= hi ? g : -1;
  };
  if (S.ez < 0) return first_in(0, l - 1);
  const int64_t ez = S.ez;
  if (!plan.kmask) {
    if (S.side != kSideRight) {
      const int64_t g = first_in(0, w - ez - 1);
      if (g >= 0) return g;
    }
    return S.side != kSideLeft ? first_in(w + ez + 1, l - 1) : -1;
  }
  const int64_t C = plan.kchunk;
  const int64_t span = l - 1 - ez;  // offsets ez + 1 .. l - 1
  if (span <= 0) return -1;
  const int64_t nch = (span + C - 1) / C;
  auto in_set = [&](int64_t c) { return ((plan.kmask[c >> 5] >> (c & 31)) & 1u) != 0; };
  if (S.side != kSideRight && w - ez - 1 >= 0) {
    // left of w: increasing j is decreasing offset
    for (int64_t c = min(nch - 1, (w - ez - 1) / C); c >= 0; --c) {
      if (!in_set(c)) continue;
      const int64_t g = first_in(w - (ez + (c + 1) * C), w - (ez + 1 + c * C));
      if (g >= 0) return g;
    }
  }
  if (S.side != kSideLeft) {
    for (int64_t c = 0; c < nch; ++c) {
      const int64_t lo = w + ez + 1 + c * C;
      if (lo > l - 1) break;
      if (!in_set(c)) continue;
      const int64_t g = first_in(lo, w + ez + (c + 1) * C);
      if (g >= 0) return g;
    }
  }
  return -1;
}

template <typename Tout>
__device__ __forceinline__ void store_out(const Outputs &o, const SeriesDesc &S, int64_t w,
                                          double P, int64_t I) {
  const int slot = S.out;
  const int64_t pos = S.p_off + w;
  reinterpret_cast<Tout *>(o.P[slot])[pos] = (Tout)P;
  o.I[slot][pos] = I;
}

}  // namespace

// --------------------------------------------------------------- finalize
// key -> P = sqrt(2 m key), I = index; then the degenerate-window rules:
//  * invalid window: (+inf, -1);
//  * constant window w: the nearest admissible constant partner at distance 0
//    if any, otherwise the smallest admissible valid partner at sqrt(m);
//  * valid window whose partner series has constant windows: the smallest
//    admissible constant partner at distance sqrt(m) competes (the sweep
//    scores such pairs too high);
//  * if the chosen partner is invalid or past the end of the partner series
//    (the sweep scores such columns like rho = 0), the window is queued for
//    an exact rescan;
//  * so is a window whose key is below `kappa` (FP32 sweep): there the
//    FP32 keys cannot order the candidates (near-exact repeats), and the
//    exact FP64 scan picks the neighbour.
// The FP64 distance of the chosen pair reads the row's own window from a
// workgroup tile of the series (staged once when the workgroup's 256
// windows lie in one series and m <= kFinTileM) and the partner's window in
// 16-byte chunks, two in flight, at eight waves per SIMD; the terms are
// summed in sample order either way.
constexpr int kFinTile = 256;
constexpr int kFinTileM = 2048;

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(256, 8) k_finalize(Plan plan, Work wk, const Tin *__restrict__ Tb,
                                                  Outputs o, int fp64_finalize, double kappa,
                                                  int64_t total_l) {
  // z_a - z_b must be exactly 0 for windows that are offset copies (as in
  // pair_dist64): no contraction into a fused multiply-add
#pragma clang fp contract(off)
  __shared__ Tin xs[kFinTile + kFinTileM];
  const int64_t w0 = (int64_t)blockIdx.x * kFinTile;
  const int s0 = find_series_w(plan, w0);
  const SeriesDesc S0 = plan.series(s0);
  const bool tiled = fp64_finalize && S0.m <= kFinTileM &&
                     s0 == find_series_w(plan, min(w0 + kFinTile, total_l) - 1);
  if (tiled) {
    const Tin *base = series_samples(plan, Tb, S0) + (w0 - S0.w_off);
    const int cnt = (int)(min(w0 + kFinTile, total_l) - w0) + S0.m - 1;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) xs[t] = base[t];
  }
  __syncthreads();
  const int64_t wi = w0 + threadIdx.x;
  if (wi >= total_l) return;
  const int si = tiled ? s0 : find_series_w(plan, wi);
  const SeriesDesc S = tiled ? S0 : plan.series(si);
  const SeriesDesc Q = plan.series(S.partner);
  const int64_t w = wi - S.w_off;
  const uint8_t fw = wk.flags[wi];
  if (!(fw & 1)) {
    store_out<Tout>(o, S, w, INFINITY, -1);
    return;
  }
  int ib = 1;
  while (((int64_t)1 << ib) < max(S.l, Q.l) + 1) ++ib;
  const uint64_t key = wk.keys[wi];
  double val = INFINITY;
  int64_t idx = -1;
  if (key != ~0ull) {
    val = unpack_key(key, ib);
    idx = unpack_idx(key, ib);
    if (!(val < kKeyInvalid)) { val = INFINITY; idx = -1; }
  }
  const int sp = wk.special[S.partner];
  const int32_t *nc = wk.next_const + Q.x_off;
  const int32_t *nv = wk.next_valid + Q.x_off;
  if (fw & 2) {  // constant window
    const int64_t jc = (sp & 2) ? first_candidate(plan, S, nc, Q.l, w) : -1;
    if (jc >= 0) {
      val = 0.0;
      idx = jc;
    } else {
      const int64_t jv = first_candidate(plan, S, (sp & 1) ? nv : nullptr, Q.l, w);
      val = jv >= 0 ? 0.5 : INFINITY;
      idx = jv;
    }
    store_out<Tout>(o, S, w, idx >= 0 ? sqrt(2.0 * S.m * val) : INFINITY, idx);
    return;
  }
  if (sp & 2) {
    const int64_t jc = first_candidate(plan, S, nc, Q.l, w);
    if (jc >= 0 && (0.5 < val || (0.5 == val && jc < idx))) {
      val = 0.5;
      idx = jc;
    }
  }
  if (idx >= Q.l || ((sp & 1) && idx >= 0 && !(wk.flags[Q.w_off + idx] & 1)) || (idx >= 0 && val < kappa)) {
    const unsigned long long pos = atomicAdd(&wk.counters[1], 1ull);
    wk.rescan[pos] = wi;
    store_out<Tout>(o, S, w, INFINITY, -1);
    return;
  }
  double P = INFINITY;
  if (idx >= 0) {
    P = sqrt(2.0 * S.m * fmax(val, 0.0));
    if (fp64_finalize && !(wk.flags[Q.w_off + idx] & 2)) {
      // both windows are valid (all samples finite) and not constant: the
      // pair_dist64 form without its non-finite guards
      const double muA = wk.mu[wi], ia = 1.0 / wk.sig[wi];
      const double muB = wk.mu[Q.w_off + idx], ib = 1.0 / wk.sig[Q.w_off + idx];
      const Tin *xa = series_samples(plan, Tb, S) + w;
      const Tin *xl = xs + threadIdx.x;
      double s2 = 0.0;
      auto pass = [&](auto a_at) {
        for_each_sample<Tin, 2>(series_samples(plan, Tb, Q) + idx, S.m, [&](int u, double vb) {
          const double za = (a_at(u) - muA) * ia;
          const double zb = (vb - muB) * ib;
          const double d = za - zb;
          s2 = fma(d, d, s2);
        });
      };
      if (tiled)
        pass([&](int u) { return (double)xl[u]; });
      else
        pass([&](int u) { return (double)xa[u]; });
      P = sqrt(s2);
    }
  }
  store_out<Tout>(o, S, w, P, idx);
}

// ------------------------------------------------------------------ rescan
// Exact row minimum for the queued windows: one workgroup per queued window
// (grid-stride over the queue), every admissible valid partner scored in
// FP64 as 1 - rho (constant partners score 1/2), smallest (key, index) wins.
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(256) k_rescan(Plan plan, Work wk, const Tin *__restrict__ Tb,
                                                Outputs o, int fp64_finalize) {
  __shared__ double bk[256];
  __shared__ int64_t bi[256];
  const unsigned long long count = wk.counters[1];
  for (unsigned long long q = blockIdx.x; q < count; q += gridDim.x) {
    const int64_t wi = wk.rescan[q];
    const int si = find_series_w(plan, wi);
    const SeriesDesc S = plan.series(si);
    const SeriesDesc Q = plan.series(S.partner);
    const int64_t w = wi - S.w_off;
    const Tin *Tw = series_samples(plan, Tb, S) + w;
    const double muw = wk.mu[wi], sgw = wk.sig[wi];
    double best = INFINITY;
    int64_t arg = -1;
    for (int64_t j = threadIdx.x; j < Q.l; j += blockDim.x) {
      if (!candidate(plan, S, w, j)) continue;
      const uint8_t fj = wk.flags[Q.w_off + j];
      if (!(fj & 1)) continue;
      double key;
      if (fj & 2) {
        key = 0.5;
      } else {
        const Tin *Tj = series_samples(plan, Tb, Q) + j;
        const double muj = wk.mu[Q.w_off + j];
        double c = 0.0;
        for (int u = 0; u < S.m; ++u) c = fma(sample(Tw + u) - muw, sample(Tj + u) - muj, c);
        key = 1.0 - c / ((double)S.m * sgw * wk.sig[Q.w_off + j]);
      }
      if (key < best) { best = key; arg = j; }  // j increases per thread
    }
    bk[threadIdx.x] = best;
    bi[threadIdx.x] = arg;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) {
        const double k2 = bk[threadIdx.x + h];
        const int64_t i2 = bi[threadIdx.x + h];
        if (i2 >= 0 && (k2 < bk[threadIdx.x] || (k2 == bk[threadIdx.x] && (bi[threadIdx.x] < 0 || i2 < bi[threadIdx.x])))) {
          bk[threadIdx.x] = k2;
          bi[threadIdx.x] = i2;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const int64_t j = bi[0];
      double P = INFINITY;
      if (j >= 0) {
        P = sqrt(2.0 * S.m * fmax(bk[0], 0.0));
        if (fp64_finalize && !(wk.flags[Q.w_off + j] & 2))
          P = pair_dist64(Tw, muw, sgw, false, series_samples(plan, Tb, Q) + j, wk.mu[Q.w_off + j],
                          wk.sig[Q.w_off + j], false, S.m);
      }
      store_out<Tout>(o, S, w, P, j);
    }
    __syncthreads();
  }
}

hipError_t launch_finalize(const Plan &plan, const Work &w, const void *T, bool t_f64,
                           const Outputs &o, bool out_f64, bool fp64_finalize, double kappa,
                           int64_t total_l, hipStream_t st) {
  const dim3 blk(256), grd((unsigned)((total_l + 255) / 256));
  const int f = fp64_finalize ? 1 : 0;
  if (t_f64) {
    if (out_f64) hipLaunchKernelGGL((k_finalize<double, double>), grd, blk, 0, st, plan, w, (const double *)T, o, f, kappa, total_l);
    else hipLaunchKernelGGL((k_finalize<double, float>), grd, blk, 0, st, plan, w, (const double *)T, o, f, kappa, total_l);
  } else {
    if (out_f64) hipLaunchKernelGGL((k_finalize<float, double>), grd, blk, 0, st, plan, w, (const float *)T, o, f, kappa, total_l);
    else hipLaunchKernelGGL((k_finalize<float, float>), grd, blk, 0, st, plan, w, (const float *)T, o, f, kappa, total_l);
  }
  return hipGetLastError();
}

hipError_t launch_rescan(const Plan &plan, const Work &w, const void *T, bool t_f64,
                         const Outputs &o, bool out_f64, bool fp64_finalize, hipStream_t st) {
  const dim3 blk(256), grd(512);
  const int f = fp64_finalize ? 1 : 0;
  if (t_f64) {
    if (out_f64) hipLaunchKernelGGL((k_rescan<double, double>), grd, blk, 0, st, plan, w, (const double *)T, o, f);
    else hipLaunchKernelGGL((k_rescan<double, float>), grd, blk, 0, st, plan, w, (const double *)T, o, f);
  } else {
    if (out_f64) hipLaunchKernelGGL((k_rescan<float, double>), grd, blk, 0, st, plan, w, (const float *)T, o, f);
    else hipLaunchKernelGGL((k_rescan<float, float>), grd, blk, 0, st, plan, w, (const float *)T, o, f);
  }
  return hipGetLastError();
}

// ------------------------------------------------------- left/right merge
// Profile of a left/right job: out[0, l) = the better of the left profile
// (out[l, 2l)) and the right profile (out[2l, 3l)); on equal distances the
// left neighbour (the smaller index) wins.
template <typename Tout>
__global__ void __launch_bounds__(256) k_lr_combine(Outputs o, int64_t l) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= l) return;
  Tout *P = reinterpret_cast<Tout *>(o.P[0]);
  int64_t *I = o.I[0];
  const Tout pl = P[l + w], pr = P[2 * l + w];
  const int64_t il = I[l + w], ir = I[2 * l + w];
  const bool right = il < 0 || (ir >= 0 && pr < pl);
  P[w] = right ? pr : pl;
  I[w] = right ? ir : il;
}

hipError_t launch_lr_combine(const Outputs &o, bool out_f64, int64_t l, hipStream_t st) {
  const dim3 blk(256), grd((unsigned)((l + 255) / 256));
  if (out_f64) hipLaunchKernelGGL((k_lr_combine<double>), grd, blk, 0, st, o, l);
  else hipLaunchKernelGGL((k_lr_combine<float>), grd, blk, 0, st, o, l);
  return hipGetLastError();
}

// ------------------------------------------------------------------ recheck
// Motif pairs: repeatedly the smallest finite P[i] not within m of an earlier
// pick, reported with its pair (i, I[i]), both members then masked; discords:
// repeatedly the largest finite P, masking within m.  One launch per pick:
// every workgroup reduces a slice to (value, index) (smallest index on ties),
// the last workgroup to finish (atomic ticket) reduces the partial results,
// re-measures the pair in FP64 and appends the new mask centres.
struct RecheckState {
  double pv[512];         // per-workgroup partial values
  int64_t pi[512];        // per-workgroup partial indices
  int64_t centres[192];   // motif members, then discords
  unsigned int ticket;
  int done;               // a pick found nothing: later picks report none
};
constexpr int kRecheckBlocks = 512;

template <typename Tin, typename Tp>
__global__ void __launch_bounds__(256)
    k_pick(const Tin *__restrict__ T, int64_t n, int m, const Tp *__restrict__ P,
           const int64_t *__restrict__ I, int discord, int q, int km, int64_t *out_idx,
           double *out_dist, RecheckState *st) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  __shared__ int64_t cen[192];
  __shared__ int last;
  const int tid = threadIdx.x;
  const int64_t l = n - m + 1;
  // mask centres of earlier picks of this kind
  const int ncen = discord ? q : 2 * q;
  const int64_t *src = st->centres + (discord ? 2 * km : 0);
  for (int c = tid; c < ncen; c += blockDim.x) cen[c] = src[c];
  __syncthreads();
  const double sign = discord ? -1.0 : 1.0;
  double best = INFINITY;
  int64_t arg = -1;
  if (!st->done) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + tid; x < l; x += (int64_t)gridDim.x * blockDim.x) {
      const double p = (double)P[x];
      if (!isfinite(p)) continue;
      bool masked = false;
      for (int c = 0; c < ncen; ++c) masked |= llabs(x - cen[c]) <= m;
      if (masked) continue;
      const double v = sign * p;
      if (v < best) { best = v; arg = x; }
    }
  }
  auto reduce = [&]() {
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
  };
  reduce();
  if (tid == 0) {
    st->pv[blockIdx.x] = bv[0];
    st->pi[blockIdx.x] = bi[0];
    __threadfence();
    last = (atomicAdd(&st->ticket, 1u) == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  best = INFINITY;
  arg = -1;
  for (int b = tid; b < (int)gridDim.x; b += blockDim.x) {
    const volatile double *pv = st->pv;
    const volatile int64_t *pi = st->pi;
    const double v = pv[b];
    const int64_t i = pi[b];
    if (i >= 0 && (arg < 0 || v < best || (v == best && i < arg))) { best = v; arg = i; }
  }
  reduce();
  // The chosen pair, re-measured in FP64 by the whole workgroup (each sum,
  // minimum and maximum over the m samples is a tree over the threads).
  const int64_t i = bi[0];
  const int64_t j = (i >= 0) ? I[i] : -1;
  __syncthreads();
  auto bred = [&](double v, int op) -> double {  // 0 sum, 1 min, 2 max
    bv[tid] = v;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
      if (tid < h) {
        const double a = bv[tid], b = bv[tid + h];
        bv[tid] = op == 0 ? a + b : (op == 1 ? fmin(a, b) : fmax(a, b));
      }
      __syncthreads();
    }
    const double r = bv[0];
    __syncthreads();
    return r;
  };
  double d = INFINITY;
  if (i >= 0 && j >= 0) {
    auto stats = [&](int64_t w, double &mu, double &sg, bool &cst) {
      double s = 0.0, lo = INFINITY, hi = -INFINITY;
      for (int u = tid; u < m; u += blockDim.x) {
        const double v = sample(T + w + u);
        lo = fmin(lo, v);
        hi = fmax(hi, v);
        s += v;
      }
      mu = bred(s, 0) / m;
      lo = bred(lo, 1);
      hi = bred(hi, 2);
      double qq = 0.0;
      for (int u = tid; u < m; u += blockDim.x) {
        const double dv = sample(T + w + u) - mu;
        qq = fma(dv, dv, qq);
      }
      sg = sqrt(bred(qq, 0) / m);
      cst = (lo == hi);
    };
    double mi, si, mj, sj;
    bool ci, cj;
    stats(i, mi, si, ci);
    stats(j, mj, sj, cj);
    const double ia = ci ? 0.0 : 1.0 / si, ib = cj ? 0.0 : 1.0 / sj;
    double acc = 0.0;
    for (int u = tid; u < m; u += blockDim.x) {
      const double e = (sample(T + i + u) - mi) * ia - (sample(T + j + u) - mj) * ib;
      acc = fma(e, e, acc);
    }
    d = sqrt(bred(acc, 0));
  }
  if (tid == 0) {
    st->ticket = 0;
    if (!discord) {
      const bool ok = (i >= 0 && j >= 0);
      out_idx[2 * q] = ok ? i : -1;
      out_idx[2 * q + 1] = ok ? j : -1;
      out_dist[q] = ok ? d : INFINITY;
      if (ok) {
        st->centres[2 * q] = i;
        st->centres[2 * q + 1] = j;
      } else {
        st->done = 1;
      }
    } else {
      out_idx[2 * km + q] = i;
      out_dist[km + q] = (i >= 0 && j >= 0) ? d : INFINITY;
      if (i >= 0) st->centres[2 * km + q] = i; else st->done = 1;
    }
  }
}

__global__ void k_recheck_init(RecheckState *st) {
  if (threadIdx.x == 0) {
    st->ticket = 0;
    st->done = 0;
  }
}

__global__ void k_recheck_phase(RecheckState *st) {
  if (threadIdx.x == 0) st->done = 0;   // discords do not depend on motif exhaustion
}

hipError_t launch_recheck(const void *T, bool t_f64, int64_t n, int32_t m, const void *P,
                          bool p_f64, const int64_t *I, int32_t km, int32_t kd, int64_t *out_idx,
                          double *out_dist, uint8_t *ws, hipStream_t st) {
  RecheckState *rs = reinterpret_cast<RecheckState *>(ws);
  const int64_t l = n - m + 1;
  const int grid = (int)std::min<int64_t>(kRecheckBlocks, std::max<int64_t>(1, (l + 255) / 256));
  hipLaunchKernelGGL(k_recheck_init, dim3(1), dim3(64), 0, st, rs);
  for (int pass = 0; pass < 2; ++pass) {
    const int k = pass == 0 ? km : kd;
    if (pass == 1) hipLaunchKernelGGL(k_recheck_phase, dim3(1), dim3(64), 0, st, rs);
    for (int q = 0; q < k; ++q) {
#define MPX_PICK(TIN, TP)                                                                      \
  hipLaunchKernelGGL((k_pick<TIN, TP>), dim3(grid), dim3(256), 0, st, (const TIN *)T, n, m,  \
                     (const TP *)P, I, pass, q, km, out_idx, out_dist, rs)
      if (t_f64) {
        if (p_f64) MPX_PICK(double, double); else MPX_PICK(double, float);
      } else {
        if (p_f64) MPX_PICK(float, double); else MPX_PICK(float, float);
      }
#undef MPX_PICK
    }
  }
  return hipGetLastError();
}

size_t recheck_state_bytes() { return sizeof(RecheckState); }

}  // namespace mpx
