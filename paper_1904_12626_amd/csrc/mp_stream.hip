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
// candidate of another in the same batch): a one-wave workgroup owns
// 64*8 - (B-1) consecutive columns and also recomputes the B-1 columns to
// their left, whose cross products it needs (a trapezoid: after step b the
// leftmost b columns hold stale values, and none of them is owned); the
// first workgroup, which starts at column 0, owns all 64*8 of its columns.  Each
// lane keeps its eight columns' terms in registers for all B rows and the
// cross products move right through registers and one DPP shift per step,
// so a column's data is read once per batch and no step needs a barrier.
#include <cmath>
#include <type_traits>
#include <utility>

#include "mp_internal.h"
#include "mp_types.h"

namespace mpx {

namespace {

// Lane `lane`'s value of x (lane index wave-uniform).
__device__ __forceinline__ double lane_value(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
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

// The same for a few windows, one wave per window (lanes split the
// samples; FP64 sums by butterfly), plus C(w, 0): column 0 has no left
// neighbour to continue from, so its cross products are direct.
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Window w_lo - 1 (an old window whose successor sample has just arrived)
// only gets its a and g terms.
template <typename Tin>
__global__ void __launch_bounds__(64) k_stream_stats_wave(StreamWork s, const Tin *__restrict__ T, int64_t n,
                                                          int m, int64_t w_lo) {
  const int64_t w = w_lo - 1 + blockIdx.x;
  const int lane = threadIdx.x;
  const Tin *x = T + w;
  if (blockIdx.x == 0) {
    if (lane == 0 && w >= 0) {
      const double a = (w + m < n) ? smp(x + m) - smp(x) : 0.0;
      s.a[w] = a;
      s.g[w] = smp(x) - s.mu[w] + a * (double)(m - 1) / (2.0 * m);
    }
    return;
  }
  bool ok = true;
  double sum = 0.0, lo = INFINITY, hi = -INFINITY;
  for (int u = lane; u < m; u += 64) {
    const double v = (double)x[u];
    if (!isfinite(v)) ok = false;
    const double c = isfinite(v) ? v : 0.0;
    lo = fmin(lo, c);
    hi = fmax(hi, c);
    sum += c;
  }
  ok = __all(ok);
  sum = wsum(sum);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  const double mu = sum / m, mu0 = s.mu[0];
  double q = 0.0, c0 = 0.0;
  for (int u = lane; u < m; u += 64) {
    const double dv = smp(x + u) - mu;
    q = fma(dv, dv, q);
    c0 = fma(dv, smp(T + u) - mu0, c0);
  }
  q = wsum(q);
  c0 = wsum(c0);
  if (lane == 0) {
    const bool cst = ok && (lo == hi || !(q > 0.0));
    s.mu[w] = mu;
    s.isd[w] = (ok && !cst) ? 1.0 / (sqrt((double)m) * sqrt(q / m)) : 0.0;
    s.flags[w] = (uint8_t)((ok ? 1 : 0) | (cst ? 2 : 0));
    const double a = (w + m < n) ? smp(x + m) - smp(x) : 0.0;
    s.a[w] = a;
    s.g[w] = smp(x) - mu + a * (double)(m - 1) / (2.0 * m);
    s.col0[w] = c0;
  }
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

// Cross products C(w, j) of window w with every j <= jmax, directly; eight
// consecutive columns per thread share their sample loads (column sample
// j0 + v meets window sample v - t in column j0 + t):
// C = sum (x_w - mu_w) x_j - mu_j sum (x_w - mu_w).
template <typename Tin>
__global__ void __launch_bounds__(256) k_stream_seed(StreamWork s, const Tin *__restrict__ T, int m,
                                                     int64_t w, int64_t jmax, double *C) {
  constexpr int K = 8;
  const int64_t j0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * K;
  if (j0 > jmax) return;
  const double mw = s.mu[w];
  double acc[K], xr[K];
#pragma unroll
  for (int t = 0; t < K; ++t) { acc[t] = 0.0; xr[t] = 0.0; }
  double Sx = 0.0;
  for (int vb = 0; vb < m + K - 1; vb += K) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int v = vb + q;
      double xn = 0.0;
      if (v < m) xn = smp(T + w + v) - mw;
      Sx += xn;
      xr[q] = xn;
      const int64_t ci = j0 + v;
      const double y = ci <= jmax + m - 1 ? smp(T + ci) : 0.0;
#pragma unroll
      for (int t = 0; t < K; ++t) acc[t] = fma(xr[(q - t + K) % K], y, acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < K; ++t)
    if (j0 + t <= jmax) C[j0 + t] = acc[t] - s.mu[j0 + t] * Sx;
}

// One batch of B new windows w0 .. w0+B-1 (see the file comment), one wave
// per workgroup.  Lane L holds the DT consecutive columns
// cbase + L*DT + t; at each step every column continues its left
// neighbour's cross product, kept in place in a register ring (slot t at
// step b works in register (t - b) mod DT, which holds slot t-1's value of
// step b-1; slot 0 takes lane L-1's through one DPP shift).  Keys carry a
// code in their low mantissa bits: the column (lane*DT + t) in the row key,
// the step b in the column key, so each minimum is one FP64 min.  Row
// minima of every step go to LDS and are reduced every 16 steps into one
// partial per wave and row; each column's minimum over the batch stays in a
// register and is merged into the profile at the end.
constexpr int kStreamSlots = 8;
constexpr int kStreamWidth = 64 * kStreamSlots;

// The low bits `mask` of v replaced by code (< mask + 1): one bitfield
// insert, (mask & code) | (~mask & low word); a per-lane code with the mask
// in a scalar register, or a wave-uniform code under the mask 63.
__device__ __forceinline__ double key_code(double v, unsigned code, unsigned mask) {
  const long long b = __double_as_longlong(v);
  unsigned lo;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(lo) : "s"(mask), "v"(code), "v"((unsigned)(b & 0xffffffffll)));
  return __longlong_as_double((b & ~0xffffffffll) | lo);
}
__device__ __forceinline__ double key_code63(double v, unsigned code) {
  const long long b = __double_as_longlong(v);
  unsigned lo;
  asm("v_bfi_b32 %0, 63, %1, %2" : "=v"(lo) : "s"(code), "v"((unsigned)(b & 0xffffffffll)));
  return __longlong_as_double((b & ~0xffffffffll) | lo);
}
__device__ __forceinline__ double key_value(double k, unsigned mask) {
  return __longlong_as_double(__double_as_longlong(k) & ~(long long)mask);
}
__device__ __forceinline__ unsigned key_code_of(double k, unsigned mask) {
  return (unsigned)(__double_as_longlong(k) & 0xffffffffll) & mask;
}
// keys are never NaN: the plain instruction, without NaN quieting
__device__ __forceinline__ double kmin(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// maximum with a wave-uniform bound (a plain instruction: no NaN arrives)
__device__ __forceinline__ double kmax_s(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(b));
  return r;
}
// lane L takes lane L-1's value; lane 0 keeps `old0`
__device__ __forceinline__ double shr1_keep(double old0, double v) {
  const long long b = __double_as_longlong(v), f = __double_as_longlong(old0);
  const int lo = __builtin_amdgcn_update_dpp((int)(f & 0xffffffffll), (int)(b & 0xffffffffll),
                                             0x138 /* wave_shr:1 */, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(b >> 32), 0x138, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename Fn, int... Ts>
__device__ __forceinline__ void sfor_impl(Fn &&f, std::integer_sequence<int, Ts...>) {
  (f(std::integral_constant<int, Ts>{}), ...);
}
template <int N, typename Fn>
__device__ __forceinline__ void sfor(Fn &&f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

template <typename Tin>
__global__ void __launch_bounds__(64) k_stream_batch(StreamWork s, const Tin *__restrict__ T, int m, int ez,
                                                     int64_t w0, int B, bool seed,
                                                     const double *__restrict__ Cprev, double *Cnew, int64_t *I,
                                                     int64_t nparts) {
  constexpr int DT = kStreamSlots, W = kStreamWidth;
  constexpr unsigned kRowMask = W - 1;  // column code: 9 bits
  constexpr unsigned kColMask = 63;     // step code: B <= 63 (key_code63)
  constexpr double kHuge = 1.0e300;
  __shared__ double lrow[16][65];
  __shared__ double lpart[64];
  __shared__ double lpd[kStreamWidth];  // profile of the owned columns
  const int lane = threadIdx.x;
  const bool first = blockIdx.x == 0;
  // Workgroup 0 owns columns 0 .. W-1 (column 0 sits in lane 0, slot 0 and
  // takes its precomputed products as the DPP fallback value); workgroup
  // k >= 1 owns W - H columns after a halo of H = B - 1.
  const int H = first ? 0 : B - 1;
  const int64_t cbase = first ? 0 : (int64_t)W + (int64_t)(blockIdx.x - 1) * (W - (B - 1)) - (B - 1);
  const int64_t jlast = w0 + B - 1 - ez - 1;  // last column any row scores
  const int64_t jprev = w0 - ez - 2;           // last column of C(w0 - 1, .)
  // the last columns of this wave become admissible during the batch
  const bool ramp = cbase + W - 1 > w0 - ez - 1;

  // Column state is read with contiguous loads (position e = lane + 64q of
  // the workgroup's columns) and handed to the lane owning it (positions
  // lane*DT .. lane*DT + DT-1) through LDS; the staging buffer is the row
  // minima buffer, unused until the first step.
  double *const lst = &lrow[0][0];
  auto pos = [](int e) { return e + (e >> 3); };  // one pad per 8 columns
  auto to_lanes = [&](const double (&v)[DT], double (&out)[DT]) {
#pragma unroll
    for (int q = 0; q < DT; ++q) lst[pos(lane + 64 * q)] = v[q];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < DT; ++t) out[t] = lst[pos(lane * DT + t)];
    __syncthreads();
  };
  unsigned code[DT];
  double aj1[DT], gj1[DT], sj[DT], vj[DT], R[DT], cm[DT];
  {
    // contiguous loads of every array first (all in flight together)
    double va[DT], vg[DT], vs[DT], vv[DT], vc[DT], vpd[DT];
    const int64_t cfirst = seed ? cbase : cbase - 1;  // C(w0, j) or C(w0 - 1, j - 1)
    const int64_t clast = seed ? w0 - ez - 1 : jprev;
#pragma unroll
    for (int q = 0; q < DT; ++q) {
      const int e = lane + 64 * q;
      const int64_t j = cbase + e;
      va[q] = 0.0;
      vg[q] = 0.0;
      vs[q] = 0.0;
      vv[q] = kHuge;  // no candidate: halo, outside the columns, invalid
      vpd[q] = INFINITY;
      if (j >= 0 && j <= jlast) {
        if (j >= 1) {
          va[q] = s.a[j - 1];
          vg[q] = s.g[j - 1];
        }
        const uint8_t f = s.flags[j];
        vs[q] = s.isd[j];
        if (e >= H && (f & 1)) vv[q] = (f & 2) ? -0.5 : 0.0;
        if (e >= H) vpd[q] = s.Pd[j];
      }
      const int64_t c = cfirst + e;
      vc[q] = (c >= 0 && c <= clast) ? Cprev[c] : 0.0;
    }
    // the profile of the owned columns waits in LDS for the final merges
#pragma unroll
    for (int q = 0; q < DT; ++q) lpd[lane + 64 * q] = vpd[q];
    to_lanes(va, aj1);
    to_lanes(vg, gj1);
    to_lanes(vs, sj);
    to_lanes(vv, vj);
    // register t feeds slot t at step 0 with C(w0 - 1, j - 1) (staged from
    // column cbase - 1, so slot t reads position lane*DT + t); register 0
    // is shifted one lane right first, so it holds this lane's last column
    // (position lane*DT + DT).  A re-seeded batch instead finds C(w0, j)
    // itself (direct products) in the same buffer, staged from cbase.
    {
#pragma unroll
      for (int q = 0; q < DT; ++q) lst[pos(lane + 64 * q)] = vc[q];
      if (lane == 0) {
        const int64_t c = cfirst + W;
        lst[pos(W)] = (c >= 0 && c <= clast) ? Cprev[c] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < DT; ++t) R[t] = lst[pos(lane * DT + (seed ? t : (t == 0 ? DT : t)))];
      __syncthreads();
    }
  }
#pragma unroll
  for (int t = 0; t < DT; ++t) {
    code[t] = (unsigned)(lane * DT + t);
    cm[t] = kHuge;
  }
  // lane 0's left neighbour at step 0 (later its first columns are stale,
  // and none of them is owned)
  const double c_left = (cbase - 1 >= 0 && cbase - 1 <= jprev) ? Cprev[cbase - 1] : 0.0;
  // The window terms of every step, lane b holding step b's (read by the
  // steps with lane reads, so that no step waits on memory): g and a of
  // window w - 1, s and the row term u of window w, and (workgroup 0)
  // C(w, 0).
  double tg = 0.0, ta = 0.0, ts = 0.0, tu = kHuge, tc0 = 0.0;
  if (lane < B) {
    const int64_t w = w0 + lane;
    tg = s.g[w - 1];
    ta = s.a[w - 1];
    ts = s.isd[w];
    const uint8_t fw = s.flags[w];
    tu = (fw & 1) ? ((fw & 2) ? 0.5 : 1.0) : kHuge;
    if (first) tc0 = s.col0[w];
  }

  int fb = 0;  // first step not yet flushed
  auto flush = [&](int nb) {
    __syncthreads();
    {
      const int r = lane & 15, g0 = (lane >> 4) * 16;
      double best = lrow[r][g0];
#pragma unroll
      for (int e = 1; e < 16; ++e) best = kmin(best, lrow[r][g0 + e]);
      lpart[lane] = best;
    }
    __syncthreads();
    if (lane < nb) {
      double best = kmin(kmin(lpart[lane], lpart[lane + 16]), kmin(lpart[lane + 32], lpart[lane + 48]));
      const double v = key_value(best, kRowMask);
      const bool hit = v < 1.0e299;
      const int64_t at = (int64_t)(fb + lane) * nparts + blockIdx.x;
      s.part_d[at] = hit ? v : INFINITY;
      s.part_j[at] = hit ? cbase + key_code_of(best, kRowMask) : -1;
    }
    __syncthreads();
  };

  // The B steps; RAMP (a uniform choice per workgroup, taken outside the
  // loop) masks the columns that are not yet admissible.
  auto run = [&](auto ramp_c) {
    constexpr bool RAMP = decltype(ramp_c)::value;
    for (int bb = 0; bb < B; bb += DT) {
      sfor<DT>([&](auto uc) {
        constexpr int u = decltype(uc)::value;
        const int b = bb + u;
        if (b < B) {
          const int64_t w = w0 + b;
          const double gw1 = lane_value(tg, b), aw1 = lane_value(ta, b), sw = lane_value(ts, b);
          const double uw = lane_value(tu, b);
          constexpr int r0 = (DT - u) % DT;  // register of slot 0
          bool direct = false;
          if constexpr (u == 0) direct = seed && b == 0;
          if (!direct) {
            const double keep = first ? lane_value(tc0, b) : (b == 0 ? c_left : R[r0]);
            R[r0] = shr1_keep(keep, R[r0]);
          }
          int lim = W;
          if constexpr (RAMP) lim = (int)min(max(w - ez - 1 - cbase, (int64_t)-1), (int64_t)W);
          double rk[DT];
#pragma unroll
          for (int t = 0; t < DT; ++t) {
            double &C = R[(t + r0) % DT];
            if (!direct) C = fma(aj1[t], gw1, fma(aw1, gj1[t], C));
            double key = kmax_s(fma(-(C * sw), sj[t], uw + vj[t]), 0x1p-1000);
            if constexpr (RAMP) {
              if ((int)code[t] > lim) key = kHuge;  // not yet admissible
            }
            rk[t] = key_code(key, code[t], kRowMask);
            cm[t] = kmin(cm[t], key_code63(key, (unsigned)b));
          }
          // the lane's row minimum as a tree (depth 3, not a chain of 8)
          static_assert(DT == 8, "tree below");
          const double rmin = kmin(kmin(kmin(rk[0], rk[1]), kmin(rk[2], rk[3])),
                                   kmin(kmin(rk[4], rk[5]), kmin(rk[6], rk[7])));
          lrow[b & 15][lane] = rmin;
          if ((b & 15) == 15) {
            flush(16);
            fb = b + 1;
          }
        }
      });
    }
  };
  if (ramp) run(std::true_type{});
  else run(std::false_type{});
  if (fb < B) flush(B - fb);

  // C(w0 + B - 1, j) for the next batch (staged through LDS for contiguous
  // stores) and the column merges (owned columns only).  The lane index is
  // passed through an empty asm so that the staging addresses are computed
  // afresh here instead of being kept in registers through the steps.
  int lane_e = lane;
  asm volatile("" : "+v"(lane_e));
  const int last = (B - 1) % DT;  // phase of the last step
  sfor<DT>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    if (p == last) {
      constexpr int r0 = (DT - p) % DT;
#pragma unroll
      for (int t = 0; t < DT; ++t) {
        const int e = lane_e * DT + t;
        const int64_t j = cbase + e;
        lst[pos(e)] = R[(t + r0) % DT];
        if (e >= H && j >= 0 && j <= jlast) {
          const double v = key_value(cm[t], kColMask);
          if (v < 1.0e299 && v < lpd[e]) {
            s.Pd[j] = v;
            I[j] = w0 + (int64_t)key_code_of(cm[t], kColMask);
          }
        }
      }
    }
  });
  __syncthreads();
#pragma unroll
  for (int q = 0; q < DT; ++q) {
    const int e = lane_e + 64 * q;
    const int64_t j = cbase + e;
    if (e >= H && j >= 0 && j <= jlast) Cnew[j] = lst[pos(e)];
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
// partial row minima: up to kStreamMaxBatch rows x one per workgroup of
// >= kStreamWidth - (kStreamMaxBatch - 1) owned columns
int64_t stream_partials(int64_t l_max) {
  constexpr int64_t owned = kStreamWidth - (kStreamMaxBatch - 1);
  return (int64_t)kStreamMaxBatch * ((l_max + owned - 1) / owned + 1);
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
    hipLaunchKernelGGL((k_stream_seed<Tin>), dim3((unsigned)((jmax / 8 + 256) / 256)), b, 0, st, s, T, m, w, jmax,
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
  hipLaunchKernelGGL((k_stream_stats_wave<Tin>), dim3((unsigned)(l_new - l_old + 1)), dim3(64), 0, st, s, T, n_new,
                     m, l_old);
  const int bmax = (int)std::min<int64_t>(kStreamMaxBatch, (int64_t)ez + 1);
  for (int64_t w0 = l_old; w0 < l_new;) {
    int B = (int)std::min<int64_t>(bmax, l_new - w0);
    // a re-seeded window (a multiple of `reseed`) always opens a batch
    const int64_t next_seed = (w0 / reseed + 1) * reseed;
    if (next_seed < w0 + B) B = (int)(next_seed - w0);
    if ((B & 1) == 0) --B;
    const bool seed = w0 % reseed == 0;
    const int64_t jlast = w0 + B - 1 - ez - 1;
    if (jlast < 0) {  // no candidates yet: one window at a time
      hipLaunchKernelGGL(k_stream_rowfin, dim3(1), dim3(256), 0, st, s, w0, (int64_t)0, I);
      ++w0;
      continue;
    }
    // workgroup 0: columns 0 .. W-1; then W - (B-1) columns each
    const int owned = kStreamWidth - (B - 1);
    const int64_t nblocks = 1 + std::max<int64_t>(0, (jlast + 1 - kStreamWidth + owned - 1) / owned);
    const int64_t nparts = nblocks;
    if (seed && w0 - ez - 1 >= 0)  // C(w0, j) by direct products into the buffer the batch reads
      hipLaunchKernelGGL((k_stream_seed<Tin>), dim3((unsigned)(((w0 - ez - 1) / 8 + 256) / 256)), b, 0, st, s, T, m,
                         w0, w0 - ez - 1, s.C[(w0 - 1) & 1]);
    hipLaunchKernelGGL((k_stream_batch<Tin>), dim3((unsigned)nblocks), dim3(64), 0, st, s, T, m, ez, w0,
                       B, seed, (const double *)s.C[(w0 - 1) & 1], s.C[(w0 + B - 1) & 1], I, nparts);
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
