// Multidimensional joins: SiMPle (Section 3.3.4: no z-normalisation, the
// distance summed over all dimensions) and the multidimensional profiles of
// Section 3.3.5 (per-dimension z-normalised distances, sorted, the
// k-dimensional distance being the mean of the k smallest).  A series has D
// dimensions sampled together, stored dimension-major: dimension d of a
// series of n samples starts d*n values after its first sample.
//
// Same diagonal order as the one-dimensional sweep (tiles of R rows of a
// strip of 64 diagonals, one wave per tile, persistent grid), with a simpler
// register layout: lane L owns diagonal k0 + L, so at row i it scores the
// cell (i, i + k0 + L).  Per dimension the centred cross product C advances
// with C += a_j g_i + a_i g_j in FP64 (seeded in FP64 at the tile's first
// row); column records are loaded per lane (consecutive lanes, consecutive
// columns), row records are wave-uniform.  Every cell yields one value per
// output profile, packed as (float value bits << 32 | partner index); row
// minima are wave reductions, column minima travel one lane down per row
// and leave through lane 0, and both merge into global words with a 64-bit
// atomic minimum (order independent: deterministic).
#include <cmath>

#include "mp_internal.h"
#include "mp_types.h"

namespace mpx {

namespace {

constexpr double kHuge = 1.0e300;

__device__ __forceinline__ double clean_md(double v) { return isfinite(v) ? v : 0.0; }

__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Load of a wave-uniform address through the constant address space, so that
// it becomes a scalar load (the records were written by an earlier kernel
// and are read-only here).
template <typename T>
__device__ __forceinline__ T ldu_md(const T *p) {
#if defined(__HIP_DEVICE_COMPILE__)
  static_assert(sizeof(T) % 4 == 0, "whole dwords");
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

// Minimum over the wave of a 32-bit value, returned wave-uniform: a
// reduction inside each row of 16 lanes by DPP row shifts (lane 15 of a row
// ends with the row's minimum), then the four row minima on the scalar unit.
__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x111 /* row_shr:1 */, 0xF, 0xF, false));
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x112 /* row_shr:2 */, 0xF, 0xF, false));
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x114 /* row_shr:4 */, 0xF, 0xF, false));
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x118 /* row_shr:8 */, 0xF, 0xF, false));
  const unsigned r0 = __builtin_amdgcn_readlane(v, 15), r1 = __builtin_amdgcn_readlane(v, 31);
  const unsigned r2 = __builtin_amdgcn_readlane(v, 47), r3 = __builtin_amdgcn_readlane(v, 63);
  return min(min(r0, r1), min(r2, r3));
}

// Lane L takes lane L+1's value; lane 63 takes `fill` (wave-uniform).
__device__ __forceinline__ unsigned shift_down1(unsigned v, unsigned fill) {
  int x = __builtin_amdgcn_update_dpp((int)v, (int)v, 0x130 /* wave_shl:1 */, 0xF, 0xF, false);
  const int f = __builtin_amdgcn_readfirstlane((int)fill);
  asm volatile("v_writelane_b32 %0, %1, 63" : "+v"(x) : "s"(f));
  return (unsigned)x;
}

__device__ __forceinline__ unsigned long long pack_md(float v, int64_t idx) {
  v = v > 0.0f ? v : 0.0f;
  return ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(uint32_t)idx;
}

__device__ __forceinline__ int find_series_md(const Plan &plan, int64_t wi) {
  return (plan.nseries > 1 && wi >= plan.s_inl[1].w_off) ? 1 : 0;
}

}  // namespace

// Per window and dimension two records.  rec = {a, g, c, e} with
// a = x[w+m] - x[w], g = x[w] - mu + a (m-1)/(2m) (the cross-product
// recurrence) and, for SiMPle, c = mu and e = Q = sum_d m sigma_d^2 (kept in
// dimension 0); for the multidimensional profiles c = s = 1/(sqrt(m) sigma)
// (0 for a constant dimension) and e = v, the column term of
// key = u_i + v_j - C s_i s_j, which is d^2/(2m) for every mix of constant
// and varying windows (u = 1 - c/2, v = -c/2, c = 1 for a constant
// dimension).  mu = {mean, u}.  A window with a non-finite sample in any
// dimension gets Q = u = v = huge; so do the 64 padding records after each
// series (and a = g = 0 there).
template <typename Tin, int MODE>
__global__ void __launch_bounds__(256) k_md_stats(Plan plan, int D, const Tin *__restrict__ Tb, Double4 *rec,
                                                  double2 *mu2, int64_t stride, int64_t total_rc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= total_rc) return;
  const int si = (plan.nseries > 1 && r >= plan.s_inl[1].rc_off) ? 1 : 0;
  const SeriesDesc S = plan.s_inl[si];
  const int64_t w = r - S.rc_off;
  if (w >= S.l) {
    for (int d = 0; d < D; ++d) {
      rec[d * stride + r] = Double4{0.0, 0.0, 0.0, kHuge};
      mu2[d * stride + r] = make_double2(0.0, kHuge);
    }
    return;
  }
  const int m = S.m;
  bool ok = true;
  double Q = 0.0;
  for (int d = 0; d < D; ++d) {
    const Tin *x = Tb + S.t_off + (int64_t)d * S.n + w;
    double s = 0.0, lo = 0.0, hi = 0.0;
    for (int u = 0; u < m; ++u) {
      const double v = (double)x[u];
      if (!isfinite(v)) ok = false;
      const double c = clean_md(v);
      if (u == 0) { lo = c; hi = c; }
      lo = fmin(lo, c);
      hi = fmax(hi, c);
      s += c;
    }
    const double mu = s / m;
    double q = 0.0;
    for (int u = 0; u < m; ++u) {
      const double dv = clean_md((double)x[u]) - mu;
      q = fma(dv, dv, q);
    }
    const double a = (w + 1 < S.l) ? clean_md((double)x[m]) - clean_md((double)x[0]) : 0.0;
    const double g = clean_md((double)x[0]) - mu + a * (double)(m - 1) / (2.0 * m);
    const bool cst = (lo == hi) || !(q > 0.0);
    const double sg = sqrt(q / m);
    Q += q;
    if (MODE == kMdSimple) {
      rec[d * stride + r] = Double4{a, g, mu, 0.0};
      mu2[d * stride + r] = make_double2(mu, 0.0);
    } else {
      rec[d * stride + r] = Double4{a, g, cst ? 0.0 : 1.0 / (sqrt((double)m) * sg), cst ? -0.5 : 0.0};
      mu2[d * stride + r] = make_double2(mu, cst ? 0.5 : 1.0);
    }
  }
  if (MODE == kMdSimple) rec[r].w = ok ? Q : kHuge;
  if (!ok && MODE == kMdMulti)
    for (int d = 0; d < D; ++d) {
      rec[d * stride + r].w = kHuge;
      mu2[d * stride + r].y = kHuge;
    }
}

__global__ void __launch_bounds__(256) k_md_clear(unsigned long long *keys, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    keys[x] = ~0ull;
}

// Sorting network (odd-even transposition) on N floats, ascending.
template <int N>
__device__ __forceinline__ void sort_net(float (&v)[N]) {
#pragma unroll
  for (int p = 0; p < N; ++p) {
#pragma unroll
    for (int i = (p & 1); i + 1 < N; i += 2) {
      const float a = v[i], b = v[i + 1];
      v[i] = fminf(a, b);
      v[i + 1] = fmaxf(a, b);
    }
  }
}

template <typename Tin, int D, int MODE>
__global__ void __launch_bounds__(64) k_md_sweep(const Plan plan, const Tin *__restrict__ Tb,
                                                 const Double4 *__restrict__ rec,
                                                 const double2 *__restrict__ mu2, int64_t stride,
                                                 const int64_t *__restrict__ seg_prefix,
                                                 const int32_t *__restrict__ seg_sweep,
                                                 unsigned long long *__restrict__ keys, int64_t kstride,
                                                 unsigned long long *__restrict__ counter, int R,
                                                 int64_t total_tiles, int64_t nseg) {
  constexpr int NP = (MODE == kMdMulti) ? D : 1;
  // column records of the 127 columns that 64 rows x 64 diagonals touch
  __shared__ Double4 lcol[D][128];
  const int lane = threadIdx.x;
  for (;;) {
    int64_t tile = 0;
    if (lane == 0) tile = (int64_t)atomicAdd(counter, 1ull);
    tile = uni(tile);
    if (tile >= total_tiles) break;
    int64_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (seg_prefix[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    const int64_t g = uni(lo);
    const SweepDesc sd = plan.sweep(seg_sweep[g]);
    const SeriesDesc RS = plan.series(sd.rs), CS = plan.series(sd.cs);
    const int64_t k0 = uni(sd.k_lo + (g - sd.seg_base) * 64);
    const int64_t L = min(RS.l, CS.l - k0);
    const int64_t i0 = uni((tile - seg_prefix[g]) * (int64_t)R);
    const int64_t nr = uni(min((int64_t)R, L - i0));
    const int64_t lc = CS.l;
    const int m = RS.m;
    const int64_t rrow = uni(RS.rc_off + i0);  // record of the tile's first row
    unsigned long long *rkeys = keys + plan.series(sd.rk).w_off;
    unsigned long long *ckeys = keys + plan.series(sd.ck).w_off;
    const int64_t j0 = i0 + k0 + lane;  // this lane's column at the tile's first row

    // FP64 seeds: C_d = sum_u (x_r - mu_r)(x_c - mu_c)
    double C[D];
    for (int d = 0; d < D; ++d) {
      double acc = 0.0;
      if (j0 < lc) {
        const Tin *xr = Tb + RS.t_off + (int64_t)d * RS.n + i0;
        const Tin *xc = Tb + CS.t_off + (int64_t)d * CS.n + j0;
        const double mr = mu2[d * stride + RS.rc_off + i0].x, mc = mu2[d * stride + CS.rc_off + j0].x;
        for (int u = 0; u < m; ++u)
          acc = fma(clean_md((double)xr[u]) - mr, clean_md((double)xc[u]) - mc, acc);
      }
      C[d] = acc;
    }
    unsigned long long CM[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) CM[p] = ~0ull;

    for (int64_t rb = 0; rb < nr; rb += 64) {
      // stage the columns of rows i0+rb .. i0+rb+63 (coalesced, two per lane)
      const int64_t cb = CS.rc_off + i0 + rb + k0;
      __syncthreads();
#pragma unroll
      for (int d = 0; d < D; ++d) {
        lcol[d][lane] = rec[d * stride + cb + lane];
        lcol[d][64 + lane] = rec[d * stride + cb + 64 + lane];
      }
      __syncthreads();
      const int rn = __builtin_amdgcn_readfirstlane((int)min((int64_t)64, nr - rb));
      for (int r = 0; r < rn; ++r) {
        const int64_t i = i0 + rb + r;
        const int64_t ri_off = uni(rrow + rb + r);
        float val[NP];
        if (MODE == kMdSimple) {
          double d2 = ldu_md(&rec[ri_off].w) + lcol[0][r + lane].w;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const Double4 ri = ldu_md(rec + d * stride + ri_off), cj = lcol[d][r + lane];
            const double dm = ri.z - cj.z;
            d2 = fma((double)m * dm, dm, d2);
            d2 = fma(-2.0, C[d], d2);
            C[d] = fma(cj.x, ri.y, C[d]);
            C[d] = fma(ri.x, cj.y, C[d]);
          }
          val[0] = (float)d2;
        } else {
          float dist[D];
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const Double4 ri = ldu_md(rec + d * stride + ri_off), cj = lcol[d][r + lane];
            const double key = ldu_md(&mu2[d * stride + ri_off].y) + cj.w - C[d] * ri.z * cj.z;
            dist[d] = sqrtf((float)(2.0 * m * fmax(key, 0.0)));
            C[d] = fma(cj.x, ri.y, C[d]);
            C[d] = fma(ri.x, cj.y, C[d]);
          }
          sort_net<D>(dist);
          float run = 0.0f;
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            run += dist[p];
            val[p] = run / (float)(p + 1);
          }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          // row minimum: the smallest value, at its first lane (the smallest
          // column on equal values)
          const float vp = val[p] > 0.0f ? val[p] : 0.0f;
          const unsigned vb = __float_as_uint(vp);
          const unsigned mn = wave_min_u32(vb);
          const unsigned long long hit = __ballot(vb == mn);
          if (lane == 0 && __uint_as_float(mn) < 1.0e30f)
            atomicMin(rkeys + p * kstride + i,
                      ((unsigned long long)mn << 32) | (unsigned long long)(uint32_t)(i + k0 + __ffsll((long long)hit) - 1));
          const unsigned long long ck = pack_md(val[p], i);
          CM[p] = ck < CM[p] ? ck : CM[p];
          // lane 0's column (i + k0) has met every row of this tile it meets
          if (lane == 0 && i + k0 < lc && (float)__uint_as_float((unsigned)(CM[p] >> 32)) < 1.0e30f)
            atomicMin(ckeys + p * kstride + i + k0, CM[p]);
          const unsigned hi = shift_down1((unsigned)(CM[p] >> 32), 0xFFFFFFFFu);
          const unsigned lo = shift_down1((unsigned)CM[p], 0xFFFFFFFFu);
          CM[p] = ((unsigned long long)hi << 32) | lo;
        }
      }
    }
    // columns still in flight: lane L holds column i0 + nr + k0 + L
    const int64_t c = i0 + nr + k0 + lane;
    unsigned long long *cdst = ckeys + c;
    for (int p = 0; p < NP; ++p) {  // CM is read through a copy so that it stays in registers
      unsigned long long v = CM[0];
#pragma unroll
      for (int q = 1; q < NP; ++q) v = q == p ? CM[q] : v;
      if (c < lc && v != ~0ull && __uint_as_float((unsigned)(v >> 32)) < 1.0e30f) atomicMin(cdst + p * kstride, v);
    }
  }
}

// Exact FP64 value of the chosen pair; (+inf, -1) for invalid rows and rows
// without a candidate.
template <typename Tin, typename Tout, int MODE>
__global__ void __launch_bounds__(256) k_md_finalize(Plan plan, int D, const Tin *__restrict__ Tb,
                                                     const Double4 *__restrict__ rec,
                                                     const double2 *__restrict__ mu2, int64_t stride,
                                                     const unsigned long long *__restrict__ keys,
                                                     int64_t kstride, int np, Outputs o, int64_t total_l) {
  const int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wi >= total_l) return;
  const int si = find_series_md(plan, wi);
  const SeriesDesc S = plan.series(si), Q = plan.series(S.partner);
  const int64_t w = wi - S.w_off;
  const int m = S.m;
  const bool valid = MODE == kMdSimple ? rec[S.rc_off + w].w < 1.0e299 : mu2[S.rc_off + w].y < 1.0e299;
  for (int p = 0; p < np; ++p) {
    const unsigned long long k = keys[p * kstride + wi];
    double P = INFINITY;
    int64_t idx = -1;
    if (valid && k != ~0ull && __uint_as_float((unsigned)(k >> 32)) < 1.0e30f) {
      idx = (int64_t)(uint32_t)(k & 0xffffffffull);
      if (MODE == kMdSimple) {
        double s = 0.0;
        for (int d = 0; d < D; ++d) {
          const Tin *a = Tb + S.t_off + (int64_t)d * S.n + w;
          const Tin *b = Tb + Q.t_off + (int64_t)d * Q.n + idx;
          for (int u = 0; u < m; ++u) {
            const double e = (double)a[u] - (double)b[u];
            s = fma(e, e, s);
          }
        }
        P = sqrt(s);
      } else {
        double dist[8];
        for (int d = 0; d < D; ++d) {
          const Double4 ra = rec[d * stride + S.rc_off + w], rb = rec[d * stride + Q.rc_off + idx];
          const double ma = mu2[d * stride + S.rc_off + w].x, mb = mu2[d * stride + Q.rc_off + idx].x;
          const Tin *a = Tb + S.t_off + (int64_t)d * S.n + w;
          const Tin *b = Tb + Q.t_off + (int64_t)d * Q.n + idx;
          const double ia = ra.z * sqrt((double)m), ib = rb.z * sqrt((double)m);  // 1/sigma or 0
          double s = 0.0;
          for (int u = 0; u < m; ++u) {
            const double e = ((double)a[u] - ma) * ia - ((double)b[u] - mb) * ib;
            s = fma(e, e, s);
          }
          dist[d] = sqrt(s);
        }
        for (int x = 1; x < D; ++x)  // insertion sort, D <= 8
          for (int y = x; y > 0 && dist[y] < dist[y - 1]; --y) {
            const double t = dist[y];
            dist[y] = dist[y - 1];
            dist[y - 1] = t;
          }
        double run = 0.0;
        for (int t = 0; t <= p; ++t) run += dist[t];
        P = run / (p + 1);
      }
    }
    Tout *out = reinterpret_cast<Tout *>(o.P[S.out]);
    out[(int64_t)p * S.l + S.p_off + w] = (Tout)P;
    o.I[S.out][(int64_t)p * S.l + S.p_off + w] = idx;
  }
}

template <typename Tin, int MODE>
hipError_t launch_md_t(int D, const Plan &plan, const Tin *T, Double4 *rec, double2 *mu2, int64_t stride,
                       int64_t total_rc, unsigned long long *keys, int64_t kstride, const int64_t *seg_prefix,
                       const int32_t *seg_sweep, unsigned long long *counter, int R, int64_t total_tiles,
                       int64_t nseg, int grid, hipEvent_t ev0, hipEvent_t ev1, hipStream_t st) {
  const dim3 b256(256);
  const int np = MODE == kMdMulti ? D : 1;
  hipLaunchKernelGGL((k_md_stats<Tin, MODE>), dim3((unsigned)((total_rc + 255) / 256)), b256, 0, st, plan, D, T,
                     rec, mu2, stride, total_rc);
  hipLaunchKernelGGL(k_md_clear, dim3((unsigned)std::min<int64_t>((np * kstride + 255) / 256, 65536)), b256, 0,
                     st, keys, np * kstride);
  if (ev0) (void)hipEventRecord(ev0, st);
  if (total_tiles > 0) {
#define MPX_MD(DD)                                                                                     \
  case DD:                                                                                             \
    hipLaunchKernelGGL((k_md_sweep<Tin, DD, MODE>), dim3((unsigned)grid), dim3(64), 0, st, plan, T,  \
                       (const Double4 *)rec, (const double2 *)mu2, stride, seg_prefix, seg_sweep, keys, \
                       kstride, counter, R, total_tiles, nseg);                                        \
    break;
    switch (D) {
      MPX_MD(1) MPX_MD(2) MPX_MD(3) MPX_MD(4) MPX_MD(5) MPX_MD(6) MPX_MD(7) MPX_MD(8)
      default: return hipErrorInvalidValue;
    }
#undef MPX_MD
  }
  if (ev1) (void)hipEventRecord(ev1, st);
  return hipGetLastError();
}

template <typename Tin, typename Tout, int MODE>
hipError_t launch_md_fin_t(int D, const Plan &plan, const Tin *T, const Double4 *rec, const double2 *mu2,
                           int64_t stride, const unsigned long long *keys, int64_t kstride, const Outputs &o,
                           int64_t total_l, hipStream_t st) {
  const int np = MODE == kMdMulti ? D : 1;
  hipLaunchKernelGGL((k_md_finalize<Tin, Tout, MODE>), dim3((unsigned)((total_l + 255) / 256)), dim3(256), 0, st,
                     plan, D, T, rec, mu2, stride, keys, kstride, np, o, total_l);
  return hipGetLastError();
}

hipError_t launch_md(int mode, int D, const Plan &plan, const void *T, bool t_f64, void *rec, void *mu2,
                     int64_t stride, int64_t total_rc, unsigned long long *keys, int64_t kstride,
                     const int64_t *seg_prefix, const int32_t *seg_sweep, unsigned long long *counter, int R,
                     int64_t total_tiles, int64_t nseg, int grid, const Outputs &o, int64_t total_l,
                     hipEvent_t ev0, hipEvent_t ev1, hipStream_t st) {
  Double4 *rc = (Double4 *)rec;
  double2 *u2 = (double2 *)mu2;
  hipError_t e;
  if (t_f64) {
    const double *Tb = (const double *)T;
    e = mode == kMdSimple
            ? launch_md_t<double, kMdSimple>(D, plan, Tb, rc, u2, stride, total_rc, keys, kstride, seg_prefix,
                                                seg_sweep, counter, R, total_tiles, nseg, grid, ev0, ev1, st)
            : launch_md_t<double, kMdMulti>(D, plan, Tb, rc, u2, stride, total_rc, keys, kstride, seg_prefix,
                                                seg_sweep, counter, R, total_tiles, nseg, grid, ev0, ev1, st);
    if (e != hipSuccess) return e;
    e = mode == kMdSimple
            ? launch_md_fin_t<double, double, kMdSimple>(D, plan, Tb, rc, u2, stride, keys, kstride, o, total_l, st)
            : launch_md_fin_t<double, double, kMdMulti>(D, plan, Tb, rc, u2, stride, keys, kstride, o, total_l, st);
  } else {
    const float *Tb = (const float *)T;
    e = mode == kMdSimple
            ? launch_md_t<float, kMdSimple>(D, plan, Tb, rc, u2, stride, total_rc, keys, kstride, seg_prefix,
                                               seg_sweep, counter, R, total_tiles, nseg, grid, ev0, ev1, st)
            : launch_md_t<float, kMdMulti>(D, plan, Tb, rc, u2, stride, total_rc, keys, kstride, seg_prefix,
                                               seg_sweep, counter, R, total_tiles, nseg, grid, ev0, ev1, st);
    if (e != hipSuccess) return e;
    e = mode == kMdSimple
            ? launch_md_fin_t<float, float, kMdSimple>(D, plan, Tb, rc, u2, stride, keys, kstride, o, total_l, st)
            : launch_md_fin_t<float, float, kMdMulti>(D, plan, Tb, rc, u2, stride, keys, kstride, o, total_l, st);
  }
  return e;
}

int md_sweep_grid(int mode, int D) {
  int dev = 0, cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    cus = prop.multiProcessorCount;
  (void)mode;
  (void)D;
  return cus * 16;
}

}  // namespace mpx
