// Multidimensional joins: SiMPle (Section 3.3.4: no z-normalisation, the
// distance summed over all dimensions) and the multidimensional profiles of
// Section 3.3.5 (per-dimension z-normalised distances, sorted, the
// k-dimensional distance being the mean of the k smallest).  A series has D
// dimensions sampled together, stored dimension-major: dimension d of a
// series of n samples starts d*n values after its first sample.
//
// Same diagonal order as the one-dimensional sweep: tiles of R rows of a
// strip of W = 64*DT diagonals, one wave per tile, persistent grid; lane L
// owns the DT diagonals k0 + L*DT + t, so at row i it scores the cells
// (i, i + k0 + L*DT + t).  Per dimension the centred cross product C
// advances with C += a_j g_i + a_i g_j in FP64 (seeded in FP64 at the tile's
// first row).  Row records are wave-uniform scalar loads; column records
// live in registers and rotate: slot t at row i+1 holds the column slot t+1
// held at row i, the last slot takes lane L+1's first through a DPP wave
// shift, and lane 63 takes the one new column of the row.  Every cell yields
// one FP64 key per output profile with the cell's diagonal in its low bits,
// so one FP64 minimum gives both the row's and the column's partner.  Column
// minima travel with their column and leave the strip through lane 0; row
// minima pass through LDS; both merge into global (float value << 32 |
// partner) words with a 64-bit atomic minimum (order independent:
// deterministic).
#include <cmath>
#include <type_traits>
#include <utility>

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

// Global minima are packed (32-bit value pattern << 32 | index), the
// pattern ordered like the value it encodes (see MdKey::value).
__device__ __forceinline__ unsigned long long pack_md(unsigned bits, int64_t idx) {
  return ((unsigned long long)bits << 32) | (unsigned long long)(uint32_t)idx;
}

// A 32-bit pattern ordered like the non-negative double v over
// [2^-511, 2^511): a 10-bit exponent and the top 22 bits of the mantissa.
// Smaller values map to 0, larger ones (the huge keys of invalid windows
// included) to the top.  SiMPle's squared distances carry the data's units,
// so they may lie far outside float's range.
__device__ __forceinline__ unsigned md_bits(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int e = (int)(b >> 52) & 0x7ff;  // biased exponent
  if (e < 1023 - 511) return 0u;
  if (e >= 1023 + 511) return 0xffffffffu;
  return ((unsigned)(e - 512) << 22) | (unsigned)((b >> 30) & 0x3fffffull);
}

// Patterns at or above this are not candidates: float 1e30 for the
// k-dimensional keys (z-normalised distances are at most 2 sqrt(m) per
// dimension), a squared distance of 2^500 for SiMPle.
__device__ __forceinline__ unsigned md_limit(bool f32) {
  return f32 ? __float_as_uint(1.0e30f) : ((unsigned)(1523 - 512) << 22);
}

__device__ __forceinline__ int find_series_md(const Plan &plan, int64_t wi) {
  return (plan.nseries > 1 && wi >= plan.s_inl[1].w_off) ? 1 : 0;
}

}  // namespace

// Per window and dimension two records.  rec = {a, g, c, e} with
// a = x[w+m] - x[w], g = x[w] - mu + a (m-1)/(2m) (the cross-product
// recurrence) and, for SiMPle, c = sqrt(m) mu and e = Q = sum_d m sigma_d^2
// (kept in dimension 0); for the multidimensional profiles c = s =
// sqrt(2)/sigma (0 for a constant dimension) and e = v, the column term of
// key = u_i + v_j - C s_i s_j, which is the squared z-normalised distance for
// every mix of constant and varying windows (u = 2m and v = 0 for a varying
// dimension, u = m and v = -m for a constant one).  mu = {mean, u}.  A window with a non-finite sample in any dimension
// gets Q = u = v = huge; so do the padding records after each series (and
// a = g = 0 there).
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
    const Tin *x = series_samples(plan, Tb, S) + (int64_t)d * S.n + w;
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
      rec[d * stride + r] = Double4{a, g, sqrt((double)m) * mu, 0.0};
      mu2[d * stride + r] = make_double2(mu, 0.0);
    } else {
      rec[d * stride + r] = Double4{a, g, cst ? 0.0 : sqrt(2.0) / sg, cst ? -(double)m : 0.0};
      mu2[d * stride + r] = make_double2(mu, cst ? (double)m : 2.0 * m);
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

// Sorting network (odd-even transposition), ascending, on the bit patterns
// of non-negative floats (+inf included), whose integer order is their order
// as floats.
template <int N>
__device__ __forceinline__ void sort_net(unsigned (&v)[N]) {
#pragma unroll
  for (int p = 0; p < N; ++p) {
#pragma unroll
    for (int i = (p & 1); i + 1 < N; i += 2) {
      const unsigned a = v[i], b = v[i + 1];
      v[i] = min(a, b);
      v[i + 1] = max(a, b);
    }
  }
}

// FP64 minimum of two keys.  Keys are never NaN, so the plain instruction is
// exact; written out so that no NaN-quieting step is added to the integer-built
// operands.
__device__ __forceinline__ double kmin_f64(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Wave shift with lane 63 keeping `in63` (the DPP source of lane 63 is out of
// range, so that lane is not written): one DPP move per dword.
__device__ __forceinline__ double md_shl_in(double in63, double v) {
  const long long b = __double_as_longlong(v), f = __double_as_longlong(in63);
  const int lo = __builtin_amdgcn_update_dpp((int)(f & 0xffffffffll), (int)(b & 0xffffffffll), 0x130, 0xF, 0xF,
                                             false);
  const int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(b >> 32), 0x130, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Tile shape of the multidimensional sweep for a mode and dimension count.
// Per slot a lane keeps its column's records (SiMPle: a, g, sqrt(m) mu per
// dimension and Q; k-dimensional: a, g, s, v per dimension), the cross
// product of every dimension and one running column minimum per output; DT
// (a power of two) is the largest slot count whose state fits the register
// budget, chosen by measurement with the row records staged and two waves
// per SIMD, where a few spilled VGPRs cost less than fewer slots:
//  * SiMPle: 120 up to 6 dimensions (n = 2^17 walk: 8, 4, 4, 2, 2, 2 slots;
//    3 dimensions 4 slots 8.3 ms; 6 dimensions 2 slots 26.2 ms vs 1 slot
//    36.7 ms), 1 slot beyond (7 dimensions: 33.5 ms vs 38.9 ms at 2);
//  * k-dimensional profiles, whose per-cell temporaries are larger: 144 up
//    to 5 dimensions and 100 beyond, where two slots spill enough to lose
//    (3 dimensions 4 slots 76.5 ms vs 2 slots 87.3 ms at n = 2^18, 4
//    dimensions 4 slots 46.1 ms vs 2 slots 38.5 ms at n = 2^17, 5
//    dimensions 2 slots vs 1 at 0.69 of the time, 6 dimensions 2 slots 2 %
//    slower).
// TP rows pass between two LDS reductions of the row minima.
template <int D, int MODE>
struct MdShape {
  static constexpr int NP = MODE == kMdMulti ? D : 1;
  static constexpr int kSlotRegs = MODE == kMdSimple ? 8 * D + 4 : 12 * D;
  static constexpr int kFit = (MODE == kMdSimple ? (D <= 6 ? 120 : 60) : (D <= 5 ? 144 : 100)) / kSlotRegs;
  static constexpr int DT = kFit >= 8 ? 8 : (kFit >= 4 ? 4 : (kFit >= 2 ? 2 : 1));
  // rows between flushes: fewer for more profiles (their row minima share
  // the LDS; at 3 profiles 4 rows leave the prefetch 4 fewer VGPRs, 46 -> 2
  // spilled, and ran 20.2 -> 19.5 ms on an n = 2^17 walk).  SiMPle at 6 and
  // 8 dimensions, whose 16-row prefetch spilled 77 and 90 VGPRs, runs faster
  // with 8 (26.2 -> 22.3 and 56.8 -> 47.7 ms); at 4, 5 and 7 dimensions 8
  // rows were slower.
  static constexpr int TP = NP == 1 ? ((D == 6 || D == 8) ? 8 : 16) : (NP == 2 ? 8 : 4);
  static constexpr int W = 64 * DT;
  // doubles of one column record set: SiMPle a, g, z per dimension and Q;
  // k-dimensional a, g, s, v per dimension
  static constexpr int NF = MODE == kMdSimple ? 3 * D + 1 : 4 * D;
  // entering-column doubles each lane prefetches for the next row block
  static constexpr int NPF = (TP * NF + 63) / 64;
  static_assert(TP % DT == 0 && 64 % TP == 0, "row blocks");
  // resident waves per SIMD the register allocation must allow (without a
  // bound the compiler hoists the LDS reads of later rows and drops to one
  // wave)
  static constexpr int kMinWaves = 2;
};

constexpr int md_code_bits(int w) { return w <= 1 ? 1 : 1 + md_code_bits((w + 1) / 2); }

// In-place wave shift of a double: lane L takes lane L+1's value, lane 63
// takes `fill` (wave-uniform).
__device__ __forceinline__ int md_shl1(int v, int fill) {
  int x = __builtin_amdgcn_update_dpp(v, v, 0x130 /* wave_shl:1 */, 0xF, 0xF, false);
  fill = __builtin_amdgcn_readfirstlane(fill);
  asm volatile("v_writelane_b32 %0, %1, 63" : "+v"(x) : "s"(fill));
  return x;
}
__device__ __forceinline__ double md_shl1d(double v, double fill) {
  const long long b = __double_as_longlong(v), f = __double_as_longlong(fill);
  const int lo = md_shl1((int)(b & 0xffffffffll), (int)(f & 0xffffffffll));
  const int hi = md_shl1((int)(b >> 32), (int)(f >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename Fn, int... Ts>
__device__ __forceinline__ void md_for_impl(Fn &&f, std::integer_sequence<int, Ts...>) {
  (f(std::integral_constant<int, Ts>{}), ...);
}
template <int N, typename Fn>
__device__ __forceinline__ void md_for(Fn &&f) {
  md_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Keys are doubles whose low bits carry the cell's diagonal inside the strip
// (its code), so one FP64 minimum serves the row (partner i + k0 + code) and
// the column (partner j - k0 - code).  SiMPle keys are the squared distance
// with its lowest mantissa bits replaced; k-dimensional keys are the bit
// pattern (float value << 32 | code), whose order as doubles is the order of
// the float values (+inf included: its pattern is a finite double).  Every
// value is kept at or above a small normal number so that no key is a
// denormal.
template <int CB>
struct MdKey {
  static constexpr unsigned kMask = (1u << CB) - 1u;
  static __device__ __forceinline__ double from_f64(double v, unsigned code) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = ((unsigned)(b & 0xffffffffll) & ~kMask) | code;
    return __longlong_as_double((b & ~0xffffffffll) | lo);
  }
  static __device__ __forceinline__ double from_f32(float v, unsigned code) {
    return __longlong_as_double((long long)(((unsigned long long)__float_as_uint(v) << 32) | code));
  }
  static __device__ __forceinline__ unsigned code(double k) {
    return (unsigned)(__double_as_longlong(k) & 0xffffffffll) & kMask;
  }
  // the pattern of the value that goes into the global packed minimum: the
  // float (negative rounding residue read as 0) or, for SiMPle's FP64 keys,
  // md_bits (the code sits in bits md_bits drops)
  static __device__ __forceinline__ unsigned value(double k, bool f32) {
    const long long b = __double_as_longlong(k);
    if (f32) {
      const float v = __uint_as_float((unsigned)((unsigned long long)b >> 32));
      return __float_as_uint(v > 0.0f ? v : 0.0f);
    }
    return md_bits(__longlong_as_double(b & ~(long long)kMask));
  }
};

template <typename Tin, int D, int MODE>
__global__ void __launch_bounds__(64, (MdShape<D, MODE>::kMinWaves)) k_md_sweep(const Plan plan, const Tin *__restrict__ Tb,
                                                 const Double4 *__restrict__ rec,
                                                 const double2 *__restrict__ mu2, int64_t stride,
                                                 const int64_t *__restrict__ seg_prefix,
                                                 const int32_t *__restrict__ seg_sweep,
                                                 unsigned long long *__restrict__ keys, int64_t kstride,
                                                 unsigned long long *__restrict__ counter, int R,
                                                 int64_t total_tiles, int64_t nseg) {
  using Sh = MdShape<D, MODE>;
  constexpr int NP = Sh::NP, DT = Sh::DT, TP = Sh::TP, W = Sh::W, NF = Sh::NF, NPF = Sh::NPF;
  constexpr int CB = md_code_bits(W);
  constexpr bool kSimple = MODE == kMdSimple;
  using K = MdKey<CB>;
  const double kBig = 1.0e300;  // above every key: an empty minimum

  __shared__ double lrow[NP][TP][65];  // per row, each lane's minimum over its slots
  __shared__ double lcol[NP][TP];      // column minima leaving the strip through lane 0
  __shared__ double lfresh[TP][NF];    // records of the columns entering at lane 63
  __shared__ double lrrec[TP][NF];     // records of the block's rows

  const int lane = threadIdx.x;
  unsigned codes[DT];
#pragma unroll
  for (int t = 0; t < DT; ++t) codes[t] = (unsigned)(lane * DT + t);

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
    const int64_t k0 = uni(sd.k_lo + (g - sd.seg_base) * (int64_t)W);
    const int64_t L = min(RS.l, CS.l - k0);
    const int64_t i0 = uni((tile - seg_prefix[g]) * (int64_t)R);
    const int64_t nr = uni(min((int64_t)R, L - i0));
    // rows past nr up to a multiple of TP are scored too: they are rows of
    // the next tile (scored twice, harmless for a minimum) or padding
    // records, whose keys are huge
    const int64_t nsteps = uni(((nr + TP - 1) / TP) * TP);
    const int64_t lc = CS.l;
    const int m = RS.m;
    const int64_t rrow = uni(RS.rc_off + i0);        // record of the tile's first row
    const int64_t newc = uni(CS.rc_off + i0 + k0 + W);  // column entering lane 63 after that row
    unsigned long long *rkeys = keys + plan.series(sd.rk).w_off;
    unsigned long long *ckeys = keys + plan.series(sd.ck).w_off;
    const int64_t c0 = i0 + k0 + (int64_t)lane * DT;  // slot 0's column at row i0

    // ---- FP64 seeds at row i0, per dimension a sliding product: column
    // sample c0+v meets row sample v-t in slot t;
    // C = sum (x_r - mu_r) x_c - mu_c sum (x_r - mu_r)
    double C[DT][D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const Tin *__restrict__ Tr = series_samples(plan, Tb, RS) + (int64_t)d * RS.n + i0;
      const Tin *__restrict__ Tc = series_samples(plan, Tb, CS) + (int64_t)d * CS.n;
      const double mur = ldu_md(&mu2[d * stride + rrow].x);
      double acc[DT], xr[DT];
#pragma unroll
      for (int t = 0; t < DT; ++t) { acc[t] = 0.0; xr[t] = 0.0; }
      double Sx = 0.0;
      const int vend = m + DT - 1;
      for (int vb = 0; vb < vend; vb += DT) {
#pragma unroll
        for (int u = 0; u < DT; ++u) {
          const int v = vb + u;
          double xn = 0.0;
          if (v < m) xn = clean_md((double)Tr[v]) - mur;
          Sx += xn;
          xr[u] = xn;
          const int64_t ci = c0 + v;
          const double y = ci < CS.n ? clean_md((double)Tc[ci]) : 0.0;
#pragma unroll
          for (int t = 0; t < DT; ++t) acc[t] = fma(xr[(u - t + DT) % DT], y, acc[t]);
        }
      }
#pragma unroll
      for (int t = 0; t < DT; ++t) {
        const int64_t cw = min(c0 + t, lc - 1);
        C[t][d] = acc[t] - mu2[d * stride + CS.rc_off + cw].x * Sx;
      }
    }

    // ---- column records of every slot (register set t holds slot t at i0)
    double A[DT][D], G[DT][D], Z[DT][D], V[DT][D], X[DT], CM[DT][NP];
#pragma unroll
    for (int t = 0; t < DT; ++t) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const Double4 r = rec[d * stride + CS.rc_off + c0 + t];
        A[t][d] = r.x;
        G[t][d] = r.y;
        Z[t][d] = r.z;
        V[t][d] = r.w;
        if (d == 0) X[t] = r.w;
      }
#pragma unroll
      for (int q = 0; q < NP; ++q) CM[t][q] = kBig;
    }

    // Records of the columns entering at lane 63 during the rows of a block
    // (column newc + row offset) and of the block's rows (row rrow + row
    // offset), spread over the lanes: element e is double f = e % NF of the
    // block's column or row e / NF.  They are loaded one block ahead and
    // staged in LDS, so no row waits on a memory load (scalar loads of each
    // row's records, waited on in every row, were slower at every mode and
    // dimension count).  A row record holds
    // the same terms as a column record except, in the k-dimensional mode,
    // u_i (from mu2) in place of v_j.
    double pf[NPF], pr[NPF];
    auto prefetch = [&](int64_t sb) {
#pragma unroll
      for (int k = 0; k < NPF; ++k) {
        const int e = lane + 64 * k;
        pf[k] = 0.0;
        pr[k] = 0.0;
        if (e < TP * NF && sb < nsteps) {
          const int u = e / NF, f = e % NF;
          int d, comp;
          if constexpr (kSimple) {
            d = f < 3 * D ? f / 3 : 0;
            comp = f < 3 * D ? f % 3 : 3;
          } else {
            d = f / 4;
            comp = f % 4;
          }
          pf[k] = reinterpret_cast<const double *>(rec + d * stride + newc + sb + u)[comp];
          if (!kSimple && comp == 3) pr[k] = mu2[d * stride + rrow + sb + u].y;
          else pr[k] = reinterpret_cast<const double *>(rec + d * stride + rrow + sb + u)[comp];
        }
      }
    };
    auto stage = [&]() {
#pragma unroll
      for (int k = 0; k < NPF; ++k) {
        const int e = lane + 64 * k;
        if (e < TP * NF) {
          lfresh[e / NF][e % NF] = pf[k];
          lrrec[e / NF][e % NF] = pr[k];
        }
      }
    };
    prefetch(0);
    __syncthreads();  // the previous tile's last block is done with lfresh
    stage();
    prefetch(TP);
    __syncthreads();

    auto emit_row = [&](int q, int64_t i, double kb) {
      const unsigned val = K::value(kb, !kSimple);
      if (val < md_limit(!kSimple)) {
        const int64_t j = i + k0 + (int64_t)K::code(kb);
        if (j < lc) atomicMin(rkeys + q * kstride + i, pack_md(val, j));
      }
    };
    auto emit_col = [&](int q, int64_t c, double kb) {
      const unsigned val = K::value(kb, !kSimple);
      if (c < lc && val < md_limit(!kSimple)) {
        const int64_t i = c - k0 - (int64_t)K::code(kb);
        atomicMin(ckeys + q * kstride + c, pack_md(val, i));
      }
    };

    for (int64_t sb = 0; sb < nsteps; sb += TP) {
      md_for<TP>([&](auto uc) {
        constexpr int u = decltype(uc)::value, r0 = u % DT;  // set of slot 0
        double ai[D], gi[D], zi[D], ui[D], qi = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          constexpr int kw = kSimple ? 3 : 4;
          ai[d] = lrrec[u][kw * d];
          gi[d] = lrrec[u][kw * d + 1];
          zi[d] = lrrec[u][kw * d + 2];
          if constexpr (!kSimple) ui[d] = lrrec[u][kw * d + 3];
        }
        if constexpr (kSimple) qi = lrrec[u][3 * D];
        double rmin[NP];
        md_for<DT>([&](auto tc) {
          constexpr int t = decltype(tc)::value, p = (t + r0) % DT;
          double key[NP];
          if constexpr (kSimple) {
            // d^2 = Q_i + Q_j + sum_d [m (mu_i - mu_j)^2 - 2 C_d]
            double d2 = qi + X[p];
#pragma unroll
            for (int d = 0; d < D; ++d) {
              const double dz = zi[d] - Z[p][d];
              d2 = fma(dz, dz, d2);
              d2 = fma(-2.0, C[t][d], d2);
              C[t][d] = fma(A[p][d], gi[d], C[t][d]);
              C[t][d] = fma(ai[d], G[p][d], C[t][d]);
            }
            key[0] = K::from_f64(fmax(d2, 0x1p-1000), codes[t]);
          } else {
            // per dimension 2m (u_i + v_j - C s_i s_j) = d^2, with u, v
            // scaled by 2m and s by sqrt(2m) in the records
            unsigned db[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
              const double k2 = fma(-(C[t][d] * zi[d]), Z[p][d], ui[d] + V[p][d]);
              // at least a small normal (the integer max also lifts negative
              // values); huge (invalid or padding) keys become +inf, which
              // the sort, the means and the key order all keep last
              const int kb = max((int)__float_as_uint((float)k2), (int)__float_as_uint(0x1p-100f));
              db[d] = __float_as_uint(__builtin_amdgcn_sqrtf(__int_as_float(kb)));
              C[t][d] = fma(A[p][d], gi[d], C[t][d]);
              C[t][d] = fma(ai[d], G[p][d], C[t][d]);
            }
            sort_net<D>(db);
            float run = 0.0f;
#pragma unroll
            for (int q = 0; q < NP; ++q) {
              run += __uint_as_float(db[q]);
              key[q] = K::from_f32(q == 0 ? run : run * (1.0f / (float)(q + 1)), codes[t]);
            }
          }
#pragma unroll
          for (int q = 0; q < NP; ++q) {
            CM[p][q] = kmin_f64(CM[p][q], key[q]);
            rmin[q] = t == 0 ? key[q] : kmin_f64(rmin[q], key[q]);
          }
        });
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          lrow[q][u][lane] = rmin[q];
          if (lane == 0) lcol[q][u] = CM[r0][q];
        }
        // set r0 moves one lane down; lane 63 takes the entering column,
        // read from LDS at a wave-uniform address
#pragma unroll
        for (int d = 0; d < D; ++d) {
          if constexpr (kSimple) {
            A[r0][d] = md_shl_in(lfresh[u][3 * d], A[r0][d]);
            G[r0][d] = md_shl_in(lfresh[u][3 * d + 1], G[r0][d]);
            Z[r0][d] = md_shl_in(lfresh[u][3 * d + 2], Z[r0][d]);
          } else {
            A[r0][d] = md_shl_in(lfresh[u][4 * d], A[r0][d]);
            G[r0][d] = md_shl_in(lfresh[u][4 * d + 1], G[r0][d]);
            Z[r0][d] = md_shl_in(lfresh[u][4 * d + 2], Z[r0][d]);
            V[r0][d] = md_shl_in(lfresh[u][4 * d + 3], V[r0][d]);
          }
        }
        if constexpr (kSimple) X[r0] = md_shl_in(lfresh[u][3 * D], X[r0]);
#pragma unroll
        for (int q = 0; q < NP; ++q) CM[r0][q] = md_shl1d(CM[r0][q], kBig);
      });
      // ---- rows sb .. sb+TP-1: the 64 lane minima of each row in two
      // passes (TP per lane, then 64/TP per row; the partials go back into
      // the row buffer, which keeps the LDS per wave small), then the merges
      __syncthreads();
      double part[NP];
      {
        const int r = lane % TP, g0 = (lane / TP) * TP;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          double best = lrow[q][r][g0];
#pragma unroll
          for (int e = 1; e < TP; ++e) best = kmin_f64(best, lrow[q][r][g0 + e]);
          part[q] = best;
        }
      }
      __syncthreads();
      double *const lpart = &lrow[0][0][0];  // [NP][64] partials
#pragma unroll
      for (int q = 0; q < NP; ++q) lpart[q * 64 + lane] = part[q];
      // the next block's entering columns (every read of this block's is done)
      stage();
      prefetch(sb + 2 * TP);
      __syncthreads();
      if (lane < TP) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          double best = lpart[q * 64 + lane];
#pragma unroll
          for (int e = 1; e < 64 / TP; ++e) best = kmin_f64(best, lpart[q * 64 + lane + e * TP]);
          const int64_t s = sb + lane;
          if (s < nr) emit_row(q, i0 + s, best);
          emit_col(q, i0 + s + k0, lcol[q][lane]);
        }
      }
      __syncthreads();
    }
    // columns still in flight: set t of lane L holds column
    // i0 + nsteps + k0 + L*DT + t
#pragma unroll
    for (int t = 0; t < DT; ++t)
#pragma unroll
      for (int q = 0; q < NP; ++q) emit_col(q, i0 + nsteps + k0 + (int64_t)lane * DT + t, CM[t][q]);
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
    if (valid && k != ~0ull && (unsigned)(k >> 32) < md_limit(MODE != kMdSimple)) {
      idx = (int64_t)(uint32_t)(k & 0xffffffffull);
      if (MODE == kMdSimple) {
        double s = 0.0;
        for (int d = 0; d < D; ++d) {
          const Tin *a = series_samples(plan, Tb, S) + (int64_t)d * S.n + w;
          const Tin *b = series_samples(plan, Tb, Q) + (int64_t)d * Q.n + idx;
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
          const Tin *a = series_samples(plan, Tb, S) + (int64_t)d * S.n + w;
          const Tin *b = series_samples(plan, Tb, Q) + (int64_t)d * Q.n + idx;
          const double ia = ra.z / sqrt(2.0), ib = rb.z / sqrt(2.0);  // 1/sigma or 0
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

namespace {
template <int MODE>
int md_width_t(int D) {
  switch (D) {
    case 1: return MdShape<1, MODE>::W;
    case 2: return MdShape<2, MODE>::W;
    case 3: return MdShape<3, MODE>::W;
    case 4: return MdShape<4, MODE>::W;
    case 5: return MdShape<5, MODE>::W;
    case 6: return MdShape<6, MODE>::W;
    case 7: return MdShape<7, MODE>::W;
    case 8: return MdShape<8, MODE>::W;
    default: return 64;
  }
}
template <int MODE>
hipError_t md_occupancy_t(int D, int *per) {
  switch (D) {
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_md_sweep<float, 1, MODE>, 64, 0);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_md_sweep<float, 2, MODE>, 64, 0);
    case 3: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_md_sweep<float, 3, MODE>, 64, 0);
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_md_sweep<float, 4, MODE>, 64, 0);
    case 5: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_md_sweep<float, 5, MODE>, 64, 0);
    case 6: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_md_sweep<float, 6, MODE>, 64, 0);
    case 7: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_md_sweep<float, 7, MODE>, 64, 0);
    case 8: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_md_sweep<float, 8, MODE>, 64, 0);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

int md_strip_width(int mode, int D) {
  return mode == kMdSimple ? md_width_t<kMdSimple>(D) : md_width_t<kMdMulti>(D);
}

int md_sweep_grid(int mode, int D) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  int per = 0;
  const hipError_t e = mode == kMdSimple ? md_occupancy_t<kMdSimple>(D, &per) : md_occupancy_t<kMdMulti>(D, &per);
  if (e != hipSuccess || per <= 0) per = 8;
  return cus * per;
}

}  // namespace mpx
