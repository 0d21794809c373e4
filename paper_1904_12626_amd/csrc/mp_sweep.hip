// The diagonal sweep: every admissible cell (i, j) of the distance matrix is
// visited once, in O(1) work, and contributes to the minimum of row i and of
// column j (matrix profile = row minima, Section 2 of the tsmp paper; the
// O(1) update of one row's dot products from the previous row is the STOMP
// idea of Section 3.3.2, applied here along diagonals so that tiles are
// independent, as in the column-independent order of Section 3.3.3).
//
// Work decomposition (one wave per tile):
//   strip   W = 64*DT consecutive diagonals k0 .. k0+W-1; lane L owns the DT
//           diagonals k0 + L*DT + t, t = 0..DT-1 ("slots").
//   tile    R consecutive rows i0 .. i0+R-1 of one strip; the cross product
//           of every diagonal is seeded in FP64 at row i0 (so R is also the
//           reseed interval of the FP32 sweep).
// At row i every lane handles cells (i, i + k0 + L*DT + t).  The per-row
// values (a_i, g_i, s_i, u_i) are wave-uniform scalar loads (the FP64 sweep
// stages them in LDS one block ahead and reads them as broadcasts).  Column values
// move one lane down per row: slot t at row i+1 reads the column slot t+1
// held at row i, so slots rotate through registers (full unroll by DT) and
// the last slot receives lane L+1's first slot through a DPP wave shift;
// lane 63 receives the one new column from a scalar load (the FP64 sweep
// reads it from LDS as the DPP fallback value instead).  Column minima
// travel the same way and leave the strip through lane 0.
//
// Per cell: key = u_i - (C s_i) s_j  (= 1 - Pearson rho for valid windows),
// the low CB bits of the key are replaced by the slot's code (its diagonal
// inside the strip), then one integer min for the column and one for the
// row; C advances with two FMAs: C += a_j g_i + a_i g_j.
// Row minima of the 64 lanes are reduced through LDS every TP rows; the
// winners are merged into global packed (key, index) words with a 64-bit
// atomic minimum, which is order independent, so results are deterministic.
#include <climits>
#include <cmath>
#include <type_traits>
#include <utility>

#include "mp_internal.h"
#include "mp_types.h"

namespace mpx {

namespace {

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

// In-place wave shift: lane L receives v from lane L+1, then lane 63 takes
// `fill` (a wave-uniform value) with one v_writelane_b32 (a VALU register
// write, no memory access).  Keeping source and destination in one register
// lets every rotating slot stay in a fixed register across the unrolled rows.
__device__ __forceinline__ int shl1(int v, int fill) {
  int x = __builtin_amdgcn_update_dpp(v, v, 0x130 /* wave_shl:1 */, 0xF, 0xF, false);
  fill = __builtin_amdgcn_readfirstlane(fill);
  asm volatile("v_writelane_b32 %0, %1, 63" : "+v"(x) : "s"(fill));
  return x;
}
__device__ __forceinline__ float shl1f(float v, float fill) {
  return __int_as_float(shl1(__float_as_int(v), __float_as_int(fill)));
}
__device__ __forceinline__ double shl1d(double v, double fill) {
  const long long b = __double_as_longlong(v), f = __double_as_longlong(fill);
  const int lo = shl1((int)(b & 0xffffffffll), (int)(f & 0xffffffffll));
  const int hi = shl1((int)(b >> 32), (int)(f >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave shift of a double with lane 63 keeping `in63` (its DPP source is out
// of range, so that lane is not written): one DPP move per dword.
__device__ __forceinline__ double shl_keep63(double in63, double v) {
  const long long b = __double_as_longlong(v), f = __double_as_longlong(in63);
  const int lo = __builtin_amdgcn_update_dpp((int)(f & 0xffffffffll), (int)(b & 0xffffffffll), 0x130, 0xF, 0xF,
                                             false);
  const int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(b >> 32), 0x130, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int64_t rfl64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (unsigned int)lo;
}

// Compile-time loop: f(integral_constant<int, 0..N-1>), fully expanded.
template <typename Fn, int... Ts>
__device__ __forceinline__ void static_for_impl(Fn &&f, std::integer_sequence<int, Ts...>) {
  (f(std::integral_constant<int, Ts>{}), ...);
}
template <int N, typename Fn>
__device__ __forceinline__ void static_for(Fn &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// In-wave key handling.  FP32 keys live as int bit patterns so that the
// minimum is an integer min (order of non-negative floats; the rare tiny
// negative key of a perfect match sorts below every positive one).
template <typename F, int CB>
struct InKey;

template <int CB>
struct InKey<float, CB> {
  using K = int;
  static constexpr int kBig = 0x7F61B1E6;  // 3.0e38f
  static constexpr unsigned kMask = (1u << CB) - 1u;
  static __device__ __forceinline__ K make(float key, unsigned code) {
    return (int)((__float_as_uint(key) & ~kMask) | code);
  }
  static __device__ __forceinline__ K kmin(K a, K b) { return min(a, b); }
  static __device__ __forceinline__ K kmin3(K a, K b, K c) { return min(min(a, b), c); }
  template <int N>
  static __device__ __forceinline__ K rowmin(const K (&k)[N]) {
    K r = min(k[0], k[1]);
    static_for<(N - 2) / 2>([&](auto q) {
      constexpr int j = 2 + 2 * decltype(q)::value;
      r = min(min(r, k[j]), k[j + 1]);
    });
    if constexpr (N % 2 == 1) r = min(r, k[N - 1]);
    return r;
  }
  static __device__ __forceinline__ K shl(K v) { return shl1(v, kBig); }
  static __device__ __forceinline__ unsigned code(K k) { return (unsigned)k & kMask; }
  static __device__ __forceinline__ double value(K k) {
    return (double)__uint_as_float((unsigned)k & ~kMask);
  }
  static __device__ __forceinline__ K big() { return kBig; }
};

template <int CB>
struct InKey<double, CB> {
  using K = double;
  static constexpr unsigned kMask = (1u << CB) - 1u;
  static __device__ __forceinline__ K make(double key, unsigned code) {
    const long long b = __double_as_longlong(key);
    const unsigned lo = ((unsigned)(b & 0xffffffffll) & ~kMask) | code;
    return __longlong_as_double((b & ~0xffffffffll) | lo);
  }
  static __device__ __forceinline__ K kmin(K a, K b) { return __builtin_fmin(a, b); }
  static __device__ __forceinline__ K kmin3(K a, K b, K c) { return __builtin_fmin(__builtin_fmin(a, b), c); }
  template <int N>
  static __device__ __forceinline__ K rowmin(const K (&k)[N]) {
    K r = k[0];
    static_for<N - 1>([&](auto q) { r = __builtin_fmin(r, k[1 + decltype(q)::value]); });
    return r;
  }
  static __device__ __forceinline__ K shl(K v) { return shl1d(v, 1.0e300); }
  static __device__ __forceinline__ unsigned code(K k) {
    return (unsigned)(__double_as_longlong(k) & 0xffffffffll) & kMask;
  }
  static __device__ __forceinline__ double value(K k) {
    const long long b = __double_as_longlong(k);
    return __longlong_as_double(b & ~(long long)kMask);
  }
  static __device__ __forceinline__ K big() { return 1.0e300; }
};

template <typename F>
__device__ __forceinline__ F shlv(F v, F fill);
template <>
__device__ __forceinline__ float shlv<float>(float v, float fill) { return shl1f(v, fill); }
template <>
__device__ __forceinline__ double shlv<double>(double v, double fill) { return shl1d(v, fill); }

// Non-finite samples read as 0 (the exponent test keeps working when the
// translation unit is compiled without NaN semantics).
__device__ __forceinline__ double clean(float v) {
  return ((__float_as_uint(v) >> 23) & 0xffu) == 0xffu ? 0.0 : (double)v;
}
__device__ __forceinline__ double clean(double v) {
  return ((__double_as_longlong(v) >> 52) & 0x7ff) == 0x7ff ? 0.0 : v;
}

// Exchange of a double between the two lanes of each pair (quad_perm
// [1, 0, 3, 2]).
__device__ __forceinline__ double swap_pair(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Load of a wave-uniform address through the constant address space, so that
// it becomes a scalar load (the data was written by an earlier kernel and is
// read-only here).
template <typename T>
__device__ __forceinline__ T ldu(const T *p) {
#if defined(__HIP_DEVICE_COMPILE__)
  static_assert(sizeof(T) % 4 == 0, "ldu loads whole dwords");
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

}  // namespace

// Minimum resident waves per SIMD the register allocation must allow.
template <typename FE, int NS>
struct SweepMinWaves {
  static constexpr int value = (sizeof(FE) == 4 && NS <= 12) ? 4 : (sizeof(FE) == 8 ? 3 : 2);
};

template <typename F, typename Tin, int DT, int TP>
__global__ void __launch_bounds__(64, (SweepMinWaves<F, DT>::value))
    k_sweep(const Plan plan, const typename FTraits<F>::V4 *__restrict__ rcb,
            const double *__restrict__ mu, const int64_t *__restrict__ seg_prefix,
            const int32_t *__restrict__ seg_sweep, const int64_t *__restrict__ seg_part,
            const SeriesDesc *__restrict__ s_ext,
            const SweepDesc *__restrict__ w_ext, const double *__restrict__ scale, uint64_t *__restrict__ keys,
            unsigned long long *__restrict__ counter, const Tin *__restrict__ Tb, const int R,
            const int64_t total_tiles, const int64_t nseg) {
  constexpr int W = 64 * DT;
  constexpr int CB = ilog2c(W - 1) + 1;  // bits for codes 0 .. W-1
  using IK = InKey<F, CB>;
  using K = typename IK::K;
  using V4 = typename FTraits<F>::V4;


  const int lane = threadIdx.x;
  auto series = [&](int i) -> SeriesDesc { return s_ext ? ldu(s_ext + i) : plan.s_inl[i]; };
  auto sweep = [&](int i) -> SweepDesc { return w_ext ? ldu(w_ext + i) : plan.w_inl[i]; };

  for (;;) {
    int64_t tile = 0;
    if (lane == 0) tile = (int64_t)atomicAdd(counter, 1ull);
    tile = rfl64(tile);
    if (tile >= total_tiles) break;

    // ---- decode the tile: strip g (binary search of the tile table; the
    // full-height tiles of all strips first, then their shorter last tiles)
    const int64_t nfull = ldu(seg_prefix + nseg);
    const bool tail = tile >= nfull;
    const int64_t *const table = tail ? seg_part : seg_prefix;
    const int64_t key = tail ? tile - nfull : tile;
    int64_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (ldu(table + mid) <= key) lo = mid; else hi = mid - 1;
    }
    const int64_t g = lo;
    const SweepDesc d = sweep(ldu(seg_sweep + g));
    const SeriesDesc RS = series(d.rs), CS = series(d.cs);
    const int64_t k0 = rfl64(d.k_lo + (g - d.seg_base) * (int64_t)W);
    const int64_t L = min(RS.l, CS.l - k0);
    const int64_t i0 = rfl64(tail ? (L / R) * (int64_t)R : (tile - ldu(seg_prefix + g)) * (int64_t)R);
    const int64_t nr = min((int64_t)R, L - i0);
    const int64_t lc = CS.l;
    // Cells outside the join read padding records: rows >= l_r give huge
    // keys; columns >= l_c score like rho = 0 and, should such a column be a
    // row's minimum, it is reported with an out-of-range index that sends the
    // row to the exact rescan.  So the last tile of a strip runs the same code.
    const int64_t nsteps = ((nr + DT - 1) / DT) * DT;
    const int m = RS.m;

    uint64_t *rkeys = keys + series(d.rk).w_off;
    uint64_t *ckeys = keys + series(d.ck).w_off;
    // wave-uniform bases (made explicit so the row loads stay scalar)
    const V4 *__restrict__ rowd = rcb + rfl64(RS.rc_off);
    const V4 *__restrict__ cold = rcb + rfl64(CS.rc_off);
    const int ib = d.idx_bits;

    // ---- FP64 seed of every slot's diagonal at row i0:
    // C = sum_u (x_r[i0+u] - mu_r) (x_c[c+u] - mu_c)
    //   = sum_u (x_r[i0+u] - mu_r) x_c[c+u] - mu_c * sum_u (x_r[i0+u] - mu_r),
    // evaluated as a sliding product: column sample c0+v meets row sample v-t.
    const int64_t c0 = i0 + k0 + (int64_t)lane * DT;
    F C[DT];
    {
      const Tin *__restrict__ Tr = series_samples(plan, Tb, RS) + i0;
      const Tin *__restrict__ Tc = series_samples(plan, Tb, CS);
      const double mur = ldu(mu + RS.w_off + i0);
      const int64_t ncol = CS.n;
      double acc[DT], xr[DT];
#pragma unroll
      for (int t = 0; t < DT; ++t) { acc[t] = 0.0; xr[t] = 0.0; }
      double Sx = 0.0;
      const int vend = m + DT - 1;
      for (int vb = 0; vb < vend; vb += DT) {
        if constexpr (std::is_same_v<F, double>) {
          // A block's loads first, at clamped (in-bounds) addresses, so that
          // they are in flight together (the FP64 sweep of a small join is
          // bound by this chain's latency); samples past either end are
          // zeroed below.  The FP32 sweeps keep the guarded loads: the same
          // change there costs spills in their row loop.
          Tin xs[DT], ys[DT];
#pragma unroll
          for (int u = 0; u < DT; ++u) {
            xs[u] = ldu(Tr + min(vb + u, m - 1));
            ys[u] = Tc[min(c0 + vb + u, ncol - 1)];
          }
#pragma unroll
          for (int u = 0; u < DT; ++u) {
            const int v = vb + u;
            const double xn = (v < m) ? clean(xs[u]) - mur : 0.0;
            Sx += xn;
            xr[u] = xn;
            const double y = (c0 + v < ncol) ? clean(ys[u]) : 0.0;
#pragma unroll
            for (int t = 0; t < DT; ++t) acc[t] = fma(xr[(u - t + DT) % DT], y, acc[t]);
          }
        } else {
#pragma unroll
          for (int u = 0; u < DT; ++u) {
            const int v = vb + u;
            double xn = 0.0;
            if (v < m) xn = clean(ldu(Tr + v)) - mur;
            Sx += xn;
            xr[u] = xn;
            const int64_t ci = c0 + v;
            const double y = (ci < ncol) ? clean(Tc[ci]) : 0.0;
#pragma unroll
            for (int t = 0; t < DT; ++t) acc[t] = fma(xr[(u - t + DT) % DT], y, acc[t]);
          }
        }
      }
      // the records carry each series' power of two (see k_stats)
      const double kk = ldu(scale + d.rs) * ldu(scale + d.cs);
#pragma unroll
      for (int t = 0; t < DT; ++t) {
        const int64_t cw = min(c0 + t, lc - 1);
        C[t] = (F)((acc[t] - mu[CS.w_off + cw] * Sx) * kk);
      }
    }

    // ---- column window and column minima
    F A[DT], G[DT], S[DT];
    K CP[DT];
#pragma unroll
    for (int t = 0; t < DT; ++t) {
      const V4 v = cold[c0 + t];
      A[t] = v.x;
      G[t] = v.y;
      S[t] = v.z;
      CP[t] = IK::big();
    }
    // the one new column per row (entering at lane 63) is a scalar load
    const V4 *__restrict__ newcol = cold + (k0 + W + i0);

    const int64_t past = ((int64_t)1 << ib) - 1;  // never a window index
    auto emit_row = [&](int64_t i, K kb) {
      const double val = IK::value(kb);
      if (val < 1.0e30) {
        int64_t j = i + k0 + (int64_t)IK::code(kb);
        if (j >= lc) j = past;
        atomicMin((unsigned long long *)(rkeys + i), (unsigned long long)pack_global(val, j, ib));
      }
    };
    auto emit_col = [&](int64_t c, K kb) {
      const double val = IK::value(kb);
      if (c < lc && val < 1.0e30) {
        const int64_t i = c - k0 - (int64_t)IK::code(kb);
        atomicMin((unsigned long long *)(ckeys + c), (unsigned long long)pack_global(val, i, ib));
      }
    };
    if constexpr (std::is_same_v<F, double>) {
      // FP64: one row at a time (there is no 3-input FP64 minimum, so row
      // pairs would only hold a second key array).  The records of a block's
      // rows and of the columns entering at lane 63 are loaded one block
      // ahead (lane u holds row u's) and staged in LDS between the two
      // barriers of the flush, so no row waits on a memory load: each row
      // reads its record as an LDS broadcast and the entering column as the
      // DPP fallback operand.  A row's 64 lane minima are halved by a DPP
      // exchange within lane pairs before they go to LDS; the 32 partials of
      // row u sit in order in a row of 33 doubles, so a row's writes are
      // contiguous and the flush's reads (lane r reads row r, partial q at
      // dword 66 r + 2 q: banks 2 (r + q) mod 64) touch distinct banks with
      // every address an immediate offset from the lane's row.  Lane 0's
      // column minimum rides in the spare slot of the entering-column
      // record.  10.5 KB of LDS per wave.
      static_assert(TP <= 32, "row-rotated partials");
      __shared__ double lrec[TP][4];   // a_i, g_i, s_i, u_i of row sb + u
      __shared__ double lent[TP][4];   // a, g, s of the column entering after row sb + u;
                                       // [3]: the column minimum leaving through lane 0
      __shared__ double lhalf[TP][33]; // row minima of lane pairs (rows padded to 33)
      V4 prow = {0.0, 0.0, 0.0, 0.0}, pcol = {0.0, 0.0, 0.0, 0.0};
      auto prefetch = [&](int64_t sb2) {
        if (lane < TP && sb2 + lane < nsteps) {
          prow = rowd[i0 + sb2 + lane];
          pcol = newcol[sb2 + lane];
        }
      };
      auto stage = [&]() {
        if (lane < TP) {
          lrec[lane][0] = prow.x;
          lrec[lane][1] = prow.y;
          lrec[lane][2] = prow.z;
          lrec[lane][3] = prow.w;
          lent[lane][0] = pcol.x;
          lent[lane][1] = pcol.y;
          lent[lane][2] = pcol.z;
        }
      };
      prefetch(0);
      stage();
      prefetch(TP);
      __syncthreads();
      const double big = IK::big();
      for (int64_t sb = 0; sb < nsteps; sb += TP) {
        const int nb = (int)min((int64_t)TP, nsteps - sb);  // a multiple of DT
        static_for<TP>([&](auto uc) {
          constexpr int u = decltype(uc)::value;
          constexpr int r0 = u % DT;  // register of slot 0
          if (u >= nb) return;
          K k[DT];
          const F ai = lrec[u][0], gi = lrec[u][1], si = lrec[u][2], ui = lrec[u][3];
          static_for<DT>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            constexpr int p = (t + r0) % DT;
            k[t] = IK::make(fma(-(C[t] * si), S[p], ui), (unsigned)(lane * DT + t));
            C[t] = fma(A[p], gi, C[t]);
            C[t] = fma(G[p], ai, C[t]);
          });
          K r = IK::rowmin(k);
          r = IK::kmin(r, swap_pair(r));
          if (!(lane & 1)) lhalf[u][lane >> 1] = r;
          // register p met slot p - r0
          static_for<DT>([&](auto pc) {
            constexpr int q = decltype(pc)::value;
            CP[q] = IK::kmin(CP[q], k[(q - r0 + DT) % DT]);
          });
          if (lane == 0) lent[u][3] = CP[r0];
          CP[r0] = shl_keep63(big, CP[r0]);
          A[r0] = shl_keep63(lent[u][0], A[r0]);
          G[r0] = shl_keep63(lent[u][1], G[r0]);
          S[r0] = shl_keep63(lent[u][2], S[r0]);
        });
        // flush, with the next block's records staged between the barriers
        // (every read of this block's is done)
        __syncthreads();
        if (lane < nb) {
          K best = lhalf[lane][0];
#pragma unroll
          for (int q = 1; q < 32; ++q) best = IK::kmin(best, lhalf[lane][q]);
          const int64_t s = sb + lane;
          if (s < nr) emit_row(i0 + s, best);
          emit_col(i0 + s + k0, lent[lane][3]);
        }
        stage();
        prefetch(sb + 2 * TP);
        __syncthreads();
      }
    } else {
    // Rows are processed in pairs: a column register receives one cell from
    // each row of the pair, so its minimum is a single 3-input min, and each
    // row's own minimum is a chain of 3-input mins.
    static_assert(TP % 2 == 0 && DT % 2 == 0, "row pairs");
    // Row partials: lane q's minimum of row u sits in component q % 4 of
    // lrow[q / 4][u].  A row's 64 writes then land on distinct banks (the
    // stride of TP + 1 records is 20 banks mod 64), and the flush (lane r
    // reduces row r) reads them as 16 contiguous 16-byte records per lane.
    __shared__ int4 lrow[16][TP + 1];
    __shared__ K lcol[TP];
    int *const lrow_w = reinterpret_cast<int *>(&lrow[lane >> 2][0]) + (lane & 3);
    // Rows [fb, fb+cnt) of this tile: reduce the 64 lane partials of each
    // row (one row per lane) and merge; merge the column minima that left
    // the strip through lane 0 at those rows.
    auto flush = [&](int64_t fb, int cnt) {
      __syncthreads();
      if (lane < cnt) {
        const int4 v0 = lrow[0][lane];
        K best = IK::kmin3(v0.x, v0.y, IK::kmin(v0.z, v0.w));
#pragma unroll
        for (int q = 1; q < 16; ++q) {
          const int4 v = lrow[q][lane];
          best = IK::kmin3(best, v.x, v.y);
          best = IK::kmin3(best, v.z, v.w);
        }
        const int64_t s = fb + lane;
        if (s < nr) emit_row(i0 + s, best);
        emit_col(i0 + s + k0, lcol[lane]);
      }
      __syncthreads();
    };
    // The row and entering-column records of a pair of rows are loaded one
    // pair ahead (scalar loads; a pair past the tile reads padding records,
    // which are never used), so their latency overlaps a pair's arithmetic.
    V4 nrd0 = ldu(rowd + i0), nrd1 = ldu(rowd + i0 + 1), nnc0 = ldu(newcol), nnc1 = ldu(newcol + 1);
    for (int64_t sb = 0; sb < nsteps; sb += TP) {
      // a multiple of DT (even); wave-uniform, kept in a scalar register so
      // that the per-pair guard below is a scalar branch
      const int nb = __builtin_amdgcn_readfirstlane((int)min((int64_t)TP, nsteps - sb));
      static_for<TP / 2>([&](auto qc) {
        constexpr int u0 = 2 * decltype(qc)::value, u1 = u0 + 1;
        constexpr int r0 = u0 % DT, r1 = u1 % DT;  // register of slot 0 in each row
        if (u0 < nb) {
          K k0[DT], k1[DT];
          const V4 rd0 = nrd0, rd1 = nrd1, nc0 = nnc0, nc1 = nnc1;
          nrd0 = ldu(rowd + i0 + sb + u0 + 2);
          nrd1 = ldu(rowd + i0 + sb + u1 + 2);
          nnc0 = ldu(newcol + sb + u0 + 2);
          nnc1 = ldu(newcol + sb + u1 + 2);
          // ---- row u0
          {
            const V4 rd = rd0;
            const F ai = rd.x, gi = rd.y, si = rd.z, ui = rd.w;
            static_for<DT>([&](auto tc) {
              constexpr int t = decltype(tc)::value;
              constexpr int p = (t + r0) % DT;
              k0[t] = IK::make(fma(-(C[t] * si), S[p], ui), (unsigned)(lane * DT + t));
              C[t] = fma(A[p], gi, C[t]);
              C[t] = fma(G[p], ai, C[t]);
            });
            lrow_w[4 * u0] = IK::rowmin(k0);
            CP[r0] = IK::kmin(CP[r0], k0[0]);
            if (lane == 0) lcol[u0] = CP[r0];
            const V4 nc = nc0;
            CP[r0] = IK::shl(CP[r0]);
            A[r0] = shlv<F>(A[r0], nc.x);
            G[r0] = shlv<F>(G[r0], nc.y);
            S[r0] = shlv<F>(S[r0], nc.z);
          }
          // ---- row u1
          {
            const V4 rd = rd1;
            const F ai = rd.x, gi = rd.y, si = rd.z, ui = rd.w;
            static_for<DT>([&](auto tc) {
              constexpr int t = decltype(tc)::value;
              constexpr int p = (t + r1) % DT;
              k1[t] = IK::make(fma(-(C[t] * si), S[p], ui), (unsigned)(lane * DT + t));
              C[t] = fma(A[p], gi, C[t]);
              C[t] = fma(G[p], ai, C[t]);
            });
            lrow_w[4 * u1] = IK::rowmin(k1);
          }
          // ---- column minima: register p met slot p-r0 in row u0 and slot
          // p-r1 in row u1; register r0 holds the column that entered after
          // row u0 and met only slot DT-1 of row u1
          static_for<DT>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            if constexpr (p == r0) {
              CP[p] = IK::kmin(CP[p], k1[DT - 1]);
            } else {
              CP[p] = IK::kmin3(CP[p], k0[(p - r0 + DT) % DT], k1[(p - r1 + DT) % DT]);
            }
          });
          if (lane == 0) lcol[u1] = CP[r1];
          const V4 nc = nc1;
          CP[r1] = IK::shl(CP[r1]);
          A[r1] = shlv<F>(A[r1], nc.x);
          G[r1] = shlv<F>(G[r1], nc.y);
          S[r1] = shlv<F>(S[r1], nc.z);
        }
      });
      flush(sb, nb);
    }
    }

    // columns still in flight after the last row: slot t of lane L holds the
    // minimum of column i0 + nsteps + k0 + L*DT + t
    static_for<DT>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      emit_col(i0 + nsteps + k0 + (int64_t)lane * DT + t, CP[t]);
    });
  }
}

int sweep_grid(bool f64_sweep, int slots) {
  // compute units of the current device (asked on every call: a process may
  // drive several devices)
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  int per = 0;
  hipError_t e;
  if (f64_sweep)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep<double, float, 8, 32>, 64, 0);
  else if (slots == 8)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep<float, float, 8, 32>, 64, 0);
  else if (slots == 12)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep<float, float, 12, 36>, 64, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep<float, float, 16, 32>, 64, 0);
  if (e != hipSuccess || per <= 0) per = 8;
  return cus * per;
}

hipError_t launch_sweep(const Plan &plan, const Work &w, const void *T, bool t_f64, bool f64_sweep,
                        int slots, int R, int64_t total_tiles, int64_t nseg, int grid,
                        hipStream_t st) {
  const dim3 blk(64), grd((unsigned)grid);
#define MPX_LAUNCH(F, TIN, DT, TP)                                                              \
  hipLaunchKernelGGL((k_sweep<F, TIN, DT, TP>), grd, blk, 0, st, plan,                         \
                     (const typename FTraits<F>::V4 *)w.rc, (const double *)w.mu,              \
                     (const int64_t *)w.seg_prefix, (const int32_t *)w.seg_sweep,               \
                     (const int64_t *)w.seg_part, plan.s_ext,                                  \
                     plan.w_ext, w.scale, w.keys, w.counters, (const TIN *)T, R, total_tiles, nseg)
  if (f64_sweep) {
    if (t_f64) MPX_LAUNCH(double, double, 8, 32);
    else MPX_LAUNCH(double, float, 8, 32);
  } else if (slots == 8) {
    if (t_f64) MPX_LAUNCH(float, double, 8, 32);
    else MPX_LAUNCH(float, float, 8, 32);
  } else if (slots == 12) {
    if (t_f64) MPX_LAUNCH(float, double, 12, 36);
    else MPX_LAUNCH(float, float, 12, 36);
  } else {
    if (t_f64) MPX_LAUNCH(float, double, 16, 32);
    else MPX_LAUNCH(float, float, 16, 32);
  }
#undef MPX_LAUNCH
  return hipGetLastError();
}

}  // namespace mpx
