// Host side of the C ABI declared in include/mp.h: argument checks, the
// workspace layout, tiling choices and the launch sequence
//   plan (tile table) -> stats -> sweep -> special tables -> finalize -> rescan.
// Nothing here allocates device memory or synchronises.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/mp.h"
#include "mp_internal.h"

using mpx::SeriesDesc;
using mpx::SweepDesc;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Options {
  bool f64 = false;      // FP64 sweep
  int slots = 12;        // diagonals per lane (FP32 default 12, FP64 8)
  int reseed = 0;        // 0 = automatic
  bool fp64_finalize = true;
  bool flat_loads = false;  // backward gather: flat loads at any size
};

mp_status parse_options(const mp_options *opt, Options &o) {
  o = Options();
  if (!opt) return MP_OK;
  if (opt->precision != MP_PREC_F64 && opt->precision != MP_PREC_F32) return MP_EINVAL;
  o.f64 = opt->precision == MP_PREC_F64;
  if (opt->tile_slots != 0 && opt->tile_slots != 8 && opt->tile_slots != 12 &&
      opt->tile_slots != 16)
    return MP_EINVAL;
  if (o.f64 && opt->tile_slots != 0 && opt->tile_slots != 8) return MP_EUNSUPPORTED;
  o.slots = opt->tile_slots ? opt->tile_slots : (o.f64 ? 8 : 12);
  if (opt->reseed_rows < 0) return MP_EINVAL;
  if (opt->reseed_rows != 0 && (opt->reseed_rows % 64 != 0 || opt->reseed_rows > (1 << 20)))
    return MP_EINVAL;
  o.reseed = opt->reseed_rows;
  if (opt->flags & ~(MP_FLAG_FP64_FINALIZE | MP_FLAG_FLAT_LOADS)) return MP_EINVAL;
  o.fp64_finalize = (opt->flags & MP_FLAG_FP64_FINALIZE) != 0;
  o.flat_loads = (opt->flags & MP_FLAG_FLAT_LOADS) != 0;
  return MP_OK;
}

int bits_for(int64_t l) {
  int b = 1;
  while (((int64_t)1 << b) < l) ++b;
  return b;
}

// Host mirror of a job: series and sweeps, sizes, and the tile count.
struct Job {
  std::vector<SeriesDesc> series;
  std::vector<SweepDesc> sweeps;
  int64_t total_l = 0, total_rc = 0, total_x = 0, total_n = 0, nseg = 0, tiles = 0, cells = 0;
  int W = 512, R = 4096;
  Options opt;
  bool t_f64 = false;
  bool lr = false;               // left/right job: outputs [P | P_left | P_right]
  int64_t out_len = -1;          // profile entries written (default total_l)
  std::vector<uint32_t> kmask;   // chunk set of a restricted self-join (empty: none)
  int64_t kchunk = 0;            // offsets per chunk
};

void add_series(Job &j, int64_t t_off, int64_t n, int32_t m, int32_t ez, int partner, int out) {
  SeriesDesc s{};
  s.t_off = t_off;
  s.n = n;
  s.l = n - m + 1;
  s.w_off = j.total_l;
  s.rc_off = j.total_rc;
  s.x_off = j.total_x;
  s.p_off = s.w_off;
  s.m = m;
  s.ez = ez;
  s.partner = partner;
  s.out = out;
  s.side = 0;
  j.total_l += s.l;
  j.total_rc += s.l + mpx::kRcPad;
  j.total_x += s.l + 1;
  j.total_n += n;
  j.series.push_back(s);
}

void add_sweep(Job &j, int rs, int cs, int rk, int ck, int64_t k_lo, int64_t k_hi) {
  SweepDesc d{};
  d.rs = rs;
  d.cs = cs;
  d.rk = rk;
  d.ck = ck;
  d.k_lo = k_lo;
  d.k_hi = k_hi;
  // one spare index value, all ones, marks a minimum outside the series
  d.idx_bits = bits_for(std::max(j.series[rk].l, j.series[ck].l) + 1);
  d.nseg = 0;
  j.sweeps.push_back(d);
}

int64_t count_tiles(const Job &j, int W, int R) {
  int64_t t = 0;
  for (const SweepDesc &d : j.sweeps) {
    const SeriesDesc &rs = j.series[d.rs], &cs = j.series[d.cs];
    if (d.k_lo > d.k_hi) continue;
    for (int64_t k0 = d.k_lo; k0 <= d.k_hi; k0 += W) {
      const int64_t L = std::min(rs.l, cs.l - k0);
      t += (L + R - 1) / R;
    }
  }
  return t;
}

// Cells of one sweep: sum over diagonals k of min(l_r, l_c - k).
int64_t sweep_cells(int64_t lr, int64_t lc, int64_t k_lo, int64_t k_hi) {
  if (k_lo > k_hi) return 0;
  int64_t c = 0;
  // split at k where l_c - k == l_r
  const int64_t kb = lc - lr;  // for k <= kb the diagonal has l_r cells
  const int64_t a_hi = std::min(k_hi, kb);
  if (a_hi >= k_lo) c += (a_hi - k_lo + 1) * lr;
  const int64_t b_lo = std::max(k_lo, kb + 1);
  if (b_lo <= k_hi) {
    // sum_{k=b_lo}^{k_hi} (lc - k)
    const int64_t n = k_hi - b_lo + 1;
    c += n * lc - (b_lo + k_hi) * n / 2;
  }
  return c;
}

// Rows per LDS flush of the sweep (a multiple of the slot count).
int flush_rows(int slots) { return slots == 12 ? 36 : (slots == 16 ? 32 : (slots == 8 ? 32 : 16)); }

// Tiling: W = 64 * slots diagonals per strip, R rows per tile (also the
// reseed interval), a multiple of the flush period.  Automatic R starts at
// 4096 and halves (down to 64) while the job has fewer than ~8 tiles per
// SIMD.
void finish_job(Job &j) {
  j.W = 64 * j.opt.slots;
  int R = j.opt.reseed ? j.opt.reseed : 4096;
  if (!j.opt.reseed) {
    while (R > 64 && count_tiles(j, j.W, R) < 8 * 1024) R /= 2;
  }
  const int tp = flush_rows(j.opt.f64 ? 8 : j.opt.slots);
  j.R = ((R + tp - 1) / tp) * tp;
  int64_t seg = 0;
  j.cells = 0;
  for (SweepDesc &d : j.sweeps) {
    d.seg_base = seg;
    d.nseg = (d.k_lo > d.k_hi) ? 0 : (d.k_hi - d.k_lo + j.W) / j.W;
    seg += d.nseg;
    j.cells += sweep_cells(j.series[d.rs].l, j.series[d.cs].l, d.k_lo, d.k_hi);
  }
  j.nseg = seg;
  j.tiles = count_tiles(j, j.W, j.R);
}

struct Layout {
  size_t mu, sig, keys, flags, nc, nv, rc, special, scale, counters, segp, segs, segq, rescan, sdesc, wdesc, kmask;
  size_t b_mu, b_isig, b_nbr, b_wrec, b_alpha, b_wsc, b_bedge, b_bgam, b_bpos, b_count, b_off, b_tmp, b_erec, b_egam,
      b_chunk, b_big,
      b_nbig;
  size_t total;
};

Layout layout_of(const Job &j, bool with_batch_tables) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t tl = (size_t)j.total_l;
  L.mu = take(8 * tl);
  L.sig = take(8 * tl);
  L.keys = take(8 * tl);
  L.flags = take(tl);
  L.nc = take(4 * (size_t)j.total_x);
  L.nv = take(4 * (size_t)j.total_x);
  L.rc = take((j.opt.f64 ? 32 : 16) * (size_t)j.total_rc);
  L.special = take(4 * j.series.size());
  L.scale = take(8 * j.series.size());
  L.counters = take(8 * 4);
  L.segp = take(8 * ((size_t)j.nseg + 1));
  L.segs = take(4 * std::max<size_t>(1, (size_t)j.nseg));
  L.segq = take(8 * ((size_t)j.nseg + 1));
  L.rescan = take(8 * tl);
  if (with_batch_tables) {
    L.b_mu = take(8 * tl);
    L.b_isig = take(8 * tl);
    L.b_nbr = take(8 * tl);
    L.b_wrec = take(sizeof(mpx::BwdWin) * tl);
    L.b_alpha = take(8 * tl);
    L.b_wsc = take(8 * tl);
    L.b_bedge = take(sizeof(mpx::BwdEdge) * tl);
    L.b_bgam = take(8 * tl);
    L.b_bpos = take(4 * tl);
    L.b_count = take(8 * tl);
    L.b_off = take(8 * (tl + 1));
    L.b_tmp = take(8 * tl);  // indexed like erec
    L.b_erec = take(sizeof(mpx::BwdEdge) * tl);
    L.b_egam = take(8 * tl);
    L.b_chunk = take(8 * ((tl + 1023) / 1024 + 1));
    L.b_big = take(8 * (tl / (size_t)mpx::kBwdSmallBucket + 1));
    L.b_nbig = take(8);
    L.sdesc = take(sizeof(SeriesDesc) * j.series.size());
    L.wdesc = take(sizeof(SweepDesc) * j.sweeps.size());
    L.kmask = take(4 * std::max<size_t>(1, j.kmask.size()));
  }
  L.total = o;
  return L;
}

mpx::Work work_of(const Layout &L, void *ws) {
  char *b = (char *)ws;
  mpx::Work w{};
  w.mu = (double *)(b + L.mu);
  w.sig = (double *)(b + L.sig);
  w.keys = (uint64_t *)(b + L.keys);
  w.flags = (uint8_t *)(b + L.flags);
  w.next_const = (int32_t *)(b + L.nc);
  w.next_valid = (int32_t *)(b + L.nv);
  w.rc = (void *)(b + L.rc);
  w.special = (int32_t *)(b + L.special);
  w.scale = (double *)(b + L.scale);
  w.counters = (unsigned long long *)(b + L.counters);
  w.seg_prefix = (int64_t *)(b + L.segp);
  w.seg_sweep = (int32_t *)(b + L.segs);
  w.seg_part = (int64_t *)(b + L.segq);
  w.rescan = (int64_t *)(b + L.rescan);
  return w;
}

mpx::BwdWork bwd_work_of(const Layout &L, void *ws) {
  char *b = (char *)ws;
  mpx::BwdWork w{};
  w.mu = (double *)(b + L.b_mu);
  w.isig = (double *)(b + L.b_isig);
  w.nbr = (int64_t *)(b + L.b_nbr);
  w.wrec = (mpx::BwdWin *)(b + L.b_wrec);
  w.alpha = (double *)(b + L.b_alpha);
  w.wsc = (double *)(b + L.b_wsc);
  w.bedge = (mpx::BwdEdge *)(b + L.b_bedge);
  w.bgam = (double *)(b + L.b_bgam);
  w.bpos = (uint32_t *)(b + L.b_bpos);
  w.count = (unsigned long long *)(b + L.b_count);
  w.off = (int64_t *)(b + L.b_off);
  w.tmp = (int64_t *)(b + L.b_tmp);
  w.erec = (mpx::BwdEdge *)(b + L.b_erec);
  w.egam = (double *)(b + L.b_egam);
  w.chunk = (int64_t *)(b + L.b_chunk);
  w.big = (int64_t *)(b + L.b_big);
  w.nbig = (unsigned long long *)(b + L.b_nbig);
  w.fmu = (const double *)(b + L.mu);
  w.fsig = (const double *)(b + L.sig);
  w.fflags = (const uint8_t *)(b + L.flags);
  return w;
}

// The backward covers self-join and AB-join plans whose windows are at most
// 2^30 samples long (the gather tests window ranges in 32 bits relative to
// a wave's first covering window: fewer than 64 + m of them).
bool backward_supported(const Job &j) {
  if (j.lr) return false;
  for (const SeriesDesc &s : j.series)
    if (s.m > (1 << 30)) return false;
  return true;
}

mpx::Plan plan_of(const Job &j, const Layout &L, void *ws, bool external) {
  mpx::Plan p{};
  p.nseries = (int32_t)j.series.size();
  p.nsweeps = (int32_t)j.sweeps.size();
  if (external) {
    p.s_ext = (const SeriesDesc *)((char *)ws + L.sdesc);
    p.w_ext = (const SweepDesc *)((char *)ws + L.wdesc);
    if (!j.kmask.empty()) {
      p.kmask = (const uint32_t *)((char *)ws + L.kmask);
      p.kchunk = j.kchunk;
    }
  } else {
    for (size_t i = 0; i < j.series.size() && i < 2; ++i) p.s_inl[i] = j.series[i];
    for (size_t i = 0; i < j.sweeps.size() && i < 2; ++i) p.w_inl[i] = j.sweeps[i];
  }
  return p;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Benchmark timing: event quadruples (start, sweep start, sweep end, end) per
// call, recycled after each query.  Calls may come from several host
// threads, so the event lists are guarded by a mutex.
struct Timing {
  std::atomic<bool> on{false};
  std::mutex mu;
  std::vector<hipEvent_t> pool;   // free events
  std::vector<hipEvent_t> rec;    // 4 per recorded call
  hipEvent_t get() {
    {
      std::lock_guard<std::mutex> g(mu);
      if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
      }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void record(const hipEvent_t (&ev)[4]) {
    std::lock_guard<std::mutex> g(mu);
    for (hipEvent_t e : ev) rec.push_back(e);
  }
};
Timing g_timing;
size_t esize(mp_dtype dt) { return dt == MP_F64 ? 8 : 4; }

mp_status check_ws(void *ws, size_t ws_bytes, size_t need) {
  if (!ws || !aligned(ws, kAlign) || ws_bytes < need) return MP_EWORKSPACE;
  return MP_OK;
}

// The full launch sequence of a job whose descriptors are reachable through
// `plan`.
// Key error floor of the FP32 sweep.  A key is 1 - rho = d^2 / (2m); the
// FP32 cross product drifts between FP64 seeds by rounding steps of about
// 2^-24 of its size, so over a tile of R rows the key error grows like
// 2^-24 sqrt(2R): measured on the n = 2^20, m = 256 planted walk at
// R = 4104, the largest key error over all rows was 4.5e-5 among rows with
// P < 3 (1e-4 at P ~ 30, where the code bits of the key dominate), i.e.
// 8 x 2^-24 sqrt(2R).  delta = 16 x 2^-24 sqrt(2R) doubles that.  Two
// candidates whose keys differ by less than 2 delta may be ordered wrongly;
// near d = 0 that costs up to sqrt(4 m delta) in d after the FP64 finalize,
// above the tolerance, so rows whose raw key is below 2 delta (near-exact
// repeats, d < sqrt(4 m delta) ~ 0.3 at m = 256) are re-found exactly by
// the FP64 rescan.  Rows above it can lose at most 2 m delta / d.
double fp32_key_floor(int R) { return 2.0 * 16.0 * std::ldexp(1.0, -24) * std::sqrt(2.0 * R); }

// `timed`: record benchmark events when timing is enabled (the entry point
// without allocations never does: creating an event is an allocation).
mp_status run_job(const Job &j, const mpx::Plan &plan, const mpx::Work &w, const void *T,
                  const mpx::Outputs &o, bool out_f64, hipStream_t st, bool timed = true) {
  const Options &op = j.opt;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  const bool rec = timed && g_timing.on;
  if (rec) {
    for (auto &e : ev) e = g_timing.get();
    if (ev[0]) (void)hipEventRecord(ev[0], st);
  }
  if (mpx::launch_plan(plan, w, T, j.t_f64, j.W, j.R, j.nseg, st) != hipSuccess) return MP_ELAUNCH;
  if (mpx::launch_stats(plan, w, T, j.t_f64, op.f64, j.total_rc, st) != hipSuccess) return MP_ELAUNCH;
  if (ev[1]) (void)hipEventRecord(ev[1], st);
  if (j.tiles > 0) {
    const int grid = (int)std::min<int64_t>(j.tiles, mpx::sweep_grid(op.f64, op.slots));
    if (mpx::launch_sweep(plan, w, T, j.t_f64, op.f64, op.slots, j.R, j.tiles, j.nseg, grid, st) !=
        hipSuccess)
      return MP_ELAUNCH;
  }
  if (ev[2]) (void)hipEventRecord(ev[2], st);
  if (mpx::launch_special(plan, w, st) != hipSuccess) return MP_ELAUNCH;
  const double kappa = (!op.f64 && op.fp64_finalize) ? fp32_key_floor(j.R) : 0.0;
  if (mpx::launch_finalize(plan, w, T, j.t_f64, o, out_f64, op.fp64_finalize, kappa, j.total_l, st) !=
      hipSuccess)
    return MP_ELAUNCH;
  if (mpx::launch_rescan(plan, w, T, j.t_f64, o, out_f64, op.fp64_finalize, st) != hipSuccess)
    return MP_ELAUNCH;
  if (j.lr && mpx::launch_lr_combine(o, out_f64, j.series[0].l, st) != hipSuccess) return MP_ELAUNCH;
  if (rec) {
    if (ev[3]) (void)hipEventRecord(ev[3], st);
    g_timing.record(ev);
  }
  return MP_OK;
}

mp_status build_selfjoin(int64_t n, int32_t m, int32_t ez, mp_dtype dt, const mp_options *opt,
                         Job &j) {
  if (dt != MP_F64 && dt != MP_F32) return MP_EINVAL;
  if (m < 2 || n < m || ez < 0) return MP_EINVAL;
  if (n - m + 1 >= ((int64_t)1 << 31)) return MP_EINVAL;
  mp_status s = parse_options(opt, j.opt);
  if (s != MP_OK) return s;
  j.t_f64 = dt == MP_F64;
  add_series(j, 0, n, m, ez, 0, 0);
  const int64_t l = n - m + 1;
  add_sweep(j, 0, 0, 0, 0, (int64_t)ez + 1, l - 1);
  finish_job(j);
  return MP_OK;
}

// B's samples: at b_off in the call's one sample array (b_sep = false, the
// AB-join plans' [A | B] layout), or at the start of a second array (b_sep).
mp_status build_abjoin(int64_t nA, int64_t nB, int64_t b_off, bool b_sep, int32_t m, mp_dtype dt,
                       const mp_options *opt, Job &j) {
  if (dt != MP_F64 && dt != MP_F32) return MP_EINVAL;
  if (m < 2 || nA < m || nB < m) return MP_EINVAL;
  if (nA - m + 1 >= ((int64_t)1 << 31) || nB - m + 1 >= ((int64_t)1 << 31)) return MP_EINVAL;
  mp_status s = parse_options(opt, j.opt);
  if (s != MP_OK) return s;
  j.t_f64 = dt == MP_F64;
  add_series(j, 0, nA, m, -1, 1, 0);
  add_series(j, b_sep ? 0 : b_off, nB, m, -1, 0, 1);
  j.series[1].tsel = b_sep ? 1 : 0;
  j.series[1].p_off = 0;  // second output array
  const int64_t lA = nA - m + 1, lB = nB - m + 1;
  add_sweep(j, 0, 1, 0, 1, 0, lB - 1);  // rows A, columns B, j >= i
  add_sweep(j, 1, 0, 1, 0, 1, lA - 1);  // rows B, columns A, i > j
  finish_job(j);
  return MP_OK;
}

}  // namespace

struct mp_batch_plan {
  Job job;
  Layout lay;
};

namespace {

// Chunks of diagonal offsets of a self-join: offsets ez + 1 .. l - 1 in
// runs of one strip width.
int64_t chunk_count(int64_t l, int32_t ez, int W) {
  const int64_t span = l - 1 - (int64_t)ez;
  return span > 0 ? (span + W - 1) / W : 0;
}

mp_status build_selfjoin_plan(int64_t n, int32_t m, int32_t ez, mp_dtype dt, const mp_options *opt,
                              int32_t sides, int64_t nchunks, const int64_t *chunks, Job &j) {
  if (dt != MP_F64 && dt != MP_F32) return MP_EINVAL;
  if (m < 2 || n < m || ez < 0) return MP_EINVAL;
  if (n - m + 1 >= ((int64_t)1 << 31)) return MP_EINVAL;
  if (sides != MP_SIDES_BOTH && sides != MP_SIDES_LEFT_RIGHT) return MP_EINVAL;
  if (nchunks < 0 || (nchunks > 0 && !chunks)) return MP_EINVAL;
  mp_status s = parse_options(opt, j.opt);
  if (s != MP_OK) return s;
  j.t_f64 = dt == MP_F64;
  const int64_t l = n - m + 1;
  const int W = 64 * j.opt.slots;
  const int64_t nch = chunk_count(l, ez, W);
  std::vector<int64_t> list;
  if (chunks) {
    j.kmask.assign((size_t)std::max<int64_t>(1, (nch + 31) / 32), 0u);
    j.kchunk = W;
    for (int64_t q = 0; q < nchunks; ++q) {
      const int64_t c = chunks[q];
      if (c < 0 || c >= nch) return MP_EINVAL;
      uint32_t &word = j.kmask[(size_t)(c >> 5)];
      if (word & (1u << (c & 31))) return MP_EINVAL;  // repeated chunk
      word |= 1u << (c & 31);
      list.push_back(c);
    }
  }
  int rows = 0;
  if (sides == MP_SIDES_BOTH) {
    add_series(j, 0, n, m, ez, 0, 0);
  } else {
    // series 0 collects the left profile (column minima), series 1 the right
    // profile (row minima); both read the same samples
    add_series(j, 0, n, m, ez, 0, 0);
    add_series(j, 0, n, m, ez, 1, 0);
    j.series[0].side = mpx::kSideLeft;
    j.series[0].p_off = l;
    j.series[1].side = mpx::kSideRight;
    j.series[1].p_off = 2 * l;
    j.lr = true;
    j.out_len = 3 * l;
    rows = 1;
  }
  const int cols_key = 0;
  if (!chunks) {
    add_sweep(j, rows, rows, rows, cols_key, (int64_t)ez + 1, l - 1);
  } else {
    for (int64_t c : list)
      add_sweep(j, rows, rows, rows, cols_key, (int64_t)ez + 1 + c * W,
                std::min<int64_t>((int64_t)ez + (c + 1) * W, l - 1));
  }
  finish_job(j);
  return MP_OK;
}

}  // namespace

extern "C" {

int mp_abi_version(void) { return MP_ABI_VERSION; }

const char *mp_strerror(mp_status s) {
  switch (s) {
    case MP_OK: return "ok";
    case MP_EINVAL: return "invalid argument";
    case MP_EWORKSPACE: return "workspace missing, misaligned or too small";
    case MP_ELAUNCH: return "kernel launch failed";
    case MP_EUNSUPPORTED: return "unsupported option combination";
    case MP_ETOOLARGE:
      return "job needs more scratch than the fixed MP_NOALLOC_SCRATCH_BYTES of mp_selfjoin_noalloc";
  }
  return "unknown status";
}

int64_t mp_selfjoin_cells(int64_t n, int32_t m, int32_t ez) {
  if (m < 2 || n < m || ez < 0) return 0;
  const int64_t l = n - m + 1;
  return sweep_cells(l, l, (int64_t)ez + 1, l - 1);
}

int64_t mp_abjoin_cells(int64_t nA, int64_t nB, int32_t m) {
  if (m < 2 || nA < m || nB < m) return 0;
  return (nA - m + 1) * (nB - m + 1);
}

size_t mp_selfjoin_workspace(int64_t n, int32_t m, mp_dtype dtype, const mp_options *opt) {
  Job j;
  if (build_selfjoin(n, m, 0, dtype, opt, j) != MP_OK) return 0;
  return layout_of(j, false).total;
}

mp_status mp_selfjoin(const void *T, int64_t n, int32_t m, int32_t ez, mp_dtype dtype,
                      const mp_options *opt, void *P, int64_t *I, void *ws, size_t ws_bytes,
                      void *stream) {
  Job j;
  mp_status s = build_selfjoin(n, m, ez, dtype, opt, j);
  if (s != MP_OK) return s;
  if (!T || !P || !I || !aligned(T, esize(dtype)) || !aligned(P, esize(dtype)) || !aligned(I, 8))
    return MP_EINVAL;
  const Layout L = layout_of(j, false);
  if ((s = check_ws(ws, ws_bytes, L.total)) != MP_OK) return s;
  const mpx::Work w = work_of(L, ws);
  const mpx::Plan p = plan_of(j, L, ws, false);
  mpx::Outputs o{};
  o.P[0] = P;
  o.I[0] = I;
  return run_job(j, p, w, T, o, dtype == MP_F64, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Fixed device scratch of mp_selfjoin_noalloc: the self-join workspace lives
// here instead of in caller memory.  Every device the library runs on holds
// one copy (at its own address) until the process ends.  In host code the
// array's name is only a stand-in; the device address comes from
// hipGetSymbolAddress, taken once per device and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[MP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The scratch address on the current device (looked up on the first call
// there).
mp_status scratch_of_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MP_ELAUNCH;
  if (dev < 0 || dev >= kMaxDevices) return MP_EUNSUPPORTED;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MP_ELAUNCH;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MP_OK;
}

}  // namespace

extern "C" {

mp_status mp_selfjoin_noalloc(const void *T, int64_t n, int32_t m, int32_t ez, mp_dtype dtype,
                              const mp_options *opt, void *P, int64_t *I, void *stream) {
  Job j;
  mp_status s = build_selfjoin(n, m, ez, dtype, opt, j);
  if (s != MP_OK) return s;
  if (!T || !P || !I || !aligned(T, esize(dtype)) || !aligned(P, esize(dtype)) || !aligned(I, 8))
    return MP_EINVAL;
  const Layout L = layout_of(j, false);
  if (L.total > (size_t)MP_NOALLOC_SCRATCH_BYTES) return MP_ETOOLARGE;
  hipStream_t st = (hipStream_t)stream;
  if (st) {
    // the scratch used is the current device's; the stream must run there
    int cur = -1;
    hipDevice_t sdev = -1;
    if (hipGetDevice(&cur) != hipSuccess || hipStreamGetDevice(st, &sdev) != hipSuccess) return MP_ELAUNCH;
    if (sdev != cur) return MP_EINVAL;
  }
  void *ws = nullptr;
  if ((s = scratch_of_current_device(&ws)) != MP_OK) return s;
  const mpx::Work w = work_of(L, ws);
  const mpx::Plan p = plan_of(j, L, ws, false);
  mpx::Outputs o{};
  o.P[0] = P;
  o.I[0] = I;
  return run_job(j, p, w, T, o, dtype == MP_F64, st, /*timed=*/false);
}

size_t mp_abjoin_workspace(int64_t nA, int64_t nB, int32_t m, mp_dtype dtype, const mp_options *opt) {
  Job j;
  if (build_abjoin(nA, nB, 0, true, m, dtype, opt, j) != MP_OK) return 0;
  return layout_of(j, false).total;
}

mp_status mp_abjoin(const void *A, int64_t nA, const void *B, int64_t nB, int32_t m, mp_dtype dtype,
                    const mp_options *opt, void *P_ab, int64_t *I_ab, void *P_ba, int64_t *I_ba,
                    void *ws, size_t ws_bytes, void *stream) {
  if (!A || !B || !P_ab || !I_ab || !P_ba || !I_ba) return MP_EINVAL;
  const size_t es = esize(dtype);
  if (!aligned(A, es) || !aligned(B, es) || !aligned(P_ab, es) || !aligned(P_ba, es) ||
      !aligned(I_ab, 8) || !aligned(I_ba, 8))
    return MP_EINVAL;
  Job j;
  mp_status s = build_abjoin(nA, nB, 0, true, m, dtype, opt, j);
  if (s != MP_OK) return s;
  const Layout L = layout_of(j, false);
  if ((s = check_ws(ws, ws_bytes, L.total)) != MP_OK) return s;
  const mpx::Work w = work_of(L, ws);
  mpx::Plan p = plan_of(j, L, ws, false);
  p.t2 = B;  // series 1 (B) reads its samples from B
  mpx::Outputs o{};
  o.P[0] = P_ab;
  o.I[0] = I_ab;
  o.P[1] = P_ba;
  o.I[1] = I_ba;
  return run_job(j, p, w, A, o, dtype == MP_F64, (hipStream_t)stream);
}

mp_status mp_batch_plan_create(int32_t nseries, const int64_t *t_off, const int32_t *m,
                               const int32_t *ez, mp_dtype dtype, const mp_options *opt,
                               mp_batch_plan **out) {
  if (!out) return MP_EINVAL;
  *out = nullptr;
  if (nseries < 1 || !t_off || !m || !ez) return MP_EINVAL;
  if (dtype != MP_F64 && dtype != MP_F32) return MP_EINVAL;
  mp_batch_plan *pl = new (std::nothrow) mp_batch_plan();
  if (!pl) return MP_EINVAL;
  Job &j = pl->job;
  mp_status s = parse_options(opt, j.opt);
  if (s != MP_OK) {
    delete pl;
    return s;
  }
  j.t_f64 = dtype == MP_F64;
  if (t_off[0] != 0) {
    delete pl;
    return MP_EINVAL;
  }
  for (int32_t i = 0; i < nseries; ++i) {
    const int64_t n = t_off[i + 1] - t_off[i];
    if (m[i] < 2 || n < m[i] || ez[i] < 0 || n - m[i] + 1 >= ((int64_t)1 << 31)) {
      delete pl;
      return MP_EINVAL;
    }
    add_series(j, t_off[i], n, m[i], ez[i], i, 0);
  }
  if (j.total_l >= ((int64_t)1 << 40)) {
    delete pl;
    return MP_EINVAL;
  }
  for (int32_t i = 0; i < nseries; ++i)
    add_sweep(j, i, i, i, i, (int64_t)ez[i] + 1, j.series[i].l - 1);
  finish_job(j);
  pl->lay = layout_of(j, true);
  *out = pl;
  return MP_OK;
}

mp_status mp_abjoin_plan_create(int64_t nA, int64_t nB, int32_t m, mp_dtype dtype,
                                const mp_options *opt, mp_batch_plan **out) {
  if (!out) return MP_EINVAL;
  *out = nullptr;
  mp_batch_plan *pl = new (std::nothrow) mp_batch_plan();
  if (!pl) return MP_EINVAL;
  const mp_status s = build_abjoin(nA, nB, nA, false, m, dtype, opt, pl->job);
  if (s != MP_OK) {
    delete pl;
    return s;
  }
  // one output array: P_ab at [0, lA), P_ba at [lA, lA + lB)
  pl->job.series[1].out = 0;
  pl->job.series[1].p_off = pl->job.series[1].w_off;
  pl->lay = layout_of(pl->job, true);
  *out = pl;
  return MP_OK;
}

int64_t mp_selfjoin_chunks(int64_t n, int32_t m, int32_t ez, const mp_options *opt,
                           int64_t *chunk_width) {
  Options o;
  if (m < 2 || n < m || ez < 0 || parse_options(opt, o) != MP_OK) return -1;
  const int W = 64 * o.slots;
  if (chunk_width) *chunk_width = W;
  return chunk_count(n - m + 1, ez, W);
}

mp_status mp_selfjoin_plan_create(int64_t n, int32_t m, int32_t ez, mp_dtype dtype,
                                  const mp_options *opt, int32_t sides, int64_t nchunks,
                                  const int64_t *chunks, mp_batch_plan **out) {
  if (!out) return MP_EINVAL;
  *out = nullptr;
  mp_batch_plan *pl = new (std::nothrow) mp_batch_plan();
  if (!pl) return MP_EINVAL;
  const mp_status s = build_selfjoin_plan(n, m, ez, dtype, opt, sides, nchunks, chunks, pl->job);
  if (s != MP_OK) {
    delete pl;
    return s;
  }
  pl->lay = layout_of(pl->job, true);
  *out = pl;
  return MP_OK;
}

mp_status mp_anytime_order(int64_t count, uint64_t seed, int64_t *order) {
  if (count < 0 || (count > 0 && !order)) return MP_EINVAL;
  // Fisher-Yates driven by SplitMix64 (Steele, Lea, Flood 2014)
  uint64_t x = seed;
  auto next = [&x]() {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  for (int64_t i = 0; i < count; ++i) order[i] = i;
  for (int64_t i = count - 1; i > 0; --i) {
    const int64_t r = (int64_t)(next() % (uint64_t)(i + 1));
    std::swap(order[i], order[r]);
  }
  return MP_OK;
}

size_t mp_batch_plan_workspace(const mp_batch_plan *pl) { return pl ? pl->lay.total : 0; }
int64_t mp_batch_plan_profile_length(const mp_batch_plan *pl) {
  if (!pl) return 0;
  return pl->job.out_len >= 0 ? pl->job.out_len : pl->job.total_l;
}
int64_t mp_batch_plan_cells(const mp_batch_plan *pl) { return pl ? pl->job.cells : 0; }

mp_status mp_batch_plan_upload(const mp_batch_plan *pl, void *ws, size_t ws_bytes, void *stream) {
  if (!pl) return MP_EINVAL;
  mp_status s = check_ws(ws, ws_bytes, pl->lay.total);
  if (s != MP_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char *b = (char *)ws;
  if (hipMemcpyAsync(b + pl->lay.sdesc, pl->job.series.data(),
                     sizeof(SeriesDesc) * pl->job.series.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return MP_ELAUNCH;
  if (hipMemcpyAsync(b + pl->lay.wdesc, pl->job.sweeps.data(),
                     sizeof(SweepDesc) * pl->job.sweeps.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return MP_ELAUNCH;
  if (!pl->job.kmask.empty() &&
      hipMemcpyAsync(b + pl->lay.kmask, pl->job.kmask.data(), 4 * pl->job.kmask.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return MP_ELAUNCH;
  return MP_OK;
}

mp_status mp_batch(const mp_batch_plan *pl, const void *T_cat, void *P_cat, int64_t *I_cat, void *ws,
                   size_t ws_bytes, void *stream) {
  if (!pl || !T_cat || !P_cat || !I_cat) return MP_EINVAL;
  const size_t es = pl->job.t_f64 ? 8 : 4;
  if (!aligned(T_cat, es) || !aligned(P_cat, es) || !aligned(I_cat, 8)) return MP_EINVAL;
  mp_status s = check_ws(ws, ws_bytes, pl->lay.total);
  if (s != MP_OK) return s;
  const mpx::Work w = work_of(pl->lay, ws);
  const mpx::Plan p = plan_of(pl->job, pl->lay, ws, true);
  mpx::Outputs o{};
  o.P[0] = P_cat;
  o.I[0] = I_cat;
  return run_job(pl->job, p, w, T_cat, o, pl->job.t_f64, (hipStream_t)stream);
}

void mp_batch_plan_destroy(mp_batch_plan *pl) { delete pl; }

mp_status mp_timing_enable(int enable) {
  g_timing.on = enable != 0;
  return MP_OK;
}

mp_status mp_timing_query(double *sweep_ms, double *total_ms, int64_t *calls) {
  double sw = 0.0, tot = 0.0;
  int64_t n = 0;
  mp_status st = MP_OK;
  std::vector<hipEvent_t> recs;
  {
    std::lock_guard<std::mutex> g(g_timing.mu);
    recs.swap(g_timing.rec);
  }
  std::vector<hipEvent_t> done;
  for (size_t q = 0; q + 3 < recs.size(); q += 4) {
    hipEvent_t *e = &recs[q];
    float a = 0.f, b = 0.f;
    if (e[0] && e[1] && e[2] && e[3] && hipEventSynchronize(e[3]) == hipSuccess &&
        hipEventElapsedTime(&a, e[1], e[2]) == hipSuccess &&
        hipEventElapsedTime(&b, e[0], e[3]) == hipSuccess) {
      sw += a;
      tot += b;
      ++n;
    } else {
      st = MP_ELAUNCH;
    }
    for (int k = 0; k < 4; ++k)
      if (e[k]) done.push_back(e[k]);
  }
  {
    std::lock_guard<std::mutex> g(g_timing.mu);
    g_timing.pool.insert(g_timing.pool.end(), done.begin(), done.end());
  }
  if (sweep_ms) *sweep_ms = sw;
  if (total_ms) *total_ms = tot;
  if (calls) *calls = n;
  return st;
}

mp_status mp_backward(const mp_batch_plan *pl, const void *T_cat, const int64_t *I_cat,
                      const void *gP_cat, void *gT_cat, void *ws, size_t ws_bytes, void *stream) {
  if (!pl || !T_cat || !I_cat || !gP_cat || !gT_cat) return MP_EINVAL;
  if (!backward_supported(pl->job)) return MP_EUNSUPPORTED;
  const size_t es = pl->job.t_f64 ? 8 : 4;
  if (!aligned(T_cat, es) || !aligned(gP_cat, es) || !aligned(gT_cat, es) || !aligned(I_cat, 8))
    return MP_EINVAL;
  mp_status s = check_ws(ws, ws_bytes, pl->lay.total);
  if (s != MP_OK) return s;
  const mpx::BwdWork w = bwd_work_of(pl->lay, ws);
  const mpx::Plan p = plan_of(pl->job, pl->lay, ws, true);
  if (mpx::launch_backward(p, w, T_cat, pl->job.t_f64, I_cat, gP_cat, gT_cat, pl->job.total_l,
                           pl->job.total_n, pl->job.opt.flat_loads, (hipStream_t)stream) != hipSuccess)
    return MP_ELAUNCH;
  return MP_OK;
}

mp_status mp_backward_after_forward(const mp_batch_plan *pl, const void *T_cat, const int64_t *I_cat,
                                    const void *P_cat, const void *gP_cat, void *gT_cat, void *ws,
                                    size_t ws_bytes, void *stream) {
  if (!pl || !T_cat || !I_cat || !P_cat || !gP_cat || !gT_cat) return MP_EINVAL;
  if (!backward_supported(pl->job) || !pl->job.opt.fp64_finalize) return MP_EUNSUPPORTED;
  const size_t es = pl->job.t_f64 ? 8 : 4;
  if (!aligned(T_cat, es) || !aligned(P_cat, es) || !aligned(gP_cat, es) || !aligned(gT_cat, es) ||
      !aligned(I_cat, 8))
    return MP_EINVAL;
  mp_status s = check_ws(ws, ws_bytes, pl->lay.total);
  if (s != MP_OK) return s;
  const mpx::BwdWork w = bwd_work_of(pl->lay, ws);
  const mpx::Plan p = plan_of(pl->job, pl->lay, ws, true);
  if (mpx::launch_backward_after_forward(p, w, T_cat, pl->job.t_f64, I_cat, P_cat, gP_cat, gT_cat,
                                         pl->job.total_l, pl->job.total_n, pl->job.opt.flat_loads,
                                         (hipStream_t)stream) != hipSuccess)
    return MP_ELAUNCH;
  return MP_OK;
}

}  // extern "C"

namespace {

// Multidimensional job: the self-join or AB-join descriptors of the
// one-dimensional path with 64-diagonal strips; every dimension of a series
// shares its windows.
struct MdLayout {
  size_t rec, mu2, keys, segp, segs, counters, special, total;
  int64_t stride;
};

// An AB-join's B is a second sample array (SeriesDesc::tsel = 1, Plan::t2).
mp_status build_md(int32_t mode, int32_t D, int64_t nA, int64_t nB, int32_t m, int32_t ez, bool self,
                   mp_dtype dt, Job &j, MdLayout &L) {
  if (dt != MP_F64 && dt != MP_F32) return MP_EINVAL;
  if (mode != MP_MD_SIMPLE && mode != MP_MD_MULTI) return MP_EINVAL;
  if (D < 1 || D > mpx::kMdMaxDims || m < 2 || nA < m) return MP_EINVAL;
  if (self && ez < 0) return MP_EINVAL;
  if (!self && nB < m) return MP_EINVAL;
  if (!self && mode == MP_MD_MULTI) return MP_EUNSUPPORTED;
  if (nA - m + 1 >= ((int64_t)1 << 31) || (!self && nB - m + 1 >= ((int64_t)1 << 31))) return MP_EINVAL;
  j.t_f64 = dt == MP_F64;
  if (self) {
    add_series(j, 0, nA, m, ez, 0, 0);
    add_sweep(j, 0, 0, 0, 0, (int64_t)ez + 1, nA - m);
  } else {
    add_series(j, 0, nA, m, -1, 1, 0);
    add_series(j, 0, nB, m, -1, 0, 1);
    j.series[1].tsel = 1;
    j.series[1].p_off = 0;
    add_sweep(j, 0, 1, 0, 1, 0, nB - m);
    add_sweep(j, 1, 0, 1, 0, 1, nA - m);
  }
  const int W = mpx::md_strip_width(mode, D);
  j.W = W;
  int R = 2048;
  while (R > 64 && count_tiles(j, W, R) < 8 * 1024) R /= 2;
  j.R = R;
  int64_t seg = 0;
  j.cells = 0;
  for (SweepDesc &d : j.sweeps) {
    d.seg_base = seg;
    d.nseg = (d.k_lo > d.k_hi) ? 0 : (d.k_hi - d.k_lo + W) / W;
    seg += d.nseg;
    j.cells += sweep_cells(j.series[d.rs].l, j.series[d.cs].l, d.k_lo, d.k_hi);
  }
  j.nseg = seg;
  j.tiles = count_tiles(j, W, R);
  const int np = mode == MP_MD_MULTI ? D : 1;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.stride = j.total_rc;
  L.rec = take(32 * (size_t)D * (size_t)j.total_rc);
  L.mu2 = take(16 * (size_t)D * (size_t)j.total_rc);
  L.keys = take(8 * (size_t)np * (size_t)j.total_l);
  L.segp = take(8 * ((size_t)j.nseg + 1));
  L.segs = take(4 * std::max<size_t>(1, (size_t)j.nseg));
  L.counters = take(8 * 4);
  L.special = take(4 * j.series.size());
  L.total = o;
  return MP_OK;
}

}  // namespace

extern "C" {

size_t mp_mdjoin_workspace(int32_t mode, int32_t D, int64_t nA, int64_t nB, int32_t m) {
  Job j;
  MdLayout L;
  const bool self = nB <= 0;
  if (build_md(mode, D, nA, nB, m, 0, self, MP_F32, j, L) != MP_OK) return 0;
  return L.total;
}

mp_status mp_mdjoin(int32_t mode, int32_t D, const void *A, int64_t nA, const void *B, int64_t nB,
                    int32_t m, int32_t ez, mp_dtype dtype, void *P, int64_t *I, void *P_ba,
                    int64_t *I_ba, void *ws, size_t ws_bytes, void *stream) {
  const bool self = B == nullptr;
  const size_t es = esize(dtype);
  if (!A || !P || !I || !aligned(A, es) || !aligned(P, es) || !aligned(I, 8)) return MP_EINVAL;
  if (!self && (!P_ba || !I_ba || !aligned(B, es) || !aligned(P_ba, es) || !aligned(I_ba, 8)))
    return MP_EINVAL;
  Job j;
  MdLayout L;
  mp_status s = build_md(mode, D, nA, nB, m, ez, self, dtype, j, L);
  if (s != MP_OK) return s;
  if ((s = check_ws(ws, ws_bytes, L.total)) != MP_OK) return s;
  char *b = (char *)ws;
  mpx::Plan p = plan_of(j, Layout{}, ws, false);
  p.t2 = self ? nullptr : B;
  mpx::Work w{};
  w.seg_prefix = (int64_t *)(b + L.segp);
  w.seg_sweep = (int32_t *)(b + L.segs);
  w.counters = (unsigned long long *)(b + L.counters);
  w.special = (int32_t *)(b + L.special);
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  if (g_timing.on) {
    for (auto &e : ev) e = g_timing.get();
    if (ev[0]) (void)hipEventRecord(ev[0], st);
  }
  if (mpx::launch_plan(p, w, A, j.t_f64, j.W, j.R, j.nseg, st) != hipSuccess) return MP_ELAUNCH;
  mpx::Outputs o{};
  o.P[0] = P;
  o.I[0] = I;
  o.P[1] = self ? nullptr : P_ba;
  o.I[1] = self ? nullptr : I_ba;
  const int grid = (int)std::min<int64_t>(std::max<int64_t>(j.tiles, 1), mpx::md_sweep_grid(mode, D));
  if (mpx::launch_md(mode, D, p, A, dtype == MP_F64, b + L.rec, b + L.mu2, L.stride, j.total_rc,
                     (unsigned long long *)(b + L.keys), j.total_l, w.seg_prefix, w.seg_sweep, w.counters,
                     j.R, j.tiles, j.nseg, grid, o, j.total_l, ev[1], ev[2], st) != hipSuccess)
    return MP_ELAUNCH;
  if (g_timing.on) {
    if (ev[3]) (void)hipEventRecord(ev[3], st);
    g_timing.record(ev);
  }
  return MP_OK;
}

}  // extern "C"

namespace {

// Stream workspace: the FP64 state for l_max windows, then the workspace of
// the initial FP64 self-join of up to n_max samples.
struct StreamLayout {
  size_t mu, isd, flags, a, g, pd, c0, c1, pdp, pjp, col0, join, total;
};

StreamLayout stream_layout(int64_t n_max, int32_t m) {
  StreamLayout L{};
  const size_t lm = (size_t)(n_max - m + 1), np = (size_t)mpx::stream_partials((int64_t)lm);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.mu = take(8 * lm);
  L.isd = take(8 * lm);
  L.flags = take(lm);
  L.a = take(8 * lm);
  L.g = take(8 * lm);
  L.pd = take(8 * lm);
  L.c0 = take(8 * lm);
  L.c1 = take(8 * lm);
  L.pdp = take(8 * np);
  L.pjp = take(8 * np);
  L.col0 = take(8 * lm);
  L.join = o;
  mp_options f64opt{MP_PREC_F64, 0, 0, (int32_t)MP_FLAG_FP64_FINALIZE};
  Job j;
  if (build_selfjoin(n_max, m, 0, MP_F64, &f64opt, j) == MP_OK) o += layout_of(j, false).total;
  L.total = align_up(o);
  return L;
}

mpx::StreamWork stream_work(const StreamLayout &L, void *ws) {
  char *b = (char *)ws;
  mpx::StreamWork s{};
  s.mu = (double *)(b + L.mu);
  s.isd = (double *)(b + L.isd);
  s.flags = (uint8_t *)(b + L.flags);
  s.a = (double *)(b + L.a);
  s.g = (double *)(b + L.g);
  s.Pd = (double *)(b + L.pd);
  s.C[0] = (double *)(b + L.c0);
  s.C[1] = (double *)(b + L.c1);
  s.part_d = (double *)(b + L.pdp);
  s.part_j = (int64_t *)(b + L.pjp);
  s.col0 = (double *)(b + L.col0);
  return s;
}

constexpr int kStreamReseed = 1024;

}  // namespace

extern "C" {

size_t mp_stream_workspace(int64_t n_max, int32_t m) {
  if (m < 2 || n_max < m || n_max - m + 1 >= ((int64_t)1 << 31)) return 0;
  return stream_layout(n_max, m).total;
}

mp_status mp_stream_init(const void *T, int64_t n, int64_t n_max, int32_t m, int32_t ez, mp_dtype dtype,
                         void *P, int64_t *I, void *ws, size_t ws_bytes, void *stream) {
  if (dtype != MP_F64 && dtype != MP_F32) return MP_EINVAL;
  if (m < 2 || ez < 0 || n < m || n > n_max || n_max - m + 1 >= ((int64_t)1 << 31)) return MP_EINVAL;
  const size_t es = esize(dtype);
  if (!T || !P || !I || !aligned(T, es) || !aligned(P, es) || !aligned(I, 8)) return MP_EINVAL;
  const StreamLayout L = stream_layout(n_max, m);
  mp_status s = check_ws(ws, ws_bytes, L.total);
  if (s != MP_OK) return s;
  // the initial profile: the FP64 self-join of the first n samples
  mp_options f64opt{MP_PREC_F64, 0, 0, (int32_t)MP_FLAG_FP64_FINALIZE};
  Job j;
  if ((s = build_selfjoin(n, m, ez, dtype, &f64opt, j)) != MP_OK) return s;
  const Layout JL = layout_of(j, false);
  if (L.join + JL.total > L.total) return MP_EWORKSPACE;
  void *jws = (char *)ws + L.join;
  const mpx::Work w = work_of(JL, jws);
  const mpx::Plan p = plan_of(j, JL, jws, false);
  mpx::Outputs o{};
  o.P[0] = P;
  o.I[0] = I;
  hipStream_t st = (hipStream_t)stream;
  if ((s = run_job(j, p, w, T, o, dtype == MP_F64, st)) != MP_OK) return s;
  if (mpx::launch_stream_init(stream_work(L, ws), T, dtype == MP_F64, n, m, ez, I, st) != hipSuccess)
    return MP_ELAUNCH;
  return MP_OK;
}

mp_status mp_stream_append(const void *T, int64_t n_old, int64_t n_new, int64_t n_max, int32_t m, int32_t ez,
                           mp_dtype dtype, void *P, int64_t *I, void *ws, size_t ws_bytes, void *stream) {
  if (dtype != MP_F64 && dtype != MP_F32) return MP_EINVAL;
  if (m < 2 || ez < 0 || n_old < m || n_new < n_old || n_new > n_max ||
      n_max - m + 1 >= ((int64_t)1 << 31))
    return MP_EINVAL;
  const size_t es = esize(dtype);
  if (!T || !P || !I || !aligned(T, es) || !aligned(P, es) || !aligned(I, 8)) return MP_EINVAL;
  const StreamLayout L = stream_layout(n_max, m);
  mp_status s = check_ws(ws, ws_bytes, L.total);
  if (s != MP_OK) return s;
  if (n_new == n_old) return MP_OK;
  hipStream_t st = (hipStream_t)stream;
  const mpx::StreamWork sw = stream_work(L, ws);
  if (mpx::launch_stream_append(sw, T, dtype == MP_F64, n_old, n_new, m, ez, kStreamReseed, I, st) !=
      hipSuccess)
    return MP_ELAUNCH;
  if (mpx::launch_stream_out(sw, n_new - m + 1, m, P, dtype == MP_F64, st) != hipSuccess) return MP_ELAUNCH;
  return MP_OK;
}

int64_t mp_mdjoin_cells(int32_t D, int64_t nA, int64_t nB, int32_t m, int32_t ez) {
  if (D < 1 || m < 2 || nA < m) return 0;
  if (nB <= 0) return ez < 0 ? 0 : mp_selfjoin_cells(nA, m, ez);
  return nB < m ? 0 : mp_abjoin_cells(nA, nB, m);
}

size_t mp_fluss_workspace(int64_t l) {
  if (l < 1 || l >= ((int64_t)1 << 31)) return 0;
  return align_up(8 * mpx::fluss_scratch_words(l));
}

mp_status mp_fluss(const int64_t *I, int64_t l, int64_t zone, int32_t k, double *cac, int64_t *segments,
                   void *ws, size_t ws_bytes, void *stream) {
  if (l < 1 || l >= ((int64_t)1 << 31) || zone < 0 || k < 0 || k > 64) return MP_EINVAL;
  if (!I || !cac || !aligned(I, 8) || !aligned(cac, 8)) return MP_EINVAL;
  if (k > 0 && (!segments || !aligned(segments, 8))) return MP_EINVAL;
  mp_status s = check_ws(ws, ws_bytes, mp_fluss_workspace(l));
  if (s != MP_OK) return s;
  if (mpx::launch_fluss(I, l, zone, k, cac, segments, (int64_t *)ws, (hipStream_t)stream) != hipSuccess)
    return MP_ELAUNCH;
  return MP_OK;
}

size_t mp_chains_workspace(int64_t l) {
  if (l < 1 || l >= ((int64_t)1 << 31)) return 0;
  return align_up(8 * mpx::chains_scratch_words(l));
}

mp_status mp_chains(const int64_t *IL, const int64_t *IR, int64_t l, int32_t min_len, int64_t *next,
                    int64_t *length, int64_t *summary, int64_t *best, void *ws, size_t ws_bytes,
                    void *stream) {
  if (l < 1 || l >= ((int64_t)1 << 31) || min_len < 1) return MP_EINVAL;
  const void *ptrs[] = {IL, IR, next, length, summary, best};
  for (const void *q : ptrs)
    if (!q || !aligned(q, 8)) return MP_EINVAL;
  mp_status s = check_ws(ws, ws_bytes, mp_chains_workspace(l));
  if (s != MP_OK) return s;
  if (mpx::launch_chains(IL, IR, l, min_len, next, length, summary, best, (int64_t *)ws,
                         (hipStream_t)stream) != hipSuccess)
    return MP_ELAUNCH;
  return MP_OK;
}

size_t mp_recheck_workspace(int64_t n, int32_t m) {
  if (m < 2 || n < m) return 0;
  return align_up(mpx::recheck_state_bytes());
}

mp_status mp_recheck(const void *T, int64_t n, int32_t m, mp_dtype dtype, const void *P,
                     const int64_t *I, int32_t k_motifs, int32_t k_discords, int64_t *out_idx,
                     double *out_dist, void *ws, size_t ws_bytes, void *stream) {
  if (dtype != MP_F64 && dtype != MP_F32) return MP_EINVAL;
  if (m < 2 || n < m || k_motifs < 0 || k_discords < 0 || k_motifs > 64 || k_discords > 64)
    return MP_EINVAL;
  if (!T || !P || !I || !out_idx || !out_dist) return MP_EINVAL;
  const size_t es = esize(dtype);
  if (!aligned(T, es) || !aligned(P, es) || !aligned(I, 8) || !aligned(out_idx, 8) ||
      !aligned(out_dist, 8))
    return MP_EINVAL;
  mp_status s = check_ws(ws, ws_bytes, mp_recheck_workspace(n, m));
  if (s != MP_OK) return s;
  if (k_motifs + k_discords == 0) return MP_OK;
  if (mpx::launch_recheck(T, dtype == MP_F64, n, m, P, dtype == MP_F64, I, k_motifs, k_discords,
                          out_idx, out_dist, (uint8_t *)ws, (hipStream_t)stream) != hipSuccess)
    return MP_ELAUNCH;
  return MP_OK;
}

}  // extern "C"
