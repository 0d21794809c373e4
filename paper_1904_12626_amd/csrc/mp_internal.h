// Internal declarations shared by the HIP translation units of libmpx.
// Nothing here is part of the public ABI (include/mp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mpx {

constexpr int kWave = 64;
// Padding (in windows) after every series' row/column data so that the
// sweep's look-ahead loads past the last window stay inside the buffer.
constexpr int64_t kRcPad = 64 * 16 + 128;
// Keys >= this value mean "no admissible neighbour".  Valid keys are
// 1 - rho in [0, 2] (plus rounding); invalid rows carry 4.
constexpr double kKeyInvalid = 3.0;

// One series as the kernels see it.  Offsets index the caller's T array and
// the concatenated per-window workspace arrays.
struct SeriesDesc {
  int64_t t_off;   // first element in the T base array
  int64_t n;       // series length
  int64_t l;       // windows, n - m + 1
  int64_t w_off;   // first window in mu/sig/flags/keys/P/I and rescan ids
  int64_t rc_off;  // first entry in the padded row/column data array
  int64_t x_off;   // first entry in next_const/next_valid (l + 1 entries)
  int64_t p_off;   // output position of window 0 within its output slot
  int32_t m;
  int32_t ez;       // >= 0: self-join zone; -1: AB side (no zone)
  int32_t partner;  // series whose windows are this series' candidates
  int32_t out;      // output slot: 0 (single array) or the AB side (0/1)
  int32_t side;     // self-join candidates: 0 both sides, kSideRight j > i, kSideLeft j < i
  int32_t tsel;     // samples in the call's T array (0) or in its second array (1, Plan::t2)
};
constexpr int32_t kSideRight = 1;
constexpr int32_t kSideLeft = 2;

// One diagonal sweep: rows from series rs, columns from series cs,
// diagonals k = j - i in [k_lo, k_hi].  Row minima go to the keys of
// series rk, column minima to the keys of series ck.
struct SweepDesc {
  int32_t rs, cs, rk, ck;
  int64_t k_lo, k_hi;
  int64_t seg_base;  // first strip (segment) of this sweep in the tile table
  int64_t nseg;      // strips
  int32_t idx_bits;  // low bits of a packed key that hold the index
  int32_t pad_;
};

// Everything the kernels need to find a series / sweep.  Passed by value;
// up to two descriptors travel inline, a batch keeps them in the workspace.
struct Plan {
  int32_t nseries, nsweeps;
  SeriesDesc s_inl[2];
  SweepDesc w_inl[2];
  const SeriesDesc *s_ext;
  const SweepDesc *w_ext;
  // Optional restriction of self-join candidates to a set of diagonal
  // chunks: chunk c holds the offsets |j - i| in
  // [ez + 1 + c * kchunk, ez + (c + 1) * kchunk]; bit c of kmask set = chunk
  // in the set.  Null = every admissible offset.
  const uint32_t *kmask;
  int64_t kchunk;
  // Second sample array of a call given two series as separate allocations
  // (the AB-joins): series with tsel = 1 index it with their t_off.
  const void *t2;

  __device__ __forceinline__ SeriesDesc series(int i) const { return s_ext ? s_ext[i] : s_inl[i]; }
  __device__ __forceinline__ SweepDesc sweep(int i) const { return w_ext ? w_ext[i] : w_inl[i]; }
};

// First sample of series S: in the call's sample array Tb, or in the second
// array of a two-array call.
template <typename Tin>
__device__ __forceinline__ const Tin *series_samples(const Plan &plan, const Tin *Tb, const SeriesDesc &S) {
  return (S.tsel ? static_cast<const Tin *>(plan.t2) : Tb) + S.t_off;
}

// Workspace arrays (device).
struct Work {
  double *mu;          // [total_l] window mean (FP64)
  double *sig;         // [total_l] window population std (FP64)
  uint64_t *keys;      // [total_l] packed (key, index) minima
  uint8_t *flags;      // [total_l] bit0 valid, bit1 constant
  int32_t *next_const; // [total_x] smallest constant window >= x (l if none)
  int32_t *next_valid; // [total_x] smallest valid window >= x (l if none)
  void *rc;            // [total_rc] row/column data {a, g, s, u} (F4)
  int32_t *special;    // [nseries] bit0 has invalid windows, bit1 has constant
  double *scale;       // [nseries] power of two the series' sweep records carry
  unsigned long long *counters;  // [4]: 0 tile counter, 1 rescan count
  int64_t *seg_prefix; // [nseg + 1] first tile of each strip; with seg_part,
                       // the full-height tiles before each strip
  int32_t *seg_sweep;  // [nseg] sweep of each strip
  int64_t *seg_part;   // [nseg + 1] strips with a shorter last tile before each
                       // strip (those tiles are numbered after every full
                       // one), or null: all tiles in strip order
  int64_t *rescan;     // [total_l] windows needing an exact row scan
};

// Backward workspace (batch plans).  The gradient of one row i -> j is a
// multiple of z_i plus a multiple of z_j on window i, and the same on window
// j.  Per window w: the multiples of its own z (its row's alpha and the
// gammas of the rows naming w as neighbour) are summed into one coefficient
// (`wsc`), and its row's multiple of z_j is the window's own edge (`wrec`).  The multiple of z_i that a row puts on its
// neighbour j is a bucket edge of j (`erec`): coefficient, source mean,
// source offset and destination.  Bucket edges are grouped by destination
// window (CSR `off`), in increasing row order.
struct BwdEdge {
  double c;      // coefficient on (x[t + delta] - mu)
  double mu;     // mean of the source window
  int64_t delta; // source window start - destination window start (samples)
  int64_t dest;  // destination window (global index)
};
struct BwdWin {
  double mu;     // mean of this window
  double oc;     // own edge: coefficient on (x[t + odelta] - omu), 0 if none
  double omu;    // own edge: mean of the neighbour window
  int64_t odelta;// own edge: neighbour start - window start (samples)
};
struct BwdWork {
  double *mu;          // [total_l] window mean
  double *isig;        // [total_l] 1/sigma, 0 for constant or non-finite windows
  int64_t *nbr;        // [total_l] neighbour window (global), -1 if the row contributes nothing
  BwdWin *wrec;        // [total_l] window records
  double *alpha;       // [total_l] per row: its multiple of its own window's z
  double *wsc;         // [total_l] per window: alpha plus its bucket's gammas, times 1/sigma
  BwdEdge *bedge;      // [total_l] per row: its bucket edge on the neighbour window
  double *bgam;        // [total_l] per row: its multiple of the neighbour's z (gamma)
  uint32_t *bpos;      // [total_l] per row: its position in the neighbour's bucket (arrival order)
  unsigned long long *count;  // [total_l] bucket rows per window
  int64_t *off;        // [total_l + 1] bucket offsets (exclusive prefix of count)
  int64_t *tmp;        // [total_l] bucket rows in arrival order (edge slots)
  BwdEdge *erec;       // [total_l] bucket edges in CSR order
  double *egam;        // [total_l] gamma of each bucket edge, same order
  int64_t *chunk;      // [ceil(total_l / 1024) + 1] scan partials
  int64_t *big;        // [total_l / kBwdSmallBucket + 1] buckets with more than kBwdSmallBucket rows
  unsigned long long *nbig;  // [1] entries of `big`
  // the forward's window statistics in the same workspace (mean, sigma,
  // flags bit0 valid / bit1 constant), read by the backward that follows it
  const double *fmu;
  const double *fsig;
  const uint8_t *fflags;
};
// Buckets of at most this many rows are ordered by a per-row count; larger
// ones (hub windows named by many rows) are sorted by one workgroup each.
constexpr int64_t kBwdSmallBucket = 64;

struct Outputs {
  void *P[2];
  int64_t *I[2];
};

// ------------------------------------------------------------- launchers
hipError_t launch_plan(const Plan &plan, const Work &w, const void *T, bool t_f64, int W, int R, int64_t nseg,
                       hipStream_t st);
hipError_t launch_stats(const Plan &plan, const Work &w, const void *T, bool t_f64, bool f64_sweep,
                        int64_t total_rc, hipStream_t st);
hipError_t launch_sweep(const Plan &plan, const Work &w, const void *T, bool t_f64, bool f64_sweep,
                        int slots, int R, int64_t total_tiles, int64_t nseg, int grid,
                        hipStream_t st);
hipError_t launch_special(const Plan &plan, const Work &w, hipStream_t st);
// kappa: rows whose key is below it are queued for the exact rescan (0: none)
hipError_t launch_finalize(const Plan &plan, const Work &w, const void *T, bool t_f64,
                           const Outputs &o, bool out_f64, bool fp64_finalize, double kappa,
                           int64_t total_l, hipStream_t st);
hipError_t launch_rescan(const Plan &plan, const Work &w, const void *T, bool t_f64,
                         const Outputs &o, bool out_f64, bool fp64_finalize, hipStream_t st);
hipError_t launch_lr_combine(const Outputs &o, bool out_f64, int64_t l, hipStream_t st);
hipError_t launch_recheck(const void *T, bool t_f64, int64_t n, int32_t m, const void *P,
                          bool p_f64, const int64_t *I, int32_t km, int32_t kd, int64_t *out_idx,
                          double *out_dist, uint8_t *ws, hipStream_t st);
size_t recheck_state_bytes();
// flat_loads: the gather reads samples with flat loads even where buffer
// loads apply (sample arrays under 2 GiB)
hipError_t launch_backward(const Plan &plan, const BwdWork &b, const void *T, bool t_f64,
                           const int64_t *I, const void *gP, void *gT, int64_t total_l,
                           int64_t total_n, bool flat_loads, hipStream_t st);
// The backward right after the forward on the same workspace and samples:
// window statistics from the forward (b.fmu / b.fsig / b.fflags), each
// row's distance from the forward's FP64-finalized profile P (P's dtype is
// the samples' dtype).
hipError_t launch_backward_after_forward(const Plan &plan, const BwdWork &b, const void *T, bool t_f64,
                                         const int64_t *I, const void *P, const void *gP, void *gT,
                                         int64_t total_l, int64_t total_n, bool flat_loads, hipStream_t st);

// Exclusive prefix sum: out[0..n] (out[n] = total) of in[0..n); `partial`
// holds ceil(n / 1024) + 1 entries of scratch.
hipError_t launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t *partial, int64_t n,
                                 hipStream_t st);

// Semantic segmentation and chains over a profile index (mp_mine.hip).
size_t fluss_scratch_words(int64_t l);
hipError_t launch_fluss(const int64_t *I, int64_t l, int64_t zone, int k, double *cac, int64_t *segments,
                        int64_t *ws, hipStream_t st);
size_t chains_scratch_words(int64_t l);
hipError_t launch_chains(const int64_t *IL, const int64_t *IR, int64_t l, int64_t min_len, int64_t *next,
                         int64_t *length, int64_t *summary, int64_t *best, int64_t *ws, hipStream_t st);

// Multidimensional joins (mp_md.hip): SiMPle (non-normalised, summed over
// dimensions, one profile) and the multidimensional profiles (one per k).
constexpr int kMdSimple = 0;
constexpr int kMdMulti = 1;
constexpr int kMdMaxDims = 8;
hipError_t launch_md(int mode, int D, const Plan &plan, const void *T, bool t_f64, void *rec, void *mu2,
                     int64_t stride, int64_t total_rc, unsigned long long *keys, int64_t kstride,
                     const int64_t *seg_prefix, const int32_t *seg_sweep, unsigned long long *counter, int R,
                     int64_t total_tiles, int64_t nseg, int grid, const Outputs &o, int64_t total_l,
                     hipEvent_t ev0, hipEvent_t ev1, hipStream_t st);
int md_sweep_grid(int mode, int D);
// Diagonals per strip of the multidimensional sweep (64 times its slots).
int md_strip_width(int mode, int D);

// Incremental self-join state (mp_stream.hip), sized for l_max windows.
struct StreamWork {
  double *mu;        // [l_max] window mean
  double *isd;       // [l_max] 1/(sqrt(m) sigma), 0 for constant or invalid windows
  uint8_t *flags;    // [l_max] bit0 valid, bit1 constant
  double *a, *g;     // [l_max] recurrence terms (a needs the window's successor sample)
  double *Pd;        // [l_max] FP64 profile as keys d^2 / (2m)
  double *C[2];      // [l_max] cross products of the newest window (window w in C[w % 2])
  double *part_d;    // per-wave row minima of a batch
  int64_t *part_j;
  double *col0;      // [l_max] C(w, 0) of the appended windows
};
int64_t stream_partials(int64_t l_max);
hipError_t launch_stream_init(const StreamWork &s, const void *T, bool t_f64, int64_t n, int m, int ez,
                              const int64_t *I, hipStream_t st);
hipError_t launch_stream_append(const StreamWork &s, const void *T, bool t_f64, int64_t n_old, int64_t n_new,
                                int m, int ez, int reseed, int64_t *I, hipStream_t st);
hipError_t launch_stream_out(const StreamWork &s, int64_t l, int m, void *P, bool out_f64, hipStream_t st);

// Occupancy-derived persistent grid for the sweep kernel.
int sweep_grid(bool f64_sweep, int slots);

}  // namespace mpx
