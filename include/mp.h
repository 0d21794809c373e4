/*
 * mp.h -- C ABI of the MI355X matrix-profile similarity-join library
 * (libmpx.so, HIP kernels for gfx950).
 *
 * The operation (tsmp paper, arXiv 1904.12626):
 *   Section 2  -- the matrix profile P of a sliding-window join is, for every
 *                 length-m window, the Euclidean distance to its nearest
 *                 neighbour; the profile index I holds that neighbour's
 *                 position (the row minimum of the distance matrix,
 *                 excluding trivial matches).
 *   Section 3.3.4 -- windows are z-normalised (SiMPle is the one mode that
 *                 is not).
 *   Section 3.2 -- one series gives a self-join, two give an AB-join; the
 *                 exclusion zone suppresses trivial matches in self-joins.
 *   Section 3.3.2 -- the dot products of one row are reused for the next
 *                 (STOMP), so every cell costs O(1); Section 3.3.3 (SCRIMP)
 *                 processes the distance matrix in an order independent of
 *                 rows; Section 3.2 states that these orders give equal
 *                 results.
 *
 * Conventions shared by every entry point
 *   - Windows: T_i = T[i .. i+m-1], i = 0 .. l-1 with l = n - m + 1.
 *   - z-normalisation uses the population standard deviation; a window whose
 *     m values are all equal normalises to the zero vector (so its distance to
 *     any other valid window is sqrt(m), and 0 to another constant window).
 *   - A window holding a NaN or +-Inf is invalid: its P is +inf, its I is -1,
 *     and it is never chosen as a neighbour.  A row with no admissible
 *     neighbour also gets (+inf, -1).  These are results, not errors.
 *   - P holds distances (not squared distances); I is 0-based and local to
 *     its series.  Equal distances go to the smallest index when the tied
 *     pairs lie in different tiles of the sweep (tile_slots x 64 diagonal
 *     offsets by reseed_rows rows); inside one tile either index may be
 *     returned.  "Equal" is at the resolution of the sweep's keys (FP32:
 *     13 significant bits of 1 - rho; FP64: 43).
 *   - Self-join: pairs with |i - j| <= ez are excluded.  AB-join: no zone.
 *
 * Memory and streams
 *   - Every array argument (T, P, I, gP, gT, workspace, offsets passed to
 *     mp_batch) is DEVICE memory owned by the caller, except where a comment
 *     says "host".  The library never allocates device memory, never frees,
 *     and never synchronises: all work is enqueued on `stream` (a
 *     hipStream_t; NULL = the legacy default stream) and the call returns at
 *     once.  Results are valid once the stream reaches that point.
 *   - The workspace must be at least the size the matching *_workspace
 *     query returns and 256-byte aligned; its contents on entry do not matter
 *     and on exit are scratch.  Two calls that share a workspace must be
 *     ordered on one stream.
 *   - Every call except mp_batch_plan_upload enqueues kernels only (no
 *     memset, no copies), so it may be captured into a HIP graph.
 *
 * Errors
 *   - Argument checks run on the host before anything is enqueued; a
 *     failing check returns MP_EINVAL / MP_EWORKSPACE / MP_EUNSUPPORTED and
 *     enqueues nothing.  A failed kernel launch returns MP_ELAUNCH.  No
 *     function throws across the ABI.
 */
#ifndef MPX_MP_H
#define MPX_MP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MP_ABI_VERSION 1

typedef enum {
  MP_OK = 0,
  MP_EINVAL = -1,        /* bad size, pointer, alignment or option      */
  MP_EWORKSPACE = -2,    /* workspace null, misaligned or too small     */
  MP_ELAUNCH = -3,       /* a kernel launch failed                      */
  MP_EUNSUPPORTED = -4,  /* valid request the library does not support  */
  MP_ETOOLARGE = -5      /* job exceeds the fixed scratch of
                            mp_selfjoin_noalloc                         */
} mp_status;

typedef enum {
  MP_F64 = 0,            /* T (and gP, gT) are double; P is double      */
  MP_F32 = 1             /* T (and gP, gT) are float;  P is float       */
} mp_dtype;

/* precision of the diagonal sweep */
#define MP_PREC_F64 0    /* FP64 sweep (the reference GPU path)          */
#define MP_PREC_F32 1    /* FP32 sweep, FP64 stats/seeds, reseeded       */
/* The FP32 sweep carries cross products of windows in FP32; each series'
 * records are scaled by a power of two (2^-500 ... 2^500) chosen from its
 * samples, so any series whose squared window sums are finite in FP64
 * (|T| up to about 1e150) stays inside FP32's range (the keys are the same
 * as without the scaling). */

/* flags */
#define MP_FLAG_FP64_FINALIZE 1u  /* recompute P[i] = dist(i, I[i]) in FP64 */
#define MP_FLAG_FLAT_LOADS 2u     /* mp_backward: read samples with flat loads, as it
                                     does anyway for sample arrays of 2 GiB or more
                                     (same results; for comparisons)            */

typedef struct {
  int32_t precision;     /* MP_PREC_F64 or MP_PREC_F32                        */
  int32_t reseed_rows;   /* rows per tile = reseed interval, a multiple of 64
                            (rounded up to the sweep's flush period);
                            0 = automatic                                   */
  int32_t tile_slots;    /* diagonals per lane: 8, 12 or 16 (the FP64 sweep
                            supports 8); 0 = automatic (12 for the FP32
                            sweep, 8 for FP64)                               */
  int32_t flags;         /* MP_FLAG_*                                        */
} mp_options;

/* ---------------------------------------------------------------- self-join
 * Section 2 / 3.2: P[i] = min over |i-j| > ez of d(i, j), I[i] = argmin.
 *   T      device, n values of `dtype`
 *   m      window, 2 <= m <= n;  ez >= 0
 *   P      device, l = n-m+1 values of `dtype`;  I  device, l int64
 *   opt    host pointer, may be NULL (= all defaults: FP32 sweep, automatic
 *          tiling, FP64 finalize on)
 */
size_t mp_selfjoin_workspace(int64_t n, int32_t m, mp_dtype dtype, const mp_options *opt);
mp_status mp_selfjoin(const void *T, int64_t n, int32_t m, int32_t ez, mp_dtype dtype,
                      const mp_options *opt, void *P, int64_t *I, void *ws, size_t ws_bytes,
                      void *stream);

/* ------------------------------------------- self-join without allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * self-join of mp_selfjoin with the same arguments minus the workspace,
 * same kernels, bitwise the same P and I.  Its scratch is a fixed device
 * array of MP_NOALLOC_SCRATCH_BYTES inside the library, one per device,
 * held from the first call on a device until the process ends; the call
 * itself allocates and frees nothing (no hipMalloc, no events; timing is
 * never recorded for it).
 *   Limit: a job whose mp_selfjoin_workspace(n, m, dtype, opt) exceeds
 *   MP_NOALLOC_SCRATCH_BYTES returns MP_ETOOLARGE and enqueues nothing
 *   (64 MiB holds the FP32 sweep's workspace up to about 1.15 million
 *   windows, the FP64 sweep's up to about 0.87 million).
 *   Device: the scratch of the current device is used; a non-NULL stream
 *   must belong to that device (else MP_EINVAL).
 *   Sharing: every call on one device uses the same scratch.  Calls that
 *   overlap on one device (two streams, two host threads) race and give
 *   undefined results; order them on one stream.  The kernels initialise
 *   every scratch entry they read, so nothing needs clearing between calls.
 */
#define MP_NOALLOC_SCRATCH_BYTES (64u << 20)
mp_status mp_selfjoin_noalloc(const void *T, int64_t n, int32_t m, int32_t ez, mp_dtype dtype,
                              const mp_options *opt, void *P, int64_t *I, void *stream);

/* ----------------------------------------------------------------- AB-join
 * Section 3.2: two series.  P_ab[i] = min_j d(A_i, B_j) (index into B),
 * P_ba[j] = min_i d(A_i, B_j) (index into A).  No exclusion zone.
 *   A, B   device, nA / nB values;  P_ab, I_ab length nA-m+1;  P_ba, I_ba
 *   length nB-m+1.
 */
size_t mp_abjoin_workspace(int64_t nA, int64_t nB, int32_t m, mp_dtype dtype, const mp_options *opt);
mp_status mp_abjoin(const void *A, int64_t nA, const void *B, int64_t nB, int32_t m,
                    mp_dtype dtype, const mp_options *opt, void *P_ab, int64_t *I_ab,
                    void *P_ba, int64_t *I_ba, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ batched joins
 * Many self-joins of uneven lengths and windows in one launch sequence.
 * Series s occupies T_cat[t_off[s] .. t_off[s+1]-1]; its profile occupies
 * P_cat/I_cat[p_off[s] .. p_off[s] + l_s - 1] with p_off[s] = sum of l over
 * the series before it.  The plan is a host object built once from host
 * copies of the offsets, windows and zones; mp_batch_plan_upload writes its
 * device tables into the workspace (hipMemcpyAsync; call it before any
 * stream capture and keep the plan alive until that copy has completed);
 * mp_batch then only enqueues kernels and may be captured and replayed.
 */
typedef struct mp_batch_plan mp_batch_plan;
mp_status mp_batch_plan_create(int32_t nseries, const int64_t *t_off_host /* [nseries+1] */,
                               const int32_t *m_host /* [nseries] */,
                               const int32_t *ez_host /* [nseries] */, mp_dtype dtype,
                               const mp_options *opt, mp_batch_plan **out);
size_t mp_batch_plan_workspace(const mp_batch_plan *plan);
int64_t mp_batch_plan_profile_length(const mp_batch_plan *plan);  /* sum of l_s */
int64_t mp_batch_plan_cells(const mp_batch_plan *plan);           /* admissible pairs */
mp_status mp_batch_plan_upload(const mp_batch_plan *plan, void *ws, size_t ws_bytes, void *stream);
mp_status mp_batch(const mp_batch_plan *plan, const void *T_cat, void *P_cat, int64_t *I_cat,
                   void *ws, size_t ws_bytes, void *stream);
void mp_batch_plan_destroy(mp_batch_plan *plan);

/* -------------------------------------------------------- AB-join plans
 * The AB-join of Section 3.2 as a batch plan, so that it can be captured
 * and differentiated: T_cat = A (nA values) followed by B (nB values);
 * the plan's profile (mp_batch_plan_profile_length = lA + lB entries) is
 * P_ab (lA entries, indices into B) followed by P_ba (lB entries, indices
 * into A).  Run with mp_batch_plan_upload / mp_batch; mp_backward then
 * gives dL/dA followed by dL/dB from gP = [gP_ab | gP_ba].
 */
mp_status mp_abjoin_plan_create(int64_t nA, int64_t nB, int32_t m, mp_dtype dtype,
                                const mp_options *opt, mp_batch_plan **out);

/* ------------------------------------ partial and one-sided self-joins
 * Sections 3.3.1 and 3.3.3 (STAMP, SCRIMP): the profile can be computed in a
 * random order of its parts and read at any point as the best-so-far
 * profile; the s_size argument of Section 3.2 stops such a run in a
 * controlled way.  Here the parts are chunks of diagonal offsets: chunk c
 * holds the pairs with |i - j| in [ez + 1 + c*W, ez + (c+1)*W] (W and the
 * number of chunks from mp_selfjoin_chunks), and a plan restricted to a set
 * of chunks returns exactly
 *   P[i] = min over j with |i - j| in the set of d(i, j)
 * (the best-so-far profile once those chunks are done; the full set gives
 * the self-join, bitwise equal to mp_selfjoin with the same options).
 * Time series chains (Section 3.4.3) and the arc counts of semantic
 * segmentation (Section 3.4.2) work on the left and right profiles:
 * P_left[i] = min over j < i - ez, P_right[i] = min over j > i + ez.  One
 * sweep gives both (row minima look right, column minima look left).
 *   sides   MP_SIDES_BOTH: the plan's profile has l entries;
 *           MP_SIDES_LEFT_RIGHT: 3l entries [P | P_left | P_right] (I alike;
 *           P is the better of the two, the left one on equal distances).
 *   chunks  host, nchunks distinct chunk numbers in [0, count), any order;
 *           NULL = every chunk.  nchunks = 0 with a non-NULL pointer is the
 *           empty set (every P is +inf).
 * The plan is a batch plan of one series: size its workspace with
 * mp_batch_plan_workspace, upload it once with mp_batch_plan_upload and run
 * it with mp_batch (T_cat = T, P_cat/I_cat of mp_batch_plan_profile_length
 * entries).  mp_backward accepts MP_SIDES_BOTH plans (gradient of the
 * restricted profile) and returns MP_EUNSUPPORTED for left/right plans.
 * mp_selfjoin_chunks returns the number of chunks (0 if l <= ez + 1, -1 on
 * invalid arguments) and stores W in *chunk_width when it is not NULL.
 */
#define MP_SIDES_BOTH 0
#define MP_SIDES_LEFT_RIGHT 1
int64_t mp_selfjoin_chunks(int64_t n, int32_t m, int32_t ez, const mp_options *opt,
                           int64_t *chunk_width);
mp_status mp_selfjoin_plan_create(int64_t n, int32_t m, int32_t ez, mp_dtype dtype,
                                  const mp_options *opt, int32_t sides, int64_t nchunks,
                                  const int64_t *chunks_host, mp_batch_plan **out);
/* A uniformly random order of `count` chunk numbers (host array of count
 * int64, written): Fisher-Yates shuffle driven by SplitMix64 seeded with
 * `seed`.  An anytime run takes a prefix of it. */
mp_status mp_anytime_order(int64_t count, uint64_t seed, int64_t *order_host);

/* ---------------------------------------------------------------- backward
 * Gradient of a loss L(P) with respect to T through the z-normalised
 * distance of each row's argmin pair (j = I[i] in the same series for a
 * self-join plan, in the other series for an AB-join plan), holding I
 * fixed (not in the paper; the derivative of d(i, j) = ||z_i - z_j||
 * through z = (x - mean)/sigma):
 *   dd/dT[i:i+m] = (rho z_i - z_j) / (sigma_i d),
 *   dd/dT[j:j+m] = (rho z_j - z_i) / (sigma_j d),   rho = z_i.z_j / m.
 * Rows with I < 0 (or I outside the series), a zero or non-finite gP, d == 0,
 * or a constant or non-finite window on either side contribute nothing.
 * Accumulation is in FP64 without atomics on values: the same inputs give
 * bitwise the same gT.  Any I is accepted (hub neighbours included); the
 * cost is O(total_l * m) plus O(h log^2 h) for a neighbour window named by
 * h > 64 rows (their order is settled by a sort).
 * Uses the batch plan's layout: T_cat / I_cat / gP_cat as for mp_batch,
 * gT_cat (n values per series, `dtype`) is overwritten.  The workspace is
 * the plan's workspace; the backward writes only its own tables there (what
 * the last mp_batch left, P's window statistics, stays).
 * MP_EUNSUPPORTED for left/right plans and for windows longer than 2^30
 * samples; MP_EINVAL for null or misaligned pointers; MP_EWORKSPACE for a
 * workspace that is null, misaligned or smaller than the plan's; MP_ELAUNCH
 * when a kernel launch fails.
 */
mp_status mp_backward(const mp_batch_plan *plan, const void *T_cat, const int64_t *I_cat,
                      const void *gP_cat, void *gT_cat, void *ws, size_t ws_bytes,
                      void *stream);

/* The same gradient for a call that follows mp_batch on the same plan,
 * workspace and T_cat, with P_cat / I_cat that mp_batch wrote (a training
 * step: forward, then backward).  It reuses what the forward left in the
 * workspace instead of recomputing it: the window means and standard
 * deviations (the same two-pass FP64 values mp_backward computes), and
 * each row's distance d = P[i] (the forward's FP64 recompute of
 * d(i, I[i]), which mp_backward forms the same way), with
 * rho = 1 - d^2/(2m) in place of the dot product; no window is read.  The
 * result equals mp_backward's up to the rounding of rho (and, for float
 * data, of d stored in a float P).
 * Requires the plan's MP_FLAG_FP64_FINALIZE (else MP_EUNSUPPORTED) and
 * MP_SIDES_BOTH.  The caller guarantees that no other mp_batch ran on this
 * workspace since the one that produced P_cat, and that T_cat is unchanged;
 * the library cannot check either.  Same layouts, ownership, errors and
 * determinism as mp_backward (it too writes only the backward tables).
 */
mp_status mp_backward_after_forward(const mp_batch_plan *plan, const void *T_cat, const int64_t *I_cat,
                                    const void *P_cat, const void *gP_cat, void *gT_cat, void *ws,
                                    size_t ws_bytes, void *stream);

/* ------------------------------------------------- multidimensional joins
 * A series with D dimensions sampled together (1 <= D <= 8), stored
 * dimension-major: dimension d of a series of n samples occupies
 * [d*n, (d+1)*n) of its array.  A window is invalid (P = +inf, I = -1,
 * never a neighbour) when any dimension holds a non-finite value in it.
 *   MP_MD_SIMPLE  Section 3.3.4 (SiMPle): no z-normalisation, the distance
 *                 summed over every dimension,
 *                   d(i, j) = sqrt( sum_d ||A^d_i - B^d_j||^2 );
 *                 self-join (B = NULL, pairs with |i - j| <= ez excluded)
 *                 or AB-join (both directions, as mp_abjoin).
 *   MP_MD_MULTI   Section 3.3.5 (multidimensional profiles, mSTOMP): per
 *                 pair the z-normalised distance of each dimension, sorted
 *                 ascending; the k-dimensional distance is the mean of the
 *                 k smallest; P holds D profiles, k = 1 .. D, profile k at
 *                 [(k-1)*l, k*l) (I alike).  Self-join only (the paper
 *                 designs it for self-joins): MP_EUNSUPPORTED otherwise.
 * Arithmetic: FP64 centred cross products and statistics; the candidate
 * values that pick each minimum are rounded to float, and P is then
 * recomputed in FP64 from the chosen pair (so P is exact for I; I can differ
 * from the exact argmin only at near-ties within float resolution).
 *   A, B   device, D*nA and D*nB values of `dtype`;  P, I, P_ba, I_ba as
 *          above (P_ba / I_ba only for the AB-join)
 *   ws     device scratch of mp_mdjoin_workspace(mode, D, nA, nB, m) bytes
 *          (nB = 0 for a self-join)
 * Enqueues kernels only.
 */
#define MP_MD_SIMPLE 0
#define MP_MD_MULTI 1
size_t mp_mdjoin_workspace(int32_t mode, int32_t D, int64_t nA, int64_t nB, int32_t m);
mp_status mp_mdjoin(int32_t mode, int32_t D, const void *A, int64_t nA, const void *B, int64_t nB,
                    int32_t m, int32_t ez, mp_dtype dtype, void *P, int64_t *I, void *P_ba,
                    int64_t *I_ba, void *ws, size_t ws_bytes, void *stream);
/* pairs a multidimensional join scores (nB = 0: self-join with zone ez) */
int64_t mp_mdjoin_cells(int32_t D, int64_t nA, int64_t nB, int32_t m, int32_t ez);

/* ---------------------------------------------------------------- streaming
 * Section 2: once computed, the join can be updated incrementally, so an
 * exact join can be kept on streaming data (the paper gives no algorithm).
 * The caller keeps a growing series in T (capacity n_max samples) and the
 * profile in P, I (capacity n_max - m + 1 entries); the library keeps FP64
 * state in the workspace.  mp_stream_init computes the self-join of the
 * first n samples (the FP64 sweep) and the state.  After the caller has
 * written samples n_old .. n_new-1 into T (ordered before the call on
 * `stream`), mp_stream_append extends P, I to the n_new - m + 1 windows so
 * that they equal the self-join of T[0, n_new): each new window gets its
 * nearest admissible earlier window, and every earlier window whose new
 * candidate is strictly closer takes it (on equal distances the older,
 * smaller index stays).  FP64: the cross products of each new window
 * continue those of its predecessor along every diagonal (O(l) per window,
 * re-seeded by direct dot products every 1024 windows); new windows are
 * processed up to min(63, ez + 1) per launch.  m, ez, n_max and the
 * workspace must stay the same for the life of the stream; nothing else may
 * write the workspace.
 *   ws   device scratch of mp_stream_workspace(n_max, m) bytes
 */
size_t mp_stream_workspace(int64_t n_max, int32_t m);
mp_status mp_stream_init(const void *T, int64_t n, int64_t n_max, int32_t m, int32_t ez,
                         mp_dtype dtype, void *P, int64_t *I, void *ws, size_t ws_bytes,
                         void *stream);
mp_status mp_stream_append(const void *T, int64_t n_old, int64_t n_new, int64_t n_max, int32_t m,
                           int32_t ez, mp_dtype dtype, void *P, int64_t *I, void *ws,
                           size_t ws_bytes, void *stream);

/* ------------------------------------------------- semantic segmentation
 * Section 3.4.2 (FLUSS, after Gharghabi et al. 2017): every window i and its
 * neighbour I[i] form an arc; the arc curve AC[x] counts the arcs with
 * min(i, I[i]) <= x < max(i, I[i]).  Few arcs cross a regime change.  The
 * corrected arc curve divides by 2x(l - x)/l, the count that arcs to
 * uniformly random positions give, and caps at 1:
 *   cac[x] = min(AC[x] / (2x(l - x)/l), 1),  cac[x] = 1 within `zone` of
 *   either end (edge effect).
 * Segment boundaries: k times the smallest cac (smallest index on ties)
 * outside the edges and farther than `zone` from every earlier boundary;
 * -1 once no position is left.
 *   I         device int64[l], a profile index (entries < 0 or >= l and
 *             I[i] == i draw no arc)
 *   zone      >= 0 (the Python layer uses 5 m);  0 <= k <= 64
 *   cac       device double[l], written;  segments  device int64[k]
 *             (may be NULL when k == 0)
 *   ws        device scratch of mp_fluss_workspace(l) bytes
 * Arc counts are integer atomics plus a prefix sum: exact and
 * deterministic.  Enqueues kernels only.
 */
size_t mp_fluss_workspace(int64_t l);
mp_status mp_fluss(const int64_t *I, int64_t l, int64_t zone, int32_t k, double *cac,
                   int64_t *segments, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ chains
 * Section 3.4.3 (time series chains, after Zhu et al. 2018): from the left
 * and right profile indices (mp_selfjoin_plan_create with
 * MP_SIDES_LEFT_RIGHT), window i links forward to j = IR[i] when the link
 * is confirmed backwards, IL[j] == i.  Confirmed links form disjoint
 * increasing paths, the chains; every window lies on exactly one.
 *   IL, IR   device int64[l] (-1 = none)
 *   next     device int64[l], written: the confirmed successor or -1
 *   length   device int64[l], written: windows from i to its chain's end
 *   summary  device int64[3], written: number of chains (counted at their
 *            first window) with at least min_len windows; first window of
 *            the longest chain (the smallest one on equal lengths); its
 *            length
 *   best     device int64[l]: its first `length` entries receive the
 *            longest chain's windows in order; the rest is left as is
 *   ws       device scratch of mp_chains_workspace(l) bytes
 * Lengths by pointer jumping (ceil(log2 l) rounds); integer work only,
 * deterministic.  Enqueues kernels only.
 */
size_t mp_chains_workspace(int64_t l);
mp_status mp_chains(const int64_t *IL, const int64_t *IR, int64_t l, int32_t min_len,
                    int64_t *next, int64_t *length, int64_t *summary, int64_t *best, void *ws,
                    size_t ws_bytes, void *stream);

/* ----------------------------------------------------------- FP64 recheck
 * Section 2: the lowest points of P are the best motif pair, the highest
 * point is the discord.  Extracts k_motifs motif pairs (repeatedly the
 * smallest finite P[i] with its pair (i, I[i]), then every index within m of
 * either member is masked) and k_discords discords (repeatedly the largest
 * finite P, masking within m), and recomputes their distances in FP64 from
 * T.  One launch per pick; meant for small k (<= 64 each).
 *   T        device, n values of `dtype`; P, I device, l values (a profile
 *            this library produced for T with window m)
 *   out_idx  device int64[2*k_motifs + k_discords]: motif pairs (i, j) first,
 *            then discord positions; -1 where fewer exist
 *   out_dist device double[k_motifs + k_discords]: FP64 distance of each
 *            motif pair, then of each discord to its neighbour I; +inf where
 *            fewer exist
 *   ws       device scratch of mp_recheck_workspace(n, m) bytes (a few KB)
 */
size_t mp_recheck_workspace(int64_t n, int32_t m);
mp_status mp_recheck(const void *T, int64_t n, int32_t m, mp_dtype dtype, const void *P,
                     const int64_t *I, int32_t k_motifs, int32_t k_discords, int64_t *out_idx,
                     double *out_dist, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ timing
 * Kernel timing for benchmarks.  While enabled, every mp_selfjoin, mp_abjoin
 * and mp_batch call also records HIP events on its stream around the sweep
 * kernel and around its whole launch sequence.  mp_timing_query waits for
 * the recorded events, returns the summed durations (milliseconds) and the
 * number of calls since the last query, then clears the record.  Host-side
 * state of the process; not for use under stream capture.
 */
mp_status mp_timing_enable(int enable);
mp_status mp_timing_query(double *sweep_ms, double *total_ms, int64_t *calls);

/* --------------------------------------------------------------- helpers */
const char *mp_strerror(mp_status status);
int mp_abi_version(void);
/* Cells (admissible pairs) of a self-join / AB-join, for throughput metrics. */
int64_t mp_selfjoin_cells(int64_t n, int32_t m, int32_t ez);
int64_t mp_abjoin_cells(int64_t nA, int64_t nB, int32_t m);

#ifdef __cplusplus
}
#endif
#endif /* MPX_MP_H */
