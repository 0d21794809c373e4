/*
 * Plain FP64 brute-force matrix-profile oracle in C + OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY: it is loaded by tests/, the smoke check and the
 * CPU-baseline leg of bench.py.  The product library never links or calls it
 * and shares nothing with it.
 *
 * It computes the same definitions as mp_oracle.py (the matrix profile is the
 * row-wise minimum non-trivial entry of the z-normalised Euclidean distance
 * matrix, tsmp paper Section 2; z-normalisation per Section 3.3.4; exclusion
 * zone for self-joins per Section 3.2), in the direct difference form
 *     d(i, j) = sqrt( sum_u ( (A[i+u]-mu_i)/sig_i - (B[j+u]-mu_j)/sig_j )^2 )
 * with a fixed left-to-right summation order, and a strict '<' scan over j
 * (ties to the smallest index).  Constant windows normalise to the zero
 * vector; windows with a non-finite value are invalid (P = +inf, I = -1) and
 * never a neighbour.  One OpenMP thread handles one requested row at a time.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Two-pass mean / population std of every window; flags: 1 = valid,
 * 2 = constant (all values equal). */
void mpo_window_stats(const double *T, int64_t n, int32_t m, double *mu,
                      double *sig, int8_t *flags) {
  int64_t l = n - m + 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < l; i++) {
    const double *w = T + i;
    int ok = 1;
    double lo = w[0], hi = w[0], s = 0.0;
    for (int32_t u = 0; u < m; u++) {
      if (!isfinite(w[u])) ok = 0;
      if (w[u] < lo) lo = w[u];
      if (w[u] > hi) hi = w[u];
      s += w[u];
    }
    if (!ok) {
      mu[i] = NAN;
      sig[i] = NAN;
      flags[i] = 0;
      continue;
    }
    double mean = s / m, v = 0.0;
    for (int32_t u = 0; u < m; u++) {
      double dv = w[u] - mean;
      v += dv * dv;
    }
    mu[i] = mean;
    sig[i] = sqrt(v / m);
    flags[i] = (int8_t)(1 | (lo == hi ? 2 : 0));
  }
}

static void znorm_window(const double *w, int32_t m, double mu, double sig,
                         int8_t flag, double *z) {
  if (flag & 2) {
    for (int32_t u = 0; u < m; u++) z[u] = 0.0;
  } else {
    for (int32_t u = 0; u < m; u++) z[u] = (w[u] - mu) / sig;
  }
}

/* Row i of A against every window of B.  ez < 0 means "no exclusion"
 * (AB-join); otherwise pairs with |i - j| <= ez are skipped (self-join).
 * Self-joins may be narrowed further: side 1 keeps j > i only, side 2 j < i
 * only; allow (may be NULL) keeps the offsets k = |i - j| with allow[k]. */
static void one_row(const double *A, const double *B, int64_t lB, int32_t m,
                    int64_t ez, int64_t i, const double *za, const double *muB,
                    const double *sgB, const int8_t *fB, double *zb,
                    const uint8_t *allow, int side, double *P, int64_t *I) {
  double best = INFINITY;
  int64_t arg = -1;
  (void)A;
  for (int64_t j = 0; j < lB; j++) {
    if (!(fB[j] & 1)) continue;
    if (ez >= 0 && llabs(i - j) <= ez) continue;
    if (ez >= 0 && side == 1 && j < i) continue;
    if (ez >= 0 && side == 2 && j > i) continue;
    if (ez >= 0 && allow && !allow[llabs(i - j)]) continue;
    znorm_window(B + j, m, muB[j], sgB[j], fB[j], zb);
    double s = 0.0;
    for (int32_t u = 0; u < m; u++) {
      double d = za[u] - zb[u];
      s += d * d;
    }
    double d = sqrt(s);
    if (d < best) {
      best = d;
      arg = j;
    }
  }
  *P = best;
  *I = arg;
}

static int join_rows(const double *A, int64_t nA, const double *B, int64_t nB,
                     int32_t m, int64_t ez, const uint8_t *allow, int side,
                     const int64_t *rows, int64_t nrows, double *P, int64_t *I) {
  int64_t lA = nA - m + 1, lB = nB - m + 1;
  if (m < 2 || lA < 1 || lB < 1) return -1;
  double *muA = malloc(sizeof(double) * lA), *sgA = malloc(sizeof(double) * lA);
  int8_t *fA = malloc(lA);
  double *muB = muA, *sgB = sgA;
  int8_t *fB = fA;
  int own_b = (B != A || nB != nA);
  if (own_b) {
    muB = malloc(sizeof(double) * lB);
    sgB = malloc(sizeof(double) * lB);
    fB = malloc(lB);
  }
  mpo_window_stats(A, nA, m, muA, sgA, fA);
  if (own_b) mpo_window_stats(B, nB, m, muB, sgB, fB);
#pragma omp parallel
  {
    double *za = malloc(sizeof(double) * m), *zb = malloc(sizeof(double) * m);
#pragma omp for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; r++) {
      int64_t i = rows[r];
      if (i < 0 || i >= lA || !(fA[i] & 1)) {
        P[r] = INFINITY;
        I[r] = -1;
        continue;
      }
      znorm_window(A + i, m, muA[i], sgA[i], fA[i], za);
      one_row(A, B, lB, m, ez, i, za, muB, sgB, fB, zb, allow, side, P + r,
              I + r);
    }
    free(za);
    free(zb);
  }
  free(muA);
  free(sgA);
  free(fA);
  if (own_b) {
    free(muB);
    free(sgB);
    free(fB);
  }
  return 0;
}

/* Exact self-join entries P[r], I[r] for row index rows[r]. */
int mpo_selfjoin_rows(const double *T, int64_t n, int32_t m, int64_t ez,
                      const int64_t *rows, int64_t nrows, double *P,
                      int64_t *I) {
  if (ez < 0) return -1;
  return join_rows(T, n, T, n, m, ez, NULL, 0, rows, nrows, P, I);
}

/* Self-join entries restricted to one side (side 1: j > i, the right
 * profile; side 2: j < i, the left profile; 0: both) and to the offsets
 * |i - j| with allow[|i - j|] != 0 (allow has l entries; NULL = all). */
int mpo_selfjoin_rows_restricted(const double *T, int64_t n, int32_t m,
                                 int64_t ez, const uint8_t *allow, int32_t side,
                                 const int64_t *rows, int64_t nrows, double *P,
                                 int64_t *I) {
  if (ez < 0 || side < 0 || side > 2) return -1;
  return join_rows(T, n, T, n, m, ez, allow, side, rows, nrows, P, I);
}

/* Exact AB-join entries P_AB[r], I_AB[r] for rows[r] of A (call with the
 * series swapped for entries of P_BA). */
int mpo_abjoin_rows(const double *A, int64_t nA, const double *B, int64_t nB,
                    int32_t m, const int64_t *rows, int64_t nrows, double *P,
                    int64_t *I) {
  return join_rows(A, nA, B, nB, m, -1, NULL, 0, rows, nrows, P, I);
}

int mpo_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
