/*
 * oracle.c -- plain FP64 CPU oracle for soft demapping and Monte-Carlo
 * achievable-information-rate estimation (MI, and bit-wise GMI under
 * bit-metric decoding) of an M-point, D-dimensional constellation over a
 * real AWGN channel.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no code,
 * header, table or constant with the GPU library; it is slow on purpose and
 * follows the textbook definitions step by step so that it can be checked
 * against the mathematics by eye.
 *
 * The paper names the quantities computed here only in its list of acronyms
 * (achievable information rate, mutual information, generalised mutual
 * information, log-likelihood ratio, bit-metric decoding, additive white
 * Gaussian noise, signal-to-noise ratio). It prints no formula for them, so
 * the definitions below are the standard ones, with these readings:
 *
 *  R1 SNR:    snr = 10^(SNR_dB/10) = Es / (D * sigma^2), where sigma^2 is the
 *             noise variance per real dimension and Es = (1/M) sum_j |x_j|^2
 *             is the average symbol energy under the uniform prior.
 *  R2 prior:  the M points are equiprobable; with a bijective labelling the
 *             m = log2 M bits are then uniform and independent.
 *  R3 LLR:    L_k = ln P(b_k = 0 | y) - ln P(b_k = 1 | y), in nats.
 *  R4 bits:   bit k of label l is (l >> k) & 1; LLR column k is bit k.
 *  R5 MC:     the estimators use the known transmitted index t_n:
 *               u_n = log2 sum_j p(y_n|x_j) - log2 p(y_n|x_t)        (>= 0)
 *               v_n = sum_k [log2 sum_j p(y_n|x_j)
 *                            - log2 sum_{j: b_k(j)=b_k(t)} p(y_n|x_j)] (>= 0)
 *               MI  = log2 M - mean(u),  GMI = m - mean(v)
 *             and SE = sample standard deviation / sqrt(N). No clamping.
 *  R6 sweep:  y_n = x_{t_n} + sigma_s z_n, formed in FP64 from the caller's
 *             unit-variance noise z_n, the same (t, z) at every SNR point.
 *
 * Every log-sum-exp is exact up to FP64 rounding at any SNR: a common shift
 * (the global maximum) is used for a bit side only when that side's sum is
 * far inside the FP64 range; otherwise the side is recomputed with its own
 * maximum as shift.
 *
 * Sums over samples use Neumaier compensated summation inside fixed chunks
 * of ORACLE_CHUNK samples, and the chunk results are added in chunk order,
 * so the result does not depend on the number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_CHUNK 1024
#define ORACLE_MAX_M 4096
#define ORACLE_MAX_D 64

enum { ORACLE_OK = 0, ORACLE_E_INVAL = -1, ORACLE_E_NOMEM = -3 };

/* ---- Neumaier (improved Kahan) summation ------------------------------ */
typedef struct { double s, c; } nsum_t;

static void nsum_add(nsum_t *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double nsum_val(const nsum_t *a) { return a->s + a->c; }

/* ---- constellation checks (R2, R4) ------------------------------------ */
/* Returns m = log2 M, or -1 if M is not a power of two in [2, 4096], D is
 * outside [1, 64], or the labels are not a bijection onto {0..M-1}. */
int oracle_bits(const uint32_t *labels, int M, int D) {
  if (M < 2 || M > ORACLE_MAX_M || (M & (M - 1)) != 0) return -1;
  if (D < 1 || D > ORACLE_MAX_D || labels == NULL) return -1;
  int m = 0;
  while ((1 << m) < M) ++m;
  char *seen = (char *)calloc((size_t)M, 1);
  if (!seen) return -1;
  for (int j = 0; j < M; ++j) {
    if (labels[j] >= (uint32_t)M || seen[labels[j]]) { free(seen); return -1; }
    seen[labels[j]] = 1;
  }
  free(seen);
  return m;
}

/* Average symbol energy Es = (1/M) sum_j sum_d X[j][d]^2 (R1). */
double oracle_es(const double *X, int M, int D) {
  nsum_t acc = {0.0, 0.0};
  for (int j = 0; j < M; ++j)
    for (int d = 0; d < D; ++d) nsum_add(&acc, X[(size_t)j * D + d] * X[(size_t)j * D + d]);
  return nsum_val(&acc) / (double)M;
}

/* Noise variance per real dimension for a given SNR in dB (R1). */
double oracle_sigma2(double es, int D, double snr_db) {
  return es / ((double)D * pow(10.0, snr_db / 10.0));
}

/* ---- one received sample ---------------------------------------------- */
/* log-sum-exp over the points j with ((labels[j] >> k) & 1) == b, shifted by
 * that side's own maximum; a[] holds the natural-log metrics. */
static double side_lse_own_shift(const double *a, const uint32_t *labels, int M, int k, int b) {
  double amax = -INFINITY;
  for (int j = 0; j < M; ++j)
    if ((int)((labels[j] >> k) & 1u) == b && a[j] > amax) amax = a[j];
  double s = 0.0;
  for (int j = 0; j < M; ++j)
    if ((int)((labels[j] >> k) & 1u) == b) s += exp(a[j] - amax);
  return amax + log(s);
}

/* Per-sample demapping of y (length D). Writes the m LLRs (nats) to llr if
 * non-NULL, and, if t >= 0, the MI and GMI terms u and v (bits).
 * a, side are scratch arrays of length M and 2*m. */
static void demap_one(const double *X, const uint32_t *labels, int M, int D, int m,
                      const double *y, double sigma2, int64_t t,
                      double *a, double *side, double *llr, double *u, double *v) {
  const double inv2s2 = 1.0 / (2.0 * sigma2);
  /* a_j = ln p(y|x_j) up to a constant common to all j:
   *       a_j = -|y - x_j|^2 / (2 sigma^2), direct differences. */
  double amax = -INFINITY;
  for (int j = 0; j < M; ++j) {
    double d2 = 0.0;
    for (int d = 0; d < D; ++d) {
      double diff = y[d] - X[(size_t)j * D + d];
      d2 += diff * diff;
    }
    a[j] = -d2 * inv2s2;
    if (a[j] > amax) amax = a[j];
  }
  /* Total log-sum-exp with the global maximum as shift. */
  double stot = 0.0;
  for (int k = 0; k < 2 * m; ++k) side[k] = 0.0;
  for (int j = 0; j < M; ++j) {
    double e = exp(a[j] - amax);
    stot += e;
    for (int k = 0; k < m; ++k) side[2 * k + ((labels[j] >> k) & 1u)] += e;
  }
  const double lse = amax + log(stot);
  /* Per bit side: the shared shift is exact while the side sum is far inside
   * the FP64 range (every dropped term is then below 1e-250 / 2^52 of it);
   * otherwise use the side's own maximum. */
  double lse_side[2 * 12];
  for (int k = 0; k < m; ++k)
    for (int b = 0; b < 2; ++b) {
      double s = side[2 * k + b];
      lse_side[2 * k + b] = (s > 1e-250) ? amax + log(s)
                                         : side_lse_own_shift(a, labels, M, k, b);
    }
  if (llr)
    for (int k = 0; k < m; ++k) llr[k] = lse_side[2 * k + 0] - lse_side[2 * k + 1];
  if (t >= 0) {
    const double ln2 = log(2.0);
    *u = (lse - a[t]) / ln2;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) {
      int bt = (int)((labels[t] >> k) & 1u);
      acc += (lse - lse_side[2 * k + bt]) / ln2;
    }
    *v = acc;
  }
}

/* ---- statistics -------------------------------------------------------- */
/* MI = log2 M - mean(u), GMI = m - mean(v), SE = sd/sqrt(N) with the sample
 * standard deviation (N-1 denominator); SE is NaN for N = 1. Sums are
 * chunked Neumaier sums; the deviation uses a second pass about the mean. */
static double chunked_sum(const double *x, int64_t N, double shift, int square) {
  int64_t nchunks = (N + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
  nsum_t total = {0.0, 0.0};
  for (int64_t c = 0; c < nchunks; ++c) {
    nsum_t part = {0.0, 0.0};
    int64_t hi = (c + 1) * ORACLE_CHUNK < N ? (c + 1) * ORACLE_CHUNK : N;
    for (int64_t n = c * ORACLE_CHUNK; n < hi; ++n) {
      double d = x[n] - shift;
      nsum_add(&part, square ? d * d : d);
    }
    nsum_add(&total, nsum_val(&part));
  }
  return nsum_val(&total);
}

static void fill_stats(const double *u, const double *v, int64_t N, int M, int m, double *stats) {
  double mu = chunked_sum(u, N, 0.0, 0) / (double)N;
  double mv = chunked_sum(v, N, 0.0, 0) / (double)N;
  stats[0] = log2((double)M) - mu;
  stats[1] = (double)m - mv;
  if (N > 1) {
    double su = chunked_sum(u, N, mu, 1) / (double)(N - 1);
    double sv = chunked_sum(v, N, mv, 1) / (double)(N - 1);
    stats[2] = sqrt(su / (double)N);
    stats[3] = sqrt(sv / (double)N);
  } else {
    stats[2] = NAN;
    stats[3] = NAN;
  }
}

/* ---- public entry points --------------------------------------------- */
/* Demap a given received block Y (N x D, row-major, FP64) at one SNR.
 *  tx:    transmitted indices (N) into X, or NULL (then no MI/GMI terms).
 *  stats: [4] = MI, GMI, SE_MI, SE_GMI (bits per D-dim symbol); needs tx.
 *  llr:   N x m LLRs in nats, or NULL.
 *  u, v:  per-sample MI/GMI terms (N each), or NULL.
 * Returns 0, or a negative error code for invalid arguments or no memory. */
static int eval_sigma2(const double *X, const uint32_t *labels, int M, int D,
                       const double *Y, const uint32_t *tx, int64_t N, double sigma2,
                       double *stats, double *llr, double *u, double *v) {
  int m = oracle_bits(labels, M, D);
  if (m < 0 || X == NULL || Y == NULL || N < 1) return ORACLE_E_INVAL;
  if (!(sigma2 > 0.0) || !isfinite(sigma2)) return ORACLE_E_INVAL;
  if ((stats || u || v) && tx == NULL) return ORACLE_E_INVAL;
  if (tx)
    for (int64_t n = 0; n < N; ++n)
      if (tx[n] >= (uint32_t)M) return ORACLE_E_INVAL;
  double *uu = u, *vv = v, *own = NULL;
  if (tx && (!u || !v)) {
    own = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    if (!own) return ORACLE_E_NOMEM;
    uu = u ? u : own;
    vv = v ? v : own + N;
  }
  int fail = 0;
#pragma omp parallel
  {
    double *a = (double *)malloc(sizeof(double) * (size_t)M);
    double side[2 * 12];
    if (!a) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(static)
      for (int64_t n = 0; n < N; ++n) {
        double du = 0.0, dv = 0.0;
        demap_one(X, labels, M, D, m, Y + (size_t)n * D, sigma2, tx ? (int64_t)tx[n] : -1,
                  a, side, llr ? llr + (size_t)n * m : NULL, &du, &dv);
        if (tx) { uu[n] = du; vv[n] = dv; }
      }
    }
    free(a);
  }
  if (!fail && stats) fill_stats(uu, vv, N, M, m, stats);
  free(own);
  return fail ? ORACLE_E_NOMEM : ORACLE_OK;
}

int oracle_eval(const double *X, const uint32_t *labels, int M, int D,
                const double *Y, const uint32_t *tx, int64_t N, double snr_db,
                double *stats, double *llr, double *u, double *v) {
  if (X == NULL || M < 1 || D < 1) return ORACLE_E_INVAL;
  return eval_sigma2(X, labels, M, D, Y, tx, N, oracle_sigma2(oracle_es(X, M, D), D, snr_db),
                     stats, llr, u, v);
}

/* ---- auxiliary-channel (mismatched) rates -----------------------------
 * The paper lists NGMI among its acronyms and measures a real link, where the
 * noise statistics are not known to the receiver. The readings:
 *  R10 auxiliary channel: the receiver's metric is the Gaussian density
 *      q(y|x) = N(x, sigma_a^2 I) with a caller-given sigma_a^2 (for example
 *      the estimate of R11). LLRs, u_n, v_n, MI and GMI are those of R3 and R5
 *      with q in place of p. With the samples drawn from the true channel,
 *      their expectations are the mismatched-decoding rates, which are lower
 *      bounds on the true channel's MI and GMI and equal them when sigma_a^2
 *      is the true noise variance.
 *  R11 noise estimate: with the transmitted points known, the per-dimension
 *      variance is s_d^2 = (1/N) sum_n (y_nd - x_{t_n},d)^2 (the maximum-
 *      likelihood estimate with known means, no N - 1 correction), and the
 *      isotropic estimate is the mean of the D values.
 *  R12 NGMI = 1 - (H(X) - GMI) / m, with H(X) = log2 M = m under the uniform
 *      prior of R2, so NGMI = GMI / m.
 */

/* ---- max-log demapping ------------------------------------------------
 * A standard receiver simplification: each bit side's log-sum-exp is replaced
 * by its largest term. The readings:
 *  R13 max-log LLR: L_k = min_{j: b_k(j)=1} |y - x_j|^2 / (2 sigma^2)
 *                       - min_{j: b_k(j)=0} |y - x_j|^2 / (2 sigma^2), nats.
 *  R14 max-log GMI: the BMD rate of a receiver that takes these LLRs as exact,
 *      v_n = sum_k log2(1 + exp(-(1 - 2 b_k(t_n)) L_nk)), GMI = m - mean(v),
 *      SE as R5. With the exact LLRs of R3 this is R5's v; with max-log LLRs
 *      it is an achievable rate of that receiver (a lower bound on its GMI).
 *      No symbol-wise MI is defined: MI, its SE and u are NaN.
 */

/* log2(1 + e^x) without overflow. */
static double log2_1p_exp(double x) {
  return (x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x))) / log(2.0);
}

static void maxlog_one(const double *X, const uint32_t *labels, int M, int D, int m,
                       const double *y, double sigma2, int64_t t, double *dmin,
                       double *llr, double *v) {
  for (int k = 0; k < 2 * m; ++k) dmin[k] = INFINITY;
  for (int j = 0; j < M; ++j) {
    double d2 = 0.0;
    for (int d = 0; d < D; ++d) {
      double diff = y[d] - X[(size_t)j * D + d];
      d2 += diff * diff;
    }
    for (int k = 0; k < m; ++k) {
      double *slot = &dmin[2 * k + ((labels[j] >> k) & 1u)];
      if (d2 < *slot) *slot = d2;
    }
  }
  double acc = 0.0;
  for (int k = 0; k < m; ++k) {
    const double L = (dmin[2 * k + 1] - dmin[2 * k]) / (2.0 * sigma2);
    if (llr) llr[k] = L;
    if (t >= 0) acc += log2_1p_exp(-(1.0 - 2.0 * (double)((labels[t] >> k) & 1u)) * L);
  }
  if (t >= 0) *v = acc;
}

/* Max-log demapping of a given block at one SNR (R13, R14); arguments as
 * oracle_eval; stats[0], stats[2] and u are NaN. */
int oracle_eval_maxlog(const double *X, const uint32_t *labels, int M, int D,
                       const double *Y, const uint32_t *tx, int64_t N, double snr_db,
                       double *stats, double *llr, double *u, double *v) {
  int m = oracle_bits(labels, M, D);
  if (m < 0 || X == NULL || Y == NULL || N < 1 || !isfinite(snr_db)) return ORACLE_E_INVAL;
  if ((stats || u || v) && tx == NULL) return ORACLE_E_INVAL;
  if (tx)
    for (int64_t n = 0; n < N; ++n)
      if (tx[n] >= (uint32_t)M) return ORACLE_E_INVAL;
  const double sigma2 = oracle_sigma2(oracle_es(X, M, D), D, snr_db);
  double *vv = v, *own = NULL;
  if (tx && !v) {
    own = (double *)malloc(sizeof(double) * (size_t)N);
    if (!own) return ORACLE_E_NOMEM;
    vv = own;
  }
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    double dmin[2 * 12];
    double dv = 0.0;
    maxlog_one(X, labels, M, D, m, Y + (size_t)n * D, sigma2, tx ? (int64_t)tx[n] : -1, dmin,
               llr ? llr + (size_t)n * m : NULL, &dv);
    if (tx) vv[n] = dv;
    if (u) u[n] = NAN;
  }
  if (stats) {
    fill_stats(vv, vv, N, M, m, stats);
    stats[0] = NAN;
    stats[2] = NAN;
  }
  free(own);
  return ORACLE_OK;
}

/* As oracle_eval, with the metric's noise variance given directly (R10). */
int oracle_eval_aux(const double *X, const uint32_t *labels, int M, int D,
                    const double *Y, const uint32_t *tx, int64_t N, double sigma2_aux,
                    double *stats, double *llr, double *u, double *v) {
  return eval_sigma2(X, labels, M, D, Y, tx, N, sigma2_aux, stats, llr, u, v);
}

/* Noise variance estimates (R11): var[d] for d < D, then the isotropic
 * estimate var[D]. Sums are the chunked Neumaier sums of chunked_sum's kind,
 * one per dimension, independent of the thread count. */
int oracle_noise_var(const double *X, int M, int D, const double *Y, const uint32_t *tx,
                     int64_t N, double *var) {
  if (X == NULL || Y == NULL || tx == NULL || var == NULL || M < 1 || D < 1 || N < 1)
    return ORACLE_E_INVAL;
  for (int64_t n = 0; n < N; ++n)
    if (tx[n] >= (uint32_t)M) return ORACLE_E_INVAL;
  const int64_t nchunk = (N + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
  double *part = (double *)malloc(sizeof(double) * (size_t)nchunk * (size_t)D);
  if (!part) return ORACLE_E_NOMEM;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < nchunk; ++q) {
    const int64_t n1 = (q + 1) * ORACLE_CHUNK < N ? (q + 1) * ORACLE_CHUNK : N;
    for (int d = 0; d < D; ++d) {
      nsum_t acc = {0.0, 0.0};
      for (int64_t n = q * ORACLE_CHUNK; n < n1; ++n) {
        const double e = Y[(size_t)n * D + d] - X[(size_t)tx[n] * D + d];
        nsum_add(&acc, e * e);
      }
      part[(size_t)q * D + d] = nsum_val(&acc);
    }
  }
  double all = 0.0;
  for (int d = 0; d < D; ++d) {
    nsum_t acc = {0.0, 0.0};
    for (int64_t q = 0; q < nchunk; ++q) nsum_add(&acc, part[(size_t)q * D + d]);
    var[d] = nsum_val(&acc) / (double)N;
    all += var[d];
  }
  var[D] = all / (double)D;
  free(part);
  return ORACLE_OK;
}

/* SNR sweep from unit noise (R6): for each of the S SNR points,
 * y_n = X[tx_n] + sigma_s * Z_n in FP64 from the FP32 noise Z (N x D), then
 * demap as oracle_eval. stats is S x 4, llr S x N x m, u and v S x N;
 * each may be NULL. Z64 may replace Z with FP64 noise (then Z is unused). */
int oracle_sweep(const double *X, const uint32_t *labels, int M, int D,
                 const uint32_t *tx, const float *Z, const double *Z64, int64_t N,
                 const double *snr_db, int S,
                 double *stats, double *llr, double *u, double *v) {
  int m = oracle_bits(labels, M, D);
  if (m < 0 || X == NULL || tx == NULL || (Z == NULL && Z64 == NULL) || N < 1 ||
      snr_db == NULL || S < 1)
    return ORACLE_E_INVAL;
  for (int64_t n = 0; n < N; ++n)
    if (tx[n] >= (uint32_t)M) return ORACLE_E_INVAL;
  const double es = oracle_es(X, M, D);
  double *y = (double *)malloc(sizeof(double) * (size_t)N * D);
  if (!y) return ORACLE_E_NOMEM;
  int rc = ORACLE_OK;
  for (int s = 0; s < S && rc == ORACLE_OK; ++s) {
    const double sigma = sqrt(oracle_sigma2(es, D, snr_db[s]));
    for (int64_t n = 0; n < N; ++n)
      for (int d = 0; d < D; ++d) {
        double z = Z64 ? Z64[(size_t)n * D + d] : (double)Z[(size_t)n * D + d];
        y[(size_t)n * D + d] = X[(size_t)tx[n] * D + d] + sigma * z;
      }
    rc = oracle_eval(X, labels, M, D, y, tx, N, snr_db[s],
                     stats ? stats + 4 * s : NULL,
                     llr ? llr + (size_t)s * N * m : NULL,
                     u ? u + (size_t)s * N : NULL,
                     v ? v + (size_t)s * N : NULL);
  }
  free(y);
  return rc;
}

/* ---- hard decisions (the paper's own metric) ---------------------------
 * The paper's receiver demaps the hard decisions of its equaliser and
 * reports the Q-factor estimated from the bit error rate, against the BER
 * thresholds of hard-decision FEC at 6.7 % and 20 % overhead (Sections II
 * and III). It prints neither the decision rule nor the BER-to-Q conversion;
 * the readings:
 *  R7 decision: the constellation point nearest to y in squared Euclidean
 *     distance, evaluated in FP32 (the receiver processes its samples in
 *     32-bit floating point, Section II): every coordinate an FP32 value, the
 *     distance accumulated over d = 0..D-1 as acc = fmaf(y_d - x_d, y_d - x_d,
 *     acc) from acc = 0, ties to the lower label. In sweep mode
 *     y_d = fmaf(sigma_f, z_d, x_t,d) with sigma_f the FP32 rounding of sigma.
 *  R8 errors: a symbol error when the decided point is not the transmitted
 *     one; its bit errors are the Hamming distance between the two labels;
 *     BER = bit errors / (N m), SER = symbol errors / N.
 *  R9 Q-factor: Q_dB = 20 log10(sqrt(2) erfcinv(2 BER)), the Gaussian-tail
 *     conversion (BER = erfc(Q / sqrt 2) / 2).
 */

/* Decided point (X row) for one FP32 received point (R7). */
static int hd_decide(const float *xf, const int *pos, int M, int D, const float *y) {
  int best = -1;
  float bd = 0.0f;
  for (int l = 0; l < M; ++l) {           /* labels in increasing order: ties keep the lower */
    const float *x = xf + (size_t)pos[l] * D;
    float acc = 0.0f;
    for (int d = 0; d < D; ++d) {
      const float df = y[d] - x[d];
      acc = fmaf(df, df, acc);
    }
    if (best < 0 || acc < bd) { best = pos[l]; bd = acc; }
  }
  return best;
}

static int hamming(uint32_t a, uint32_t b) {
  int c = 0;
  for (uint32_t x = a ^ b; x; x >>= 1) c += (int)(x & 1u);
  return c;
}

/* Hard decisions of a given FP32 block Y (N x D).
 *  tx:      transmitted indices or NULL; counts [2] = symbol errors, bit
 *           errors (needs tx; may be NULL).
 *  decided: N decided X rows, or NULL. */
int oracle_hd(const double *X, const uint32_t *labels, int M, int D, const float *Y,
              const uint32_t *tx, int64_t N, uint32_t *decided, uint64_t *counts) {
  int m = oracle_bits(labels, M, D);
  if (m < 0 || X == NULL || Y == NULL || N < 1 || (counts && !tx)) return ORACLE_E_INVAL;
  if (tx)
    for (int64_t n = 0; n < N; ++n)
      if (tx[n] >= (uint32_t)M) return ORACLE_E_INVAL;
  float *xf = (float *)malloc(sizeof(float) * (size_t)M * D);
  int *pos = (int *)malloc(sizeof(int) * (size_t)M);
  if (!xf || !pos) { free(xf); free(pos); return ORACLE_E_NOMEM; }
  for (int64_t i = 0; i < (int64_t)M * D; ++i) xf[i] = (float)X[i];
  for (int j = 0; j < M; ++j) pos[labels[j]] = j;
  uint64_t se = 0, be = 0;
#pragma omp parallel for schedule(static) reduction(+ : se, be)
  for (int64_t n = 0; n < N; ++n) {
    const int j = hd_decide(xf, pos, M, D, Y + (size_t)n * D);
    if (decided) decided[n] = (uint32_t)j;
    if (tx && (uint32_t)j != tx[n]) {
      se += 1;
      be += (uint64_t)hamming(labels[j], labels[tx[n]]);
    }
  }
  if (counts) { counts[0] = se; counts[1] = be; }
  free(xf);
  free(pos);
  return ORACLE_OK;
}

/* Hard decisions of the SNR sweep: y = fmaf(sigma_f, z, x_t) in FP32 (R7).
 * decided is S x N or NULL, counts S x 2. */
int oracle_hd_sweep(const double *X, const uint32_t *labels, int M, int D, const uint32_t *tx,
                    const float *Z, int64_t N, const double *snr_db, int S, uint32_t *decided,
                    uint64_t *counts) {
  int m = oracle_bits(labels, M, D);
  if (m < 0 || X == NULL || tx == NULL || Z == NULL || N < 1 || snr_db == NULL || S < 1 ||
      counts == NULL)
    return ORACLE_E_INVAL;
  for (int64_t n = 0; n < N; ++n)
    if (tx[n] >= (uint32_t)M) return ORACLE_E_INVAL;
  const double es = oracle_es(X, M, D);
  float *y = (float *)malloc(sizeof(float) * (size_t)N * D);
  if (!y) return ORACLE_E_NOMEM;
  int rc = ORACLE_OK;
  for (int s = 0; s < S && rc == ORACLE_OK; ++s) {
    const float sf = (float)sqrt(oracle_sigma2(es, D, snr_db[s]));
    for (int64_t n = 0; n < N; ++n)
      for (int d = 0; d < D; ++d)
        y[(size_t)n * D + d] = fmaf(sf, Z[(size_t)n * D + d], (float)X[(size_t)tx[n] * D + d]);
    rc = oracle_hd(X, labels, M, D, y, tx, N, decided ? decided + (size_t)s * N : NULL, counts + 2 * s);
  }
  free(y);
  return rc;
}

/* erfc^-1 by bisection on erfc (decreasing on the real line), then the
 * Q-factor in dB of a bit error rate in (0, 0.5) (R9); NaN outside. */
double oracle_q_db(double ber) {
  if (!(ber > 0.0 && ber < 0.5)) return NAN;
  const double target = 2.0 * ber;          /* erfc(x) = 2 BER, x = Q / sqrt 2 > 0 */
  double lo = 0.0, hi = 30.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (erfc(mid) > target) lo = mid;
    else hi = mid;
  }
  return 20.0 * log10(sqrt(2.0) * 0.5 * (lo + hi));
}

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---- per-SNR summaries of the rates (readings R12, R15, R16) -------------
 *
 * The paper evaluates each format by its bit error rate against the
 * thresholds of two hard-decision FEC codes, of 6.7 % and 20 % overhead,
 * and plots the net throughput of the formats that meet a threshold
 * (Section III); it prints neither the threshold BERs nor a formula for the
 * net rate. Readings:
 *  R12 NGMI:  1 - (H(X) - GMI) / m with H(X) = m under the uniform prior,
 *             i.e. GMI / m; its standard error is SE_GMI / m.
 *  R15 HD-FEC: a code of overhead OH (fraction: 0.067, 0.2) and threshold
 *             BER th is met when BER <= th (a NaN BER meets nothing).
 *  R16 net rate: a code of overhead OH carries m / (1 + OH) information
 *             bits per symbol (code rate 1 / (1 + OH)); the net rate is the
 *             largest such value over the codes that are met, times the
 *             symbol rate, and 0 when none is met. Ties keep the code listed
 *             first.
 */

/* NGMI and its SE for S points of MI/GMI statistics (S x 4: MI, GMI, SE_MI,
 * SE_GMI); out is S x 2. */
int oracle_ngmi(const double *stats, int S, int m, double *out) {
  if (!stats || !out || S < 1 || m < 1) return ORACLE_E_INVAL;
  for (int s = 0; s < S; ++s) {
    const double gmi = stats[4 * s + 1], se = stats[4 * s + 3];
    const double hx = (double)m;                 /* entropy of the uniform input, bits */
    out[2 * s] = 1.0 - (hx - gmi) / (double)m;
    out[2 * s + 1] = se / (double)m;
  }
  return ORACLE_OK;
}

/* BER, SER and Q-factor (dB) of S points of hard-decision error counts
 * (S x 2: symbol errors, bit errors) over N symbols of m bits (R8, R9);
 * out is S x 3. */
int oracle_hd_rates(const uint64_t *counts, int S, int64_t N, int m, double *out) {
  if (!counts || !out || S < 1 || N < 1 || m < 1) return ORACLE_E_INVAL;
  for (int s = 0; s < S; ++s) {
    const double ser = (double)counts[2 * s] / (double)N;
    const double ber = (double)counts[2 * s + 1] / ((double)N * (double)m);
    out[3 * s] = ber;
    out[3 * s + 1] = ser;
    out[3 * s + 2] = oracle_q_db(ber);
  }
  return ORACLE_OK;
}

/* HD-FEC pass/fail and net rate for S points of BERs (ber[s * stride]) and F
 * codes (overhead[f], threshold[f]) (R15, R16).
 *  pass: S x F (1 met, 0 not), or NULL
 *  net:  S net rates (symbol_rate x bits per symbol), or NULL
 *  best: S indices of the code that gives the net rate (-1: none), or NULL */
int oracle_fec_net(const double *ber, int64_t stride, int S, int m, const double *overhead,
                   const double *threshold, int F, double symbol_rate, int32_t *pass, double *net,
                   int32_t *best) {
  if (!ber || stride < 1 || S < 1 || m < 1 || !overhead || !threshold || F < 1) return ORACLE_E_INVAL;
  for (int f = 0; f < F; ++f)
    if (!(overhead[f] >= 0.0) || !(threshold[f] >= 0.0)) return ORACLE_E_INVAL;
  for (int s = 0; s < S; ++s) {
    const double b = ber[(int64_t)s * stride];
    double top = 0.0;
    int arg = -1;
    for (int f = 0; f < F; ++f) {
      const int ok = b <= threshold[f];          /* false for a NaN BER */
      if (pass) pass[(int64_t)s * F + f] = ok;
      const double rate = (double)m / (1.0 + overhead[f]);
      if (ok && rate > top) {
        top = rate;
        arg = f;
      }
    }
    if (net) net[s] = symbol_rate * top;
    if (best) best[s] = arg;
  }
  return ORACLE_OK;
}
