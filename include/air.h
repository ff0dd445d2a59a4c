/*
 * air.h -- C ABI of libair: soft demapping (per-bit LLRs) and Monte-Carlo
 * achievable-information-rate estimation (MI, and bit-wise GMI under
 * bit-metric decoding) of D-dimensional constellations over real AWGN, on
 * one AMD Instinct MI355X (gfx950).
 *
 * The paper (a software-defined GPU receiver) only names these quantities in
 * its list of acronyms -- achievable information rate, mutual information,
 * generalised mutual information, log-likelihood ratio, bit-metric decoding,
 * additive white Gaussian noise, signal-to-noise ratio -- and its receiver
 * demaps the hard decisions of its adaptive equaliser (Section II). The
 * definitions used here are the standard ones, with these readings:
 *
 *  - SNR:   snr = 10^(snr_db/10) = Es / (D sigma^2); sigma^2 is the noise
 *           variance per real dimension, Es = (1/M) sum_j |x_j|^2 the average
 *           energy of the constellation under a uniform prior.
 *  - LLR:   L_k = ln P(b_k=0 | y) - ln P(b_k=1 | y), natural log (nats).
 *  - Bits:  bit k of a label l is (l >> k) & 1; LLR column k is bit k.
 *  - MI:    log2 M - mean_n log2( sum_j p(y_n|x_j) / p(y_n|x_{t_n}) )
 *  - GMI:   m - mean_n sum_k log2( sum_j p(y_n|x_j)
 *                                / sum_{j: b_k(j) = b_k(t_n)} p(y_n|x_j) )
 *           with m = log2 M. Both in bits per D-dimensional symbol, with
 *           standard errors sd/sqrt(N) (sample standard deviation). No clamping.
 *  - Sweep: y_n = x_{t_n} + sigma_s z_n from the caller's unit-variance noise
 *           z_n; the same (t, z) is used at every SNR point.
 *
 * Conventions for every call:
 *  - Every function returns an air_status and never throws across the ABI.
 *    On failure air_last_error() describes the cause.
 *  - Pointers named *_dev are device memory owned by the caller (for example
 *    the storage of a torch tensor on the context's device); pointers named
 *    *_host are host memory. Layouts are dense and row-major.
 *  - Work is enqueued asynchronously on the context's HIP stream; results in
 *    device buffers are valid once the stream has reached that point
 *    (air_sync, or any later operation on the same stream).
 *  - A context is not thread-safe; use one per host thread.
 *  - The constellation X is given in FP64 on the host and kept on the device.
 *    Transmitted indices tx index the rows of X (not labels).
 */
#ifndef LIBAIR_AIR_H
#define LIBAIR_AIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct air_ctx air_ctx;
typedef struct air_const air_const;

typedef enum {
  AIR_OK = 0,
  AIR_E_INVAL = -1,        /* invalid argument (null pointer, bad size, bad labels...) */
  AIR_E_UNSUPPORTED = -2,  /* valid request this build or precision cannot serve        */
  AIR_E_NOMEM = -3,        /* device or host allocation failed                          */
  AIR_E_DEVICE = -4,       /* a HIP runtime call failed                                 */
  AIR_E_BUSY = -5,         /* resource temporarily unavailable                          */
  AIR_E_RANGE = -6         /* device data out of range (a tx index >= M was seen)       */
} air_status;

/* Arithmetic of the demapping kernels.
 *  AIR_FP64    FP64 throughout (distances, log-sum-exp, sums). Y / Z / LLR are double.
 *  AIR_FP32    FP32 vector ALU, squared distances by direct differences.
 *  AIR_BF16X3  exponent tile on the matrix cores from bfloat16 splits of both
 *              factors into hi + mid + lo parts (six cross products per term,
 *              ~2^-24 relative) with FP32 accumulation; FP32 log-sum-exp.
 *  AIR_FP16X3  the exponent tile from half-precision hi + lo splits (three
 *              cross products per term, ~2^-22 relative); as AIR_BF16X3 otherwise.
 * Except AIR_FP64, Y / Z are float and LLRs float. Sums over samples are
 * always FP64. A result the fast FP32 frame cannot hold to the stated
 * accuracy (very large |LLR|, a received point far from every constellation
 * point) is recomputed: by a second tier with every term in an FP64 frame
 * (AIR_FP32, AIR_BF16X3, AIR_FP16X3), and beyond that (or in AIR_FP64) by an
 * exact per-sample path relative to the nearest point. */
typedef enum {
  AIR_FP64 = 0,
  AIR_FP32 = 1,
  AIR_BF16X3 = 2,
  AIR_FP16X3 = 3
} air_prec;

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the default stream). *out receives the context. */
air_status air_create(air_ctx **out, int device, void *hip_stream);

/* Release a context and its workspace (synchronises its stream first). NULL is ignored. */
void air_destroy(air_ctx *ctx);

/* Issue subsequent work on another stream of the same device. Waits first for
 * the work already issued on the current stream (the next call reuses the
 * context's workspace), so the current stream must still exist; returns
 * AIR_E_DEVICE if that wait fails. */
air_status air_set_stream(air_ctx *ctx, void *hip_stream);

/* Message describing the last failure on this context ("" if none). Owned by the context. */
const char *air_last_error(const air_ctx *ctx);

/* Wait for all work issued on the context's stream. Returns AIR_E_RANGE (and
 * clears the flag) if a kernel saw a transmitted index >= M since the last
 * air_sync; the statistics of the affected calls are then NaN. */
air_status air_sync(air_ctx *ctx);

/* Upload a constellation.
 *  X_host:      M x D FP64 points, row-major.
 *  labels_host: M bit labels, a bijection onto {0, ..., M-1}.
 *  M = 2^m with 2 <= M <= 4096; 1 <= D <= 16.
 * The handle owns device copies in every layout the kernels use (label order,
 * FP64 / FP32 coordinates, split half / bfloat16 operands). It lives on the
 * context's device and may only be used with the context that created it. */
air_status air_const_create(air_ctx *ctx, const double *X_host, const uint32_t *labels_host,
                            int M, int D, air_const **out);

/* Release a constellation (waits for device work that may still read it). NULL is ignored.
 * May be called after its context was destroyed. */
void air_const_destroy(air_const *c);

/* Bits per label, m = log2 M, of a constellation (0 if c is NULL). */
int air_const_bits(const air_const *c);

/* Soft demapping of a received block at one SNR.
 *  Y_dev:   N x D received points (double for AIR_FP64, else float).
 *  llr_dev: N x m LLRs in nats (double for AIR_FP64, else float).
 * N >= 1. Calls in AIR_FP16X3 and AIR_BF16X3, and the exact (not max-log)
 * calls in AIR_FP32, take at most 2^32 - 128 samples (32-bit sample indices)
 * and return AIR_E_UNSUPPORTED beyond; this holds for every call below that
 * takes N. */
air_status air_llr(air_ctx *ctx, const air_const *c, const void *Y_dev, int64_t N,
                   double snr_db, air_prec prec, void *llr_dev);

/* Monte-Carlo MI and GMI of a received block at one SNR, with known
 * transmitted indices.
 *  Y_dev:     N x D received points (double for AIR_FP64, else float).
 *  tx_dev:    N transmitted indices into the rows of X (uint32).
 *  stats_dev: 4 doubles: MI, GMI, SE_MI, SE_GMI (bits per symbol); SE is NaN for N = 1.
 *  llr_dev:   N x m LLRs (nats), or NULL to skip the LLR output. */
air_status air_mi_gmi(air_ctx *ctx, const air_const *c, const void *Y_dev,
                      const uint32_t *tx_dev, int64_t N, double snr_db, air_prec prec,
                      double *stats_dev, void *llr_dev);

/* SNR sweep in one launch: for every SNR point s, y = x_t + sigma_s z.
 *  tx_dev:      N transmitted indices into the rows of X (uint32).
 *  Z_dev:       N x D unit-variance noise (double for AIR_FP64, else float).
 *  snr_db_host: S SNR points in dB, S >= 1.
 *  stats_dev:   S x 4 doubles (MI, GMI, SE_MI, SE_GMI per SNR point).
 *  llr_dev:     S x N x m LLRs (nats), or NULL.
 * Without LLRs (here and in air_mi_gmi) only the bit sides that MI and GMI use
 * must stay inside the FP32 frame, so at high SNR far fewer items need the
 * second tier; the statistics agree with those of the same call with LLRs to
 * FP32 rounding, not bit for bit. */
air_status air_sweep(air_ctx *ctx, const air_const *c, const uint32_t *tx_dev,
                     const void *Z_dev, int64_t N, const double *snr_db_host, int S,
                     air_prec prec, double *stats_dev, void *llr_dev);

/* air_sweep for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc. The
 * same computation, arguments, layouts and errors as air_sweep; it calls no
 * hipMalloc / hipFree or other allocating routine, and launches untimed
 * (air_set_timing does not apply). The second tier's per-launch workspace
 * comes from one 48 MiB device array per GPU, allocated with the library's
 * code on that GPU and kept until the process ends; a launch takes as many
 * SNR points (at most 64) as fit in it: per point about 4.3 bytes per sample
 * plus up to 1.7 MB for the launch's waves (5 MB at N = 1e6). N beyond what
 * one SNR point fits (about 1.1e7 samples) returns AIR_E_INVAL before any
 * launch. Every call on a GPU shares that GPU's array: calls that can overlap
 * on one GPU (other contexts or streams) race and must be ordered by the
 * caller. Each launch writes every
 * part of the array it reads before reading it, so nothing carries over
 * between calls. Requires that a context was created on the device
 * (air_create looks the array up); AIR_E_DEVICE otherwise. */
air_status air_sweep_noalloc(air_ctx *ctx, const air_const *c, const uint32_t *tx_dev,
                             const void *Z_dev, int64_t N, const double *snr_db_host, int S,
                             air_prec prec, double *stats_dev, void *llr_dev);

/* Number of (sample, SNR) items the last call on this context did not finish
 * in its first tier's sums (starved bit sides: |LLR| beyond the FP32 frame's
 * range, or a received point far from every constellation point): finished by
 * the second tier or the exact path. Synchronises. Returns -1 on error. */
int64_t air_last_recomputed(air_ctx *ctx);

/* Of those items, the number that needed the exact path (beyond the FP64
 * second-tier window, |LLR| of roughly 1300 nats; for AIR_FP64 every
 * recomputed item). Synchronises. -1 on error. */
int64_t air_last_exact(air_ctx *ctx);

/* Kernel timing for measurement tools. While enabled, each launch of a call's
 * main demapping kernel (the vector kernel, or the first tier of the
 * matrix-core forms; not their second tier or the small reduction kernel that
 * follows) sets a pair of HIP events to the kernel's own start and end
 * (hipExtLaunchKernel: no marker commands are added to the stream). Enabling
 * or disabling discards the recorded pairs. */
air_status air_set_timing(air_ctx *ctx, int enable);

/* Sum of the demapping-kernel durations recorded since timing was enabled or
 * last read (ms), and the number of launches; synchronises, then discards the
 * recorded pairs. */
air_status air_kernel_time(air_ctx *ctx, double *total_ms, int64_t *launches);

/* Rates of the units that bound the demapping path on the context's device,
 * measured by microbenchmark kernels (each timed with HIP events after one
 * untimed launch; all CUs busy, independent chains per lane). For measurement
 * tools: the roof fractions reported for the demapping kernels are taken
 * against these units. */
typedef struct {
  double exp_per_s;          /* v_exp_f32 results per second                               */
  double explog_per_s;       /* exp2 and log2 in turn: transcendental results per second  */
  double fma_per_s;          /* FP32 FMA results per second (non-packed)                  */
  double exp_fma_ratio[3];   /* time of (1 exp2 + K FMAs), K = 1, 2, 4, over the sum of the
                                two kinds' separate times: 1 = they share one issue budget,
                                ~0.5 = they overlap fully                                   */
  double mfma_f16_flops;     /* v_mfma_f32_32x32x16_f16, flop/s                            */
  double mfma_bf16_flops;    /* v_mfma_f32_32x32x16_bf16, flop/s                           */
  double copy_bytes_per_s;   /* bytes read + written per second by a 1 GiB device copy     */
} air_roofs;

/* Run the microbenchmarks on the context's stream (about 0.1 s; allocates and
 * frees 2 GiB of device memory and synchronises). */
air_status air_measure_roofs(air_ctx *ctx, air_roofs *out);

/* ---------------------------------------------------------------------------
 * Auxiliary-channel (mismatched) rates. The paper measures a real link and
 * lists the normalised GMI among its acronyms; there the receiver does not
 * know the noise statistics and demaps with a Gaussian model of the channel
 * whose variance it estimates. MI and GMI computed with that metric on
 * samples of the true channel are achievable rates of the mismatched
 * receiver: lower bounds that equal the matched rates when the model's
 * variance is the true one. NGMI = 1 - (H(X) - GMI) / m = GMI / m under the
 * uniform prior.
 * ------------------------------------------------------------------------- */

/* Noise variance estimates with known transmitted points (maximum likelihood
 * with known means, no N - 1 correction).
 *  Y_dev:   N x D received points (double for AIR_FP64, else float).
 *  tx_dev:  N transmitted indices into the rows of X.
 *  var_dev: D + 1 doubles (device): (1/N) sum_n (y_nd - x_{t_n},d)^2 for each
 *           dimension d, then their mean (the isotropic estimate). All NaN
 *           and AIR_E_RANGE at the next air_sync if an index is >= M.
 * Sums are FP64 in a fixed order: repeated calls give identical bits. */
air_status air_noise_var(air_ctx *ctx, const air_const *c, const void *Y_dev,
                         const uint32_t *tx_dev, int64_t N, air_prec prec, double *var_dev);

/* air_llr and air_mi_gmi with the receiver's Gaussian metric of noise
 * variance sigma2_aux per real dimension (> 0, finite; a host value, for
 * example the isotropic estimate of air_noise_var) in place of the variance
 * that an SNR point implies. Arguments, layouts and errors as air_llr /
 * air_mi_gmi. */
air_status air_llr_aux(air_ctx *ctx, const air_const *c, const void *Y_dev, int64_t N,
                       double sigma2_aux, air_prec prec, void *llr_dev);
air_status air_mi_gmi_aux(air_ctx *ctx, const air_const *c, const void *Y_dev,
                          const uint32_t *tx_dev, int64_t N, double sigma2_aux, air_prec prec,
                          double *stats_dev, void *llr_dev);

/* The chain a receiver runs on measured data, in one call: the isotropic
 * noise-variance estimate of air_noise_var, then air_mi_gmi_aux with that
 * variance, then the NGMI of air_ngmi. Synchronises (the estimate is read
 * back to form the metric).
 *  var_host:   D + 1 doubles (host) receiving the estimates as air_noise_var
 *              writes them, or NULL.
 *  rates_host: 7 doubles (host): sigma2 (the isotropic estimate), MI, GMI,
 *              SE_MI, SE_GMI, NGMI, SE_NGMI.
 * AIR_E_RANGE, with NaN rates, if a tx index is >= M or the estimate is zero
 * (received points equal to the transmitted ones). */
air_status air_aux_rates(air_ctx *ctx, const air_const *c, const void *Y_dev,
                         const uint32_t *tx_dev, int64_t N, air_prec prec, double *var_host,
                         double *rates_host);

/* Normalised GMI of S points of statistics, host arithmetic on host arrays:
 * NGMI = 1 - (H(X) - GMI) / m with H(X) = m bits under the uniform prior over
 * M = 2^m points (so GMI / m), and its standard error SE_GMI / m.
 *  stats_host: S x 4 doubles as air_mi_gmi / air_sweep write them (MI, GMI,
 *              SE_MI, SE_GMI), copied to the host by the caller.
 *  ngmi_host:  S x 2 doubles: NGMI, SE_NGMI.
 * AIR_E_INVAL for null pointers, S < 1 or m < 1. */
air_status air_ngmi(const double *stats_host, int S, int m, double *ngmi_host);

/* ---------------------------------------------------------------------------
 * Max-log demapping, the usual receiver simplification of soft demapping:
 * each bit side's log-sum-exp is replaced by its largest term, so that
 *   L_k = min_{j: b_k(j)=1} |y - x_j|^2 / (2 sigma^2)
 *       - min_{j: b_k(j)=0} |y - x_j|^2 / (2 sigma^2)   (nats),
 * with no exponentials or logarithms per point. Its GMI is the bit-metric
 * rate of a receiver that takes these LLRs as exact:
 *   GMI = m - mean_n sum_k log2(1 + exp(-(1 - 2 b_k(t_n)) L_nk)),
 * an achievable rate of that receiver (no more than the exact GMI). No
 * symbol-wise MI is defined: stats[0] (MI) and stats[2] (SE_MI) are NaN.
 * Precisions, layouts and errors as air_llr / air_mi_gmi / air_sweep.
 * ------------------------------------------------------------------------- */
air_status air_llr_maxlog(air_ctx *ctx, const air_const *c, const void *Y_dev, int64_t N,
                          double snr_db, air_prec prec, void *llr_dev);
air_status air_gmi_maxlog(air_ctx *ctx, const air_const *c, const void *Y_dev,
                          const uint32_t *tx_dev, int64_t N, double snr_db, air_prec prec,
                          double *stats_dev, void *llr_dev);
air_status air_sweep_maxlog(air_ctx *ctx, const air_const *c, const uint32_t *tx_dev,
                            const void *Z_dev, int64_t N, const double *snr_db_host, int S,
                            air_prec prec, double *stats_dev, void *llr_dev);

/* ---------------------------------------------------------------------------
 * Hard decisions. The paper's receiver demaps the hard decisions of its
 * equaliser and reports the Q-factor estimated from the bit error rate
 * against hard-decision FEC thresholds (Sections II and III). The decision is
 * the constellation point nearest to y in squared Euclidean distance, taken
 * in FP32 as the receiver processes its samples in 32-bit floating point:
 * acc = fma(y_d - x_d, y_d - x_d, acc) over d = 0..D-1 from 0, ties to the
 * lower label. A symbol error is a decided point other than the transmitted
 * one; its bit errors are the Hamming distance of the two labels.
 * BER = bit errors / (N m), SER = symbol errors / N.
 * ------------------------------------------------------------------------- */

/* Decisions for a received block Y (float, N x D, device).
 *  tx_dev:      N transmitted indices, or NULL (needed for counts_dev).
 *  decided_dev: N decided X rows (uint32), or NULL.
 *  counts_dev:  2 uint64: symbol errors, bit errors; or NULL. */
air_status air_hard_decide(air_ctx *ctx, const air_const *c, const float *Y_dev,
                           const uint32_t *tx_dev, int64_t N, uint32_t *decided_dev,
                           uint64_t *counts_dev);

/* Decisions over an SNR sweep, y = fma(sigma_s, z, x_t) in FP32 with sigma_s
 * the FP32 rounding of the SNR point's noise deviation.
 *  counts_dev:  S x 2 uint64 (symbol errors, bit errors per SNR point).
 *  decided_dev: S x N decided X rows, or NULL. */
air_status air_hard_sweep(air_ctx *ctx, const air_const *c, const uint32_t *tx_dev,
                          const float *Z_dev, int64_t N, const double *snr_db_host, int S,
                          uint64_t *counts_dev, uint32_t *decided_dev);

/* Q-factor in dB of a bit error rate: 20 log10(sqrt(2) erfcinv(2 BER)), the
 * Gaussian-tail conversion (the paper quotes Q estimated from the BER without
 * printing the conversion). NaN unless 0 < BER < 0.5. */
double air_q_factor_db(double ber);

/* BER, SER and Q-factor of S points of hard-decision error counts, host
 * arithmetic on host arrays (the paper evaluates every format by its
 * Q-factor estimated from the BER; Sections II and III).
 *  counts_host: S x 2 uint64 as air_hard_sweep writes them (symbol errors,
 *               bit errors), copied to the host by the caller.
 *  N, m:        symbols per SNR point and bits per symbol.
 *  rates_host:  S x 3 doubles: BER = bit errors / (N m), SER = symbol
 *               errors / N, Q_dB = air_q_factor_db(BER) (NaN unless
 *               0 < BER < 0.5).
 * AIR_E_INVAL for null pointers, S < 1, N < 1 or m < 1. */
air_status air_hd_rates(const uint64_t *counts_host, int S, int64_t N, int m, double *rates_host);

/* Hard-decision FEC pass/fail and net rate of S points of BERs against F
 * codes, host arithmetic on host arrays. The paper compares each format's
 * BER with the thresholds of a 6.7 % and a 20 % overhead hard-decision FEC
 * and plots the net throughput of the formats that meet one (Section III);
 * it prints neither the threshold BERs nor the net-rate formula, so the
 * codes are the caller's and the readings are:
 *  - a code of overhead OH (a fraction, e.g. 0.067) and threshold BER th is
 *    met when BER <= th (a NaN BER meets none);
 *  - the code carries m / (1 + OH) information bits per symbol (code rate
 *    1 / (1 + OH));
 *  - the net rate is the largest of those over the codes met, times
 *    symbol_rate (symbols per second, or 1 for bits per symbol), and 0 when
 *    no code is met; ties keep the code listed first.
 *  ber_host:   BER of point s at ber_host[s * stride] (stride 3 reads the BER
 *              column of air_hd_rates' output).
 *  overhead, threshold: F doubles each (>= 0, overhead finite).
 *  pass_host:  S x F int32 (1 met, 0 not), or NULL.
 *  net_host:   S doubles, or NULL.
 *  code_host:  S int32: the code that gives the net rate, -1 for none; or NULL.
 * AIR_E_INVAL for null inputs, stride < 1, S < 1, m < 1, F < 1, a negative
 * or non-finite overhead, a negative or NaN threshold, or a negative or
 * non-finite symbol_rate. */
air_status air_fec_net(const double *ber_host, int64_t stride, int S, int m, const double *overhead,
                       const double *threshold, int F, double symbol_rate, int32_t *pass_host,
                       double *net_host, int32_t *code_host);

/* ---------------------------------------------------------------------------
 * Per-buffer streaming from host memory. The paper's receiver moves buffers
 * of samples to the GPU by DMA, runs each buffer on its own stream and writes
 * the demapped results back to host memory; it is real time because buffers
 * are processed faster than they arrive (Section II). A pipe runs each pushed
 * buffer as H2D copy (the slot's stream) -> the air_llr kernels (the
 * context's stream) -> D2H copy of the LLRs (the slot's stream); with
 * `depth` slots the copies of one buffer overlap the kernels of another.
 * Kernels of different buffers run in push order on the context's stream,
 * and each buffer's LLRs are bitwise those of air_llr on the same data.
 * ------------------------------------------------------------------------- */
typedef struct air_pipe air_pipe;

/* Create a pipe for buffers of at most max_symbols received symbols of the
 * constellation c, demapped at precision prec (LLRs as air_llr).
 * depth: 2..8 slots. Allocates, per slot, device buffers for one input and
 * one LLR buffer and the same in pinned host staging. The pipe must be
 * destroyed before its context; c must outlive every push. */
air_status air_pipe_create(air_ctx *ctx, const air_const *c, int64_t max_symbols, int depth,
                           air_prec prec, air_pipe **out);

/* Queue one buffer: Y_host is N x D received symbols, llr_host receives N x m
 * LLRs (nats), both host memory (double for AIR_FP64, else float); 1 <= N <=
 * max_symbols. Pinned buffers (hipHostMalloc) are copied directly; pageable
 * ones through the pipe's staging: Y_host is then read before the call
 * returns. Returns once the buffer is queued; the oldest slot is waited for
 * first when all are busy. llr_host (and a pinned Y_host) must stay valid
 * and untouched until air_pipe_wait returns. */
air_status air_pipe_push(air_pipe *p, const void *Y_host, int64_t N, double snr_db, void *llr_host);

/* Wait until every pushed buffer's LLRs are in their host buffers; then
 * air_sync on the context (reports its errors). */
air_status air_pipe_wait(air_pipe *p);

/* Release a pipe. Waits for its queued work; the LLRs of buffers pushed since
 * the last air_pipe_wait are then not delivered to pageable llr_host buffers
 * (pinned ones receive them). NULL is ignored. */
void air_pipe_destroy(air_pipe *p);

/* ---------------------------------------------------------------------------
 * Serving loop. Demapping jobs of uneven size (constellation, N, SNR) arrive
 * at any time, the way a software receiver hands over one buffer after
 * another (the paper streams buffers of samples to the GPU and gives each
 * buffer its own stream, trading buffer size against latency; Section II).
 * A server owns one device arena of a fixed byte budget, allocated at
 * creation, and a worker thread that
 *  - admits jobs in arrival order while their footprint fits in the arena
 *    and fewer than max_inflight jobs are admitted or running; the footprint
 *    is the job's staged inputs (host Y / Z and tx), staged LLRs (host llr),
 *    and its per-item FP64 partial sums and tile lists;
 *  - batches whatever is admitted when one of its launch slots (one stream
 *    each) is free, and runs the batch: input copies, the batched
 *    matrix-core kernels (one launch per kernel class of jobs), a
 *    fixed-order reduction per job, result copies;
 *  - stamps completion when the batch's event has completed and queues the
 *    results for air_server_poll.
 * Each job's reduction order is fixed by the job alone, so its statistics
 * and LLRs are bitwise the same whether it runs alone or in any mix.
 * Jobs use the matrix-core forms (AIR_FP16X3, AIR_BF16X3) with M >= 16.
 * A server must be destroyed before its context; a job's constellation and
 * buffers must stay valid until its result has been polled.
 * ------------------------------------------------------------------------- */
typedef struct air_server air_server;

typedef struct {
  const air_const *c;    /* constellation (created on the server's context) */
  const float *in;       /* N x D float: received points y, or unit noise z if noise_in;
                            device memory of the context, or host memory (pinned
                            memory copies asynchronously; pageable memory works) */
  const uint32_t *tx;    /* N transmitted indices (device or host), or NULL: LLRs
                            only, the statistics are NaN */
  int64_t N;             /* samples, >= 1 */
  double snr_db;
  int32_t noise_in;      /* 1: in holds z and y = x_tx + sigma z is formed on the device */
  int32_t prec;          /* air_prec: AIR_FP16X3 or AIR_BF16X3 */
  float *llr;            /* N x m LLRs (nats): device or host memory, or NULL */
  uint64_t t_arrival_ns; /* arrival time on the steady clock (CLOCK_MONOTONIC);
                            0 = stamped at submission */
  uint64_t tag;          /* caller's value, returned with the result */
} air_job;

typedef struct {
  uint64_t id, tag;
  int32_t status;        /* air_status: AIR_OK; AIR_E_RANGE (a tx index >= M was seen:
                            statistics NaN, LLRs of those samples NaN); AIR_E_DEVICE */
  int32_t pad;
  double mi, gmi, se_mi, se_gmi;   /* bits per symbol, as air_mi_gmi */
  uint64_t recomputed;   /* samples finished by the second tier or the exact path */
  uint64_t t_arrival_ns, t_admit_ns, t_launch_ns, t_done_ns;   /* steady clock */
  uint64_t footprint;    /* arena bytes the job held from admission to completion */
} air_result;

typedef struct {
  uint64_t submitted, completed, batches;
  uint64_t in_use, peak_in_use, budget;   /* arena bytes */
  int32_t max_batch;     /* most jobs in one launch so far */
  int32_t queued;        /* jobs waiting for admission */
} air_server_info;

/* Create a server on ctx's device with an arena of hbm_budget_bytes (>= 4096)
 * and at most max_inflight (>= 1) jobs admitted or running at a time. */
air_status air_server_create(air_ctx *ctx, size_t hbm_budget_bytes, int max_inflight,
                             air_server **out);

/* Queue one job; *id_out receives its id (> 0). Returns at once: the job
 * waits for admission inside the server. AIR_E_NOMEM if its footprint alone
 * exceeds the budget, AIR_E_UNSUPPORTED for a precision or M the serving
 * kernels do not cover, AIR_E_INVAL for invalid fields, AIR_E_DEVICE after a
 * device failure of the server, AIR_E_BUSY while it shuts down. The message
 * is in air_server_last_error (one submitting thread at a time). */
air_status air_server_submit(air_server *s, const air_job *job, uint64_t *id_out);

/* Move up to max finished results into out (completion order); returns how
 * many, or a negative air_status for invalid arguments. Never blocks. */
int air_server_poll(air_server *s, air_result *out, int max);

/* Wait until every submitted job has finished (timeout_ms < 0: no limit).
 * AIR_E_BUSY on timeout; AIR_E_DEVICE if the server failed. */
air_status air_server_drain(air_server *s, int timeout_ms);

/* Counters of the server (see air_server_info). */
air_status air_server_query(air_server *s, air_server_info *info);

/* Message of the last failed submission ("" if none). Owned by the server. */
const char *air_server_last_error(const air_server *s);

/* Finish every submitted job, stop the worker and release the arena and
 * streams. Results not yet polled are discarded. Returns AIR_E_DEVICE if the
 * server had failed on the device (its unfinished jobs are then dropped),
 * else AIR_OK; AIR_E_INVAL for NULL. */
air_status air_server_destroy(air_server *s);

#ifdef __cplusplus
}
#endif
#endif /* LIBAIR_AIR_H */
