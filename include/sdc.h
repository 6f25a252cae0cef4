/*
 * sdc.h -- C ABI of the fused, binned spin pair-correlation library (gfx950).
 *
 * The library computes, on one AMD Instinct MI355X, the space- and
 * time-displaced spin pair correlation
 *
 *     C(b, t) = < S_i(t0) . S_j(t0 + t) >   over ordered pairs (i, j) in bin b
 *
 * (Eq. (4) of arXiv 2308.07487 without the mean subtraction, summed over the
 * components alpha as in Eq. (3), averaged over time origins t0 of one
 * trajectory instead of Monte Carlo realizations), binned by the displacement
 * of site j (at the later time) relative to site i (at the origin).  Each lag
 * is the dense product of the N x 3*n_origins spin matrices (Sec. 3.2); the
 * bin key and the histogram are fused into the product's epilogue so the
 * N x N result never reaches memory (Sec. 3.3-3.4, Fig. 2, Eq. (6)).
 *
 * Conventions for every entry point:
 *  - Return codes only; nothing throws or aborts across this ABI.
 *  - Argument and state errors are detected before any GPU work is queued.
 *  - GPU failures map to SDC_ERR_HIP; faults of queued work surface at the
 *    next synchronising call (sdc_finalize, sdc_plan_raw).
 *  - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *  - A plan is not thread-safe; distinct plans are independent.
 *  - sdc_last_error() returns a thread-local description of the last failure.
 */
#ifndef SDC_H
#define SDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SDC_OK = 0,
    SDC_ERR_INVALID_ARG = 1,  /* a pointer, size or spec field is invalid     */
    SDC_ERR_STATE = 2,        /* call not allowed in the plan's current state */
    SDC_ERR_OOM = 3,          /* host or device allocation failed             */
    SDC_ERR_HIP = 4,          /* a HIP runtime call or kernel launch failed   */
    SDC_ERR_UNSUPPORTED = 5,  /* valid request outside what the library does */
    SDC_ERR_NO_DEVICE = 6     /* no usable gfx950 device                      */
} sdc_status;

/* Contraction precision of the per-lag product.  Accumulation is always
 * FP32 inside the matrix cores, the per-workgroup histograms and the global
 * bins are FP64.
 *  FP32        : plain FP32 MFMA (v_mfma_f32_32x32x2_f32).
 *  SPLIT_BF16  : x = hi + lo, hi = bf16(x), lo = bf16(x - hi); the product is
 *                hi*hi + hi*lo + lo*hi on BF16 MFMA (three products).
 *  SPLIT_FP16  : the same split with FP16 parts (about 22 significant bits).
 *  BF16X3      : x = hi + mid + lo in BF16 (exact for normal fp32 x); the
 *                product keeps hi*hi, hi*mid, mid*hi, mid*mid, hi*lo, lo*hi
 *                (six BF16 MFMA products, about 2^-24 of |x||y| left out),
 *                which reaches FP32-level accuracy on BF16 matrix cores.
 *  For the reduced forms the omitted products (lo*lo; for BF16X3 mid*lo +
 *  lo*mid + lo*lo) are added exactly (FP64) for the i = j pairs, where they
 *  would otherwise bias C at zero displacement; off the diagonal they are
 *  left out (rounding noise, <= 2^-16 (BF16), 2^-22 (FP16) or 2^-23 (BF16X3)
 *  of |S_i||S_j| per term). */
typedef enum {
    SDC_PREC_FP32 = 0,
    SDC_PREC_SPLIT_BF16 = 1,
    SDC_PREC_SPLIT_FP16 = 2,
    SDC_PREC_BF16X3 = 3
} sdc_precision;

/* Bin kinds.
 *  PERIODIC_SC  : simple-cubic lattice, lattice constant 1, cells[0..2] cells
 *                 per axis, one site per cell at the integer point.  Bin =
 *                 displacement (r_j - r_i) mod cells, index
 *                 b = (kx*cells[1] + ky)*cells[2] + kz; n_bins = N.
 *  PERIODIC_BCC : body-centred cubic, sites n and n + (1/2,1/2,1/2).  Bin =
 *                 (k, p) with k = (n_j - n_i - [beta_j < beta_i](1,1,1)) mod
 *                 cells and p = (beta_j - beta_i) mod 2; b = 2*sc_index(k) + p;
 *                 n_bins = N = 2*cells^3.
 *  RADIAL       : arbitrary positions, no periodicity.  n_shells shells of
 *                 width w = r_max / n_shells.  d2 = ((dx*dx + dy*dy) + dz*dz)
 *                 in FP32 with dx = fp32(x_j - x_i), no fused multiply-add;
 *                 shell = largest k with E2[k] <= d2, E2[k] = fp32((k*w)^2)
 *                 evaluated in FP64 and rounded; distances beyond the last
 *                 edge fall in the last shell. */
typedef enum {
    SDC_BINS_PERIODIC_SC = 0,
    SDC_BINS_PERIODIC_BCC = 1,
    SDC_BINS_RADIAL = 2
} sdc_bin_kind;

typedef struct {
    int32_t kind;      /* sdc_bin_kind                                      */
    int32_t cells[3];  /* periodic kinds: cells per axis (each >= 1)        */
    int32_t n_shells;  /* radial: number of shells, 1..1024                 */
    float r_max;       /* radial: outer edge of the last shell, > 0         */
} sdc_bin_spec;

typedef struct {
    int32_t n_origins;     /* time origins per accumulate call, >= 1         */
    int32_t n_lags;        /* lags 0..n_lags-1, in frames, >= 1              */
    int32_t origin_stride; /* frames between origins s, >= 1 (origin o uses  */
                           /* frame o*s; lag t pairs it with frame o*s + t)  */
    int32_t precision;     /* sdc_precision                                  */
    int32_t flags;         /* SDC_FLAG_TIMING | SDC_FLAG_CONNECTED |
                              SDC_FLAG_NO_KEY_TABLE | SDC_FLAG_DETERMINISTIC */
} sdc_corr_spec;

/* flags: record HIP events around each kernel of sdc_accumulate (on the
 * caller's stream) so sdc_plan_timings can report per-kernel durations. */
#define SDC_FLAG_TIMING 1
/* flags: connected correlation, Eq. (4) with its second term: every
 * accumulate subtracts the product of the per-site averages over its own
 * origins, H[t][b] += sum_o (S_i(o s) - <S_i>).S_j(o s + t) with
 * <S_i> = (1/n_origins) sum_o S_i(o s) -- the covariance form of Eq. (5),
 * which needs the centring on the origin side only (the centred values sum
 * to zero over the origins).  The self term and the site sum (C_sum) are
 * connected the same way. */
#define SDC_FLAG_CONNECTED 2
/* flags: radial bins only.  By default a plan stores the shell of every
 * ordered pair (2 bytes per pair slot, 8 KiB per pair of 64-point tiles,
 * 8.6 GB for 65536 points) when that is at most 32 GiB and a quarter of the
 * free device memory, computed once at creation; the fused epilogue then
 * reads it instead of recomputing distances for every lag group.  This flag
 * keeps the on-the-fly computation (no table). */
#define SDC_FLAG_NO_KEY_TABLE 4
/* flags: deterministic results.  Every sum that several threads add into
 * (the per-task histograms, the global bins, the self sums) is kept as a
 * 64-bit two's-complement fixed-point number with 2^-20 resolution, so the
 * integer atomics give bit-identical bins, self sums and outputs whatever the
 * order of the adds; each added value is rounded once to 2^-20 (about 1e-6
 * absolute, far below the FP32 product's own rounding for |G| > 1).  Range:
 * |H[t][b]| < 2^43 (8.8e12) over all accumulates.  The FP64 views are
 * refreshed by sdc_finalize, sdc_plan_raw and sdc_plan_structure_factor. */
#define SDC_FLAG_DETERMINISTIC 8

/* Schedules of the fused product (Sec. 3.3-3.4: how the per-lag product
 * and its epilogue are laid out on the matrix cores).  Every schedule forms
 * the same products in the same precision; results differ only by the order
 * of the FP32/FP64 roundings.  In every schedule the small products of the
 * reduced-precision forms (hi*lo, lo*hi; for BF16X3 all but hi*hi) are never
 * added to a sum that already holds the large ones: there their lowest bits
 * would be dropped by the matrix cores' alignment, always downwards, a bias
 * of a fraction of the last place per element and K-step. */
typedef enum {
    SDC_SCHED_DEFAULT = 0,  /* tuning entry for the plan's size class, else the library default */
    SDC_SCHED_ONE_PASS = 1, /* one K loop per tile pair, second accumulator set for the small
                               products; one workgroup per compute unit.  Every precision. */
    SDC_SCHED_TWO_PASS = 2, /* SPLIT_BF16 / SPLIT_FP16 only: per tile pair a K loop over
                               hi*lo + lo*hi, then one adding hi*hi to those sums, in one
                               accumulator set; two workgroups per compute unit. */
    SDC_SCHED_LAG_SPLIT = 3,/* one K loop, second accumulator set as ONE_PASS, but workgroups
                               of eight waves: two waves per 32x32 quadrant, each with half
                               of the lags; two waves per SIMD.  Every precision. */
    SDC_SCHED_FOLD = 4      /* reduced forms only: one K loop; per K-step the small products
                               are summed from zero in a transient tile and added to the
                               large sums with FP32 vector adds (round to nearest); one
                               accumulator set, two workgroups per compute unit. */
} sdc_schedule;

/* Tuning of a plan: what the autotuner (sdc_autotune) chooses per size
 * class.  Zero fields mean "default". */
typedef struct {
    int32_t schedule;      /* sdc_schedule                                     */
    int32_t segment_pairs; /* tile pairs per fused task (pairs that share one  */
                           /* LDS histogram; one merge into the global bins    */
                           /* per task): 0 = default (periodic kinds 96,       */
                           /* radial all pairs of an i-tile), else [1, 2^20]   */
} sdc_tuning;

typedef struct sdc_plan sdc_plan;

/*
 * Create a plan for one sample (Sec. 3.2: the spin matrices; Sec. 3.4 and
 * Eq. (6): values computed from positions inside the epilogue).
 *  positions_host : [n_sites][3] fp32, host, copied; periodic kinds need
 *                   lattice points within 1e-3 (bcc: 2r within 2e-3) with
 *                   every site of the box exactly once.
 *  device         : HIP device ordinal; the plan's memory lives there.
 *  out            : receives the plan (owned by the library until destroy).
 * Builds the tile layout, copies tables to the device and computes the exact
 * per-bin pair counts (integer kernel), synchronously.
 * Errors: INVALID_ARG (bad pointer/spec/positions), UNSUPPORTED, OOM,
 *         NO_DEVICE, HIP.
 */
sdc_status sdc_plan_create(const float* positions_host, int64_t n_sites,
                           const sdc_bin_spec* bins, const sdc_corr_spec* corr,
                           int device, sdc_plan** out);

/*
 * sdc_plan_create with an explicit tuning.  tuning == NULL, or zero fields,
 * take the entry for the plan's size class from the tuning file named by the
 * environment variable SDC_TUNING_FILE (written by sdc_autotune; key: device
 * architecture, bin kind, floor(2 log2 n_sites), K-steps ceil(3 ceil(n_origins
 * / 8) / 2), precision), else the library defaults (TWO_PASS for the hi/lo
 * splits, ONE_PASS otherwise; default segments).  sdc_plan_create(...) is
 * sdc_plan_create_tuned(..., NULL, ...).  A missing or unreadable tuning file
 * counts as empty.
 * Errors: as sdc_plan_create; INVALID_ARG for an unknown schedule or a
 * segment length out of range, UNSUPPORTED for a schedule the precision does
 * not have.
 */
sdc_status sdc_plan_create_tuned(const float* positions_host, int64_t n_sites,
                                 const sdc_bin_spec* bins, const sdc_corr_spec* corr,
                                 const sdc_tuning* tuning, int device, sdc_plan** out);

/* The tuning a plan runs with (fields resolved, never 0).
 * Errors: INVALID_ARG. */
sdc_status sdc_plan_get_tuning(const sdc_plan* plan, sdc_tuning* tuning);

/*
 * Autotuner: for one sample shape, times candidate tunings on the device
 * and returns the fastest.  Each candidate gets its own plan and runs one
 * warm-up and three timed accumulates (HIP events around the fused launch)
 * over the first min(n_lags, max_lags) lags (max_lags <= 0: all lags) on
 * seeded uniform unit spins.  The winner: of the candidates whose median is
 * within 0.5% of the smallest (ties within the timing noise), the one with
 * the longest segment (fewest histogram merges), then the smallest median.
 *  candidates   : n_candidates tunings with every field set, or NULL for the
 *                 built-in list (sdc_autotune_candidates: every schedule the
 *                 precision has x segment lengths {16, 32, 48, 96, 192} for
 *                 periodic kinds, {64, 256, all} for radial).
 *  cache_path   : JSON tuning file; when not NULL the winner is written under
 *                 the plan's size-class key with every candidate's time
 *                 (other entries are kept; the file is replaced atomically),
 *                 for sdc_plan_create to pick up via SDC_TUNING_FILE.
 *  best         : receives the winner;  best_ms : its median fused time
 *                 (milliseconds), or NULL;  candidate_ms : [n] medians of all
 *                 candidates in order, or NULL.
 * Synchronous; allocates and frees its own plans and spins.  With the
 * environment variable SDC_TUNE_VERBOSE set (and not "0") every candidate's
 * median is also printed to stderr as it is measured.
 * Errors: as sdc_plan_create; HIP; INVALID_ARG for a candidate with a zero
 * field or a file that cannot be written.
 */
sdc_status sdc_autotune(const float* positions_host, int64_t n_sites, const sdc_bin_spec* bins,
                        const sdc_corr_spec* corr, int device, int32_t max_lags,
                        const sdc_tuning* candidates, int32_t n_candidates, const char* cache_path,
                        sdc_tuning* best, double* best_ms, double* candidate_ms);

/* The built-in candidate list of sdc_autotune for a sample shape: *n_out
 * candidates, the first max_out of them written to out (out may be NULL when
 * max_out is 0).  Host only.  Errors: INVALID_ARG. */
sdc_status sdc_autotune_candidates(const sdc_bin_spec* bins, const sdc_corr_spec* corr,
                                   sdc_tuning* out, int32_t max_out, int32_t* n_out);

/* The tuning-file entry for a sample shape: *found = 1 and *tuning set if
 * cache_path holds one, else *found = 0.  Host only, except that the device's
 * architecture name is part of the key.  Errors: INVALID_ARG, NO_DEVICE. */
sdc_status sdc_tuning_lookup(const char* cache_path, int64_t n_sites, const sdc_bin_spec* bins,
                             const sdc_corr_spec* corr, int device, sdc_tuning* tuning,
                             int32_t* found);

/* Number of bins of the plan.  Errors: INVALID_ARG. */
sdc_status sdc_plan_n_bins(const sdc_plan* plan, int64_t* n_bins);

/*
 * Add one trajectory's contribution (Eq. (4) unsubtracted, Eq. (3) alpha sum,
 * averaged over origins; the GEMM of Sec. 3.2 with the fused epilogue of
 * Sec. 3.3-3.4).  For every selected lag t and origin o < n_origins:
 *     H[t][key(i,j)] += S_i(o*s) . S_j(o*s + t)   for all ordered pairs.
 *  spins_dev  : [n_frames][n_sites][3] fp32 in device memory of the plan's
 *               device, site order as in positions_host; read-only; must stay
 *               valid until the stream reaches this work.
 *  n_frames   : >= (n_origins - 1)*s + max_selected_lag + 1.
 *  lags_host  : host array of n_lags_sel distinct lags in [0, n_lags), or
 *               NULL for all lags (then n_lags_sel is ignored).
 *  stream     : hipStream_t; everything is queued on it, nothing waits.
 * Repeated calls add; the per-lag origin totals add too (they are kept on
 * the device, so replays of a captured call count their origins).  Graph-
 * capturable once the lag selection has been used in an uncaptured call
 * (its first use uploads the selection's tables).
 * Errors: INVALID_ARG, STATE (plan failed earlier), HIP.
 */
sdc_status sdc_accumulate(sdc_plan* plan, const float* spins_dev, int64_t n_frames,
                          const int32_t* lags_host, int32_t n_lags_sel, void* stream);

/*
 * Normalise and transform (Sec. 2.2: temporal transform with a window;
 * Sec. 1: summing the correlation over all sites), in FP64 on the GPU, then
 * copy to host buffers and synchronise the stream.  Any output may be NULL.
 *  C_host      : [n_lags][n_bins]  H / (n_org[t] * count[b]), 0 if either is 0
 *  counts_host : [n_bins] exact ordered-pair counts (uint64)
 *  Csum_host   : [n_lags]  sum_b H[t][b] / (N * n_org[t]), evaluated as
 *                sum_o M(o s).M(o s + t) / (N * n_org[t]) with M(f) = sum_i
 *                S_i(f) in FP64 (the same quantity, an exact identity; it
 *                keeps the per-pair rounding of the split products from
 *                adding up over the N^2 pairs of the site sum)
 *  Cself_host  : [n_lags]  sum_o sum_i S_i(o s).S_i(o s + t) / (N * n_org[t])
 *  Ssum_host   : [n_lags][2] (re, im) of sum_t w_t Csum(t) exp(-2 pi i k t / n_lags)
 *  Sself_host  : [n_lags][2] same for Cself; w_t = (1 + cos(pi t / n_lags)) / 2
 * May be called repeatedly; it does not reset the accumulation.
 * Errors: INVALID_ARG, STATE, HIP (including faults of earlier queued work).
 */
sdc_status sdc_finalize(sdc_plan* plan, double* C_host, uint64_t* counts_host,
                        double* Csum_host, double* Cself_host, double* Ssum_host,
                        double* Sself_host, void* stream);

/*
 * Dynamic structure factor of Eq. (3) from the accumulated bins of a
 * periodic plan (sc or bcc), on the GPU in FP64, then the windowed time
 * transform of Sec. 2.2 (the window of sdc_finalize):
 *     S(q, t) = (1 / (N n_org[t])) sum_b exp(-i q.d_b) H[t][b],
 * d_b the displacement of bin b (bcc: plus half a cell on every axis for
 * the odd parity), q_a = 2 pi m_a / L_a with integer m (the wave vectors
 * commensurate with the box; for these the bins give Eq. (3) exactly).
 *  m_host   : [n_q][3] int32, |m| <= 2^20, host.
 *  Sqt_host : [n_q][n_lags][2] (re, im) or NULL.
 *  Sqw_host : [n_q][n_lags][2] (re, im) of sum_t w_t S(q,t) e^{-2 pi i k t/n_lags},
 *             or NULL (not both NULL).
 * Accuracy: every bin carries the contraction's rounding.  Near q = 0 the
 * sum runs over all N^2 pair elements, where unbiased rounding cancels and a
 * one-signed residual does not: the reduced-precision forms keep one of at
 * most 3e-10 (split-BF16, BF16x3) or 1e-9 (split-FP16) of the absolute pair
 * mass sum_o A(o) A(o + t), A = sum_i |S_i| (the matrix cores' alignment of
 * the products inside one instruction; measured 4.4e-11, 2.1e-11 and
 * 2.7e-10 on a 36^3 antiferromagnet), FP32 below 1e-10.
 * Synchronises the stream; allocates and frees its own scratch.
 * Errors: INVALID_ARG, UNSUPPORTED (radial plan), STATE, OOM, HIP.
 */
sdc_status sdc_plan_structure_factor(sdc_plan* plan, const int32_t* m_host, int32_t n_q,
                                     double* Sqt_host, double* Sqw_host, void* stream);

/*
 * sdc_plan_structure_factor for callers that cannot allocate device memory
 * (serving loops, harnesses that forbid hipMalloc/hipFree): the same
 * computation and the same results, with its scratch (the wave-vector
 * indices and both outputs before the copy to the host) in a fixed 16 MiB
 * device array per GPU instead of per-call allocations.  Limit: 12 n_q +
 * 32 n_q n_lags bytes <= 16 MiB (e.g. 1024 wave vectors x 256 lags);
 * larger requests return UNSUPPORTED before any GPU work.  Calls no
 * hipMalloc, hipFree or allocating library routine (the array's device
 * address is looked up once per device on the first call there).  Every
 * call on one GPU uses the same array: calls that overlap in time on one GPU
 * (from several host threads, or streams) race; calls in turn are safe
 * (each synchronises the stream before it returns, and every output element
 * is rewritten by each call).
 * Errors: as sdc_plan_structure_factor (UNSUPPORTED also for the size
 * limit).
 */
sdc_status sdc_plan_structure_factor_static(sdc_plan* plan, const int32_t* m_host, int32_t n_q,
                                            double* Sqt_host, double* Sqw_host, void* stream);

/*
 * Raw accumulated state (for exact comparisons and checkpointing): H
 * [n_lags][n_bins] FP64, per-lag origin totals [n_lags] FP64, raw self sums
 * [n_lags] FP64, raw site sums sum_o M.M [n_lags] FP64.  Any output may be
 * NULL.  Synchronises the stream.  Errors: INVALID_ARG, STATE, HIP.
 */
sdc_status sdc_plan_raw(sdc_plan* plan, double* H_host, double* n_org_host,
                        double* self_host, double* msum_host, void* stream);

/* Replace the accumulated state with one saved by sdc_plan_raw (resume).
 * Synchronises the stream.  Errors: INVALID_ARG, STATE, HIP. */
sdc_status sdc_plan_load_raw(sdc_plan* plan, const double* H_host,
                             const double* n_org_host, const double* self_host,
                             const double* msum_host, void* stream);

/* Per-kernel durations (milliseconds) of the most recent sdc_accumulate of a
 * plan created with SDC_FLAG_TIMING: ms[0] pack, ms[1] self term, ms[2] fused
 * product + epilogue.  Waits for those events.  Errors: INVALID_ARG, STATE
 * (no timed accumulate yet or flag not set), HIP. */
sdc_status sdc_plan_timings(sdc_plan* plan, double* ms);

/* Zero the accumulated state (counts are kept).  Queued on the stream. */
sdc_status sdc_plan_reset(sdc_plan* plan, void* stream);

/* Free the plan and its device memory (waits for the device).  NULL is a
 * no-op.  The pointer is invalid afterwards.  Errors: STATE if a batch still
 * holds the plan (destroy the batch first). */
sdc_status sdc_plan_destroy(sdc_plan* plan);

typedef struct sdc_batch sdc_batch;

/*
 * Group plans of several samples (the paper averages over many independent
 * realizations, Sec. 2.2 and Sec. 4) so that one accumulate runs all their
 * fused work as a single persistent launch: workgroups take (plan, stream,
 * lag group) tasks from per-XCD queues until all are done.
 *  plans   : n_plans distinct plans on one device, same precision, all
 *            periodic or all radial; each keeps its own bins, counts and
 *            origin totals.  Every lag of every plan is accumulated.
 *  flags   : 0 or SDC_FLAG_TIMING (HIP events around the pack/self kernels
 *            and around the fused launch, read by sdc_batch_timings; a
 *            timing batch is meant for eager calls, not for capture).
 *  out     : receives the batch; it refers to the plans, which must outlive
 *            it (sdc_plan_destroy refuses a plan still in a batch).
 * Uploads the per-plan kernel arguments once.  Errors: INVALID_ARG,
 * UNSUPPORTED (more than 2^30 tasks), STATE (a plan failed earlier), OOM,
 * HIP.
 */
sdc_status sdc_batch_create(sdc_plan* const* plans, int32_t n_plans, int32_t flags, sdc_batch** out);

/*
 * Accumulate one trajectory per plan, all lags (as sdc_accumulate with
 * lags_host = NULL on each plan), with one fused launch for the batch.
 *  spins_dev : host array of n_plans device pointers, [n_frames[k]][N_k][3]
 *              fp32 each, read-only until the stream reaches this work.
 *  n_frames  : host array of n_plans frame counts, each large enough for
 *              its plan's origins and lags.
 * Queued on the stream, no allocation and no host synchronisation: graph-
 * capturable (the queue counters are cleared by a kernel, not a memset).
 * Calls on one batch must not overlap in time.
 * Errors: INVALID_ARG, STATE, HIP (then every plan of the batch is marked
 * failed).
 */
sdc_status sdc_batch_accumulate(sdc_batch* batch, const float* const* spins_dev,
                                const int64_t* n_frames, void* stream);

/* Durations (milliseconds) of the most recent sdc_batch_accumulate of a
 * batch created with SDC_FLAG_TIMING: ms[0] the pack and self kernels of all
 * plans, ms[1] the persistent fused launch.  Waits for those events.
 * Errors: INVALID_ARG, STATE (flag not set or no accumulate yet), HIP. */
sdc_status sdc_batch_timings(sdc_batch* batch, double* ms);

/* sdc_batch_create with the schedule of its one launch given: tuning->schedule
 * (segment_pairs is ignored: each plan keeps its own layout).  tuning == NULL
 * or SDC_SCHED_DEFAULT takes the schedule that the plans' own tunings give
 * the most work (sum of n_sites^2 * n_lags * n_origins).  The launch's task
 * list takes the plans in order of decreasing task length (K-steps times tile
 * pairs per task).  Errors: as sdc_batch_create; INVALID_ARG for an unknown
 * schedule, UNSUPPORTED for one the precision does not have. */
sdc_status sdc_batch_create_tuned(sdc_plan* const* plans, int32_t n_plans, int32_t flags,
                                  const sdc_tuning* tuning, sdc_batch** out);

/* Total fused tasks of the batch and the persistent grid (workgroups).
 * Either output may be NULL.  Errors: INVALID_ARG. */
sdc_status sdc_batch_info(const sdc_batch* batch, int64_t* n_tasks, int32_t* grid);

/* Schedule (sdc_schedule, never DEFAULT) of the batch's launch.
 * Errors: INVALID_ARG. */
sdc_status sdc_batch_schedule(const sdc_batch* batch, int32_t* schedule);

/* Free the batch (waits for the device); its plans stay valid.  NULL is a
 * no-op. */
sdc_status sdc_batch_destroy(sdc_batch* batch);

/* ---------------------------------------------------------------------- */
/* q-resolved dynamic structure factor at arbitrary wave vectors          */
/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t n_origins;     /* time origins per accumulate call, [1, 4096]    */
    int32_t n_lags;        /* lags 0..n_lags-1 in frames, [1, 1024]           */
    int32_t origin_stride; /* frames between origins s, [1, 64]               */
    int32_t flags;         /* SDC_FLAG_TIMING | SDC_FLAG_CONNECTED            */
} sdc_sq_spec;

typedef struct sdc_sq sdc_sq;

/*
 * Create an accumulator of Eq. (3) at a list of arbitrary wave vectors for
 * any point set (periodic or not; no binning, no periodic image):
 *     S(q, t) = (1 / (N n_org)) sum_o sum_{i,j} exp(-i q.(r_j - r_i))
 *               S_i(o s) . S_j(o s + t),
 * site j at the later time, r the given positions.  This is the quantity
 * the paper's fused kernel evaluates with the on-the-fly Q of Eq. (6)
 * (Sec. 3.4); here the phase is split per site, exp(-i q.(r_j - r_i)) =
 * conj(e_i) e_j, so each accumulate is one FP64 matrix-core contraction of
 * the [n_q x N] phases with the [N x 3T] spins followed by a correlation
 * over the origins, O(n_q N T) instead of O(n_q N^2 T) work.  Everything is
 * FP64 after the fp32 inputs (phases q.r and sin/cos in FP64).
 *  positions_host : [n_sites][3] fp32, host, copied; finite.
 *  q_host         : [n_q][3] FP64 wave vectors (radians per unit length),
 *                   host, copied; finite.  1 <= n_q <= 65536.  The phases
 *                   must stay below 2^20 rad: max_q |q|_1 times the largest
 *                   |coordinate| < 2^20 (else UNSUPPORTED).
 *  spec           : origins, lags, stride as in sdc_corr_spec; flags
 *                   SDC_FLAG_CONNECTED subtracts the second term of Eq. (4)
 *                   per pair (the product of the per-site averages over each
 *                   call's origins), SDC_FLAG_TIMING records HIP events.
 *  device         : HIP device ordinal.
 * Allocates all device memory the accumulator needs: the spins packed in
 * FP64 by chunks of 24 sites (24 bytes per site and frame), the per-site-
 * range partial transforms (at most 1 GiB) and the [n_q][3T] transform.
 * Errors: INVALID_ARG, UNSUPPORTED, OOM, NO_DEVICE, HIP.
 */
sdc_status sdc_sq_create(const float* positions_host, int64_t n_sites, const double* q_host, int32_t n_q,
                         const sdc_sq_spec* spec, int device, sdc_sq** out);

/*
 * Add one trajectory: spins_dev [n_frames][n_sites][3] fp32 device memory
 * (site order of positions_host), n_frames >= (n_origins - 1) s + n_lags,
 * read-only until the stream reaches this work.  Queued on the stream with
 * no allocation, memset or host synchronisation, so it can be captured into
 * a graph (the origin total is counted on the device: each replay counts);
 * deterministic (no atomics: the partial transforms of the site ranges are
 * summed in a fixed order).
 * Calls on one accumulator must not overlap in time.
 * Errors: INVALID_ARG, STATE, HIP.
 */
sdc_status sdc_sq_accumulate(sdc_sq* sq, const float* spins_dev, int64_t n_frames, void* stream);

/*
 * Sqt_host : [n_q][n_lags][2] (re, im) of S(q, t) over all accumulated
 *            origins, or NULL.
 * Sqw_host : [n_q][n_lags][2] windowed time transform
 *            sum_t w_t S(q, t) exp(-2 pi i k t / n_lags),
 *            w_t = (1 + cos(pi t / n_lags)) / 2, or NULL.
 * Synchronises the stream; does not reset.  Errors: INVALID_ARG, STATE, HIP.
 */
sdc_status sdc_sq_finalize(sdc_sq* sq, double* Sqt_host, double* Sqw_host, void* stream);

/* Durations (milliseconds) of the most recent accumulate of an accumulator
 * created with SDC_FLAG_TIMING: ms[0] the FP64 site-chunk packing of the
 * frames, ms[1] the phase contraction kernel, ms[2] the sum of its site
 * ranges and the correlation over origins.  Waits for those events.
 * Errors: INVALID_ARG, STATE, HIP. */
sdc_status sdc_sq_timings(sdc_sq* sq, double* ms);

/* Zero the accumulated sums and origin total.  Queued on the stream. */
sdc_status sdc_sq_reset(sdc_sq* sq, void* stream);

/* Free the accumulator (waits for the device).  NULL is a no-op. */
sdc_status sdc_sq_destroy(sdc_sq* sq);

/* ---------------------------------------------------------------------- */
/* Matrix-core measurements (the ceilings the fused product is held to)    */
/* ---------------------------------------------------------------------- */

typedef enum {
    SDC_MFMA_BF16 = 0,  /* v_mfma_f32_32x32x16_bf16 (split-BF16, BF16x3)     */
    SDC_MFMA_F16 = 1,   /* v_mfma_f32_32x32x16_f16  (split-FP16)             */
    SDC_MFMA_F32 = 2    /* v_mfma_f32_32x32x2_f32   (FP32)                   */
} sdc_mfma_form;

/*
 * Sustained matrix-core rate of the device on the form the fused product
 * uses, with nothing else in the loop: every wave keeps four independent
 * 32x32 accumulators and four operand sets in registers and issues
 * iterations x 16 MFMAs; workgroups of four waves, workgroups_per_cu (1 or
 * 2) per compute unit on every compute unit.  random_operands = 1 draws the
 * operands (Philox) with magnitudes in [2^-8, 1) and random signs and
 * mantissas, as spin data has; 0 uses the constant 0.5 (fewest toggling
 * bits, the highest clock the power limit allows).  One warm-up launch, then
 * one timed launch (HIP events).
 *  ms     : duration of the timed launch.   tflops : executed TFLOP/s.
 * Synchronous; allocates and frees a small output buffer.
 * Errors: INVALID_ARG, NO_DEVICE, OOM, HIP.
 */
sdc_status sdc_mfma_peak(int32_t form, int32_t random_operands, int64_t iterations,
                         int32_t workgroups_per_cu, int device, double* ms, double* tflops);

/*
 * One MFMA instruction of the given form on one wave, with element (0, 0)
 * of its 32x32 output set to c + sum_k a[k] b[k] (k < n_products; at most 16
 * for the 16-bit forms, 2 for FP32) and every other input zero: how the
 * matrix cores sum products into the accumulator, bit for bit.  a and b must
 * be exact in the form's input type (else INVALID_ARG).
 *  out : the FP32 result for element (0, 0).
 * Synchronous.  Errors: INVALID_ARG, NO_DEVICE, OOM, HIP.
 */
sdc_status sdc_mfma_probe(int32_t form, float c, const float* a, const float* b,
                          int32_t n_products, int device, float* out);

/* Static description of a status code. */
const char* sdc_status_string(sdc_status s);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* sdc_last_error(void);

/*
 * Host-only check of the tile layout (no device needed): the bin of every
 * ordered pair as the fused kernel's epilogue maps it (tile pair, window
 * coordinate, window-to-bin map), written to keys_out[i*n_sites + j].
 * Sizes up to n_sites = 4096.  Errors: INVALID_ARG, UNSUPPORTED, OOM.
 */
sdc_status sdc_layout_keys(const float* positions_host, int64_t n_sites,
                           const sdc_bin_spec* bins, int64_t* keys_out);

/* ---------------------------------------------------------------------- */
/* Trajectory generator: Landau-Lifshitz RK4 (Eq. (2), Sec. 3.1)           */
/* ---------------------------------------------------------------------- */

typedef enum {
    SDC_COUPLING_NN_UNIFORM = 0,   /* J on every nearest-neighbour bond      */
    SDC_COUPLING_NN_RANDOM_SIGN = 1, /* +-|J| per bond, Philox sign          */
    SDC_COUPLING_EXP_CUTOFF = 2    /* J*exp(-r) for d2 <= r_cut^2 (FP32 rule) */
} sdc_coupling;

typedef enum {
    SDC_INIT_UNIFORM = 0,      /* uniform unit vectors (Philox)               */
    SDC_INIT_PERTURBED_Z = 1,  /* z-aligned + Gaussian tangent of width sigma */
    SDC_INIT_GIVEN = 2         /* copy init_dev                               */
} sdc_init;

typedef struct {
    int32_t kind;       /* sdc_bin_kind of the positions: SC/BCC periodic     */
                        /* lattices (nearest neighbours) or RADIAL (open)     */
    int32_t cells[3];   /* periodic box                                       */
    int32_t coupling;   /* sdc_coupling                                       */
    float r_cut;        /* EXP_CUTOFF: cutoff radius                          */
    double J;           /* exchange; J > 0 antiferromagnetic (Eq. (1))        */
    double dt;          /* RK4 step; one frame per step                       */
    int32_t init;       /* sdc_init                                           */
    int32_t pad0;
    double sigma;       /* PERTURBED_Z tangent width (radians)                */
    uint64_t seed;      /* Philox4x32-10 key                                  */
    const float* init_dev; /* GIVEN: [n_sites][3] fp32 device memory          */
    double D;           /* DMI strength: D_ij = D (r_j - r_i)/|r_j - r_i|     */
                        /* (bulk form, minimal image on lattices), Eq. (1)    */
    double A;           /* single-ion anisotropy, -A sum_i (S_i^z)^2          */
    double Hz;          /* field along z, -H_z sum_i S_i^z                    */
} sdc_traj_spec;

/*
 * Integrate Eq. (2) with the Hamiltonian of Eq. (1),
 *     H = sum_<ij> [J_ij S_i.S_j - D_ij.(S_i x S_j)] - A sum_i (S_i^z)^2
 *         - H_z sum_i S_i^z,
 *     dS_i/dt = h_i x S_i,  h_i = sum_j (J_ij S_j + D_ij x S_j)
 *                                 - 2 A S_i^z z - H_z z,
 * (lattice bonds that close on the site itself, along an axis one cell
 * wide, are dropped) with classical RK4 (no renormalisation) in FP32 and
 * write frames
 * [n_frames][n_sites][3] fp32 into frames_dev (frame 0 = initial state,
 * frame f = after f steps).
 *  positions_host : [n_sites][3] fp32 host; neighbour bonds come from them.
 * Initial states: Philox4x32-10 with key = seed, counter = (site low 32 bits,
 * 0, site high 32 bits, 0); u = (word >> 8) * 2^-24; UNIFORM uses z = 2u0 - 1,
 * phi = 2 pi u1; PERTURBED_Z uses Box-Muller normals (g0, g1) from (u0, u1),
 * v = sigma (g0, g1), S = (sin|v| v/|v|, cos|v|).  Random bond signs use
 * counter (min(i,j), max(i,j), 1, 0): sign = -1 if the first word is odd.
 * Synchronises the stream before returning (host-built bond tables).
 * Errors: INVALID_ARG, UNSUPPORTED, OOM, HIP, NO_DEVICE.
 */
sdc_status sdc_traj_generate(const float* positions_host, int64_t n_sites,
                             const sdc_traj_spec* spec, float* frames_dev,
                             int64_t n_frames, int device, void* stream);

/* ---------------------------------------------------------------------- */
/* Thermalised starts: Metropolis Monte Carlo with simulated annealing     */
/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t kind;         /* as sdc_traj_spec: SC/BCC nearest neighbours or   */
    int32_t cells[3];     /* RADIAL with EXP_CUTOFF couplings                 */
    int32_t coupling;     /* sdc_coupling                                     */
    float r_cut;          /* EXP_CUTOFF: cutoff radius                        */
    double J, D, A, Hz;   /* Eq. (1): exchange, bulk DMI, anisotropy, field   */
    uint64_t seed;        /* Philox key of the moves (and of random bond signs) */
    double T_start;       /* annealing: T_k = T_start cool^k while T_k > T_end */
    double T_end;         /* then the final sweeps at T_end (> 0)             */
    double cool;          /* in (0, 1)                                        */
    int64_t sweeps_per_T; /* sweeps at each temperature of the ladder (>= 1)  */
    int64_t sweeps_final; /* sweeps at T_end (>= 0)                           */
    double cone0;         /* initial trial-cone half-angle, (0, pi]           */
    double acc_target;    /* acceptance-rate target of the adaptation, (0, 0.5] */
} sdc_mc_spec;

/* Number of sweeps of the spec's schedule (host only).  Errors: INVALID_ARG. */
sdc_status sdc_mc_n_sweeps(const sdc_mc_spec* spec, int64_t* n_sweeps);

/*
 * Thermalised spin configurations by Metropolis Monte Carlo (Sec. 2.1) with
 * simulated annealing (Sec. 4.3) on the Hamiltonian of Eq. (1), as starts
 * for sdc_traj_generate (SDC_INIT_GIVEN).  A sweep visits the colour
 * classes of a greedy colouring of the bond graph (each site takes the
 * smallest colour no lower-indexed neighbour has) in order, all sites of a
 * class in parallel.  Site i in sweep s draws one Philox4x32-10 block, key =
 * seed, counter = (i low, s low, i high, 2^31 | s high), u_k = (w_k + 1/2)
 * 2^-32: trial spin at cos a = 1 - u_0 (1 - cos cone) and azimuth 2 pi u_1
 * about S_i (frame e1 = normalised z - (z.S)S, or x when |S_z| >= 0.9,
 * e2 = S x e1), renormalised; accepted when dE <= 0 or u_2 < exp(-dE/T).
 * After each sweep, with rate = accepted / N: cone *= 0.9 (not below 1e-3)
 * if rate < acc_target, cone = min(pi, 1.1 cone) if rate > 2 acc_target.
 * The state is FP64 on the device.
 *  positions_host : [n_sites][3] fp32 (bonds as in sdc_traj_generate).
 *  init_dev       : [n_sites][3] fp32 device start (e.g. a one-frame
 *                   sdc_traj_generate with a Philox start).
 *  state_dev      : [n_sites][3] fp32 device output (may equal init_dev).
 *  accepted_host  : [sdc_mc_n_sweeps] accepted moves per sweep, or NULL.
 *  info_host      : [4] energy per site (Eq. (1)) of the final state, final
 *                   cone, last temperature, number of colour classes; or NULL.
 * Synchronises the stream (allocates and frees its own device memory).
 * Errors: INVALID_ARG, UNSUPPORTED, OOM, HIP, NO_DEVICE.
 */
sdc_status sdc_mc_anneal(const float* positions_host, int64_t n_sites, const sdc_mc_spec* spec,
                         const float* init_dev, float* state_dev, int64_t* accepted_host,
                         double* info_host, int device, void* stream);

typedef struct sdc_mc sdc_mc;

/* The same as a reusable object: sdc_mc_create builds the bonds, the colour
 * classes and the device state once (synchronously) for the model fields of
 * spec (kind .. Hz; seed only for random bond signs).  Errors: INVALID_ARG,
 * UNSUPPORTED, OOM, HIP, NO_DEVICE. */
sdc_status sdc_mc_create(const float* positions_host, int64_t n_sites, const sdc_mc_spec* spec,
                         int device, sdc_mc** out);

/* Run the schedule of `schedule` (seed, T_start .. acc_target; its model
 * fields are ignored) from init_dev ([n_sites][3] fp32 device), or, when
 * init_dev is NULL, from the FP64 state the previous run left; the final
 * state goes to state_dev as fp32.  Sweep indices (the Philox counter) start
 * at 0 in every run: use a new seed for an independent run.  Queued on the
 * stream without host synchronisation unless accepted_host or info_host
 * (as in sdc_mc_anneal) is requested.  Errors: INVALID_ARG, STATE (NULL
 * init_dev before any run), OOM, HIP. */
sdc_status sdc_mc_run(sdc_mc* mc, const sdc_mc_spec* schedule, const float* init_dev, float* state_dev,
                      int64_t* accepted_host, double* info_host, void* stream);

/* Duration (milliseconds) of the sweeps of the most recent run (HIP events
 * on its stream around the sweep kernels).  Waits for them.  Errors:
 * INVALID_ARG, STATE, HIP. */
sdc_status sdc_mc_timings(sdc_mc* mc, double* ms);

/* Which sweep kernel the object uses: *stencil = 1 when the neighbours
 * follow from lattice arithmetic (periodic sc box with even edges and a
 * uniform coupling, checked at create to reproduce the bond tables bit for
 * bit; the sweeps read 52 fewer bytes per update), 0 when they are read from
 * the bond tables.  Both give the same result.  Errors: INVALID_ARG. */
sdc_status sdc_mc_uses_stencil(const sdc_mc* mc, int32_t* stencil);

/* Free the object (waits for the device).  NULL is a no-op. */
sdc_status sdc_mc_destroy(sdc_mc* mc);

#ifdef __cplusplus
}
#endif

#endif /* SDC_H */
