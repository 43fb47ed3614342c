/*
 * gbs_lhaf.h -- C ABI of the MI355X (gfx950) loop-hafnian library.
 *
 * The library evaluates the loop hafnian of a complex symmetric matrix by the
 * power-trace subset sum that Quesada et al., "Quadratic speedup for simulating
 * Gaussian boson sampling" (arXiv:2010.15595, "the paper") benchmark in Sec. IV,
 * and the pure-state photon-number probability of Sec. II, Eq. (12), built on
 * it.  All arithmetic runs in HIP kernels on the GPU; the host code only
 * validates, expands photon patterns, factorises the 2M x 2M matrix Q and
 * assembles the final probability.
 *
 * Conventions
 *   - Complex numbers are gbs_z {re, im}: the layout of C99 double _Complex,
 *     std::complex<double> and torch.complex128.
 *   - Matrices are row-major with an explicit leading dimension (in elements).
 *   - Host-pointer entry points are synchronous.  Device-pointer entry points
 *     are ordered on the HIP stream passed in (NULL = the null stream) and
 *     return before the GPU work finishes.
 *   - The return code is the only error channel.  On error, outputs are left
 *     untouched and gbs_last_error() returns a thread-local description.
 *   - The caller owns every buffer it passes.  The library owns per-device
 *     workspace, created by gbs_init() and released by gbs_finalize().
 *   - lhaf(0 x 0) = 1.  An odd dimension is padded with one vertex that has
 *     loop weight 1 and no edges (the value is unchanged).  Pairs of the
 *     subset sum are (i, i + n), n = ceil(N / 2).
 *   - Largest supported dimension after expansion: GBS_MAX_DIM for single
 *     evaluations, GBS_MAX_BATCH_DIM for batch plans and the sampling chain.
 */
#ifndef GBS_LHAF_H
#define GBS_LHAF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GBS_MAX_DIM 64
/* Batch plans and the sampling chain run only the register-tile kernels, whose
 * largest tile holds a 56 x 56 subset matrix without register spills. */
#define GBS_MAX_BATCH_DIM 56
/* Size of the fixed per-device scratch array of gbs_lhaf_device_noalloc. */
#define GBS_NOALLOC_SCRATCH_BYTES (32 << 20)
/* Largest number of shards of gbs_lhaf_device_shard. */
#define GBS_MAX_SHARDS 65536

typedef struct { double re, im; } gbs_z;

typedef enum {
    GBS_OK = 0,
    GBS_E_ARG = -1,           /* null pointer, negative size, bad enum, bad leading dimension */
    GBS_E_NOT_SYMMETRIC = -2, /* |A_ij - A_ji| > 1e-12 * max|A| */
    GBS_E_NONFINITE = -3,     /* NaN or Inf in an input */
    GBS_E_TOO_LARGE = -4,     /* expanded dimension > GBS_MAX_DIM, or batch too large */
    GBS_E_NOT_PURE = -5,      /* Q does not describe a pure state (probability only) */
    GBS_E_NOT_PD = -6,        /* Q singular or not Hermitian positive definite */
    GBS_E_DEVICE = -7,        /* no usable GPU, or a HIP call failed */
    GBS_E_NOMEM = -8,         /* device or host allocation failed */
    GBS_E_UNSUPPORTED = -9    /* valid request the library does not implement */
} gbs_status;

typedef enum {
    GBS_FP64 = 0,      /* all steps in IEEE binary64 */
    GBS_FP32_COMP = 1, /* Hessenberg reduction and all cross-lane / final sums in
                          binary64; La Budde, power-trace series and the per-lane
                          compensated (TwoSum) sums in complex binary32 */
    GBS_DD = 2,        /* every step of every subset term and every sum in
                          double-double (~106-bit significand; the paper's CPU
                          code uses x87 long double, 64 bits): single
                          evaluations with N <= 56 only (GBS_E_TOO_LARGE above,
                          GBS_E_UNSUPPORTED for batch plans and the sampler).
                          The result is hi + lo: out receives hi, and
                          gbs_diag.lhaf_lo the low part */
    GBS_PRECISION_MAX_ENUM = 0x7FFFFFFF /* not a precision: makes every non-negative
                          int32 value representable, so an unknown value is
                          rejected (GBS_E_ARG) rather than undefined */
} gbs_precision;

/* Optional diagnostics of one loop-hafnian evaluation. */
typedef struct {
    double abs_sum;        /* sum over subsets of |t_S|                         */
    double kappa;          /* abs_sum / |lhaf| (cancellation ratio; inf if 0)   */
    uint64_t subset_terms; /* 2^n                                               */
    double kernel_ms;      /* GPU time of the subset sum (HIP events)           */
    int32_t n_pairs;       /* n                                                 */
    int32_t launches;      /* kernel launches issued                            */
    gbs_z lhaf_lo;         /* GBS_DD: low part of the result (lhaf = out + lhaf_lo);
                              0 for the other precisions                         */
} gbs_diag;

/* ---- library lifetime ---------------------------------------------------- */

/* Select `device` (HIP ordinal) and create its workspace.  Idempotent per
 * device.  Returns GBS_E_DEVICE when no GPU is visible. */
gbs_status gbs_init(int device);
/* Release all device workspace created by gbs_init.  Safe to call twice. */
void gbs_finalize(void);
const char *gbs_status_string(gbs_status status);
/* Thread-local detail for the last failing call on this thread ("" if none). */
const char *gbs_last_error(void);
int32_t gbs_max_dim(void);

/* ---- host helpers (no GPU needed) ---------------------------------------- */

/* Pattern expansion, Sec. II (text after Eqs. (7) and (11)): row/column i of B
 * (M x M, leading dim ldb) repeated mult[i] times, dropped when mult[i] = 0,
 * then the main diagonal replaced by gamma repeated the same way (filldiag).
 * gamma NULL keeps B's diagonal; mult NULL means all ones.  Writes the
 * N x N result (N = sum mult) row-major into out (capacity out_cap elements)
 * and N into *N_out.  B must be symmetric. */
gbs_status gbs_expand(const gbs_z *B, int32_t M, int64_t ldb, const gbs_z *gamma,
                      const int32_t *mult, gbs_z *out, int64_t out_cap, int32_t *N_out);

/* Pure-state parameters from Q = Sigma + I/2 (2M x 2M, Eq. (3)) and the mean
 * vector alpha = [a; conj(a)] (2M, Eq. (8)):
 *   B      = (X (I - Q^-1))[:M, :M]                 (Eq. (4); A = B (+) conj(B))
 *   gamma  = (Q^-1 alpha)[M:] = conj(a) - B a       (Eq. (9), see note)
 *   p_vac  = exp(-alpha^H Q^-1 alpha / 2) / sqrt(det Q)   (Eq. (10))
 * Note: Eq. (9) printed with this block order pairs the loop weights with
 * conj(B); the half used here is the one that pairs with B, which is what a
 * Fock-space computation of the same state confirms.  Any of B_out, gamma_out,
 * p_vac_out may be NULL.  Errors: GBS_E_NOT_PD for singular / non-positive Q,
 * GBS_E_NOT_PURE when A is not of the form B (+) conj(B) to 1e-10. */
gbs_status gbs_pure_state(const gbs_z *Q, const gbs_z *alpha, int32_t M, gbs_z *B_out,
                          gbs_z *gamma_out, double *p_vac_out);

/* ---- single evaluations, host pointers, synchronous ---------------------- */

/* lhaf(filldiag(A_S, gamma_S)) for the expansion described at gbs_expand.
 * A: M x M symmetric, leading dim lda.  *out receives the loop hafnian.
 * diag may be NULL. */
gbs_status gbs_lhaf(const gbs_z *A, int32_t M, int64_t lda, const gbs_z *gamma,
                    const int32_t *mult, gbs_precision prec, gbs_z *out, gbs_diag *diag);

/* haf(A) (Eq. (6)) of an N x N symmetric matrix: the loop hafnian of A with a
 * zero diagonal.  Odd N gives 0. */
gbs_status gbs_haf(const gbs_z *A, int32_t N, int64_t lda, gbs_precision prec, gbs_z *out,
                   gbs_diag *diag);

/* Characteristic-polynomial method of the reference kernels. */
typedef enum {
    GBS_CHARPOLY_LABUDDE = 0, /* La Budde over the Hessenberg form (the paper's method, Sec. IV) */
    GBS_CHARPOLY_EIGEN = 1,   /* eigenvalues of the Hessenberg form by the single-shift complex QR
                                 algorithm, multiplied out: the diagonalisation the paper compares
                                 La Budde with (Sec. IV) */
    GBS_CHARPOLY_MAX_ENUM = 0x7FFFFFFF /* not a method (see GBS_PRECISION_MAX_ENUM) */
} gbs_charpoly;

/* lhaf of an N x N symmetric matrix A (leading dim lda, diagonal = loop weights)
 * on the LDS-resident reference kernels (one workgroup per subset, the same
 * formulation as gbs_lhaf) with the characteristic polynomials from `method`:
 * for comparing the two methods in one framework.  prec GBS_FP64 (either
 * method, N <= 64) or GBS_DD (La Budde only, N <= 56; diag->lhaf_lo holds the
 * low part); GBS_E_UNSUPPORTED otherwise.  GBS_E_NONFINITE when a subset's QR
 * iteration needs more than 30 sweeps for one eigenvalue.  Host pointers;
 * synchronous; diag may be NULL. */
gbs_status gbs_lhaf_method(const gbs_z *A, int32_t N, int64_t lda, gbs_precision prec, gbs_charpoly method,
                           gbs_z *out, gbs_diag *diag);

/* Pure-state photon-number probability, Eq. (12):
 *   p(S) = p(vac) |lhaf(filldiag(B_S, gamma_S))|^2 / prod_i s_i!
 * Q: 2M x 2M (row-major, dense), alpha: 2M, pattern: M photon counts >= 0.
 * lhaf_out and diag may be NULL. */
gbs_status gbs_probability(const gbs_z *Q, const gbs_z *alpha, const int32_t *pattern,
                           int32_t M, gbs_precision prec, double *p_out, gbs_z *lhaf_out,
                           gbs_diag *diag);

/* Photon-number probability of a general (mixed) Gaussian state, Eq. (11):
 *   p(S) = p(vac) lhaf(filldiag(A_S, gamma_S)) / prod_i s_i!,   A = X (I - Q^-1) (Eq. (4)),
 * where A_S repeats rows/columns i and i + M s_i times (a 2N x 2N matrix for N photons,
 * so N <= GBS_MAX_DIM / 2) and the loop weight of index k is entry X(k) of Q^-1 alpha
 * (X swaps the two halves: the weights that pair with each block of A; for a pure state
 * this reduces to Eq. (12)).  Q: 2M x 2M Hermitian positive definite of the form
 * [[K, L], [conj(L), conj(K)]] (GBS_E_ARG otherwise); alpha: 2M of the form [a; conj(a)]
 * or NULL (no displacement); pattern: M counts >= 0 (GBS_E_TOO_LARGE above 32 photons).
 * p_out receives the real part (the loop hafnian of a valid state is real and >= 0;
 * lhaf_out, nullable, returns it unrounded).  Host pointers; synchronous. */
gbs_status gbs_probability_mixed(const gbs_z *Q, const gbs_z *alpha, const int32_t *pattern,
                                 int32_t M, gbs_precision prec, double *p_out, gbs_z *lhaf_out,
                                 gbs_diag *diag);

/* Signed subset terms t_S of the power-trace sum for an explicit list of pair
 * subsets (bit i of masks[j] set = pair (i, i+n) kept).  A: N x N, its diagonal
 * holds the loop weights.  terms_out[j] receives t_S; sum over all 2^n masks
 * gives lhaf(A).  Host pointers, synchronous.  Diagnostic / parity use. */
gbs_status gbs_lhaf_terms(const gbs_z *A, int32_t N, int64_t lda, const uint64_t *masks,
                          int64_t count, gbs_precision prec, gbs_z *terms_out);

/* ---- device-resident evaluation, stream-ordered -------------------------- */

/* lhaf of the N x N row-major matrix A_dev (device memory, diagonal = loop
 * weights, leading dim N).  Writes the result to out_dev[0] and, when
 * abs_sum_dev is non-NULL, sum_S |t_S| to abs_sum_dev[0] (device memory).
 * Symmetry is not checked here (the caller owns the device data).  Ordered on
 * `stream` (a hipStream_t, NULL = null stream); asynchronous. */
gbs_status gbs_lhaf_device(const gbs_z *A_dev, int32_t N, gbs_precision prec, gbs_z *out_dev,
                           double *abs_sum_dev, void *stream);

/* One GPU's share of the subset sum, for splitting one loop hafnian over
 * several GPUs: the power-trace sum is a sum of independent subset terms
 * (Sec. IV), so shard g of G takes colex ranks [C_s g / G, C_s (g + 1) / G) of
 * every size class s (C_s = C(n, s), integer division); the G shards cover
 * every subset once and take the same share of every class.  Writes the
 * shard's compensated partial sum, five doubles, to partial_dev[0..4] (device
 * memory): (sum re, compensation re, sum im, compensation im, sum |t_S|).
 * gbs_combine_partials folds the G records into the loop hafnian.  A, N and
 * stream as in gbs_lhaf_device (asynchronous, ordered on `stream`); GBS_FP64
 * or GBS_FP32_COMP (GBS_E_UNSUPPORTED for GBS_DD); 0 <= shard < nshards <=
 * GBS_MAX_SHARDS (GBS_E_ARG otherwise).  N = 0 puts its single term, 1, in
 * shard 0.  With nshards = 1 the combined result is bitwise that of
 * gbs_lhaf_device; with more, it agrees to rounding (the terms are grouped
 * differently). */
gbs_status gbs_lhaf_device_shard(const gbs_z *A_dev, int32_t N, gbs_precision prec, int32_t shard,
                                 int32_t nshards, double *partial_dev, void *stream);

/* Folds `count` partial records of gbs_lhaf_device_shard (host memory, five
 * doubles each, in shard order) with TwoSum in index order: out = the loop
 * hafnian, abs_sum (nullable) = sum_S |t_S|.  count >= 1 (GBS_E_ARG
 * otherwise).  Host only; the same merge as the device reductions. */
gbs_status gbs_combine_partials(const double *partials, int32_t count, gbs_z *out, double *abs_sum);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * loop hafnian as gbs_lhaf_device (same arguments, device pointers, ordered on
 * `stream`, asynchronous) with no allocation, no freeing and no autotuning in
 * the call.  Every buffer beyond the caller's input and outputs lives in one
 * fixed device array of GBS_NOALLOC_SCRATCH_BYTES (32 MiB) per device, which
 * the library holds until the process ends; it keeps the last call's
 * contents, and every value a call reads from it is written by that call
 * first.  gbs_init(device) must have been called for the current device
 * (GBS_E_ARG otherwise).  N <= GBS_MAX_DIM (GBS_E_TOO_LARGE above);
 * GBS_FP64 or GBS_FP32_COMP (GBS_E_UNSUPPORTED for GBS_DD).  Lane grids are
 * those of earlier tuning or gbs_set_layout, else the defaults.  All calls on
 * one device share the array: calls that overlap in time on one GPU (on
 * different streams, or from several threads with their streams running
 * concurrently) race and give wrong results.  The result agrees with
 * gbs_lhaf_device to rounding: the sum is folded per chunk of subsets, a
 * different order of the same compensated additions. */
gbs_status gbs_lhaf_device_noalloc(const gbs_z *A_dev, int32_t N, gbs_precision prec, gbs_z *out_dev,
                                   double *abs_sum_dev, void *stream);

/* ---- batches of loop hafnians: plan once, replay many times -------------- */

typedef struct gbs_plan gbs_plan;

typedef struct {
    int32_t items;           /* loop hafnians per run                             */
    int32_t tiles;           /* work tiles (runs of subsets of one size class)    */
    int32_t rounds;          /* rounds over the two coefficient buffers           */
    int32_t kernel_nodes;    /* kernel launches captured in the graph             */
    int64_t subset_terms;    /* sum over items of 2^n_i                           */
    int64_t tile_subsets;    /* subsets per tile (autotuned or default)           */
    int64_t workspace_bytes; /* device memory owned by the plan                   */
    double yardstick_flops;  /* flop yardstick of one run (gbs_yardstick_flops)   */
    double tune_ms;          /* time of the fastest tile size when autotuned     */
} gbs_batch_info;

#define GBS_PLAN_AUTOTUNE 1

/* Plans a batch of `count` loop hafnians of dimensions dims[i] <= GBS_MAX_BATCH_DIM
 * (the conditional-sampling chain of the paper's Sec. III produces such
 * batches: many loop hafnians of uneven size).  The input of a run is the
 * packed concatenation of the matrices: item i is an N_i x N_i row-major
 * block (diagonal = loop weights) at element offset sum_{j<i} N_j^2.  The plan
 * splits every item's subset sum into tiles (runs of subsets of one size
 * class), processes them with persistent per-subset kernels that take tiles
 * largest first from a device counter, then the series kernels and a
 * fixed-order compensated reduction per item; the whole schedule is captured
 * once into a HIP graph.  Tiles hold 256 subsets; flags = GBS_PLAN_AUTOTUNE
 * instead times the lane grid of every n in the batch and candidate tile sizes
 * (64, 128, 256, 1024, 4096, ... subsets in turn, one replay each, until one
 * is slower than the best) on the device and keeps the fastest.  Owns its device workspace (including its own copies of the
 * library's binomial and lane-map tables, so it stays valid across
 * gbs_finalize / gbs_init) until gbs_batch_plan_destroy.  GBS_E_TOO_LARGE
 * when an item exceeds GBS_MAX_BATCH_DIM. */
gbs_status gbs_batch_plan_create(const int32_t *dims, int32_t count, gbs_precision prec, int32_t flags,
                                 gbs_plan **plan);
gbs_status gbs_batch_plan_info(const gbs_plan *plan, gbs_batch_info *info);
/* Runs the plan: mats_dev packed inputs (device memory), out_dev[count]
 * results and abs_sum_dev[count] (sum_S |t_S|, nullable), both device memory.
 * Ordered on `stream` (hipStream_t, NULL = null stream); asynchronous.  Runs
 * of one plan must not overlap. */
gbs_status gbs_batch_run(gbs_plan *plan, const gbs_z *mats_dev, gbs_z *out_dev, double *abs_sum_dev,
                         void *stream);
void gbs_batch_plan_destroy(gbs_plan *plan);

/* ---- conditional sampling chain ------------------------------------------ */

typedef struct {
    int64_t loop_hafnians; /* loop hafnians evaluated: nsamples * M * (cutoff + 1)     */
    int64_t subset_terms;  /* sum over them of 2^n                                      */
    int32_t max_dim;       /* largest loop-hafnian dimension met                        */
    int32_t groups;        /* lockstep groups of samples (up to 8192 samples each)      */
    double setup_ms;       /* host conditioning of the covariance, once per call        */
    double total_ms;       /* wall time of the call                                     */
} gbs_sample_info;

/* Photon-number samples of a pure Gaussian state by the algorithm of Sec. III:
 * heterodyne outcomes beta_2..beta_M are drawn from the Husimi distribution
 * (mean and augmented covariance: alpha and Q of those modes); then for
 * k = 1..M the photon number of mode k is drawn from the probabilities
 * (Eq. (12)) of the patterns (s_1, .., s_{k-1}, j), j = 0..cutoff, of the pure
 * state of modes 1..k conditioned on beta_{k+1}..beta_M (Gaussian conditioning,
 * Sec. II), normalised over j.
 * Q (2M x 2M) and alpha (2M) as for gbs_probability; M <= 128.  All randomness
 * is passed in, row-major per sample:
 *   normals  (nsamples x 2(M-1)): x = m + L z with z these normals, L the lower
 *            Cholesky factor and m the mean of x = (Re beta_2..Re beta_M,
 *            Im beta_2..Im beta_M); NULL allowed when M = 1;
 *   uniforms (nsamples x M) in [0, 1): s_k = #{j : cdf_j <= u_k}, at most
 *            cutoff, with cdf_j the running sum of the normalised probabilities.
 * samples_out (nsamples x M) receives the patterns; probs_out (nullable,
 * nsamples x M x (cutoff + 1)) the normalised conditional probabilities each
 * draw used.  Every loop hafnian runs on the GPU; GBS_E_TOO_LARGE when a
 * sample's photons so far plus cutoff exceed GBS_MAX_BATCH_DIM (never when
 * M * cutoff <= GBS_MAX_BATCH_DIM), GBS_E_NONFINITE when a step's probabilities are
 * not finite or all zero.  Host pointers; synchronous.  info may be NULL. */
gbs_status gbs_sample_pure(const gbs_z *Q, const gbs_z *alpha, int32_t M, int32_t cutoff,
                           const double *normals, const double *uniforms, int32_t nsamples,
                           gbs_precision prec, int32_t *samples_out, double *probs_out,
                           gbs_sample_info *info);

/* ---- kernel layout selection and autotuning ------------------------------ */

/* Lane grid of the per-subset kernel (rows x columns of lanes per subset). */
typedef enum {
    GBS_LAYOUT_DEFAULT = -1, /* heuristic, or the autotuned choice when one exists */
    GBS_LAYOUT_4x4 = 0,      /* 16 lanes per subset, 4 subsets per wavefront, m <= 24 */
    GBS_LAYOUT_8x4 = 1,      /* 32 lanes per subset, 2 subsets per wavefront, m <= 40 */
    GBS_LAYOUT_8x8 = 2,      /* 64 lanes per subset, m <= 56 (larger subsets of a
                                single evaluation run on an LDS-resident FP64 kernel) */
    GBS_LAYOUT_8x4_ONE_TEAM = 3 /* 8x4 grid, one 64-lane La Budde team serving both subsets
                                   in turn (half the LDS of two 32-lane teams), m <= 40 */
} gbs_layout;

/* Use `layout` for subsets of size s (m = 2s vertices) whenever the loop
 * hafnian has n pairs; n = 0 applies to every n, s = 0 to every size the
 * grid can hold (other sizes keep their setting).  GBS_LAYOUT_DEFAULT clears
 * the setting.  GBS_E_ARG if s > 0 and the grid cannot hold m x m.  Affects
 * the current device. */
gbs_status gbs_set_layout(int32_t n, int32_t s, int32_t layout);

typedef struct {
    int32_t n;
    int32_t layout[33];           /* chosen grid per subset size s = 1..n    */
    double ns_per_subset[33][4];  /* measured time per subset, 0 = not valid */
} gbs_tune_report;

/* Project autotuner: for every subset size s of an n-pair loop hafnian, times
 * each valid lane grid on a sample of that size class (HIP events, synthetic
 * matrix; the work is data-independent) and keeps the fastest for the current
 * device (report->ns_per_subset holds those single-evaluation timings).
 * Batch plans use the fastest grid other than GBS_LAYOUT_8x4_ONE_TEAM
 * (measured slower when many launches share the device), timed in the form
 * batch tiles run: the subset block at tile offset 0.  GBS_FP32_COMP
 * evaluations run GBS_LAYOUT_8x4 where GBS_LAYOUT_8x4_ONE_TEAM was chosen.
 * With GBS_AUTOTUNE_CACHE=<path> in the environment the choices are
 * appended to / read from that file; GBS_AUTOTUNE_LAYOUTS=<bit mask of
 * gbs_layout values> restricts the candidates.  report may be NULL. */
gbs_status gbs_autotune(int32_t n, gbs_tune_report *report);

/* ---- diagnostics --------------------------------------------------------- */

/* Per-kernel timing of the subset-sum kernels, measured with HIP events
 * recorded on the launch stream around every launch while enabled.  While
 * enabled, the launches that otherwise overlap run one at a time: the size
 * classes of a single loop hafnian on the caller's stream, gbs_batch_run
 * issues its captured schedule eagerly with every branch on the caller's
 * stream, and so do the per-step batches of gbs_sample_pure; each duration is
 * that of the kernel alone on the device. */
typedef struct {
    double charpoly_ms;        /* summed durations of the per-subset kernels (Hessenberg + La Budde) */
    double series_ms;          /* summed durations of the per-subset series kernels                 */
    double reduce_ms;          /* summed durations of the final reductions                          */
    int64_t charpoly_launches;
    int64_t series_launches;
    int64_t reduce_launches;
    double charpoly_flops;     /* algorithmic flops of the profiled subsets (see gbs_yardstick_flops) */
    double subset_terms;       /* subsets processed by the profiled launches                        */
    char dominant_kernel[96];  /* per-subset kernel instance with the largest summed duration    */
    double dominant_ms;        /* its summed duration                                           */
    double dominant_flops;     /* its algorithmic flops (yardstick of its subsets)             */
    int64_t dominant_launches; /* its launches                                                  */
} gbs_profile;

/* on = 1 clears the counters and starts recording; on = 0 stops recording. */
gbs_status gbs_profile_enable(int on);
/* Waits for the recorded events, writes the totals since the last enable or
 * read into *out and clears them. */
gbs_status gbs_profile_read(gbs_profile *out);
/* Algorithmic real-flop count of the subset sum of an N x N loop hafnian:
 * sum over subset sizes s of C(n, s) [(40/3) m^3 + (4/3) m^3 + 8 min(n-1, m-1) m^2],
 * m = 2s -- Householder Hessenberg reduction, characteristic polynomial and the
 * loop-term mat-vecs of the power-trace method, one complex FMA = 8 flops. */
double gbs_yardstick_flops(int32_t N);

/* Runs the device self-check of the wavefront cross-lane sums, broadcasts and
 * lane shifts the kernels rely on, against host arithmetic.  *failures
 * receives the number of mismatching lanes (0 = pass). */
gbs_status gbs_selftest(int32_t *failures);

#ifdef __cplusplus
}
#endif

#endif /* GBS_LHAF_H */
