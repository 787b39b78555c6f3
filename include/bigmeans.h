/*
 * bigmeans.h -- C ABI of the Big-means library for one AMD Instinct MI355X.
 *
 * Big-means (Mussabayev, Mladenovic, Mussabayev, Jarboui, "How to Use K-means
 * for Big Data Clustering?", Alg. 1 and Sec. 3) clusters n points in d
 * dimensions into k clusters by repeatedly drawing a uniform sample of s
 * points, reseeding the degenerate (empty) centroids of the best solution so
 * far with K-means++, running K-means (Lloyd) on the sample from there, and
 * keeping the result when its sample objective is lower.  A final pass assigns
 * every point to its nearest centroid and returns the objective of Eq. (1),
 * the sum of squared distances of points to their nearest centroids.
 *
 * Naming: n = number of points, d = number of features (the paper's m and n).
 *
 * Conventions shared by every entry point
 *   - All functions return a bm_status; BM_OK (0) on success, a negative code
 *     otherwise, with a message available from bm_last_error() (per thread).
 *     No exception or abort crosses this boundary.
 *   - Buffers named "device" are device pointers on the current HIP device
 *     (for example torch tensors' data_ptr()); "host" buffers are ordinary
 *     host memory.  The caller owns every buffer it passes.  The library owns
 *     only an internal scratch pool, kept between calls and released by
 *     bm_release_scratch().
 *   - Arrays are row-major: X is n x d, centroids are k x d FP32.  A degenerate
 *     centroid (Sec. 3.3: an empty cluster, or one never initialised) is
 *     reported with degenerate[j] = 1 and NaN coordinates, and receives no
 *     points.
 *   - Calls are synchronous with respect to the host: they enqueue on
 *     opt->stream (NULL = the null stream) and return when the results are
 *     ready.  Calls from several host threads must use distinct streams and
 *     are serialised on the scratch pool.
 *   - Random numbers come from the counter-based stream documented in
 *     bm_rng.h (Philox4x32-10 keyed by seed); the same (seed, sample index)
 *     always yields the same sample and the same K-means++ draws.
 */
#ifndef BIGMEANS_H
#define BIGMEANS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bm_status;

enum {
  BM_OK = 0,
  BM_EINVAL = -1,      /* invalid argument (sizes, null pointers, options) */
  BM_ENOMEM = -2,      /* device or host allocation failed                 */
  BM_EDEVICE = -3,     /* a HIP call or a kernel failed                    */
  BM_ENOTSUP = -4,     /* a valid request this library cannot serve        */
  BM_ECANCELLED = -5,  /* the work was cancelled                           */
  BM_ETIMEDOUT = -6    /* a wait ran out of time (the work goes on)        */
};

enum { BM_F32 = 0, BM_BF16 = 1 };               /* element type of X       */
enum { BM_STOP_SHIFT = 0, BM_STOP_REL_OBJ = 1 }; /* Lloyd stop rule         */
enum { BM_CMP_FOPT = 0, BM_CMP_RESAMPLE = 1 };   /* keep-the-best reference */
enum { BM_PREC_FP32 = 0, BM_PREC_BF16_MFMA = 1 }; /* distance arithmetic    */
enum { BM_INIT_KMEANSPP = 0, BM_INIT_FORGY = 1 };  /* (re)initialisation     */
enum { BM_FINAL_ASSIGN = 0, BM_FINAL_POLISH = 1 }; /* last step of a fit     */

#define BM_ABI_VERSION 2

/* Options.  Fill with bm_default_options(); fields are read only when
 * struct_size covers them, so callers built against an older header keep
 * working. */
typedef struct bm_options {
  uint32_t struct_size;   /* sizeof(bm_options)                                   */
  int32_t x_dtype;        /* BM_F32 (default) or BM_BF16 (uint16 bit patterns)    */
  int32_t max_iter;       /* Lloyd assign+update rounds per sample (default 100)  */
  double tol;             /* stop tolerance (default 1e-4)                        */
  int32_t stop_rule;      /* BM_STOP_SHIFT: stop when no centroid moves by tol    */
                          /* or more; BM_STOP_REL_OBJ: stop when the relative     */
                          /* decrease of the objective is <= tol (Sec. 5 rule)    */
  int32_t n_local_trials; /* K-means++ candidates per new centre (default 3,      */
                          /* Sec. 5); 1 is plain D^2 sampling                     */
  int32_t compare_rule;   /* BM_CMP_FOPT: replace the incumbent when f(C'',P) <   */
                          /* f_opt (Alg. 1); BM_CMP_RESAMPLE: when f(C'',P) <     */
                          /* f(C,P) of the incumbent on the new sample (Sec. 3.2) */
  int32_t precision;      /* BM_PREC_FP32 (default): FP32 direct differences.     */
                          /* BM_PREC_BF16_MFMA (X must be BM_BF16): the full-data */
                          /* assignment (kmeans_assign, the final pass of         */
                          /* bigmeans_fit) takes x.c on the matrix cores with the */
                          /* centroids split into two BF16 parts, and recomputes  */
                          /* on the FP32 path every point whose two best          */
                          /* candidates are within a proven error bound, so the   */
                          /* labels equal BM_PREC_FP32's; needs d <= 256, k <= 128 */
                          /* and the split centroids in LDS (else BM_ENOTSUP)     */
  void* stream;           /* hipStream_t to run on; NULL = null stream            */
  int32_t grid;           /* workgroups of the cooperative solver; 0 = automatic  */
  int32_t t_start;        /* index of the first sample (resume); default 0        */
  int32_t resume;         /* 1: centroids (device), degenerate (host) and         */
                          /* f_opt_in carry an incumbent into bigmeans_fit        */
  double f_opt_in;        /* incumbent objective when resume = 1                  */
  uint32_t spin_limit;    /* bound on a grid-barrier wait, in polls; 0 = default; */
                          /* a wait that exceeds it aborts the call (BM_EDEVICE)  */
  int32_t* sample_idx;    /* optional device out, n_samples x s sampled indices   */
  double* sample_f;       /* optional host out, n_samples objectives f(C'',P)     */
  /* --- ABI version 2 --- */
  int32_t init_method;    /* how degenerate centroids are (re)initialised on a    */
                          /* sample (Sec. 3.3 allows other strategies):           */
                          /* BM_INIT_KMEANSPP (default; Sec. 2, greedy with       */
                          /* n_local_trials candidates, Sec. 5) or BM_INIT_FORGY  */
                          /* (each takes a uniformly drawn sample row, draws from */
                          /* the K-means++ stream, independent per slot)          */
  int32_t final_mode;     /* bigmeans_fit's last step: BM_FINAL_ASSIGN (default,  */
                          /* Alg. 1: assign every point to the incumbent) or      */
                          /* BM_FINAL_POLISH (Sec. 3.4: K-means on all of X from  */
                          /* the incumbent, with this struct's stop rule,         */
                          /* tolerance and cap; then labels and sse belong to the */
                          /* polished centroids; FP32 X only, else BM_ENOTSUP)    */
  double time_budget_ms;  /* > 0: the stop condition of Sec. 5 -- the sample loop */
                          /* stops before the first sample that starts after this */
                          /* much device time (sample 0 always runs); n_samples   */
                          /* is then a cap; stats->samples tells how many ran.    */
                          /* Processing s samples gives exactly the result of a   */
                          /* run with n_samples = s.  0 (default): no budget      */
} bm_options;

/* Per-call counters (all optional; pass NULL). */
typedef struct bm_stats {
  uint32_t struct_size;   /* sizeof(bm_stats)                                     */
  int32_t samples;        /* samples processed                                    */
  int32_t replacements;   /* incumbent replacements (keep-the-best)               */
  int32_t grid;           /* workgroups the solver ran with                       */
  int64_t lloyd_iters;    /* assignment passes over samples inside K-means        */
  int64_t reseeded;       /* centroids placed by K-means++                        */
  int64_t n_d;            /* distance evaluations at sample level (Sec. 5's n_d)  */
  int64_t boundary_draws; /* D^2 draws that fell within rounding of a boundary of */
                          /* the running sum, retaken with row-order sums         */
  double f_opt;           /* objective of the incumbent on its own sample         */
  double ms_solver;       /* device time of the sample loop                       */
  double ms_final;        /* device time of the final assignment pass             */
  double ms_sampling;     /* share of ms_solver spent drawing and gathering samples */
  double ms_seeding;      /* ... in K-means++ reseeding                           */
  double ms_lloyd;        /* ... in K-means on the samples                        */
  double ms_lloyd_pass;   /* ... of which assignment passes (incl. their barrier) */
  double ms_lloyd_post;   /* ... of which reading the reductions + updating        */
  double ms_lloyd_wait;   /* ... of which waiting in the assignment-pass barrier  */
  int64_t rechecked;      /* final pass, BM_PREC_BF16_MFMA: points recomputed on  */
                          /* the FP32 path (near-ties)                            */
  /* --- ABI version 2 --- */
  int32_t final_passes;   /* BM_FINAL_POLISH: assignment passes over all of X     */
  int32_t pad_;
} bm_stats;

/* Fill *opt with defaults (struct_size set).  Returns BM_EINVAL on NULL. */
bm_status bm_default_options(bm_options* opt);

/* Message of the last failure on this thread ("" if none).  Owned by the
 * library, valid until the next call on this thread. */
const char* bm_last_error(void);

/* Release the library's device scratch pool (it is re-created on demand). */
bm_status bm_release_scratch(void);

/* BM_ABI_VERSION of the built library. */
int32_t bm_abi_version(void);

/*
 * bigmeans_fit -- Big-means, Alg. 1, followed by the final assignment of
 * Sec. 3.4.
 *   X           device, n x d, FP32 (or BF16 bit patterns when opt->x_dtype is
 *               BM_BF16); read only.
 *   n, d, k, s  1 <= k <= s <= n, d >= 1, n < 2^31.
 *   n_samples   number of samples processed (the stop condition; >= 1).
 *   seed        key of the random stream.
 *   opt         options, or NULL for defaults.
 *   centroids   device, k x d FP32, out (in/out when opt->resume = 1).
 *               Degenerate rows are NaN.
 *   sse         host, out: objective of Eq. (1) on all of X, summed in FP64;
 *               may be NULL to skip the final pass together with labels.
 *   labels      device, n int32, out: nearest non-degenerate centroid of every
 *               point (exact ties to the lowest index); may be NULL.
 *   degenerate  host, k bytes, out (in/out when resuming); may be NULL unless
 *               resuming.
 *   stats       host, out; may be NULL.
 * Errors: BM_EINVAL for bad sizes/pointers/options, BM_ENOMEM when scratch
 * cannot be allocated, BM_ENOTSUP when k x d exceeds what a workgroup can
 * stage, BM_EDEVICE on a HIP failure or an aborted grid barrier.
 */
bm_status bigmeans_fit(const void* X, int64_t n, int32_t d, int32_t k, int64_t s,
                       int32_t n_samples, uint64_t seed, const bm_options* opt,
                       float* centroids, double* sse, int32_t* labels, uint8_t* degenerate,
                       bm_stats* stats);

/*
 * bigmeans_fit_collective -- the collective parallel form of Big-means
 * (Sec. 3.6, third scheme) on one GPU: n_rounds rounds of n_workers workers.
 * Worker w of round r clusters its own sample, index t = r * n_workers + w of
 * the random stream, starting from the incumbent of the previous rounds (all
 * degenerate in round 0): it reinitialises the incumbent's degenerate
 * centroids on its sample (opt->init_method) and runs K-means there.  All
 * workers of a round run their K-means together in the batched kernels
 * (kmeans_lloyd_batched).  After the round the worker with the smallest
 * sample objective (ties to the lowest w) replaces the incumbent if that
 * objective is below f_opt (Alg. 1's keep-the-best).  Then the final
 * assignment (Alg. 1 last step).  With n_workers = 1 this is bigmeans_fit.
 *   X, n, d, k, s, seed, centroids, sse, labels, degenerate, stats: as for
 *               bigmeans_fit (stats->samples = rounds x workers; the
 *               per-phase times are not filled).
 *   n_workers   1..1024; n_rounds >= 1; n_rounds x n_workers < 2^32.
 *   opt         as for bigmeans_fit, except that compare_rule must be
 *               BM_CMP_FOPT, and resume, t_start, time_budget_ms,
 *               final_mode, sample_idx and sample_f are not used.
 *   worker_f    host, n_rounds x n_workers out: every worker's f(C'', P), or NULL.
 * Errors: as bigmeans_fit; BM_ENOTSUP for compare_rule BM_CMP_RESAMPLE.
 */
bm_status bigmeans_fit_collective(const void* X, int64_t n, int32_t d, int32_t k, int64_t s,
                                  int32_t n_workers, int32_t n_rounds, uint64_t seed,
                                  const bm_options* opt, float* centroids, double* sse,
                                  int32_t* labels, uint8_t* degenerate, bm_stats* stats,
                                  double* worker_f);

/*
 * bigmeans_sample_size_sweep -- the rule of thumb of Sec. 5 for choosing s:
 * run bigmeans_fit with s = s_min, 2 s_min, 4 s_min, ... (capped at s_max and
 * n) while the final objective on X keeps decreasing; stop at the first size
 * that does not improve on the best so far (or at the cap), and return the
 * best size's fit.
 *   s_min, s_max  k <= s_min <= s_max.
 *   n_samples, seed, opt  as for bigmeans_fit, for every run (final_mode must
 *               be BM_FINAL_ASSIGN; resume is not used).
 *   centroids, degenerate, sse, labels  the best run's outputs (device k x d,
 *               host k, host, device n or NULL); sse is required.
 *   s_best      host out: the best sample size.
 *   s_tried, sse_tried  host out, the sizes run and their objectives, up to
 *               max_tried entries (either may be NULL); n_tried host out.
 */
bm_status bigmeans_sample_size_sweep(const void* X, int64_t n, int32_t d, int32_t k,
                                     int64_t s_min, int64_t s_max, int32_t n_samples,
                                     uint64_t seed, const bm_options* opt, float* centroids,
                                     double* sse, int32_t* labels, uint8_t* degenerate,
                                     int64_t* s_best, int64_t* s_tried, double* sse_tried,
                                     int32_t max_tried, int32_t* n_tried);

/*
 * kmeans_assign -- assignment step (Sec. 2) and objective, Eq. (1): every row
 * of X goes to its nearest non-degenerate centroid (exact ties to the lowest
 * index), distances in FP32 by direct differences, the sum in FP64.
 *   X        device n x d (FP32 or BF16 per opt->x_dtype).
 *   C        device k x d FP32.
 *   deg      host k bytes (1 = skip this centroid) or NULL (all active).
 *   labels   device n int32 out, or NULL.
 *   min_d2   device n FP32 out (squared distance to the chosen centroid), or NULL.
 *   sse      host FP64 out, or NULL.
 * At least one centroid must be active.
 */
bm_status kmeans_assign(const void* X, int64_t n, int32_t d, const float* C, const uint8_t* deg,
                        int32_t k, const bm_options* opt, int32_t* labels, float* min_d2,
                        double* sse);

/*
 * kmeans_assign_noalloc -- kmeans_assign for callers that cannot allocate
 * device memory (code running under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * kmeans_assign (labels and objective identical); it calls no hipMalloc,
 * hipFree or allocating library routine.  Its scratch (the flags, one FP64
 * partial per workgroup and the objective) is a fixed 64 KiB
 * array in device memory that every GPU the library runs on holds until the
 * process ends; calls whose scratch would exceed it (k plus the workgroup
 * count of the call: about 7,000 workgroup partials with k <= 8,000) return
 * BM_EINVAL.  Calls on one GPU share that array: the library serialises them
 * within the process (each returns after its work is done); work from such
 * calls that a caller captures and replays concurrently with another call
 * would race.
 */
bm_status kmeans_assign_noalloc(const void* X, int64_t n, int32_t d, const float* C,
                                const uint8_t* deg, int32_t k, const bm_options* opt,
                                int32_t* labels, float* min_d2, double* sse);

/*
 * kmeanspp_seed -- K-means++ (Sec. 2, greedy form of Sec. 5) applied to the
 * degenerate slots of C, as in the reseeding step of Alg. 1 (Sec. 3.3).
 *   P          device s x d FP32: the points to seed from (a sample).
 *   C          device k x d FP32, in/out: slots with deg[j] = 0 are kept.
 *   deg        host k bytes, in/out: 1 = fill this slot.  Slots are filled in
 *              ascending order; if every remaining D^2 is zero they stay 1.
 *   seed, stream_id  the draws use sample index t = stream_id (< 2^32).
 *   opt        n_local_trials (1..8) is read from here.
 * A D^2 draw takes the first row whose running sum of weights, in row order,
 * exceeds u W (W the sum of all weights, u the draw's uniform); the sums are
 * formed by chunks and scans, and a draw that lands within their rounding
 * bound of a row boundary is taken again with W and the running sum added
 * one row at a time, so every pick is the row-order definition's.
 */
bm_status kmeanspp_seed(const float* P, int64_t s, int32_t d, int32_t k, float* C, uint8_t* deg,
                        uint64_t seed, uint64_t stream_id, const bm_options* opt);

/*
 * kmeans_lloyd -- K-means local search (Sec. 2) on the rows of P from C, with
 * the stop rule, tolerance and iteration cap of opt; a centroid whose cluster
 * empties becomes degenerate (Sec. 3.3).
 *   P        device s x d FP32.
 *   C        device k x d FP32, in/out.      deg  host k bytes, in/out.
 *   labels   device s int32 out (assignment to the returned C), or NULL.
 *   f        host out: objective of the returned C on P (FP64), or NULL.
 *   passes   host out: assignment passes run, or NULL.
 */
bm_status kmeans_lloyd(const float* P, int64_t s, int32_t d, int32_t k, float* C, uint8_t* deg,
                       const bm_options* opt, int32_t* labels, double* f, int32_t* passes);

/*
 * bm_sample_indices -- the uniform sample of s distinct indices out of n that
 * bigmeans_fit uses for sample index t (Sec. 3.1, 3.5): the s points with the
 * smallest (key, index) pairs, in ascending index order.
 *   idx   device s int32 out.
 */
bm_status bm_sample_indices(int64_t n, int64_t s, uint64_t seed, int32_t t, int32_t* idx,
                            const bm_options* opt);

/*
 * bm_gather_rows -- P[r] = X[idx[r]] for r < s, widened to FP32 (the sample
 * matrix of Alg. 1 built from a sample's indices, Sec. 3.1).
 *   X    device n x d (FP32, or BF16 per opt->x_dtype).
 *   idx  device s int32 row indices, each in [0, n) (else BM_EINVAL, P partly written).
 *   P    device s x d FP32 out.
 */
bm_status bm_gather_rows(const void* X, int64_t n, int32_t d, const int32_t* idx, int64_t s,
                         float* P, const bm_options* opt);

/*
 * kmeans_lloyd_batched -- kmeans_lloyd (K-means, Sec. 2) on n_solves
 * independent problems at once, as the parallel workers of Big-means run it
 * on their own samples (Sec. 3.6): every round assigns all rows of every
 * unfinished problem and updates its centroids, with each problem's stop rule,
 * tolerance and cap from opt, and stops a problem exactly where kmeans_lloyd
 * would.  One graph launch per round on an internal stream ordered after
 * opt->stream.
 *   P        device, the problems' rows concatenated: problem j owns
 *            s[j] rows starting after those of problems 0 .. j-1; FP32, d wide.
 *   s, k     host n_solves each: rows and centroids per problem, 1 <= k <= s.
 *   C        device, the problems' k[j] x d centroids concatenated, in/out.
 *   deg      host, sum(k) bytes, in/out (1 = degenerate, as kmeans_lloyd).
 *   labels   device, sum(s) int32 out (nearest centroid within the problem,
 *            for the returned centroids), or NULL.
 *   f        host n_solves out: objective of each returned C on its rows (FP64), or NULL.
 *   passes   host n_solves out: assignment passes per problem, or NULL.
 * The row tile per work item is tuned once per shape (timed) and cached.
 * Errors: BM_EINVAL for bad sizes or pointers, BM_ENOTSUP when d > 256 or
 * the largest k x d does not fit the workgroup's LDS, BM_EDEVICE on a HIP
 * failure.
 */
bm_status kmeans_lloyd_batched(int32_t n_solves, const float* P, int32_t d, const int64_t* s,
                               const int32_t* k, float* C, uint8_t* deg, const bm_options* opt,
                               int32_t* labels, double* f, int32_t* passes);

/* ------------------------------------------------------------------------
 * Serving: a context runs many bigmeans_fit jobs concurrently on one GPU.
 *
 * A context has `slots` workers, each with its own HIP stream and device
 * scratch; jobs start strictly in submission order, each as soon as a slot is
 * idle and the scratch it needs fits in hbm_budget together with what the
 * other slots hold (X and the outputs are the caller's and are not counted).
 * A job's cooperative grid is capped (CUs / slots by default) so that the
 * solver kernels of all slots are co-resident.  A job gives the result
 * bigmeans_fit gives for it alone (integer outputs identical; objectives and
 * centroids equal to rounding).  Every entry point is thread safe.
 */
typedef struct bm_ctx bm_ctx;

enum { BM_JOB_QUEUED = 0, BM_JOB_RUNNING = 1, BM_JOB_DONE = 2, BM_JOB_FAILED = 3,
       BM_JOB_CANCELLED = 4 };

enum { BM_SERVE_FITS = 0, BM_SERVE_ROUNDS = 1 };

typedef struct bm_serve_config {
  uint32_t struct_size;   /* sizeof(bm_serve_config)                              */
  int32_t slots;          /* concurrent jobs, 1..64 (default 4)                   */
  int64_t hbm_budget;     /* device scratch the context may hold, bytes (8 GiB)   */
  int32_t device;         /* HIP device; -1 = the caller's current device         */
  int32_t grid_per_job;   /* cap of a job's cooperative grid; 0 = CUs / slots     */
                          /* (BM_SERVE_FITS only)                                 */
  int32_t mode;           /* BM_SERVE_FITS (default): each slot runs whole fits   */
                          /* with the persistent solver.  BM_SERVE_ROUNDS: one    */
                          /* engine keeps up to `slots` jobs in flight, draws and */
                          /* seeds each job's samples, and runs the Lloyd rounds  */
                          /* of all of them together in the batched kernels;      */
                          /* jobs join and leave at round boundaries              */
  int32_t round_max_k;    /* BM_SERVE_ROUNDS: largest k of a job (default 64)     */
  int64_t round_max_s;    /* BM_SERVE_ROUNDS: largest sample size (default 50000) */
} bm_serve_config;

/* One job: the arguments of bigmeans_fit.  opt.stream is ignored (the slot's
 * stream is used); every pointer must stay valid until the job is finished. */
typedef struct bm_job {
  uint32_t struct_size;   /* sizeof(bm_job)                                       */
  const void* X;          /* device n x d (FP32, or BF16 per opt.x_dtype)         */
  int64_t n;
  int32_t d, k;
  int64_t s;
  int32_t n_samples;
  uint64_t seed;
  bm_options opt;         /* filled by bm_default_options, then adjusted          */
  float* centroids;       /* device k x d out                                     */
  int32_t* labels;        /* device n out, or NULL                                */
  uint8_t* degenerate;    /* host k out, or NULL                                  */
  double* sse;            /* host out, or NULL (with labels NULL: no final pass)  */
  bm_stats* stats;        /* host out, or NULL                                    */
} bm_job;

typedef struct bm_job_info {
  uint32_t struct_size;   /* sizeof(bm_job_info)                                  */
  int32_t state;          /* BM_JOB_*                                             */
  bm_status result;       /* the job's status once finished                       */
  int32_t slot;           /* slot it ran on, -1 before it starts                  */
  int64_t footprint;      /* device scratch it needs, bytes                       */
  double t_submit_ms, t_start_ms, t_end_ms;  /* steady clock, from bm_ctx_create  */
  char error[160];        /* bm_last_error of a failed job                        */
} bm_job_info;

typedef struct bm_serve_info {
  uint32_t struct_size;   /* sizeof(bm_serve_info)                                */
  int32_t slots, grid_per_job;
  int64_t submitted, completed, failed, cancelled, queued, running;
  int64_t reserved_bytes, peak_reserved_bytes;  /* scratch held by the slots      */
} bm_serve_info;

/* Defaults for *cfg (struct_size set). */
bm_status bm_serve_default_config(bm_serve_config* cfg);
/* Create a context (cfg NULL = defaults); its worker threads start at once. */
bm_status bm_ctx_create(const bm_serve_config* cfg, bm_ctx** ctx);
/* Queue a job (validated as bigmeans_fit validates it; BM_ENOMEM when it needs
 * more scratch than the whole budget).  Returns at once with its id.  In
 * BM_SERVE_ROUNDS mode a job also needs compare_rule BM_CMP_FOPT, s <=
 * round_max_s and k <= round_max_k (else BM_ENOTSUP); its result agrees with
 * bigmeans_fit's to rounding (the batched kernels sum in another order), and
 * its stats carry samples, replacements, lloyd_iters, reseeded and f_opt. */
bm_status bm_ctx_submit(bm_ctx* ctx, const bm_job* job, int64_t* job_id);
/* State of a job (info->struct_size must be set). */
bm_status bm_ctx_poll(bm_ctx* ctx, int64_t job_id, bm_job_info* info);
/* Block until the job has finished (timeout_ms < 0: no limit); BM_ETIMEDOUT
 * if it has not finished in time.  info may be NULL. */
bm_status bm_ctx_wait(bm_ctx* ctx, int64_t job_id, int32_t timeout_ms, bm_job_info* info);
/* Cancel a queued job (BM_EINVAL once it has started). */
bm_status bm_ctx_cancel(bm_ctx* ctx, int64_t job_id);
/* Forget a finished job's record. */
bm_status bm_ctx_release(bm_ctx* ctx, int64_t job_id);
/* Counters of the context. */
bm_status bm_ctx_info(bm_ctx* ctx, bm_serve_info* info);
/* Cancel queued jobs, wait for running ones, free everything.  NULL is a no-op. */
bm_status bm_ctx_destroy(bm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* BIGMEANS_H */
