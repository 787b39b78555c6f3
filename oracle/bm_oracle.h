/*
 * bm_oracle.h -- plain, slow FP64 CPU oracle for Big-means.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the GPU library (different sources, different Philox implementation, no
 * common headers); the two meet only through seeded inputs.
 *
 * What it computes (Mussabayev et al., "How to Use K-means for Big Data
 * Clustering?"):
 *   - the MSSC objective, Eq. (1), with each point charged to its nearest
 *     centroid (the surrounding text of Sec. 1 says "nearest");
 *   - K-means (Lloyd) local search, Sec. 2: assign to the nearest centre, move
 *     each centre to the mean of its cell, repeat;
 *   - K-means++ D^2 seeding, Sec. 2, in the greedy form of Sec. 5 (several
 *     candidates per new centre, keep the best);
 *   - Big-means, Alg. 1 with Sec. 3.2-3.5: uniform sample without replacement,
 *     reseed only degenerate centroids, Lloyd from the incumbent, keep the best
 *     by sample objective, final assignment of every point.
 * Every free choice the paper leaves open (random stream layout, tie rules,
 * stop rules) is fixed in the comments of bm_oracle.c.
 *
 * Notation: n points, d features (the paper's m and n), k clusters, s sample
 * size.  Arrays are row-major; centroids are FP64 here; a degenerate centroid
 * has deg[j] = 1 and NaN coordinates.
 */
#ifndef BM_ORACLE_H
#define BM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_F32 = 0, ORC_BF16 = 1 };
enum { ORC_STOP_SHIFT = 0, ORC_STOP_REL_OBJ = 1 };
enum { ORC_CMP_FOPT = 0, ORC_CMP_RESAMPLE = 1 };
enum { ORC_INIT_KMEANSPP = 0, ORC_INIT_FORGY = 1 };

typedef struct orc_opts {
    int32_t max_iter;       /* Lloyd assign+update rounds per sample          */
    double  tol;            /* shift or relative-objective tolerance          */
    int32_t stop_rule;      /* ORC_STOP_SHIFT | ORC_STOP_REL_OBJ              */
    int32_t n_local_trials; /* K-means++ candidates per new centre (>= 1)     */
    int32_t compare_rule;   /* ORC_CMP_FOPT | ORC_CMP_RESAMPLE                */
    int32_t init_method;    /* ORC_INIT_KMEANSPP | ORC_INIT_FORGY: how the    */
                            /* degenerate centroids are (re)initialised       */
} orc_opts;

typedef struct orc_stats {
    int32_t samples;
    int32_t replacements;
    int64_t lloyd_iters;    /* assignment passes run inside Lloyd             */
    int64_t reseeded;       /* centroids placed by K-means++                  */
    int64_t n_d;            /* distance evaluations at sample level           */
    double  f_opt;          /* incumbent objective on its own sample          */
} orc_stats;

/* Threads the per-point loops use: 1, or OpenMP's count in the threaded
 * build (whose results are bit-identical to the single-threaded build's). */
int orc_threads(void);

/* Philox4x32 with 10 rounds (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* 64-bit word of the draw-stream block q of sample t (stream tag 1). */
uint64_t orc_seed_word(uint64_t seed, uint32_t t, uint64_t q);
/* 64-bit selection key of point i for sample t (stream tag 0). */
uint64_t orc_sample_key(uint64_t seed, uint32_t t, int64_t i);

/* Uniform sample of s distinct indices out of n, ascending. */
int orc_sample(int64_t n, int64_t s, uint64_t seed, uint32_t t, int32_t* idx);

/* Squared Euclidean distance by direct differences, FMA in dimension order. */
double orc_dist2(const double* x, const double* c, int32_t d);

/* Nearest active centroid of every row; returns the SSE (index-order sum). */
double orc_assign(const double* P, int64_t s, int32_t d, const double* C,
                  const uint8_t* deg, int32_t k, int32_t* labels, double* mind);

/* One D^2 draw: the smallest i whose running sum of w (row order) exceeds
 * target; if none does (rounding), the last i with w[i] > 0; -1 if all zero. */
int64_t orc_d2_pick(const double* w, int64_t s, double target);

/* K-means++ reseed of the slots with deg[j] = 1 on the rows of P. */
int orc_kmeanspp(const double* P, int64_t s, int32_t d, int32_t k, double* C,
                 uint8_t* deg, uint64_t seed, uint32_t t, int32_t trials,
                 orc_stats* st);

/* Forgy-style (re)initialisation of the slots with deg[j] = 1: each takes a
 * uniformly drawn row of P, slots in ascending order, draws from the same
 * stream as K-means++ (Sec. 3.3 allows initialisations other than K-means++). */
int orc_forgy(const double* P, int64_t s, int32_t d, int32_t k, double* C,
              uint8_t* deg, uint64_t seed, uint32_t t, orc_stats* st);

/* Lloyd from C on P; returns the SSE of the returned C on P. */
double orc_lloyd(const double* P, int64_t s, int32_t d, int32_t k, double* C,
                 uint8_t* deg, const orc_opts* o, int32_t* labels,
                 int32_t* iters, orc_stats* st);

/* Big-means, Alg. 1.  X is FP32 or BF16 (raw uint16) row-major n x d.
 * resume = 0: C/deg/f_opt are outputs only; resume = 1: they carry the
 * incumbent in and out, and samples t_start .. t_start+T-1 are processed.
 * labels (n) and sse may be NULL.  sample_f (T) gets f(C'',P) per sample,
 * sample_idx (T*s) the sampled indices; both may be NULL. */
int orc_bigmeans_fit(const void* X, int32_t x_dtype, int64_t n, int32_t d,
                     int32_t k, int64_t s, int32_t T, uint64_t seed,
                     const orc_opts* o, int32_t t_start, int32_t resume,
                     double* C, uint8_t* deg, double* f_opt, int32_t* labels,
                     double* sse, double* sample_f, int32_t* sample_idx,
                     orc_stats* st);

/* Collective parallel Big-means (Sec. 3.6, third scheme): W workers per
 * round, worker w of round r clusters sample t = r*W + w starting from the
 * incumbent of the previous rounds (all degenerate in round 0); after each
 * round the worker with the smallest f(C'',P) (ties to the lowest w) replaces
 * the incumbent when its objective is below f_opt.  R rounds, then the final
 * assignment.  worker_f (R*W, may be NULL) gets every worker's f(C'',P). */
int orc_bigmeans_collective(const void* X, int32_t x_dtype, int64_t n, int32_t d,
                            int32_t k, int64_t s, int32_t W, int32_t R, uint64_t seed,
                            const orc_opts* o, double* C, uint8_t* deg, double* f_opt,
                            int32_t* labels, double* sse, double* worker_f,
                            orc_stats* st);

/* The sample-size rule of thumb (Sec. 5): s = s_min, 2 s_min, 4 s_min, ...
 * (capped at s_max and n), one Big-means run of T samples each with its final
 * objective on X, continued while the objective decreases; stops at the
 * first s that does not improve on the best so far.  s_tried / sse_tried get
 * the sizes run and their objectives (capacity 64), *n_tried their count;
 * returns the best s (or < 0 on bad arguments). */
int64_t orc_sample_size_sweep(const void* X, int32_t x_dtype, int64_t n, int32_t d,
                              int32_t k, int64_t s_min, int64_t s_max, int32_t T,
                              uint64_t seed, const orc_opts* o, int64_t* s_tried,
                              double* sse_tried, int32_t* n_tried);

#ifdef __cplusplus
}
#endif
#endif
