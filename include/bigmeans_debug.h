/*
 * bigmeans_debug.h -- diagnostics and test hooks of libbigmeans.so.
 *
 * Not part of the clustering API (bigmeans.h): these report per-thread
 * details of the last call for tests and measurement, or switch internal
 * paths so tests can reach them.  All are thread-safe in the sense that they
 * read or write only the calling thread's records (bm_debug_presample is
 * process-wide).
 */
#ifndef BIGMEANS_DEBUG_H
#define BIGMEANS_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Presampling before the persistent solver: mode 0 = automatic, 1 = never
 * (the solver draws every sample), 2 = report a predicted-window miss (the
 * solver then draws every sample itself).  Returns the previous mode, or -1
 * for a mode outside 0..2.  Process-wide. */
int32_t bm_debug_presample(int32_t mode);

/* BF16 points with BM_PREC_BF16_MFMA: 1 (default) runs the sample-level
 * K-means on the matrix cores, 0 runs it on the FP32 persistent solver (both
 * give the same labels).  Returns the previous setting, or -1 for another
 * value.  Process-wide. */
int32_t bm_debug_mfma_lloyd(int32_t on);

/* FP32 points: 1 (default) lets the full-data assignment (final pass,
 * kmeans_assign) run on the matrix cores when d >= 8, k >= 8 and
 * k d >= 256, 0 keeps it
 * on the VALU direct-difference kernel (both give the same labels).  Returns
 * the previous setting, or -1 for another value.  Process-wide. */
int32_t bm_debug_fp32_mfma(int32_t on);

/* K-means++ D^2 draws (Sec. 2): 1 takes every draw with W and the running
 * sum added one row at a time in row order, 0 (default) only the draws that
 * the chunked sums leave within rounding of a row boundary (the others pick
 * the same row either way); each such draw adds one to boundary_draws.
 * Returns the previous setting, or -1 for another value.  Process-wide. */
int32_t bm_debug_exact_draws(int32_t on);

/* Copies the first n raw device counters of this thread's last bigmeans_fit
 * (passes, reseeds, replacements, n_d, boundary draws, samples, sampler
 * passes, then per-phase clock ticks) into out.  BM_EINVAL for out NULL or
 * n < 1. */
int32_t bm_debug_counters(int64_t* out, int32_t n);

/* Points this thread's last BM_PREC_BF16_MFMA kmeans_assign recomputed on
 * the FP32 path (near ties). */
int64_t bm_debug_rechecked(void);

/* Device time in ms (HIP events on the call's stream, bracketing only the
 * assignment kernel) of this thread's last kmeans_assign. */
double bm_debug_assign_ms(void);

/* Rounds and rows per work tile of this thread's last kmeans_lloyd_batched;
 * either pointer may be NULL.  Returns 0. */
int32_t bm_debug_batch_info(int32_t* rounds, int32_t* tile_rows);

/* Device time in ms of round i of this thread's last kmeans_lloyd_batched
 * (0 when i is out of range). */
double bm_debug_batch_round_ms(int32_t i);

#ifdef __cplusplus
}
#endif
#endif /* BIGMEANS_DEBUG_H */
