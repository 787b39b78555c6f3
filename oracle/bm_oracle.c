/*
 * bm_oracle.c -- plain, slow FP64 CPU oracle for Big-means.
 *
 * TEST INFRASTRUCTURE ONLY (see bm_oracle.h).  Written for a reader holding the
 * paper: every step follows the passage named in its comment, in the paper's
 * order, with no blocking, fusion or reordering.  Every sum has one fixed
 * order: the index order of its terms.
 *
 * Threads: the same source builds a single-threaded library and an OpenMP one
 * (-fopenmp; used to time the oracle on all host cores and to compute stored
 * results of large workloads).  Only loops whose iterations are independent
 * per point are shared out (distances, keys, row loads); each writes its
 * per-point terms to an array, and every sum over points is then taken by one
 * thread in index order.  So both builds return bit-identical results.
 *
 * Random stream (the paper names no generator; this is the fixed reading):
 *   Philox4x32-10, key = (low 32 bits of seed, high 32 bits of seed), counter
 *   (c0, c1, c2, c3) with c2 = sample index t and c3 = stream tag
 *   (0 = sampling, 1 = K-means++ draws).
 *     sampling: block b = i / 2 has counter (lo32(b), hi32(b), t, 0); point i
 *       takes the words (out0, out1) if i is even, (out2, out3) if odd, as the
 *       64-bit key  hi << 32 | lo.
 *     K-means++: draw q of sample t has counter (lo32(q), hi32(q), t, 1) and
 *       yields w = out0 << 32 | out1.
 *   A uniform double is (w >> 11) * 2^-53 in [0, 1); a uniform integer in
 *   [0, N) is the high 64 bits of the 128-bit product w * N.
 */
#include "bm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the per-point loops use (1 in the single-threaded build). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  One round multiplies
 * counter words 0 and 2 by fixed odd constants, and mixes the high halves with
 * the other two words and the round key; the key is advanced by two Weyl
 * increments between rounds.                                                 */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void seed_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
}

uint64_t orc_sample_key(uint64_t seed, uint32_t t, int64_t i)
{
    uint32_t key[2], ctr[4], out[4];
    uint64_t b = (uint64_t)i >> 1;
    seed_key(seed, key);
    ctr[0] = (uint32_t)b; ctr[1] = (uint32_t)(b >> 32); ctr[2] = t; ctr[3] = 0u;
    orc_philox4x32_10(ctr, key, out);
    if ((i & 1) == 0) return ((uint64_t)out[0] << 32) | out[1];
    return ((uint64_t)out[2] << 32) | out[3];
}

uint64_t orc_seed_word(uint64_t seed, uint32_t t, uint64_t q)
{
    uint32_t key[2], ctr[4], out[4];
    seed_key(seed, key);
    ctr[0] = (uint32_t)q; ctr[1] = (uint32_t)(q >> 32); ctr[2] = t; ctr[3] = 1u;
    orc_philox4x32_10(ctr, key, out);
    return ((uint64_t)out[0] << 32) | out[1];
}

static double word_to_unit(uint64_t w)
{
    return (double)(w >> 11) * 0x1.0p-53;
}

static uint64_t word_below(uint64_t w, uint64_t N)
{
    unsigned __int128 p = (unsigned __int128)w * (unsigned __int128)N;
    return (uint64_t)(p >> 64);
}

/* ------------------------------------------------------------------------ */
/* Sampling, Sec. 3.1 and 3.5: a simple random sample of s distinct points.
 * Reading: every point gets an independent uniform 64-bit key and the sample
 * is the s points with the smallest (key, index) pairs -- a uniformly random
 * s-subset.  Returned in ascending index order.                              */
typedef struct { uint64_t key; int64_t i; } keyed;

static int cmp_keyed(const void* a, const void* b)
{
    const keyed* x = (const keyed*)a;
    const keyed* y = (const keyed*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

int orc_sample(int64_t n, int64_t s, uint64_t seed, uint32_t t, int32_t* idx)
{
    if (n < 1 || s < 1 || s > n || n > 2147483647LL) return -1;
    keyed* all = (keyed*)malloc((size_t)n * sizeof(keyed));
    if (!all) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        all[i].key = orc_sample_key(seed, t, i);
        all[i].i = i;
    }
    qsort(all, (size_t)n, sizeof(keyed), cmp_keyed);
    for (int64_t r = 0; r < s; ++r) idx[r] = (int32_t)all[r].i;
    free(all);
    qsort(idx, (size_t)s, sizeof(int32_t), cmp_i32);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. (1) term: squared Euclidean distance, by direct differences.          */
double orc_dist2(const double* x, const double* c, int32_t d)
{
    double acc = 0.0;
    for (int32_t t = 0; t < d; ++t) {
        double diff = x[t] - c[t];
        acc = fma(diff, diff, acc);
    }
    return acc;
}

/* Assignment step (Sec. 2) and the objective of Eq. (1): each row goes to the
 * nearest non-degenerate centroid; an exact tie goes to the lowest index.   */
double orc_assign(const double* P, int64_t s, int32_t d, const double* C,
                  const uint8_t* deg, int32_t k, int32_t* labels, double* mind)
{
    double* md = mind ? mind : (double*)malloc((size_t)s * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s; ++i) {
        const double* x = P + (size_t)i * d;
        int32_t best = -1;
        double bestd = INFINITY;
        for (int32_t j = 0; j < k; ++j) {
            if (deg && deg[j]) continue;
            double dd = orc_dist2(x, C + (size_t)j * d, d);
            if (dd < bestd) { bestd = dd; best = j; }
        }
        if (labels) labels[i] = best;
        md[i] = bestd;
    }
    double f = 0.0;
    for (int64_t i = 0; i < s; ++i) f += md[i];
    if (!mind) free(md);
    return f;
}

static int32_t count_active(const uint8_t* deg, int32_t k)
{
    int32_t a = 0;
    for (int32_t j = 0; j < k; ++j) a += deg[j] ? 0 : 1;
    return a;
}

/* ------------------------------------------------------------------------ */
/* K-means++ (Sec. 2; greedy variant with several candidates, Sec. 5), used by
 * Alg. 1 to (re)initialise only the degenerate centroids (Sec. 3.3).
 * Readings: the point set is the current sample; slots are filled in
 * ascending order; with no active centroid the first pick is uniform; a new
 * centre is drawn with probability proportional to D^2 (the squared distance
 * to the nearest already-placed centre) by inverting the running sum in row
 * order; among the candidates the one with the smallest potential
 * sum_i min(D_i^2, |p_i - c|^2) wins, ties to the earlier draw; if every D^2
 * is zero the remaining slots stay degenerate.                              */
/* One D^2 draw: the smallest row i whose running sum w_0 + ... + w_i (added
 * in row order) exceeds target; if rounding leaves no such row, the last row
 * with w_i > 0; -1 if every w_i is zero.                                    */
int64_t orc_d2_pick(const double* w, int64_t s, double target)
{
    double run = 0.0;
    for (int64_t i = 0; i < s; ++i) {
        run += w[i];
        if (run > target) return i;
    }
    for (int64_t i = s - 1; i >= 0; --i)
        if (w[i] > 0.0) return i;
    return -1;
}

int orc_kmeanspp(const double* P, int64_t s, int32_t d, int32_t k, double* C,
                 uint8_t* deg, uint64_t seed, uint32_t t, int32_t trials,
                 orc_stats* st)
{
    if (s < 1 || d < 1 || k < 1 || trials < 1) return -1;
    double* w = (double*)malloc((size_t)s * sizeof(double));
    double* term = (double*)malloc((size_t)s * sizeof(double));
    if (!w || !term) { free(w); free(term); return -2; }
    uint64_t q = 0;
    int32_t active = count_active(deg, k);

    if (active > 0) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < s; ++i) {
            double best = INFINITY;
            for (int32_t j = 0; j < k; ++j) {
                if (deg[j]) continue;
                double dd = orc_dist2(P + (size_t)i * d, C + (size_t)j * d, d);
                if (dd < best) best = dd;
            }
            w[i] = best;
        }
        if (st) st->n_d += s * (int64_t)active;
    }

    for (int32_t j = 0; j < k; ++j) {
        if (!deg[j]) continue;
        int64_t pick;
        if (active == 0) {
            pick = (int64_t)word_below(orc_seed_word(seed, t, q++), (uint64_t)s);
        } else {
            double W = 0.0;
            for (int64_t i = 0; i < s; ++i) W += w[i];
            if (W == 0.0) break;
            pick = -1;
            double best_phi = INFINITY;
            for (int32_t l = 0; l < trials; ++l) {
                double target = word_to_unit(orc_seed_word(seed, t, q++)) * W;
                int64_t cand = orc_d2_pick(w, s, target);
                if (trials == 1) { pick = cand; break; }
                /* potential of the candidate: sum_i min(w_i, |p_i - cand|^2) */
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < s; ++i) {
                    double dd = orc_dist2(P + (size_t)i * d, P + (size_t)cand * d, d);
                    term[i] = dd < w[i] ? dd : w[i];
                }
                double phi = 0.0;
                for (int64_t i = 0; i < s; ++i) phi += term[i];
                if (st) st->n_d += s;
                if (phi < best_phi) { best_phi = phi; pick = cand; }
            }
        }
        memcpy(C + (size_t)j * d, P + (size_t)pick * d, (size_t)d * sizeof(double));
        deg[j] = 0;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < s; ++i) {
            double dd = orc_dist2(P + (size_t)i * d, C + (size_t)j * d, d);
            if (active == 0 || dd < w[i]) w[i] = dd;
        }
        if (st) { st->n_d += s; st->reseeded += 1; }
        active += 1;
    }
    free(w);
    free(term);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Another initialisation (Sec. 3.3: the first sample may be initialised
 * otherwise, e.g. at random, and degenerate clusters may be handled by other
 * strategies): every degenerate slot, in ascending order, takes the row of P
 * at a uniformly drawn index -- independent draws, so two slots may take the
 * same row; the later one then empties and is reinitialised at the next
 * sample.  Draw q of sample t is the same stream word K-means++ uses.        */
int orc_forgy(const double* P, int64_t s, int32_t d, int32_t k, double* C,
              uint8_t* deg, uint64_t seed, uint32_t t, orc_stats* st)
{
    if (s < 1 || d < 1 || k < 1) return -1;
    uint64_t q = 0;
    for (int32_t j = 0; j < k; ++j) {
        if (!deg[j]) continue;
        int64_t pick = (int64_t)word_below(orc_seed_word(seed, t, q++), (uint64_t)s);
        memcpy(C + (size_t)j * d, P + (size_t)pick * d, (size_t)d * sizeof(double));
        deg[j] = 0;
        if (st) st->reseeded += 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* K-means / Lloyd (Sec. 2): assign, then move each centre to the mean of its
 * cell.  Stop rules: ORC_STOP_REL_OBJ is the rule of Sec. 5 (stop when the
 * relative decrease of two consecutive objective values is below tol, or after
 * max_iter rounds); ORC_STOP_SHIFT stops when no centre moves by tol or more
 * (Euclidean).  A centre whose cell empties becomes degenerate (Sec. 3.3) and
 * stays so for the rest of this run.  The value returned is always the
 * objective of the returned centroids on P.                                 */
double orc_lloyd(const double* P, int64_t s, int32_t d, int32_t k, double* C,
                 uint8_t* deg, const orc_opts* o, int32_t* labels,
                 int32_t* iters, orc_stats* st)
{
    int32_t* lab = labels ? labels : (int32_t*)malloc((size_t)s * sizeof(int32_t));
    double* sums = (double*)malloc((size_t)k * d * sizeof(double));
    int64_t* cnt = (int64_t*)malloc((size_t)k * sizeof(int64_t));
    double f = 0.0, f_prev = INFINITY;
    int32_t passes = 0;
    int converged_by_objective = 0;

    for (int32_t it = 1; it <= o->max_iter; ++it) {
        f = orc_assign(P, s, d, C, deg, k, lab, NULL);
        passes++;
        if (st) st->n_d += s * (int64_t)count_active(deg, k);
        if (o->stop_rule == ORC_STOP_REL_OBJ && it > 1 && (f_prev - f) <= o->tol * f_prev) {
            converged_by_objective = 1;
            break;
        }
        memset(sums, 0, (size_t)k * d * sizeof(double));
        memset(cnt, 0, (size_t)k * sizeof(int64_t));
        for (int64_t i = 0; i < s; ++i) {
            int32_t j = lab[i];
            for (int32_t t = 0; t < d; ++t) sums[(size_t)j * d + t] += P[(size_t)i * d + t];
            cnt[j] += 1;
        }
        double shift = 0.0;
        for (int32_t j = 0; j < k; ++j) {
            if (deg[j]) continue;
            double* c = C + (size_t)j * d;
            if (cnt[j] == 0) {
                deg[j] = 1;
                for (int32_t t = 0; t < d; ++t) c[t] = NAN;
                continue;
            }
            double moved = 0.0;
            for (int32_t t = 0; t < d; ++t) {
                double m = sums[(size_t)j * d + t] / (double)cnt[j];
                double diff = m - c[t];
                moved += diff * diff;
                c[t] = m;
            }
            moved = sqrt(moved);
            if (moved > shift) shift = moved;
        }
        f_prev = f;
        if (o->stop_rule == ORC_STOP_SHIFT && shift < o->tol) break;
    }
    if (!converged_by_objective) {
        f = orc_assign(P, s, d, C, deg, k, lab, NULL);
        passes++;
        if (st) st->n_d += s * (int64_t)count_active(deg, k);
    }
    if (iters) *iters = passes;
    if (st) st->lloyd_iters += passes;
    free(sums);
    free(cnt);
    if (!labels) free(lab);
    return f;
}

/* ------------------------------------------------------------------------ */
static double bf16_to_double(uint16_t h)
{
    uint32_t bits = (uint32_t)h << 16;
    float v;
    memcpy(&v, &bits, sizeof v);
    return (double)v;
}

static void load_row(const void* X, int32_t x_dtype, int64_t i, int32_t d, double* out)
{
    if (x_dtype == ORC_BF16) {
        const uint16_t* r = (const uint16_t*)X + (size_t)i * d;
        for (int32_t t = 0; t < d; ++t) out[t] = bf16_to_double(r[t]);
    } else {
        const float* r = (const float*)X + (size_t)i * d;
        for (int32_t t = 0; t < d; ++t) out[t] = (double)r[t];
    }
}

static double final_pass(const void* X, int32_t x_dtype, int64_t n, int32_t d, int32_t k,
                         const double* C, const uint8_t* deg, int32_t* labels);

/* Big-means, Alg. 1 (Sec. 3.2): start with every centroid degenerate and
 * f_opt = infinity; per sample draw P, copy the incumbent, reseed its
 * degenerate centroids with K-means++, run K-means on P, and replace the
 * incumbent when the new sample objective is strictly smaller.  Finally
 * assign every point of X and return the objective on X.
 * compare_rule ORC_CMP_FOPT compares with the stored f_opt as Alg. 1 does;
 * ORC_CMP_RESAMPLE compares with the incumbent re-evaluated on the new sample,
 * as the prose of Sec. 3.2 words it.                                        */
int orc_bigmeans_fit(const void* X, int32_t x_dtype, int64_t n, int32_t d,
                     int32_t k, int64_t s, int32_t T, uint64_t seed,
                     const orc_opts* o, int32_t t_start, int32_t resume,
                     double* C, uint8_t* deg, double* f_opt, int32_t* labels,
                     double* sse, double* sample_f, int32_t* sample_idx,
                     orc_stats* st)
{
    if (n < 1 || d < 1 || k < 1 || s < k || s > n || T < 0 || t_start < 0) return -1;
    if (n > 2147483647LL || o->max_iter < 1 || o->n_local_trials < 1) return -1;

    int32_t* idx = (int32_t*)malloc((size_t)s * sizeof(int32_t));
    double* P = (double*)malloc((size_t)s * d * sizeof(double));
    double* Cp = (double*)malloc((size_t)k * d * sizeof(double));
    uint8_t* degp = (uint8_t*)malloc((size_t)k);
    if (!idx || !P || !Cp || !degp) return -2;

    if (!resume) {
        for (size_t z = 0; z < (size_t)k * d; ++z) C[z] = NAN;
        memset(deg, 1, (size_t)k);
        *f_opt = INFINITY;
    }

    for (int32_t tt = 0; tt < T; ++tt) {
        uint32_t t = (uint32_t)(t_start + tt);
        orc_sample(n, s, seed, t, idx);
        if (sample_idx) memcpy(sample_idx + (size_t)tt * s, idx, (size_t)s * sizeof(int32_t));
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < s; ++r) load_row(X, x_dtype, idx[r], d, P + (size_t)r * d);

        memcpy(Cp, C, (size_t)k * d * sizeof(double));
        memcpy(degp, deg, (size_t)k);
        if (count_active(degp, k) < k) {
            if (o->init_method == ORC_INIT_FORGY)
                orc_forgy(P, s, d, k, Cp, degp, seed, t, st);
            else
                orc_kmeanspp(P, s, d, k, Cp, degp, seed, t, o->n_local_trials, st);
        }

        double f = orc_lloyd(P, s, d, k, Cp, degp, o, NULL, NULL, st);
        if (sample_f) sample_f[tt] = f;

        double reference = *f_opt;
        if (o->compare_rule == ORC_CMP_RESAMPLE) {
            reference = count_active(deg, k) > 0
                            ? orc_assign(P, s, d, C, deg, k, NULL, NULL)
                            : INFINITY;
        }
        if (reference > f) {
            memcpy(C, Cp, (size_t)k * d * sizeof(double));
            memcpy(deg, degp, (size_t)k);
            *f_opt = f;
            if (st) st->replacements += 1;
        }
        if (st) st->samples += 1;
    }

    if (labels || sse) {
        double total = final_pass(X, x_dtype, n, d, k, C, deg, labels);
        if (sse) *sse = total;
    }
    if (st) st->f_opt = *f_opt;
    free(idx); free(P); free(Cp); free(degp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Final assignment (Alg. 1 last step, Sec. 3.4) of every row of X to the
 * nearest active centroid; returns the objective on X (index-order sum).    */
static double final_pass(const void* X, int32_t x_dtype, int64_t n, int32_t d, int32_t k,
                         const double* C, const uint8_t* deg, int32_t* labels)
{
    double* md = (double*)malloc((size_t)n * sizeof(double));
    if (!md) return NAN;
#pragma omp parallel
    {
        double* xr = (double*)malloc((size_t)d * sizeof(double));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            load_row(X, x_dtype, i, d, xr);
            int32_t best = -1;
            double bestd = INFINITY;
            for (int32_t j = 0; j < k; ++j) {
                if (deg[j]) continue;
                double dd = orc_dist2(xr, C + (size_t)j * d, d);
                if (dd < bestd) { bestd = dd; best = j; }
            }
            if (labels) labels[i] = best;
            md[i] = bestd;
        }
        free(xr);
    }
    double total = 0.0;
    for (int64_t i = 0; i < n; ++i) total += md[i];
    free(md);
    return total;
}

/* Collective parallel Big-means (Sec. 3.6, third scheme; see bm_oracle.h).
 * Each worker of a round does what one sample of Alg. 1 does, starting from
 * the same incumbent; the round's best worker result then goes through
 * Alg. 1's keep-the-best comparison.                                        */
int orc_bigmeans_collective(const void* X, int32_t x_dtype, int64_t n, int32_t d,
                            int32_t k, int64_t s, int32_t W, int32_t R, uint64_t seed,
                            const orc_opts* o, double* C, uint8_t* deg, double* f_opt,
                            int32_t* labels, double* sse, double* worker_f,
                            orc_stats* st)
{
    if (n < 1 || d < 1 || k < 1 || s < k || s > n || W < 1 || R < 1) return -1;
    if (n > 2147483647LL || o->max_iter < 1 || o->n_local_trials < 1) return -1;
    if ((int64_t)R * W > 4294967295LL) return -1;
    int32_t* idx = (int32_t*)malloc((size_t)s * sizeof(int32_t));
    double* P = (double*)malloc((size_t)s * d * sizeof(double));
    double* Cw = (double*)malloc((size_t)k * d * sizeof(double));
    uint8_t* degw = (uint8_t*)malloc((size_t)k);
    double* Cbest = (double*)malloc((size_t)k * d * sizeof(double));
    uint8_t* degbest = (uint8_t*)malloc((size_t)k);
    if (!idx || !P || !Cw || !degw || !Cbest || !degbest) return -2;

    for (size_t z = 0; z < (size_t)k * d; ++z) C[z] = NAN;
    memset(deg, 1, (size_t)k);
    *f_opt = INFINITY;

    for (int32_t r = 0; r < R; ++r) {
        double round_best = INFINITY;
        for (int32_t w = 0; w < W; ++w) {
            uint32_t t = (uint32_t)((int64_t)r * W + w);
            orc_sample(n, s, seed, t, idx);
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < s; ++q) load_row(X, x_dtype, idx[q], d, P + (size_t)q * d);
            memcpy(Cw, C, (size_t)k * d * sizeof(double));
            memcpy(degw, deg, (size_t)k);
            if (count_active(degw, k) < k) {
                if (o->init_method == ORC_INIT_FORGY)
                    orc_forgy(P, s, d, k, Cw, degw, seed, t, st);
                else
                    orc_kmeanspp(P, s, d, k, Cw, degw, seed, t, o->n_local_trials, st);
            }
            double f = orc_lloyd(P, s, d, k, Cw, degw, o, NULL, NULL, st);
            if (worker_f) worker_f[(size_t)r * W + w] = f;
            if (st) st->samples += 1;
            if (f < round_best) {      /* strict: ties go to the lowest worker */
                round_best = f;
                memcpy(Cbest, Cw, (size_t)k * d * sizeof(double));
                memcpy(degbest, degw, (size_t)k);
            }
        }
        if (*f_opt > round_best) {
            memcpy(C, Cbest, (size_t)k * d * sizeof(double));
            memcpy(deg, degbest, (size_t)k);
            *f_opt = round_best;
            if (st) st->replacements += 1;
        }
    }
    if (labels || sse) {
        double total = final_pass(X, x_dtype, n, d, k, C, deg, labels);
        if (sse) *sse = total;
    }
    if (st) st->f_opt = *f_opt;
    free(idx); free(P); free(Cw); free(degw); free(Cbest); free(degbest);
    return 0;
}

/* The sample-size rule of thumb of Sec. 5 (see bm_oracle.h): grow s by
 * doubling while the final objective on X keeps decreasing.                 */
int64_t orc_sample_size_sweep(const void* X, int32_t x_dtype, int64_t n, int32_t d,
                              int32_t k, int64_t s_min, int64_t s_max, int32_t T,
                              uint64_t seed, const orc_opts* o, int64_t* s_tried,
                              double* sse_tried, int32_t* n_tried)
{
    if (s_min < k || s_min > s_max || T < 1) return -1;
    if (s_max > n) s_max = n;
    if (s_min > s_max) return -1;
    double* C = (double*)malloc((size_t)k * d * sizeof(double));
    uint8_t* deg = (uint8_t*)malloc((size_t)k);
    if (!C || !deg) return -2;
    int64_t best_s = -1;
    double best = INFINITY;
    int32_t m = 0;
    for (int64_t s = s_min;; ) {
        double f_opt = 0.0, sse = 0.0;
        int rc = orc_bigmeans_fit(X, x_dtype, n, d, k, s, T, seed, o, 0, 0, C, deg, &f_opt,
                                  NULL, &sse, NULL, NULL, NULL);
        if (rc != 0) { free(C); free(deg); return -3; }
        if (m < 64) { s_tried[m] = s; sse_tried[m] = sse; }
        ++m;
        if (!(sse < best)) break;          /* no improvement: the sweet spot is behind */
        best = sse;
        best_s = s;
        if (s >= s_max || m >= 64) break;
        s = (s > s_max / 2) ? s_max : 2 * s;
    }
    *n_tried = m < 64 ? m : 64;
    free(C); free(deg);
    return best_s;
}
