// bm_internal.h -- declarations shared by the library's translation units
// (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bigmeans.h"
#include "bm_device.h"

namespace bm {

constexpr int kMaxTrials = 8;       // K-means++ candidates per centre
constexpr int kReplicas = 1;        // copies of the cluster-sum accumulators (workgroup g
                                    // adds into copy g % kReplicas); one measured best
constexpr int kMaxGrid = 1024;      // solver workgroups
constexpr int kNumCounters = 28;
constexpr unsigned int kDefaultSpinLimit = 1u << 24;

enum Counter {
  kCntPasses = 0,      // Lloyd assignment passes
  kCntReseeded = 1,    // centroids placed by K-means++
  kCntReplaced = 2,    // incumbent replacements
  kCntND = 3,          // distance evaluations at sample level
  kCntBoundary = 4,    // D^2 draws within rounding of a running-sum boundary
  kCntSamples = 5,     // samples processed
  kCntSelectPasses = 6, // histogram passes of the sampler (all samples)
  kCntTicksSample = 8,   // device wall-clock ticks spent per phase (workgroup 0)
  kCntTicksSeed = 9,
  kCntTicksLloyd = 10,
  kCntTicksPass = 11,    // Lloyd: assign + accumulate + flush + barrier
  kCntTicksPost = 12,    // Lloyd: gather of the reductions + centroid update
  kCntTicksBarrier = 13, // Lloyd: waiting in the pass barrier
  kCntTicksCollect = 14, // sampler: collect pass / its barrier wait / select / emit
  kCntTicksCollectWait = 15,
  kCntTicksSelect = 16,
  kCntTicksEmit = 17,
  kCntTicksAssign = 18,  // Lloyd pass: assignment + local accumulation / global flush
  kCntTicksFlush = 19,
  kCntTicksSeedInit = 20,    // K-means++: D^2 to the active slots (with its barrier)
  kCntTicksSeedLocate = 21,  //   per pick: total weight, owner search, candidates (barrier)
  kCntTicksSeedPot = 22,     //   potentials of the candidates (barrier)
  kCntTicksSeedUpdate = 23,  //   placement and D^2 update (barrier)
  kCntTicksAssignInit = 24,  // Lloyd pass: clearing the ring slot and the LDS sums
  kCntTicksAssignRows = 25,  //   the rows: nearest slot, objective term, LDS accumulation
  kCntTicksAssignSum = 26,   //   the workgroup's objective sum
};

enum SolverError {
  kErrNone = 0,
  kErrBarrier = 1,     // a grid-barrier wait exceeded its bound
  kErrSelect = 2,      // sampler bookkeeping inconsistent
  kErrSeed = 3,        // K-means++ found no candidate
};

// Everything the cooperative solver kernel needs; passed by value.
struct SolverArgs {
  const void* X;
  int64_t n;
  int64_t s;
  int32_t d;
  int32_t k;
  int32_t x_bf16;
  int32_t T;
  uint64_t seed;
  int32_t t0;
  int32_t max_iter;
  double tol;
  int32_t stop_rule;
  int32_t trials;
  int32_t cmp_rule;
  int32_t do_sample;
  int32_t do_gather;
  int32_t do_seed;
  int32_t do_lloyd;
  int32_t do_keep;
  int32_t init_incumbent;
  int32_t init_forgy;        // 1: degenerate slots take uniform rows (Forgy), not K-means++
  uint64_t budget_ticks;     // > 0: stop before a sample once this many wall-clock
                             // ticks have passed since the launch (sample 0 always runs)
  int32_t* stop_flag;        // workgroup 0's budget decision, read after a grid barrier
  int32_t sums_in_lds;       // replicas (1, 2, 4) of the FP64 cluster sums in LDS; 0: global ring
  int32_t c64_in_lds;
  int64_t cand_cap;          // capacity of the global candidate list
  uint64_t win_lo;           // predicted key window of the sampler (inclusive)
  uint64_t win_hi;
  uint32_t spin_limit;
  int32_t exact_draws;       // 1: every K-means++ draw takes the row-order sums (a test hook)
  int32_t sbatch;            // samples drawn per batch (slots of the buffers below)
  int32_t presampled;        // 1: every sample was drawn before the solver launch
  int32_t* presample_miss;   // 1: a presampled window missed (the solver samples)
  // sample-sized buffers (sbatch slots of each when sampling)
  float* P;                  // sbatch x s x d
  int32_t* idx;              // sbatch x s
  int32_t* labels;           // s
  double* w;                 // s (K-means++ D^2 weights)
  double* dcache;            // kMaxTrials x s: FP64 distances of streamed rows to the
                             // K-means++ candidates of the current centre
  // incumbent
  float* Cinc;               // k x d
  uint8_t* deg_inc;          // k
  double* f_opt;             // 1
  // reductions
  double* c64;               // 2 x k x d: FP64 centroid means (old / new)
  double* sums;              // 3 x kReplicas x k x d ring
  int32_t* cnt;              // 3 x kReplicas x k ring
  double* sse_part;          // 2 x kMaxGrid
  double* wsum;              // kMaxGrid
  double* phi_part;          // kMaxGrid x kMaxTrials
  int64_t* cand;             // kMaxTrials
  // sampler
  uint32_t* hist;            // 3 x 256 ring
  uint32_t* wg_lo;           // sbatch x kMaxGrid
  uint32_t* wg_off;          // sbatch x kMaxGrid
  uint64_t* cand_key;        // sbatch x cand_cap
  int32_t* cand_idx;         // sbatch x cand_cap
  uint32_t* cand_count;      // sbatch
  uint8_t* selcode;          // sbatch x n: key below (1), inside (2), above (0) the window
  uint64_t* thr;             // sbatch x 2: threshold key, index
  int32_t* smiss;            // sbatch: the predicted window missed
  // outputs / control
  int32_t* sample_idx_out;   // T x s or null
  double* sample_f;          // T
  int64_t* counters;         // kNumCounters
  GridBarrier* bar;
  int32_t* err;
};

// Device scratch pool (per process, current device); grows on demand.  A
// thread may switch to a pool of its own (serving slots); nullptr restores the
// shared pool.
struct ScratchPool {
  void* ptr = nullptr;
  size_t bytes = 0;
};
void* scratch_get(size_t bytes, hipStream_t stream, bm_status* st);
void scratch_release();
void scratch_set_thread_pool(ScratchPool* p);
void scratch_pool_free(ScratchPool* p);
bm_status scratch_pool_reserve(ScratchPool* p, size_t bytes);  // exactly `bytes` if it grows

// bigmeans_fit in parts (bm_api.hip), for the serving engine.
bm_status fit_validate(const void* X, int64_t n, int32_t d, int32_t k, int64_t s,
                       int32_t n_samples, const bm_options* opt_in, float* centroids,
                       uint8_t* degenerate, bm_stats* stats, bm_options* o);
size_t fit_scratch_bytes(int64_t n, int32_t d, int32_t k, int64_t s, int32_t n_samples,
                         bool final_pass);
bm_status fit_run(const void* X, int64_t n, int32_t d, int32_t k, int64_t s, int32_t n_samples,
                  uint64_t seed, const bm_options& o, float* centroids, double* sse,
                  int32_t* labels, uint8_t* degenerate, bm_stats* stats, int grid_cap);
bm_status solver_coresident_blocks(int d, int k, int64_t s, int64_t n, int* blocks);

// Options with defaults filled in and validated (bm_api.hip).
bm_status resolve_options(const bm_options* in, bm_options* out);

// Error reporting for the ABI layer.
bm_status set_error(bm_status code, const char* fmt, ...);
void clear_error();

// Launchers (defined in bm_solver.hip / bm_assign.hip).
size_t solver_lds_bytes(int dm, int k, int d, int sums_reps, bool c64_in_lds);
void sampler_window(int64_t n, int64_t s, uint64_t* lo, uint64_t* hi, int64_t* cap);
// Samples drawn per batch by bigmeans_fit: all T when their buffers (rows,
// indices, codes, candidates) fit in kSampleBatchBytes, else fewer (>= 1).
constexpr double kSampleBatchBytes = 4096.0 * 1024 * 1024;
int sample_slots(int64_t n, int64_t s, int d, int T, int64_t cand_cap);
int padded_dim(int d);
bm_status launch_solver(const SolverArgs& a, int grid, size_t lds, hipStream_t stream);
// All a.T samples drawn into their slots by ordinary launches (a.sbatch == a.T);
// sets a.presampled.
bm_status launch_presample(SolverArgs& a, size_t lds, hipStream_t stream, bool force_miss = false);
bm_status solver_max_grid(int dm, size_t lds, int* max_grid);
bm_status max_lds_per_block(size_t* bytes);
// Raises kernel fn's dynamic-LDS limit on the current device to at least
// `bytes` (nothing to do up to 64 KiB).  The attribute is set once per
// function, device and larger size, under a lock, not on every launch.
bm_status reserve_lds(const void* fn, size_t bytes);

// HIP events destroyed when the scope ends, on every return path.
template <int N>
struct EventSet {
  hipEvent_t e[N] = {};
  EventSet() = default;
  EventSet(const EventSet&) = delete;
  EventSet& operator=(const EventSet&) = delete;
  ~EventSet() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
  hipError_t create() {
    for (auto& x : e) {
      const hipError_t r = hipEventCreate(&x);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  }
  hipEvent_t& operator[](int i) { return e[i]; }
};

bm_status launch_assign(const void* X, int x_bf16, int64_t n, int d, const float* C,
                        const uint8_t* deg_dev, int k, int32_t* labels, float* min_d2,
                        double* partial, double* sse_dev, int grid, hipStream_t stream);
int assign_grid(int64_t n, int d);
// *out = the np partials added in a fixed order (one workgroup).
bm_status launch_sum_partials(const double* partial, int np, double* out, hipStream_t stream);

// Batched Lloyd (bm_batch.hip): per-solve state, laid out in device memory.
constexpr int kSolveRunning = 0;  // next round: assignment + update
constexpr int kSolveFinal = 1;    // next round: the last assignment only
constexpr int kSolveDone = 2;
struct BatchSolve {
  int64_t row0, s;      // rows of P
  int32_t c0, k;        // rows of C
  int32_t tile0, ntiles;
  int32_t status, iter;  // iter: 1-based index of the next assignment
  int32_t passes, pad;
  double f, f_prev;
  int64_t nd;           // distance evaluations of its assignment passes (s x active slots)
};
size_t batch_assign_lds(int d, int kmax, bool sums_lds);
bm_status batch_assign_grid(int d, int kmax, bool sums_lds, int* grid);
// Pp: rows DM = padded_dim(d) wide, zero padded (launch_pad_rows).
bm_status launch_batch_assign(const float* Pp, int d, const float* C, const float* Cpad,
                              const uint8_t* deg, const BatchSolve* sv, const int32_t* tile_solve,
                              int ntiles, int tile_rows, int kmax, bool sums_lds, double* sums,
                              int32_t* cnt, double* tile_f, int32_t* labels, int dry, int grid,
                              hipStream_t stream, const int32_t* labels_in = nullptr,
                              double* partials = nullptr, int32_t* pcnt = nullptr);
// One solve (sv[0]) accumulated as per-workgroup partial blocks (partials:
// grid x k x DM, pcnt: grid x k, from launch_batch_assign): sums and counts
// added in workgroup order.
bm_status launch_batch_reduce(const double* partials, const int32_t* pcnt, int nparts, int k, int d,
                              double* sums, int32_t* cnt, const BatchSolve* sv, hipStream_t stream);
// One solve (sv[0]) with labels given: FP64 sums, counts (partial blocks,
// grid x k x DM and grid x k) and the objective partials (tile_f, grid) of
// d-wide BF16 rows (grid <= s workgroups, each a contiguous range of rows).
size_t labels_accum_lds(int d, int k);
bm_status launch_labels_accum(const uint16_t* P, int64_t s, int d, int k, const float* C,
                              const int32_t* labels, const BatchSolve* sv, double* partials,
                              int32_t* pcnt, double* tile_f, int grid, hipStream_t stream);
// P[r] = X[idx[r]] for BF16 rows (bit copies); idx from the sampler.
bm_status launch_gather_rows_bf16(const uint16_t* X, int d, const int32_t* idx, int64_t s,
                                  uint16_t* P, hipStream_t stream);
bm_status launch_batch_update(BatchSolve* sv, int n_solves, const double* tile_f, double* sums,
                              int32_t* cnt, float* C, float* Cpad, double* C64, uint8_t* deg, int d,
                              int max_iter, double tol, int stop_rule, int* running,
                              hipStream_t stream, int kmax);
// One solve's start (sv[0] = init; working centroids and flags copied from
// the incumbent; sums and counts cleared).
bm_status launch_solve_start(const float* Cinc, const uint8_t* deginc, float* cw, uint8_t* degw,
                             BatchSolve* sv, const BatchSolve& init, double* sums, int32_t* cnt, int k,
                             int d, hipStream_t stream);
bm_status launch_batch_init(const float* C, double* C64, float* Cpad, int64_t rows, int d,
                            hipStream_t stream);
bm_status launch_pad_rows(const float* P, float* Pp, int64_t rows, int d, hipStream_t stream);
bm_status launch_gather_rows(const void* X, int x_bf16, int64_t n, int d, const int32_t* idx,
                             int64_t s, float* P, int* bad, hipStream_t stream);

// BF16 matrix-core assignment (bm_assign_mfma.hip): plan checks the shape and
// picks the grid; the launch writes the same outputs as launch_assign and
// adds the number of points it recomputed on the FP32 path to *rechecked.
bm_status plan_assign_mfma(const void* X, int64_t n, int d, int k, int* grid);
// FP32 X on the matrix cores (bm_assign_mfma32.hip): labels of the FP32
// direct-difference path; launch_assign takes this form when it applies.
bm_status plan_assign_mfma32(const void* X, int64_t n, int d, int k, int* grid);
bm_status launch_assign_mfma32(const float* X, int64_t n, int d, const float* C, const uint8_t* deg_dev,
                               int k, int32_t* labels, float* min_d2, double* partial,
                               double* sse_dev, unsigned long long* rechecked, int grid,
                               hipStream_t stream);
bool fp32_mfma_enabled();
bool exact_draws_forced();  // every K-means++ draw takes the row-order sums (test hook)
// The batched assignment with matrix-core labels (same results as
// launch_batch_assign's kernel; no labels_in / partial-block modes).
size_t batch_assign_mfma32_lds(int d, int kmax, bool sums_lds);
bm_status launch_batch_assign_mfma32(const float* Pp, int d, const float* C, const uint8_t* deg,
                                     const BatchSolve* sv, const int32_t* tile_solve, int ntiles,
                                     int tile_rows, int kmax, bool sums_lds, double* sums,
                                     int32_t* cnt, double* tile_f, int32_t* labels, int dry,
                                     hipStream_t stream);
// With `stop` (a solve's status word) the launch does nothing once the solve
// is done; partial == nullptr leaves the objective out (labels only).
bm_status launch_assign_mfma(const uint16_t* X, int64_t n, int d, const float* C,
                             const uint8_t* deg_dev, int k, int32_t* labels, float* min_d2,
                             double* partial, double* sse_dev, unsigned long long* rechecked,
                             int grid, hipStream_t stream,
                             const int32_t* stop = nullptr);

}  // namespace bm
