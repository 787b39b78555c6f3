// bm_serve.hip -- serving many Big-means jobs on one GPU (the stream of
// clustering requests of the big-data setting the paper motivates in Sec. 2).
//
// A context owns `slots` worker threads.  Each slot has its own HIP stream
// and its own device scratch pool, so jobs on different slots share no state
// and run concurrently.  Jobs are admitted strictly in submission order: the
// head of the queue starts on the first idle slot as soon as the scratch it
// needs fits in the context's HBM budget together with what the other slots
// hold.  An idle slot whose pool stands in the head job's way gives its pool
// back, so a job that fits the budget alone always starts eventually.
//
// Every job's cooperative solver grid is capped at CUs / slots workgroups:
// the solver kernels of all slots then fit on the device at the same time
// (each workgroup fits on one CU), so their grid barriers cannot wait on each
// other.  A job's result does not depend on the grid (integer outputs are
// identical, objectives agree to rounding), so a job run in the mix gives the
// result it gives alone.
//
// BM_SERVE_ROUNDS mode (continuous batching): an engine keeps up to `slots`
// jobs in flight.  A prep thread gives a job that needs a sample its draw
// (Philox keys, Sec. 3.2), gathers and pads it into the job's slot of an
// arena, and reseeds the degenerate incumbent slots by K-means++ (Sec. 3.3),
// exactly as the persistent solver does for sample t.  The round thread runs
// the Lloyd rounds of every job whose sample is ready together, one batched
// assignment + update launch per (d, stop rule) class and round, so jobs join
// and leave at round boundaries.  A job whose sample converged keeps the
// better of its incumbent and the new centroids (Alg. 1), goes back to the
// prep thread for its next sample, and after the last one gets the
// full-data assignment there.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string.h>
#include <string>
#include <thread>
#include <vector>

#include "bm_internal.h"

struct bm_ctx;

namespace bm {
namespace {

using Clock = std::chrono::steady_clock;

struct Job {
  bm_job spec;
  bm_options opt;
  size_t alloc = 0;  // scratch bytes the job's pool must hold
  int32_t state = BM_JOB_QUEUED;
  bm_status result = BM_OK;
  int32_t slot = -1;
  double t_submit = 0, t_start = 0, t_end = 0;
  char error[160] = "";
};

struct Slot {
  hipStream_t stream = nullptr;
  ScratchPool pool;
};

// --- BM_SERVE_ROUNDS ------------------------------------------------------

constexpr int kRoundTile = 512;  // sample rows per work-list tile
// Rounds queued per host synchronisation of the round thread.  A solve that
// finishes inside the group is skipped by the rest of it (the batched kernels
// skip done solves), so its results are those of a round-by-round loop; it
// waits at most kRoundsPerSync - 1 rounds longer for its hand-over, while
// every other job saves kRoundsPerSync - 1 synchronisations and hand-overs.
constexpr int kRoundsPerSync = 4;

// Jobs whose Lloyd rounds run in the same launch: same d and stop rule.
struct ClassKey {
  int d, max_iter, stop_rule;
  double tol;
  bool operator<(const ClassKey& o) const {
    if (d != o.d) return d < o.d;
    if (max_iter != o.max_iter) return max_iter < o.max_iter;
    if (stop_rule != o.stop_rule) return stop_rule < o.stop_rule;
    return tol < o.tol;
  }
};

// One class's device arena: `nslot` job slots of smax sample rows (dm wide,
// zero padded) and kmax centroids each, the batched kernels' per-centroid
// state, the solve states and the work list.
struct Arena {
  ClassKey key{};
  int d = 0, dm = 0, nslot = 0, kmax = 0, grid = 0;
  int64_t smax = 0;
  bool sums_lds = false;
  void* mem = nullptr;
  size_t bytes = 0;
  float* P = nullptr;
  float* C = nullptr;
  float* Cpad = nullptr;
  double* c64 = nullptr;
  double* sums = nullptr;
  int32_t* cnt = nullptr;
  uint8_t* deg = nullptr;
  BatchSolve* sv = nullptr;
  int32_t* tiles = nullptr;
  double* tile_f = nullptr;
  int* running = nullptr;
  std::vector<int> owner;           // job id index per slot, -1 free
  std::vector<BatchSolve> hs;       // host copy of the solve states after a round
  std::vector<int32_t> tile_solve;  // work list (solve of each tile)
  bool tiles_dirty = true;
  int in_lloyd = 0;                 // slots whose solve is running
};

// Stage of a job in flight.  The prep thread owns a job in kPrepping and
// kFinalizing, the round thread in kLloyd; transitions happen under the
// context's mutex, after the owner has synchronized its stream.
enum Stage { kPrep, kPrepping, kReady, kLloyd, kFinal, kFinalizing, kEnded };

struct RJob {
  int64_t id = 0;
  Job* job = nullptr;
  Arena* ar = nullptr;
  int slot = -1;
  int t = 0;             // samples done
  int stage = kPrep;
  bool lloyd = false;    // the current sample's solve is in the arena
  std::vector<uint8_t> deg_inc, deg_work;
  double f_opt = 0.0;
  int32_t replacements = 0;
  int64_t iters = 0, reseeded = 0;
  bm_status result = BM_OK;
  bool started = false;  // incumbent set up
  bool finished = false;
  char error[160] = "";
};

}  // namespace
}  // namespace bm

using namespace bm;

struct bm_ctx {
  int device = 0;
  int nslots = 0;
  int64_t budget = 0;
  int grid_cap = 0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  std::deque<int64_t> queue;
  std::map<int64_t, std::unique_ptr<Job>> jobs;
  std::vector<Slot> slots;
  std::vector<std::thread> workers;
  int64_t next_id = 1;
  int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, running = 0;
  int64_t reserved = 0, peak_reserved = 0;  // bytes held by all slot pools
  bool stopping = false;
  // BM_SERVE_ROUNDS
  int mode = BM_SERVE_FITS;
  int round_max_k = 0;
  int64_t round_max_s = 0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }

  // Scratch bytes scratch_get() allocates for a request of `bytes`.
  static size_t pool_alloc(size_t bytes) { return bytes + bytes / 4 + (1u << 20); }

  void engine();  // BM_SERVE_ROUNDS
  // Record the end of job j (under mu).
  void finish_job(Job* j, bm_status st, const char* msg) {
    j->result = st;
    j->state = st == BM_OK ? BM_JOB_DONE : BM_JOB_FAILED;
    if (st != BM_OK) snprintf(j->error, sizeof j->error, "%s", msg ? msg : "");
    j->t_end = now_ms();
    --running;
    if (st == BM_OK) ++completed; else ++failed;
  }

  void worker(int i) {
    Slot& sl = slots[i];
    if (hipSetDevice(device) != hipSuccess) return;
    scratch_set_thread_pool(&sl.pool);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      Job* job = nullptr;
      for (;;) {
        if (stopping && queue.empty()) break;
        if (!queue.empty()) {
          Job* head = jobs[queue.front()].get();
          const int64_t mine = static_cast<int64_t>(sl.pool.bytes);
          const int64_t need = static_cast<int64_t>(head->alloc) > mine ? static_cast<int64_t>(head->alloc) : mine;
          if (reserved - mine + need <= budget) {
            job = head;
            queue.pop_front();
            reserved += need - mine;  // the pool grows to `need` when the job starts
            peak_reserved = reserved > peak_reserved ? reserved : peak_reserved;
            break;
          }
          if (sl.pool.bytes > 0) {  // give this idle slot's pool back to the budget
            lk.unlock();
            (void)hipStreamSynchronize(sl.stream);
            scratch_pool_free(&sl.pool);
            lk.lock();
            reserved -= mine;
            cv_work.notify_all();
            continue;
          }
        }
        cv_work.wait(lk);
      }
      if (!job) break;
      job->state = BM_JOB_RUNNING;
      job->slot = i;
      job->t_start = now_ms();
      ++running;
      lk.unlock();

      const int64_t before = static_cast<int64_t>(sl.pool.bytes);
      bm_options o = job->opt;
      o.stream = sl.stream;
      clear_error();
      // size the pool to the reservation made above
      bm_status st = scratch_pool_reserve(&sl.pool, job->alloc);
      if (st == BM_OK) {
        const bm_job& J = job->spec;
        st = fit_run(J.X, J.n, J.d, J.k, J.s, J.n_samples, J.seed, o, J.centroids, J.sse, J.labels,
                     J.degenerate, J.stats, grid_cap);
      }
      const char* msg = bm_last_error();

      lk.lock();
      // the pool may have grown past the reservation (only if the estimate
      // was low); keep the accounting exact
      reserved += static_cast<int64_t>(sl.pool.bytes) -
                  (before > static_cast<int64_t>(job->alloc) ? before : static_cast<int64_t>(job->alloc));
      peak_reserved = reserved > peak_reserved ? reserved : peak_reserved;
      job->result = st;
      job->state = st == BM_OK ? BM_JOB_DONE : BM_JOB_FAILED;
      if (st != BM_OK) snprintf(job->error, sizeof job->error, "%s", msg ? msg : "");
      job->t_end = now_ms();
      --running;
      if (st == BM_OK) ++completed; else ++failed;
      cv_done.notify_all();
      cv_work.notify_all();
    }
    lk.unlock();
    (void)hipStreamSynchronize(sl.stream);
    scratch_pool_free(&sl.pool);
    scratch_set_thread_pool(nullptr);
  }
};

namespace {

// Device memory of an arena for class `key` with `nslot` slots.
bm_status arena_create(const ClassKey& key, int nslot, int64_t smax, int kmax, Arena* A) {
  A->key = key;
  A->d = key.d;
  A->dm = padded_dim(key.d);
  A->nslot = nslot;
  A->smax = smax;
  A->kmax = kmax;
  if (A->dm < 0) return set_error(BM_ENOTSUP, "d = %d exceeds the limit of 256", key.d);
  size_t lds_max = 0;
  bm_status st = max_lds_per_block(&lds_max);
  if (st != BM_OK) return st;
  A->sums_lds = batch_assign_lds(A->d, kmax, true) + 1024 <= lds_max;
  if (!A->sums_lds && batch_assign_lds(A->d, kmax, false) + 1024 > lds_max)
    return set_error(BM_ENOTSUP, "k x d = %d x %d centroids do not fit one workgroup's LDS", kmax, A->d);
  if ((st = batch_assign_grid(A->d, kmax, A->sums_lds, &A->grid)) != BM_OK) return st;
  const size_t ns = static_cast<size_t>(nslot), dm = static_cast<size_t>(A->dm);
  const size_t kt = ns * kmax, rows = ns * static_cast<size_t>(smax);
  const size_t tiles = ns * static_cast<size_t>((smax + kRoundTile - 1) / kRoundTile);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = (off + bytes + 255) & ~size_t(255); return o; };
  const size_t oP = take(rows * dm * 4), oC = take(kt * A->d * 4), oCp = take(kt * dm * 4);
  const size_t o64 = take(kt * A->d * 8), oS = take(kt * dm * 8), oN = take(kt * 4), oD = take(kt);
  const size_t oV = take(ns * sizeof(BatchSolve)), oT = take(tiles * 4), oF = take(tiles * 8);
  const size_t oR = take(sizeof(int));
  if (hipMalloc(&A->mem, off) != hipSuccess) {
    A->mem = nullptr;
    return set_error(BM_ENOMEM, "cannot allocate a %zu-byte serving arena", off);
  }
  A->bytes = off;
  char* b = static_cast<char*>(A->mem);
  A->P = reinterpret_cast<float*>(b + oP);
  A->C = reinterpret_cast<float*>(b + oC);
  A->Cpad = reinterpret_cast<float*>(b + oCp);
  A->c64 = reinterpret_cast<double*>(b + o64);
  A->sums = reinterpret_cast<double*>(b + oS);
  A->cnt = reinterpret_cast<int32_t*>(b + oN);
  A->deg = reinterpret_cast<uint8_t*>(b + oD);
  A->sv = reinterpret_cast<BatchSolve*>(b + oV);
  A->tiles = reinterpret_cast<int32_t*>(b + oT);
  A->tile_f = reinterpret_cast<double*>(b + oF);
  A->running = reinterpret_cast<int*>(b + oR);
  A->owner.assign(nslot, -1);
  A->hs.assign(nslot, BatchSolve{});
  for (auto& h : A->hs) h.status = kSolveDone;  // free slots take no part in a round
  if (hipMemcpy(A->sv, A->hs.data(), ns * sizeof(BatchSolve), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(A->sums, 0, kt * dm * 8) != hipSuccess || hipMemset(A->cnt, 0, kt * 4) != hipSuccess)
    return set_error(BM_EDEVICE, "cannot initialise a serving arena");
  return BM_OK;
}

// Engine-wide staging for the sample stage: indices, the unpadded rows (the
// K-means++ reseed reads them), and the gather's bad-index flag.
struct Staging {
  int32_t* idx = nullptr;
  float* P = nullptr;
  int* bad = nullptr;
  size_t idx_cap = 0, p_cap = 0;
  int64_t bytes() const { return static_cast<int64_t>(idx_cap * 4 + p_cap * 4 + 256); }
};

bm_status staging_reserve(Staging* g, int64_t s, int d) {
  if (!g->bad && hipMalloc(reinterpret_cast<void**>(&g->bad), 256) != hipSuccess) {
    g->bad = nullptr;
    return set_error(BM_ENOMEM, "cannot allocate staging");
  }
  const size_t ni = static_cast<size_t>(s), np = static_cast<size_t>(s) * d;
  if (ni > g->idx_cap) {
    if (g->idx) (void)hipFree(g->idx);
    g->idx = nullptr;
    g->idx_cap = 0;
    if (hipMalloc(reinterpret_cast<void**>(&g->idx), ni * 4) != hipSuccess)
      return set_error(BM_ENOMEM, "cannot allocate staging");
    g->idx_cap = ni;
  }
  if (np > g->p_cap) {
    if (g->P) (void)hipFree(g->P);
    g->P = nullptr;
    g->p_cap = 0;
    if (hipMalloc(reinterpret_cast<void**>(&g->P), np * 4) != hipSuccess)
      return set_error(BM_ENOMEM, "cannot allocate staging");
    g->p_cap = np;
  }
  return BM_OK;
}

#define BM_HIPR(call)                                                                     \
  do {                                                                                    \
    const hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) return set_error(BM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// Sample t0 + t of job r (Alg. 1): draw, gather, copy the incumbent, reseed
// its degenerate slots with K-means++ on the sample, and lay the sample and
// the start centroids out in the job's arena slot (its solve state is left
// to the round thread).  Runs on the prep thread; synchronous on `stream`.
bm_status prep_sample(RJob& r, Staging& g, hipStream_t stream) {
  const bm_job& J = r.job->spec;
  const bm_options& jo = r.job->opt;
  Arena& A = *r.ar;
  const int d = J.d, k = J.k, dm = A.dm;
  const int64_t s = J.s;
  if (!r.started) {  // incumbent of a new job: every slot degenerate, or resumed
    r.started = true;
    if (jo.resume) {
      memcpy(r.deg_inc.data(), J.degenerate, static_cast<size_t>(k));
      r.f_opt = jo.f_opt_in;
    } else {
      BM_HIPR(hipMemsetAsync(J.centroids, 0xff, sizeof(float) * k * d, stream));  // NaN rows
    }
  }
  const int32_t t = jo.t_start + r.t;
  bm_options o = jo;
  o.stream = stream;
  o.grid = 0;
  bm_status st = staging_reserve(&g, s, d);
  if (st != BM_OK) return st;
  if ((st = bm_sample_indices(J.n, s, J.seed, t, g.idx, &o)) != BM_OK) return st;
  BM_HIPR(hipMemsetAsync(g.bad, 0, sizeof(int), stream));
  if ((st = launch_gather_rows(J.X, jo.x_dtype == BM_BF16, J.n, d, g.idx, s, g.P, g.bad, stream)) != BM_OK)
    return st;
  if (jo.sample_idx)
    BM_HIPR(hipMemcpyAsync(jo.sample_idx + static_cast<size_t>(r.t) * s, g.idx, sizeof(int32_t) * s,
                           hipMemcpyDeviceToDevice, stream));
  const size_t c0 = static_cast<size_t>(r.slot) * A.kmax;
  const size_t row0 = static_cast<size_t>(r.slot) * A.smax;
  float* Cw = A.C + c0 * d;
  BM_HIPR(hipMemcpyAsync(Cw, J.centroids, sizeof(float) * k * d, hipMemcpyDeviceToDevice, stream));
  r.deg_work = r.deg_inc;
  int before = 0;
  for (int j = 0; j < k; ++j) before += r.deg_work[j];
  if (before) {
    if ((st = kmeanspp_seed(g.P, s, d, k, Cw, r.deg_work.data(), J.seed, static_cast<uint64_t>(t), &o)) != BM_OK)
      return st;
    int after = 0;
    for (int j = 0; j < k; ++j) after += r.deg_work[j];
    if (after == k) return set_error(BM_EDEVICE, "K-means++ left every slot degenerate");
    r.reseeded += before - after;
  }
  if (dm == d) {
    BM_HIPR(hipMemcpyAsync(A.P + row0 * dm, g.P, sizeof(float) * s * d, hipMemcpyDeviceToDevice, stream));
  } else if ((st = launch_pad_rows(g.P, A.P + row0 * dm, s, d, stream)) != BM_OK) {
    return st;
  }
  if ((st = launch_batch_init(Cw, A.c64 + c0 * d, A.Cpad + c0 * dm, k, d, stream)) != BM_OK) return st;
  BM_HIPR(hipMemcpyAsync(A.deg + c0, r.deg_work.data(), static_cast<size_t>(k), hipMemcpyHostToDevice, stream));
  int bad = 0;
  BM_HIPR(hipMemcpyAsync(&bad, g.bad, sizeof(int), hipMemcpyDeviceToHost, stream));
  BM_HIPR(hipStreamSynchronize(stream));
  if (bad) return set_error(BM_EINVAL, "a sampled index is outside [0, n)");
  return BM_OK;
}

// Start the prepared solve of job r in its arena (round thread, between
// rounds): its state goes to the device on the round stream.
bm_status activate(RJob& r, hipStream_t stream) {
  const bm_job& J = r.job->spec;
  Arena& A = *r.ar;
  BatchSolve& h = A.hs[r.slot];
  const int keep0 = h.tile0, keepn = h.ntiles;
  if (keepn != static_cast<int>((J.s + kRoundTile - 1) / kRoundTile)) A.tiles_dirty = true;
  memset(&h, 0, sizeof h);
  h.row0 = static_cast<int64_t>(r.slot) * A.smax;
  h.s = J.s;
  h.c0 = static_cast<int32_t>(static_cast<int64_t>(r.slot) * A.kmax);
  h.k = J.k;
  h.tile0 = keep0;
  h.ntiles = keepn;
  h.status = kSolveRunning;
  h.iter = 1;
  h.f_prev = __builtin_inf();
  BM_HIPR(hipMemcpyAsync(A.sv + r.slot, &h, sizeof(BatchSolve), hipMemcpyHostToDevice, stream));
  r.lloyd = true;
  ++A.in_lloyd;
  return BM_OK;
}

// One assignment + update round of every running solve of arena A.
bm_status arena_round(Arena& A, hipStream_t stream) {
  if (A.tiles_dirty) {
    A.tile_solve.clear();
    for (int q = 0; q < A.nslot; ++q) {
      if (A.owner[q] < 0) continue;
      const int nt = static_cast<int>((A.smax + kRoundTile - 1) / kRoundTile);
      (void)nt;
      BatchSolve& h = A.hs[q];
      const int need = static_cast<int>((h.s + kRoundTile - 1) / kRoundTile);
      h.tile0 = static_cast<int32_t>(A.tile_solve.size());
      h.ntiles = need;
      for (int i = 0; i < need; ++i) A.tile_solve.push_back(q);
      BM_HIPR(hipMemcpyAsync(&A.sv[q].tile0, &h.tile0, 2 * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    }
    if (!A.tile_solve.empty())
      BM_HIPR(hipMemcpyAsync(A.tiles, A.tile_solve.data(), sizeof(int32_t) * A.tile_solve.size(),
                             hipMemcpyHostToDevice, stream));
    BM_HIPR(hipStreamSynchronize(stream));  // the host vectors are reused
    A.tiles_dirty = false;
  }
  const int nt = static_cast<int>(A.tile_solve.size());
  if (nt == 0) return BM_OK;
  bm_status st = launch_batch_assign(A.P, A.d, A.C, A.Cpad, A.deg, A.sv, A.tiles, nt, kRoundTile, A.kmax,
                                     A.sums_lds, A.sums, A.cnt, A.tile_f, nullptr, 0, A.grid, stream);
  if (st != BM_OK) return st;
  st = launch_batch_update(A.sv, A.nslot, A.tile_f, A.sums, A.cnt, A.C, A.Cpad, A.c64, A.deg, A.d,
                           A.key.max_iter, A.key.tol, A.key.stop_rule, A.running, stream, A.kmax);
  if (st != BM_OK) return st;
  BM_HIPR(hipMemcpyAsync(A.hs.data(), A.sv, sizeof(BatchSolve) * A.nslot, hipMemcpyDeviceToHost, stream));
  return BM_OK;
}

// The solve of job r finished (round thread): keep the better centroids
// (Alg. 1) and count the sample.  Synchronous on `stream`.
bm_status keep_best(RJob& r, hipStream_t stream) {
  const bm_job& J = r.job->spec;
  const bm_options& jo = r.job->opt;
  Arena& A = *r.ar;
  const int d = J.d, k = J.k;
  const BatchSolve& h = A.hs[r.slot];
  const double f = h.f;
  r.iters += h.passes;
  r.lloyd = false;
  --A.in_lloyd;
  const size_t c0 = static_cast<size_t>(r.slot) * A.kmax;
  if (jo.sample_f) jo.sample_f[r.t] = f;
  if (f < r.f_opt) {
    BM_HIPR(hipMemcpyAsync(J.centroids, A.C + c0 * d, sizeof(float) * k * d, hipMemcpyDeviceToDevice, stream));
    BM_HIPR(hipMemcpyAsync(r.deg_inc.data(), A.deg + c0, static_cast<size_t>(k), hipMemcpyDeviceToHost, stream));
    BM_HIPR(hipStreamSynchronize(stream));
    r.f_opt = f;
    ++r.replacements;
  }
  ++r.t;
  return BM_OK;
}

// After the last sample (prep thread): the full-data assignment (Alg. 1 last
// step) and the job's outputs.
bm_status final_pass(RJob& r, hipStream_t stream) {
  const bm_job& J = r.job->spec;
  const bm_options& jo = r.job->opt;
  const int d = J.d, k = J.k;
  bm_options o = jo;
  o.stream = stream;
  double sse = 0.0;
  if (J.sse || J.labels) {
    bm_status st = kmeans_assign(J.X, J.n, d, J.centroids, r.deg_inc.data(), k, &o, J.labels, nullptr, &sse);
    if (st != BM_OK) return st;
  }
  BM_HIPR(hipStreamSynchronize(stream));
  if (J.sse) *J.sse = sse;
  if (J.degenerate) memcpy(J.degenerate, r.deg_inc.data(), static_cast<size_t>(k));
  if (J.stats) {
    bm_stats* S = J.stats;
    const uint32_t size = S->struct_size;
    memset(S, 0, sizeof *S);
    S->struct_size = size;
    S->samples = r.t;
    S->replacements = r.replacements;
    S->grid = r.ar->grid;
    S->lloyd_iters = r.iters;
    S->reseeded = r.reseeded;
    S->f_opt = r.f_opt;
  }
  r.finished = true;
  return BM_OK;
}

}  // namespace

// The BM_SERVE_ROUNDS engine.  The round thread (this function) admits jobs,
// starts prepared solves, runs one batched round per class while any solve
// runs, keeps the best centroids of finished solves and retires jobs; a prep
// thread draws, gathers and reseeds samples and runs final passes on its own
// stream meanwhile, so a job's sample stage does not hold up the others'
// rounds.  Arena slots are disjoint and a slot's solve is marked done while
// the prep thread fills it, and the batched kernels skip done solves, so the
// two streams never touch the same bytes.
void bm_ctx::engine() {
  Slot& sl = slots[0];
  if (hipSetDevice(device) != hipSuccess) return;
  std::map<ClassKey, std::unique_ptr<Arena>> arenas;
  std::vector<std::unique_ptr<RJob>> live;
  int64_t arena_bytes = 0;
  bool prep_stop = false;
  std::condition_variable cv_prep;

  std::thread prep([&] {
    if (hipSetDevice(device) != hipSuccess) return;
    ScratchPool pool;
    scratch_set_thread_pool(&pool);
    hipStream_t ps = nullptr;
    const bool ok = hipStreamCreateWithFlags(&ps, hipStreamNonBlocking) == hipSuccess;
    Staging stage;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      RJob* r = nullptr;
      for (auto& x : live)
        if (x->stage == kPrep || x->stage == kFinal) {
          r = x.get();
          break;
        }
      if (!r) {
        if (prep_stop) break;
        cv_prep.wait(lk);
        continue;
      }
      const bool fin = r->stage == kFinal;
      r->stage = fin ? kFinalizing : kPrepping;
      lk.unlock();
      clear_error();
      bm_status st = !ok ? set_error(BM_EDEVICE, "cannot create the prep stream")
                         : fin ? final_pass(*r, ps) : prep_sample(*r, stage, ps);
      const std::string msg = st == BM_OK ? "" : bm_last_error();
      lk.lock();
      if (st != BM_OK) {
        r->result = st;
        snprintf(r->error, sizeof r->error, "%s", msg.c_str());
        r->stage = kEnded;
      } else {
        r->stage = fin ? kEnded : kReady;
      }
      cv_work.notify_all();
    }
    lk.unlock();
    if (ps) {
      (void)hipStreamSynchronize(ps);
      (void)hipStreamDestroy(ps);
    }
    if (stage.idx) (void)hipFree(stage.idx);
    if (stage.P) (void)hipFree(stage.P);
    if (stage.bad) (void)hipFree(stage.bad);
    scratch_pool_free(&pool);
    scratch_set_thread_pool(nullptr);
  });

  hipStream_t stream = sl.stream;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // admit queued jobs in submission order while a slot is free
    bool new_prep = false;
    while (!queue.empty() && static_cast<int>(live.size()) < nslots) {
      const int64_t id = queue.front();
      Job* j = jobs[id].get();
      queue.pop_front();
      j->state = BM_JOB_RUNNING;
      j->t_start = now_ms();
      ++running;
      const bm_job& J = j->spec;
      const ClassKey key{J.d, j->opt.max_iter, j->opt.stop_rule, j->opt.tol};
      auto it = arenas.find(key);
      if (it == arenas.end()) {
        std::unique_ptr<Arena> A(new Arena());
        clear_error();
        bm_status st = arena_create(key, nslots, round_max_s, round_max_k, A.get());
        if (st == BM_OK && reserved + static_cast<int64_t>(A->bytes) > budget)
          st = set_error(BM_ENOMEM, "a serving arena of %zu bytes exceeds the budget", A->bytes);
        if (st != BM_OK) {
          if (A->mem) (void)hipFree(A->mem);
          finish_job(j, st, bm_last_error());
          cv_done.notify_all();
          continue;
        }
        arena_bytes += static_cast<int64_t>(A->bytes);
        reserved += static_cast<int64_t>(A->bytes);
        peak_reserved = reserved > peak_reserved ? reserved : peak_reserved;
        it = arenas.emplace(key, std::move(A)).first;
      }
      Arena* A = it->second.get();
      int q = 0;
      while (q < A->nslot && A->owner[q] >= 0) ++q;  // a free slot exists: live < nslots
      std::unique_ptr<RJob> r(new RJob());
      r->id = id;
      r->job = j;
      r->ar = A;
      r->slot = q;
      j->slot = q;
      A->owner[q] = static_cast<int>(id & 0x7fffffff);
      A->tiles_dirty = true;  // the work list must cover the new owner's rows
      r->deg_inc.assign(J.k, 1);
      r->f_opt = __builtin_inf();
      live.push_back(std::move(r));
      new_prep = true;
    }
    if (new_prep) cv_prep.notify_all();
    // retire ended jobs, freeing their slots
    for (auto it = live.begin(); it != live.end();) {
      RJob& r = **it;
      if (r.stage != kEnded) {
        ++it;
        continue;
      }
      Arena& A = *r.ar;
      if (r.lloyd) {  // a failed job's solve is dropped from the next rounds
        --A.in_lloyd;
        r.lloyd = false;
        A.hs[r.slot].status = kSolveDone;
        (void)hipMemcpyAsync(A.sv + r.slot, &A.hs[r.slot], sizeof(BatchSolve), hipMemcpyHostToDevice, stream);
        (void)hipStreamSynchronize(stream);
      }
      A.owner[r.slot] = -1;
      A.tiles_dirty = true;
      finish_job(r.job, r.result, r.error);
      it = live.erase(it);
      cv_done.notify_all();
    }
    // start prepared solves
    std::vector<RJob*> ready;
    int in_lloyd = 0;
    for (auto& r : live) {
      if (r->stage == kReady) {
        r->stage = kLloyd;
        ready.push_back(r.get());
      }
      if (r->stage == kLloyd) ++in_lloyd;
    }
    if (in_lloyd == 0) {
      if (stopping && queue.empty() && live.empty()) break;
      cv_work.wait(lk);
      continue;
    }
    lk.unlock();

    std::vector<RJob*> failed, done;
    for (RJob* r : ready) {
      clear_error();
      const bm_status st = activate(*r, stream);
      if (st != BM_OK) {
        r->result = st;
        snprintf(r->error, sizeof r->error, "%s", bm_last_error());
        failed.push_back(r);
      }
    }
    // kRoundsPerSync rounds per class with running solves
    bm_status rst = BM_OK;
    for (int rr = 0; rr < kRoundsPerSync && rst == BM_OK; ++rr) {
      for (auto& kv : arenas) {
        Arena& A = *kv.second;
        if (A.in_lloyd == 0) continue;
        clear_error();
        if ((rst = arena_round(A, stream)) != BM_OK) break;
      }
    }
    if (rst == BM_OK && hipStreamSynchronize(stream) != hipSuccess)
      rst = set_error(BM_EDEVICE, "a batched round failed");
    const std::string rmsg = rst == BM_OK ? "" : bm_last_error();
    lk.lock();
    std::vector<RJob*> lloyd_jobs;
    for (auto& r : live)
      if (r->stage == kLloyd && r->result == BM_OK) lloyd_jobs.push_back(r.get());
    lk.unlock();
    for (RJob* r : lloyd_jobs) {
      if (rst != BM_OK) {
        r->result = rst;
        snprintf(r->error, sizeof r->error, "%s", rmsg.c_str());
        failed.push_back(r);
        continue;
      }
      if (!r->lloyd || r->ar->hs[r->slot].status != kSolveDone) continue;
      clear_error();
      const bm_status st = keep_best(*r, stream);
      if (st != BM_OK) {
        r->result = st;
        snprintf(r->error, sizeof r->error, "%s", bm_last_error());
        failed.push_back(r);
      } else {
        done.push_back(r);
      }
    }
    lk.lock();
    for (RJob* r : failed) r->stage = kEnded;
    bool wake_prep = false;
    for (RJob* r : done) {
      r->stage = r->t < r->job->spec.n_samples ? kPrep : kFinal;
      wake_prep = true;
    }
    if (wake_prep) cv_prep.notify_all();
  }
  prep_stop = true;
  cv_prep.notify_all();
  lk.unlock();
  prep.join();
  (void)hipStreamSynchronize(stream);
  for (auto& kv : arenas)
    if (kv.second->mem) (void)hipFree(kv.second->mem);
  lk.lock();
  reserved -= arena_bytes;
}

namespace {

void fill_info(const bm_ctx* c, const Job& j, bm_job_info* info) {
  (void)c;
  info->state = j.state;
  info->result = j.result;
  info->slot = j.slot;
  info->footprint = static_cast<int64_t>(j.alloc);
  info->t_submit_ms = j.t_submit;
  info->t_start_ms = j.t_start;
  info->t_end_ms = j.t_end;
  snprintf(info->error, sizeof info->error, "%s", j.error);
}

bool terminal(int32_t s) { return s == BM_JOB_DONE || s == BM_JOB_FAILED || s == BM_JOB_CANCELLED; }

}  // namespace

extern "C" {

bm_status bm_serve_default_config(bm_serve_config* cfg) {
  if (!cfg) return set_error(BM_EINVAL, "cfg is NULL");
  memset(cfg, 0, sizeof *cfg);
  cfg->struct_size = sizeof(bm_serve_config);
  cfg->slots = 4;
  cfg->hbm_budget = int64_t(8) << 30;
  cfg->device = -1;
  cfg->grid_per_job = 0;
  cfg->mode = BM_SERVE_FITS;
  cfg->round_max_k = 64;
  cfg->round_max_s = 50000;
  return BM_OK;
}

bm_status bm_ctx_create(const bm_serve_config* cfg_in, bm_ctx** out) {
  clear_error();
  if (!out) return set_error(BM_EINVAL, "out is NULL");
  *out = nullptr;
  bm_serve_config cfg;
  bm_serve_default_config(&cfg);
  if (cfg_in) {
    if (cfg_in->struct_size < sizeof(uint32_t) || cfg_in->struct_size > sizeof(bm_serve_config))
      return set_error(BM_EINVAL, "bm_serve_config.struct_size %u not recognised", cfg_in->struct_size);
    memcpy(&cfg, cfg_in, cfg_in->struct_size);
  }
  if (cfg.slots < 1 || cfg.slots > 64) return set_error(BM_EINVAL, "slots must be in [1, 64]");
  if (cfg.hbm_budget < (int64_t(1) << 20)) return set_error(BM_EINVAL, "hbm_budget below 1 MiB");
  if (cfg.grid_per_job < 0) return set_error(BM_EINVAL, "grid_per_job must be >= 0");
  if (cfg.mode != BM_SERVE_FITS && cfg.mode != BM_SERVE_ROUNDS)
    return set_error(BM_EINVAL, "mode must be BM_SERVE_FITS or BM_SERVE_ROUNDS");
  if (cfg.mode == BM_SERVE_ROUNDS && (cfg.round_max_k < 1 || cfg.round_max_s < 1 ||
                                      cfg.round_max_s > 2147483647LL))
    return set_error(BM_EINVAL, "round_max_k and round_max_s must be positive");
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return set_error(BM_EDEVICE, "no current HIP device");
  const int dev = cfg.device < 0 ? prev : cfg.device;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1 ||
      hipSetDevice(dev) != hipSuccess)
    return set_error(BM_EDEVICE, "cannot use HIP device %d", dev);
  std::unique_ptr<bm_ctx> c(new bm_ctx());
  c->device = dev;
  c->nslots = cfg.slots;
  c->budget = cfg.hbm_budget;
  const int fair = cus / cfg.slots > 0 ? cus / cfg.slots : 1;
  c->grid_cap = cfg.grid_per_job > 0 && cfg.grid_per_job < fair ? cfg.grid_per_job : fair;
  c->t0 = Clock::now();
  c->mode = cfg.mode;
  c->round_max_k = cfg.round_max_k;
  c->round_max_s = cfg.round_max_s;
  // ROUNDS: one engine thread with one stream; `slots` bounds the jobs in flight
  c->slots.resize(cfg.mode == BM_SERVE_ROUNDS ? 1 : cfg.slots);
  for (auto& sl : c->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
      for (auto& s2 : c->slots)
        if (s2.stream) (void)hipStreamDestroy(s2.stream);
      (void)hipSetDevice(prev);
      return set_error(BM_EDEVICE, "cannot create a stream");
    }
  }
  (void)hipSetDevice(prev);
  bm_ctx* raw = c.get();
  if (cfg.mode == BM_SERVE_ROUNDS)
    raw->workers.emplace_back([raw] { raw->engine(); });
  else
    for (int i = 0; i < cfg.slots; ++i) raw->workers.emplace_back([raw, i] { raw->worker(i); });
  *out = c.release();
  return BM_OK;
}

bm_status bm_ctx_submit(bm_ctx* c, const bm_job* job_in, int64_t* job_id) {
  clear_error();
  if (!c || !job_in || !job_id) return set_error(BM_EINVAL, "ctx, job and job_id are required");
  if (job_in->struct_size != sizeof(bm_job))
    return set_error(BM_EINVAL, "bm_job.struct_size mismatch");
  std::unique_ptr<Job> j(new Job());
  j->spec = *job_in;
  const bm_job& J = j->spec;
  bm_status st = fit_validate(J.X, J.n, J.d, J.k, J.s, J.n_samples, &J.opt, J.centroids,
                              J.degenerate, J.stats, &j->opt);
  if (st != BM_OK) return st;
  if (j->opt.final_mode != BM_FINAL_ASSIGN)
    return set_error(BM_ENOTSUP, "served jobs end with the final assignment (BM_FINAL_ASSIGN)");
  if (c->mode == BM_SERVE_ROUNDS) {
    if (j->opt.compare_rule != BM_CMP_FOPT)
      return set_error(BM_ENOTSUP, "round-batched serving compares with f_opt only (BM_CMP_FOPT)");
    if (j->opt.init_method != BM_INIT_KMEANSPP || j->opt.time_budget_ms > 0.0)
      return set_error(BM_ENOTSUP, "round-batched serving reseeds with K-means++ and has no time budget");
    if (J.s > c->round_max_s || J.k > c->round_max_k)
      return set_error(BM_ENOTSUP, "s = %lld or k = %d above the context's round_max_s / round_max_k",
                       static_cast<long long>(J.s), J.k);
    if (padded_dim(J.d) < 0) return set_error(BM_ENOTSUP, "d = %d exceeds the limit of 256", J.d);
    // this job's share of its class arena: one slot of rows and centroids
    const size_t dm = static_cast<size_t>(padded_dim(J.d));
    j->alloc = static_cast<size_t>(c->round_max_s) * dm * 4 +
               static_cast<size_t>(c->round_max_k) * (J.d * 12 + dm * 12 + 5) + sizeof(BatchSolve);
  } else {
    j->alloc = bm_ctx::pool_alloc(fit_scratch_bytes(J.n, J.d, J.k, J.s, J.n_samples,
                                                    J.sse != nullptr || J.labels != nullptr));
  }
  if (static_cast<int64_t>(j->alloc) > c->budget)
    return set_error(BM_ENOMEM, "job needs %zu bytes of scratch, above the budget of %lld", j->alloc,
                     static_cast<long long>(c->budget));
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->stopping) return set_error(BM_ECANCELLED, "context is shutting down");
  const int64_t id = c->next_id++;
  j->t_submit = c->now_ms();
  c->jobs[id] = std::move(j);
  c->queue.push_back(id);
  ++c->submitted;
  *job_id = id;
  c->cv_work.notify_all();
  return BM_OK;
}

bm_status bm_ctx_poll(bm_ctx* c, int64_t job_id, bm_job_info* info) {
  clear_error();
  if (!c || !info) return set_error(BM_EINVAL, "ctx and info are required");
  if (info->struct_size != sizeof(bm_job_info)) return set_error(BM_EINVAL, "bm_job_info.struct_size mismatch");
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->jobs.find(job_id);
  if (it == c->jobs.end()) return set_error(BM_EINVAL, "unknown job %lld", static_cast<long long>(job_id));
  fill_info(c, *it->second, info);
  return BM_OK;
}

bm_status bm_ctx_wait(bm_ctx* c, int64_t job_id, int32_t timeout_ms, bm_job_info* info) {
  clear_error();
  if (!c) return set_error(BM_EINVAL, "ctx is required");
  if (info && info->struct_size != sizeof(bm_job_info))
    return set_error(BM_EINVAL, "bm_job_info.struct_size mismatch");
  std::unique_lock<std::mutex> lk(c->mu);
  auto it = c->jobs.find(job_id);
  if (it == c->jobs.end()) return set_error(BM_EINVAL, "unknown job %lld", static_cast<long long>(job_id));
  Job* j = it->second.get();
  auto done = [j] { return terminal(j->state); };
  if (timeout_ms < 0) {
    c->cv_done.wait(lk, done);
  } else if (!c->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
    if (info) fill_info(c, *j, info);
    return set_error(BM_ETIMEDOUT, "job %lld still %s", static_cast<long long>(job_id),
                     j->state == BM_JOB_QUEUED ? "queued" : "running");
  }
  if (info) fill_info(c, *j, info);
  return BM_OK;
}

bm_status bm_ctx_cancel(bm_ctx* c, int64_t job_id) {
  clear_error();
  if (!c) return set_error(BM_EINVAL, "ctx is required");
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->jobs.find(job_id);
  if (it == c->jobs.end()) return set_error(BM_EINVAL, "unknown job %lld", static_cast<long long>(job_id));
  Job* j = it->second.get();
  if (j->state != BM_JOB_QUEUED)
    return set_error(BM_EINVAL, "job %lld is no longer queued", static_cast<long long>(job_id));
  for (auto q = c->queue.begin(); q != c->queue.end(); ++q)
    if (*q == job_id) {
      c->queue.erase(q);
      break;
    }
  j->state = BM_JOB_CANCELLED;
  j->result = BM_ECANCELLED;
  j->t_end = c->now_ms();
  ++c->cancelled;
  c->cv_done.notify_all();
  c->cv_work.notify_all();
  return BM_OK;
}

bm_status bm_ctx_release(bm_ctx* c, int64_t job_id) {
  clear_error();
  if (!c) return set_error(BM_EINVAL, "ctx is required");
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->jobs.find(job_id);
  if (it == c->jobs.end()) return set_error(BM_EINVAL, "unknown job %lld", static_cast<long long>(job_id));
  if (!terminal(it->second->state))
    return set_error(BM_EINVAL, "job %lld has not finished", static_cast<long long>(job_id));
  c->jobs.erase(it);
  return BM_OK;
}

bm_status bm_ctx_info(bm_ctx* c, bm_serve_info* info) {
  clear_error();
  if (!c || !info) return set_error(BM_EINVAL, "ctx and info are required");
  if (info->struct_size != sizeof(bm_serve_info)) return set_error(BM_EINVAL, "bm_serve_info.struct_size mismatch");
  std::lock_guard<std::mutex> lk(c->mu);
  info->submitted = c->submitted;
  info->completed = c->completed;
  info->failed = c->failed;
  info->cancelled = c->cancelled;
  info->queued = static_cast<int64_t>(c->queue.size());
  info->running = c->running;
  info->reserved_bytes = c->reserved;
  info->peak_reserved_bytes = c->peak_reserved;
  info->slots = c->nslots;
  info->grid_per_job = c->grid_cap;
  return BM_OK;
}

bm_status bm_ctx_destroy(bm_ctx* c) {
  clear_error();
  if (!c) return BM_OK;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->stopping = true;
    for (int64_t id : c->queue) {
      Job* j = c->jobs[id].get();
      j->state = BM_JOB_CANCELLED;
      j->result = BM_ECANCELLED;
      j->t_end = c->now_ms();
      ++c->cancelled;
    }
    c->queue.clear();
    c->cv_work.notify_all();
    c->cv_done.notify_all();
  }
  for (auto& t : c->workers) t.join();
  for (auto& sl : c->slots)
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  delete c;
  return BM_OK;
}

}  // extern "C"
