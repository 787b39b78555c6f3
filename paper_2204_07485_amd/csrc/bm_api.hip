// bm_api.hip -- the C ABI (include/bigmeans.h): argument checks, option
// defaults, the device scratch pool, launches and error mapping.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <vector>

#include "bm_internal.h"

namespace bm {

// ---------------------------------------------------------------------------
// errors

static thread_local char g_err[512] = "";
static thread_local int64_t g_last_counters[kNumCounters];
// Presampling before the solver: 0 automatic, 1 never, 2 always report a
// window miss (the solver then samples itself); a test hook, not in the header.
static std::atomic<int> g_presample_mode{0};
// BF16 matrix-core fits: 1 = the sample-level K-means on the matrix cores
// (default), 0 = the FP32 persistent solver for it (a test hook).
static std::atomic<int> g_mfma_lloyd{1};
static std::atomic<int> g_fp32_mfma{1};
bool fp32_mfma_enabled() { return g_fp32_mfma.load() != 0; }
// 1: every K-means++ draw is taken with the row-order sums, not only those
// near a boundary (a test hook).
static std::atomic<int> g_exact_draws{0};
bool exact_draws_forced() { return g_exact_draws.load() != 0; }
static thread_local int64_t g_last_rechecked = 0;
static thread_local double g_last_assign_ms = 0.0;
static thread_local int32_t g_last_batch_rounds = 0;
static thread_local int32_t g_last_batch_tile = 0;
static thread_local std::vector<float> g_last_batch_ms;  // device time of each round's graph

bm_status set_error(bm_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_err[0] = '\0'; }

#define BM_HIP(call)                                                                      \
  do {                                                                                    \
    const hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                                 \
      return set_error(BM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));        \
  } while (0)

// ---------------------------------------------------------------------------
// scratch pool: one growing device allocation per device, guarded by a mutex

static std::mutex g_mu;
static std::mutex g_launch_mu;
static ScratchPool g_pool[64];
// The batched Lloyd's scratch when it runs inside a call that keeps its own
// buffers in g_pool (the full-data polish, the collective mode), under g_mu.
static ScratchPool g_pool_inner[64];
static thread_local bool t_inner = false;
// A serving slot's worker thread uses its own pool (no shared state, no lock).
static thread_local ScratchPool* t_pool = nullptr;

void scratch_set_thread_pool(ScratchPool* p) { t_pool = p; }

void scratch_pool_free(ScratchPool* p) {
  if (p->ptr) (void)hipFree(p->ptr);
  p->ptr = nullptr;
  p->bytes = 0;
}

bm_status scratch_pool_reserve(ScratchPool* p, size_t bytes) {
  if (p->bytes >= bytes) return BM_OK;
  scratch_pool_free(p);
  if (hipMalloc(&p->ptr, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p->ptr = nullptr;
    return set_error(BM_ENOMEM, "cannot allocate %zu bytes of device scratch", bytes);
  }
  p->bytes = bytes;
  return BM_OK;
}

void* scratch_get(size_t bytes, hipStream_t stream, bm_status* st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    *st = set_error(BM_EDEVICE, "no current HIP device");
    return nullptr;
  }
  ScratchPool& p = t_inner ? g_pool_inner[dev] : (t_pool ? *t_pool : g_pool[dev]);
  if (p.bytes >= bytes) {
    *st = BM_OK;
    return p.ptr;
  }
  if (p.ptr) {
    (void)hipStreamSynchronize(stream);
    (void)hipFree(p.ptr);
    p.ptr = nullptr;
    p.bytes = 0;
  }
  size_t want = bytes + bytes / 4 + (1u << 20);
  if (hipMalloc(&p.ptr, want) != hipSuccess) {
    (void)hipGetLastError();
    p.ptr = nullptr;
    *st = set_error(BM_ENOMEM, "cannot allocate %zu bytes of device scratch", want);
    return nullptr;
  }
  p.bytes = want;
  *st = BM_OK;
  return p.ptr;
}

void scratch_release() {
  for (ScratchPool* pools : {g_pool, g_pool_inner}) {
    for (int i = 0; i < 64; ++i) {
      ScratchPool& p = pools[i];
      if (p.ptr) (void)hipFree(p.ptr);
      p.ptr = nullptr;
      p.bytes = 0;
    }
  }
}

// While alive, scratch_get() on this thread hands out the inner pool.
struct InnerScratch {
  bool prev;
  InnerScratch() : prev(t_inner) { t_inner = true; }
  ~InnerScratch() { t_inner = prev; }
};

// Bump layout over the scratch block: first pass sizes, second pass binds.
struct Layout {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (count ? count : 1);
    return p;
  }
};

// ---------------------------------------------------------------------------
// options

static void defaults(bm_options* o) {
  memset(o, 0, sizeof *o);
  o->struct_size = sizeof(bm_options);
  o->x_dtype = BM_F32;
  o->max_iter = 100;
  o->tol = 1e-4;
  o->stop_rule = BM_STOP_SHIFT;
  o->n_local_trials = 3;
  o->compare_rule = BM_CMP_FOPT;
  o->precision = BM_PREC_FP32;
}

static bm_status resolve(const bm_options* in, bm_options* out) {
  defaults(out);
  if (in) {
    if (in->struct_size < sizeof(uint32_t) || in->struct_size > sizeof(bm_options))
      return set_error(BM_EINVAL, "bm_options.struct_size %u not recognised", in->struct_size);
    memcpy(out, in, in->struct_size);
    out->struct_size = sizeof(bm_options);
  }
  if (out->x_dtype != BM_F32 && out->x_dtype != BM_BF16)
    return set_error(BM_EINVAL, "x_dtype %d", out->x_dtype);
  if (out->max_iter < 1) return set_error(BM_EINVAL, "max_iter must be >= 1");
  if (!(out->tol >= 0.0)) return set_error(BM_EINVAL, "tol must be >= 0");
  if (out->stop_rule != BM_STOP_SHIFT && out->stop_rule != BM_STOP_REL_OBJ)
    return set_error(BM_EINVAL, "stop_rule %d", out->stop_rule);
  if (out->n_local_trials < 1 || out->n_local_trials > kMaxTrials)
    return set_error(BM_EINVAL, "n_local_trials must be in [1, %d]", kMaxTrials);
  if (out->compare_rule != BM_CMP_FOPT && out->compare_rule != BM_CMP_RESAMPLE)
    return set_error(BM_EINVAL, "compare_rule %d", out->compare_rule);
  if (out->precision != BM_PREC_FP32 && out->precision != BM_PREC_BF16_MFMA)
    return set_error(BM_EINVAL, "precision %d", out->precision);
  if (out->precision == BM_PREC_BF16_MFMA && out->x_dtype != BM_BF16)
    return set_error(BM_EINVAL, "BM_PREC_BF16_MFMA needs BF16 points (x_dtype = BM_BF16)");
  if (out->grid < 0 || out->grid > kMaxGrid) return set_error(BM_EINVAL, "grid %d", out->grid);
  if (out->t_start < 0) return set_error(BM_EINVAL, "t_start must be >= 0");
  if (out->init_method != BM_INIT_KMEANSPP && out->init_method != BM_INIT_FORGY)
    return set_error(BM_EINVAL, "init_method %d", out->init_method);
  if (out->final_mode != BM_FINAL_ASSIGN && out->final_mode != BM_FINAL_POLISH)
    return set_error(BM_EINVAL, "final_mode %d", out->final_mode);
  if (!(out->time_budget_ms >= 0.0) || out->time_budget_ms > 1e12)
    return set_error(BM_EINVAL, "time_budget_ms must be in [0, 1e12]");
  return BM_OK;
}

bm_status resolve_options(const bm_options* in, bm_options* out) { return resolve(in, out); }

// ---------------------------------------------------------------------------
// solver configuration shared by the entry points that run the solver

struct SolverPlan {
  int dm = 0;
  int grid = 0;
  int gmax = 0;  // co-resident workgroups of this configuration on the device
  int64_t cand_cap = 0;
  uint64_t win_lo = 0, win_hi = 0;
  int sums_in_lds = 0;  // replicas of the FP64 sums in LDS (0: global ring)
  bool c64_in_lds = false;
  size_t lds = 0;
};

static bm_status plan_solver(int d, int k, int64_t s, int64_t n_points, int grid_req,
                             SolverPlan* sp) {
  sp->dm = padded_dim(d);
  if (sp->dm < 0) return set_error(BM_ENOTSUP, "d = %d exceeds the limit of 256", d);
  size_t lds_max = 0;
  bm_status st = max_lds_per_block(&lds_max);
  if (st != BM_OK) return st;
  const size_t budget = lds_max > 2048 ? lds_max - 2048 : lds_max;  // static LDS of the kernel
  // prefer, in order: FP64 sums (4, then 2 replicas) and means in LDS, then
  // FP64 sums in LDS, then FP64 means in LDS
  bool found = false;
  const int modes[6][2] = {{4, 1}, {2, 1}, {1, 1}, {1, 0}, {0, 1}, {0, 0}};
  for (int mi = 0; mi < 6 && !found; ++mi) {
    const int sl = modes[mi][0];
    const bool cl = modes[mi][1] != 0;
    const size_t need = solver_lds_bytes(sp->dm, k, d, sl, cl);
    if (need <= budget) {
      sp->sums_in_lds = sl;
      sp->c64_in_lds = cl;
      sp->lds = need;
      found = true;
    }
  }
  sampler_window(n_points, s, &sp->win_lo, &sp->win_hi, &sp->cand_cap);
  if (!found)
    return set_error(BM_ENOTSUP, "k*d = %d*%d centroids do not fit in one workgroup's LDS", k, d);
  int gmax = 0;
  st = solver_max_grid(sp->dm, sp->lds, &gmax);
  if (st != BM_OK) return st;
  sp->gmax = gmax;
  int g = grid_req;
  if (g <= 0) {
    const int64_t want = (s + 511) / 512;
    g = static_cast<int>(want < 1 ? 1 : (want > gmax ? gmax : want));
  }
  if (g > gmax) g = gmax;
  const int64_t pairs = (n_points + 1) / 2;
  if (g > s) g = static_cast<int>(s);
  if (g > pairs) g = static_cast<int>(pairs);
  if (g < 1) g = 1;
  sp->grid = g;
  return BM_OK;
}

struct SolverBuffers {
  SolverArgs a;
  double* partial = nullptr;      // final assignment pass: per-workgroup objective
  double* sse_dev = nullptr;      //   the objective
  unsigned long long* rechecked = nullptr;  //   points recomputed on the FP32 path (MFMA form)
  size_t bytes = 0;
  size_t ctrl_bytes = 0;  // prefix cleared before each launch
};

// Lay out every solver buffer; with base == nullptr only the size is computed.
static void layout_solver(char* base, int64_t n, int64_t s, int d, int k, int T, int64_t cand_cap, bool own_P,
                          bool own_idx, bool no_labels, bool own_inc, int final_grid, int sbatch,
                          SolverBuffers* b) {
  Layout L;
  L.base = base;
  SolverArgs& a = b->a;
  const size_t B = static_cast<size_t>(sbatch);
  a.sbatch = sbatch;
  a.bar = L.take<GridBarrier>(1);
  a.err = L.take<int32_t>(1);
  a.presample_miss = L.take<int32_t>(1);
  a.stop_flag = L.take<int32_t>(1);
  a.counters = L.take<int64_t>(kNumCounters);
  a.cand_count = L.take<uint32_t>(B);
  a.hist = L.take<uint32_t>(3 * 256);
  a.sums = L.take<double>(3 * static_cast<size_t>(kReplicas) * k * d);
  a.cnt = L.take<int32_t>(3 * static_cast<size_t>(kReplicas) * k);
  b->ctrl_bytes = L.off;
  a.c64 = L.take<double>(2 * static_cast<size_t>(k) * d);
  a.thr = L.take<uint64_t>(2 * B);
  a.smiss = L.take<int32_t>(B);
  a.sse_part = L.take<double>(2 * kMaxGrid);
  a.wsum = L.take<double>(kMaxGrid);
  a.phi_part = L.take<double>(static_cast<size_t>(kMaxGrid) * kMaxTrials);
  a.cand = L.take<int64_t>(kMaxTrials);
  a.wg_lo = L.take<uint32_t>(B * kMaxGrid);
  a.wg_off = L.take<uint32_t>(B * kMaxGrid);
  a.cand_key = L.take<uint64_t>(B * static_cast<size_t>(cand_cap));
  a.cand_idx = L.take<int32_t>(B * static_cast<size_t>(cand_cap));
  a.selcode = L.take<uint8_t>(B * ((static_cast<size_t>(n) + 15) & ~size_t(15)));  // 16-byte slots
  a.w = L.take<double>(s);
  a.dcache = L.take<double>(static_cast<size_t>(kMaxTrials) * s);
  a.sample_f = L.take<double>(T > 0 ? T : 1);
  float* P = L.take<float>(own_P ? B * static_cast<size_t>(s) * d : 1);
  int32_t* idx = L.take<int32_t>(own_idx ? B * static_cast<size_t>(s) : 1);
  float* Cinc = L.take<float>(own_inc ? static_cast<size_t>(k) * d : 1);
  uint8_t* deg = L.take<uint8_t>(k);
  double* fopt = L.take<double>(1);
  if (own_P) a.P = P;
  if (own_idx) a.idx = idx;
  if (no_labels) a.labels = nullptr;  // sample labels are then not written at all
  if (own_inc) a.Cinc = Cinc;
  a.deg_inc = deg;
  a.f_opt = fopt;
  b->partial = L.take<double>(final_grid > 0 ? final_grid : 1);
  b->sse_dev = L.take<double>(1);
  b->rechecked = L.take<unsigned long long>(1);
  b->bytes = L.off + 256;
}

static bm_status prepare_solver(hipStream_t stream, int64_t n, int64_t s, int d, int k, int T,
                                int64_t cand_cap,
                                bool own_P, bool own_idx, bool no_labels, bool own_inc,
                                int final_grid, int sbatch, SolverBuffers* b) {
  SolverArgs keep = b->a;
  layout_solver(nullptr, n, s, d, k, T, cand_cap, own_P, own_idx, no_labels, own_inc, final_grid,
                sbatch, b);
  bm_status st = BM_OK;
  char* base = static_cast<char*>(scratch_get(b->bytes, stream, &st));
  if (!base) return st;
  b->a = keep;
  layout_solver(base, n, s, d, k, T, cand_cap, own_P, own_idx, no_labels, own_inc, final_grid,
                sbatch, b);
  BM_HIP(hipMemsetAsync(base, 0, b->ctrl_bytes, stream));
  if (final_grid > 0) {
    BM_HIP(hipMemsetAsync(b->rechecked, 0, sizeof(unsigned long long), stream));
  }
  return BM_OK;
}

static bm_status solver_error(int32_t code) {
  switch (code) {
    case kErrNone: return BM_OK;
    case kErrBarrier:
      return set_error(BM_EDEVICE, "solver aborted: a grid-barrier wait exceeded its bound");
    case kErrSelect: return set_error(BM_EDEVICE, "solver aborted: sampler bookkeeping inconsistent");
    case kErrSeed: return set_error(BM_EDEVICE, "solver aborted: K-means++ found no candidate");
    default: return set_error(BM_EDEVICE, "solver aborted with code %d", code);
  }
}

static bm_status check_solver_error(const SolverArgs& a, hipStream_t stream, int32_t* code_out) {
  int32_t code = 0;
  BM_HIP(hipMemcpyAsync(&code, a.err, sizeof code, hipMemcpyDeviceToHost, stream));
  BM_HIP(hipStreamSynchronize(stream));
  if (code_out) *code_out = code;
  return solver_error(code);
}

static bm_status check_sizes(int64_t n, int d, int k, int64_t s) {
  if (n < 1 || n > 2147483647LL) return set_error(BM_EINVAL, "n = %lld out of [1, 2^31)", (long long)n);
  if (d < 1) return set_error(BM_EINVAL, "d = %d must be >= 1", d);
  if (k < 1) return set_error(BM_EINVAL, "k = %d must be >= 1", k);
  if (s < k || s > n) return set_error(BM_EINVAL, "need k <= s <= n (k=%d, s=%lld, n=%lld)", k,
                                       (long long)s, (long long)n);
  return BM_OK;
}

static float elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

// ---------------------------------------------------------------------------
// batched Lloyd: host-side plan

struct BatchShape {
  int d, kmax, n_solves;
  int64_t rows;
  bool operator<(const BatchShape& o) const {
    if (d != o.d) return d < o.d;
    if (kmax != o.kmax) return kmax < o.kmax;
    if (n_solves != o.n_solves) return n_solves < o.n_solves;
    return rows < o.rows;
  }
};
static std::map<BatchShape, int> g_tile_cache;  // tuned rows per tile (under g_mu)

// Work list for a tile size: tile -> solve, and each solve's first tile.
static int build_tiles(const std::vector<int64_t>& s, int tile_rows, std::vector<int32_t>* tile_solve,
                       std::vector<int32_t>* tile0, std::vector<int32_t>* ntiles) {
  tile_solve->clear();
  tile0->assign(s.size(), 0);
  ntiles->assign(s.size(), 0);
  for (size_t j = 0; j < s.size(); ++j) {
    const int64_t nt = (s[j] + tile_rows - 1) / tile_rows;
    (*tile0)[j] = static_cast<int32_t>(tile_solve->size());
    (*ntiles)[j] = static_cast<int32_t>(nt);
    for (int64_t q = 0; q < nt; ++q) tile_solve->push_back(static_cast<int32_t>(j));
  }
  return static_cast<int>(tile_solve->size());
}

// kmeans_lloyd_batched after option resolution; the caller holds g_mu.
static bm_status batched_run(int32_t n_solves, const float* P, int32_t d, const int64_t* s,
                             const int32_t* k, float* C, uint8_t* deg, const bm_options& o,
                             int32_t* labels, double* f, int32_t* passes) {
  bm_status st = BM_OK;
  if (n_solves < 1 || d < 1) return set_error(BM_EINVAL, "need n_solves >= 1 and d >= 1");
  if (!P || !s || !k || !C || !deg) return set_error(BM_EINVAL, "P, s, k, C and deg are required");
  if (padded_dim(d) < 0) return set_error(BM_ENOTSUP, "d = %d exceeds the limit of 256", d);
  std::vector<int64_t> sv_s(n_solves);
  std::vector<BatchSolve> hs(n_solves);
  int64_t rows = 0, ktot = 0;
  int kmax = 0;
  for (int j = 0; j < n_solves; ++j) {
    if (s[j] < 1 || k[j] < 1 || k[j] > s[j])
      return set_error(BM_EINVAL, "solve %d: need 1 <= k <= s (s=%lld, k=%d)", j, (long long)s[j], k[j]);
    int active = 0;
    for (int q = 0; q < k[j]; ++q) active += deg[ktot + q] ? 0 : 1;
    if (!active) return set_error(BM_EINVAL, "solve %d: every centroid is degenerate", j);
    sv_s[j] = s[j];
    memset(&hs[j], 0, sizeof(BatchSolve));
    hs[j].row0 = rows;
    hs[j].s = s[j];
    hs[j].c0 = static_cast<int32_t>(ktot);
    hs[j].k = k[j];
    hs[j].status = kSolveRunning;
    hs[j].iter = 1;
    hs[j].f_prev = __builtin_inf();
    rows += s[j];
    ktot += k[j];
    kmax = k[j] > kmax ? k[j] : kmax;
    if (rows > 2147483647LL || ktot > 2147483647LL)
      return set_error(BM_EINVAL, "more than 2^31 rows or centroids in the batch");
  }
  size_t lds_max = 0;
  if ((st = max_lds_per_block(&lds_max)) != BM_OK) return st;
  const bool sums_lds = batch_assign_lds(d, kmax, true) + 1024 <= lds_max;
  if (!sums_lds && batch_assign_lds(d, kmax, false) + 1024 > lds_max)
    return set_error(BM_ENOTSUP, "k x d = %d x %d centroids do not fit in one workgroup's LDS", kmax, d);
  hipStream_t user = static_cast<hipStream_t>(o.stream);
  int grid = 0;
  if ((st = batch_assign_grid(d, kmax, sums_lds, &grid)) != BM_OK) return st;

  // scratch: solve states, work list (sized for the smallest tile), tile
  // objectives, FP64 sums, counts, FP64 means, flags, running counter
  constexpr int kMinTile = 256;
  int64_t max_tiles = 0;
  for (int j = 0; j < n_solves; ++j) max_tiles += (s[j] + kMinTile - 1) / kMinTile;
  BatchSolve* sv_d = nullptr;
  int32_t* tiles_d = nullptr;
  double* tile_f = nullptr;
  double* sums = nullptr;
  int32_t* cnt = nullptr;
  double* c64 = nullptr;
  float* cpad = nullptr;
  float* ppad = nullptr;
  uint8_t* deg_d = nullptr;
  int* running = nullptr;
  char* base = nullptr;
  for (int round = 0; round < 2; ++round) {
    Layout L;
    L.base = base;
    sv_d = L.take<BatchSolve>(n_solves);
    tiles_d = L.take<int32_t>(max_tiles);
    tile_f = L.take<double>(max_tiles);
    sums = L.take<double>(ktot * padded_dim(d));
    cnt = L.take<int32_t>(ktot);
    c64 = L.take<double>(ktot * d);
    cpad = L.take<float>(ktot * padded_dim(d));
    ppad = L.take<float>(padded_dim(d) == d ? 1 : rows * padded_dim(d));
    deg_d = L.take<uint8_t>(ktot);
    running = L.take<int>(1);
    if (round == 0) {
      base = static_cast<char*>(scratch_get(L.off + 256, user, &st));
      if (!base) return st;
    }
  }
  // an internal stream (capturable; default priority) ordered after the caller's
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto cleanup = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (stream) (void)hipStreamDestroy(stream);
  };
  auto fail = [&](bm_status code) {
    if (stream) (void)hipStreamSynchronize(stream);
    cleanup();
    return code;
  };
#define BM_HIPB(call)                                                                          \
  do {                                                                                         \
    const hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                      \
      return fail(set_error(BM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)));       \
  } while (0)
  BM_HIPB(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  BM_HIPB(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
  BM_HIPB(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
  BM_HIPB(hipEventRecord(ev_in, user));
  BM_HIPB(hipStreamWaitEvent(stream, ev_in, 0));
  BM_HIPB(hipMemcpyAsync(deg_d, deg, static_cast<size_t>(ktot), hipMemcpyHostToDevice, stream));
  BM_HIPB(hipMemsetAsync(sums, 0, sizeof(double) * ktot * padded_dim(d), stream));
  BM_HIPB(hipMemsetAsync(cnt, 0, sizeof(int32_t) * ktot, stream));
  if ((st = launch_batch_init(C, c64, cpad, ktot, d, stream)) != BM_OK) return fail(st);
  // rows DM wide for guard-free loads (a copy only when d is not already DM)
  const float* Pp = P;
  if (padded_dim(d) != d) {
    if ((st = launch_pad_rows(P, ppad, rows, d, stream)) != BM_OK) return fail(st);
    Pp = ppad;
  }

  // rows per tile: tuned once per shape by timing a dry assignment pass
  std::vector<int32_t> tile_solve, tile0, ntiles;
  const BatchShape shape{d, kmax, n_solves, rows};
  int tile_rows = 0;
  auto it_cache = g_tile_cache.find(shape);
  auto upload = [&](int tr) -> bm_status {
    const int nt = build_tiles(sv_s, tr, &tile_solve, &tile0, &ntiles);
    for (int j = 0; j < n_solves; ++j) {
      hs[j].tile0 = tile0[j];
      hs[j].ntiles = ntiles[j];
    }
    BM_HIP(hipMemcpyAsync(tiles_d, tile_solve.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, stream));
    BM_HIP(hipMemcpyAsync(sv_d, hs.data(), sizeof(BatchSolve) * n_solves, hipMemcpyHostToDevice, stream));
    BM_HIP(hipStreamSynchronize(stream));  // the host vectors are reused
    return BM_OK;
  };
  if (it_cache != g_tile_cache.end()) {
    tile_rows = it_cache->second;
  } else if (rows < 65536) {
    tile_rows = 512;
  } else {
    EventSet<2> tev;
    BM_HIPB(tev.create());
    hipEvent_t t0 = tev[0], t1 = tev[1];
    float best = 0.f;
    for (int tr : {256, 512, 1024, 2048, 4096}) {
      bm_status su = upload(tr);
      if (su != BM_OK) return fail(su);
      const int nt = static_cast<int>(tile_solve.size());
      float ms = 0.f;
      for (int rep = 0; rep < 2 && su == BM_OK; ++rep) {  // first run warms caches
        BM_HIPB(hipEventRecord(t0, stream));
        su = launch_batch_assign(Pp, d, C, cpad, deg_d, sv_d, tiles_d, nt, tr, kmax, sums_lds, sums,
                                 cnt, tile_f, nullptr, 1, grid, stream);
        BM_HIPB(hipEventRecord(t1, stream));
        BM_HIPB(hipEventSynchronize(t1));
        BM_HIPB(hipEventElapsedTime(&ms, t0, t1));
      }
      if (su != BM_OK) return fail(su);
      if (tile_rows == 0 || ms < best) {
        best = ms;
        tile_rows = tr;
      }
    }
    g_tile_cache[shape] = tile_rows;
  }
  if ((st = upload(tile_rows)) != BM_OK) return fail(st);
  const int nt = static_cast<int>(tile_solve.size());

  // one round = assignment + update, captured once and launched per round
  BM_HIPB(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  bm_status cs = launch_batch_assign(Pp, d, C, cpad, deg_d, sv_d, tiles_d, nt, tile_rows, kmax,
                                     sums_lds, sums, cnt, tile_f, labels, 0, grid, stream);
  if (cs == BM_OK)
    cs = launch_batch_update(sv_d, n_solves, tile_f, sums, cnt, C, cpad, c64, deg_d, d, o.max_iter,
                             o.tol, o.stop_rule, running, stream, kmax);
  const hipError_t ce = hipStreamEndCapture(stream, &graph);
  if (cs != BM_OK) return fail(cs);
  if (ce != hipSuccess)
    return fail(set_error(BM_EDEVICE, "graph capture failed: %s", hipGetErrorString(ce)));
  BM_HIPB(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  int still = 1;
  int rounds = 0;
  EventSet<2> rev;
  BM_HIPB(rev.create());
  hipEvent_t r0 = rev[0], r1 = rev[1];
  g_last_batch_ms.clear();
  for (; rounds <= o.max_iter && still; ++rounds) {
    BM_HIPB(hipMemsetAsync(running, 0, sizeof(int), stream));
    BM_HIPB(hipEventRecord(r0, stream));
    BM_HIPB(hipGraphLaunch(exec, stream));
    BM_HIPB(hipEventRecord(r1, stream));
    BM_HIPB(hipMemcpyAsync(&still, running, sizeof(int), hipMemcpyDeviceToHost, stream));
    BM_HIPB(hipStreamSynchronize(stream));
    g_last_batch_ms.push_back(elapsed_ms(r0, r1));
  }
  if (still) return fail(set_error(BM_EDEVICE, "batched Lloyd did not finish in max_iter + 1 rounds"));
  BM_HIPB(hipMemcpyAsync(hs.data(), sv_d, sizeof(BatchSolve) * n_solves, hipMemcpyDeviceToHost, stream));
  BM_HIPB(hipMemcpyAsync(deg, deg_d, static_cast<size_t>(ktot), hipMemcpyDeviceToHost, stream));
  BM_HIPB(hipEventRecord(ev_out, stream));
  BM_HIPB(hipStreamWaitEvent(user, ev_out, 0));
  BM_HIPB(hipStreamSynchronize(stream));
#undef BM_HIPB
  for (int j = 0; j < n_solves; ++j) {
    if (hs[j].status != kSolveDone) return fail(set_error(BM_EDEVICE, "solve %d did not finish", j));
    if (f) f[j] = hs[j].f;
    if (passes) passes[j] = hs[j].passes;
  }
  g_last_batch_rounds = rounds;
  g_last_batch_tile = tile_rows;
  cleanup();
  return BM_OK;
}

}  // namespace bm

using namespace bm;

// ---------------------------------------------------------------------------
// public entry points

extern "C" {

bm_status bm_default_options(bm_options* opt) {
  if (!opt) return set_error(BM_EINVAL, "opt is NULL");
  defaults(opt);
  return BM_OK;
}

const char* bm_last_error(void) { return g_err; }

int32_t bm_abi_version(void) { return BM_ABI_VERSION; }

// Diagnostics and test hooks, declared in include/bigmeans_debug.h.
// Test hook: presampling mode (0 automatic, 1 never, 2 force a window miss);
// returns the previous mode.
int32_t bm_debug_presample(int32_t mode) {
  if (mode < 0 || mode > 2) return -1;
  return g_presample_mode.exchange(mode);
}

// Test hook: BF16 fits' sample-level K-means on the matrix cores (1) or on
// the FP32 persistent solver (0); returns the previous setting.
int32_t bm_debug_mfma_lloyd(int32_t on) {
  if (on < 0 || on > 1) return -1;
  return g_mfma_lloyd.exchange(on);
}

// Test hook: FP32 full-data assignment on the matrix cores (1) or on the VALU
// kernel (0); returns the previous setting.
int32_t bm_debug_fp32_mfma(int32_t on) {
  if (on != 0 && on != 1) return -1;
  return g_fp32_mfma.exchange(on);
}

// Test hook: every K-means++ draw with the row-order sums (1) or only the
// draws near a running-sum boundary (0); returns the previous setting.
int32_t bm_debug_exact_draws(int32_t on) {
  if (on != 0 && on != 1) return -1;
  return g_exact_draws.exchange(on);
}

// Raw per-phase counters of the last bigmeans_fit on this thread.
int32_t bm_debug_counters(int64_t* out, int32_t n) {
  if (!out || n < 1) return BM_EINVAL;
  for (int i = 0; i < n && i < kNumCounters; ++i) out[i] = g_last_counters[i];
  return BM_OK;
}

// Points the last BM_PREC_BF16_MFMA kmeans_assign on this thread recomputed
// on the FP32 path.
int64_t bm_debug_rechecked(void) { return g_last_rechecked; }

// Device time (HIP events on the call's stream) of the assignment kernel of
// the last kmeans_assign on this thread, in ms.
double bm_debug_assign_ms(void) { return g_last_assign_ms; }

bm_status bm_release_scratch(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  (void)hipDeviceSynchronize();
  scratch_release();
  return BM_OK;
}

}  // extern "C"

namespace bm {

bm_status fit_validate(const void* X, int64_t n, int32_t d, int32_t k, int64_t s,
                       int32_t n_samples, const bm_options* opt_in, float* centroids,
                       uint8_t* degenerate, bm_stats* stats, bm_options* o) {
  bm_status st = resolve(opt_in, o);
  if (st != BM_OK) return st;
  if ((st = check_sizes(n, d, k, s)) != BM_OK) return st;
  if (n_samples < 1) return set_error(BM_EINVAL, "n_samples must be >= 1");
  if (!X || !centroids) return set_error(BM_EINVAL, "X and centroids are required");
  if (o->resume && !degenerate) return set_error(BM_EINVAL, "resume needs the degenerate flags");
  if (static_cast<int64_t>(o->t_start) + n_samples > 4294967295LL)
    return set_error(BM_EINVAL, "sample indices exceed 2^32");
  if (stats && stats->struct_size != sizeof(bm_stats))
    return set_error(BM_EINVAL, "bm_stats.struct_size mismatch");
  if (o->final_mode == BM_FINAL_POLISH && o->x_dtype != BM_F32)
    return set_error(BM_ENOTSUP, "BM_FINAL_POLISH needs FP32 points");
  return BM_OK;
}

bm_status solver_coresident_blocks(int d, int k, int64_t s, int64_t n, int* blocks) {
  SolverPlan sp;
  const bm_status st = plan_solver(d, k, s, n, 0, &sp);
  if (st != BM_OK) return st;
  *blocks = sp.gmax;
  return BM_OK;
}

size_t fit_scratch_bytes(int64_t n, int32_t d, int32_t k, int64_t s, int32_t n_samples,
                         bool final_pass) {
  uint64_t lo = 0, hi = 0;
  int64_t cap = 0;
  sampler_window(n, s, &lo, &hi, &cap);
  SolverBuffers b;
  memset(&b.a, 0, sizeof b.a);
  const int final_grid = final_pass ? 2048 : 0;  // an upper bound of either final kernel's grid
  layout_solver(nullptr, n, s, d, k, n_samples, cap, true, true, true, true, final_grid,
                sample_slots(n, s, d, n_samples, cap), &b);
  return b.bytes;
}

// Device buffers of the matrix-core sample K-means (one problem at a time).
// Pinned host memory for the small per-sample transfers of the matrix-core
// fit, so they queue behind the kernels instead of stalling the host; one
// block per thread, kept until the process ends.
struct MfmaStage {
  BatchSolve hs;                // the solve record after a group of rounds
  int64_t cnt[kNumCounters];    // reseeding counters
  int32_t err;                  // reseeding error code
  int32_t pad;
  uint8_t deg[256];             // the working flags after a group of rounds (k <= 256)
};
static thread_local MfmaStage* t_mfma_stage = nullptr;

static bm_status mfma_stage(MfmaStage** out) {
  if (!t_mfma_stage) {
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(MfmaStage), hipHostMallocDefault) != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_error(BM_ENOMEM, "cannot allocate pinned host staging");
    }
    t_mfma_stage = static_cast<MfmaStage*>(p);
  }
  *out = t_mfma_stage;
  return BM_OK;
}

struct MfmaLloydBuffers {
  uint16_t* p16 = nullptr;   // s x d BF16 rows of the sample
  float* ppad = nullptr;     // s x DM FP32 rows when d != DM
  int32_t* lab = nullptr;    // s labels from the matrix cores
  int* bad = nullptr;        // set by the FP32 row gather on an index outside X
  BatchSolve* sv = nullptr;
  int32_t* tiles = nullptr;
  double* tile_f = nullptr;
  double* sums = nullptr;    // k x DM
  int32_t* cnt = nullptr;
  double* c64 = nullptr;     // k x d
  float* cpad = nullptr;     // k x DM
  float* cw = nullptr;       // k x d: the sample's centroids
  uint8_t* degw = nullptr;   // k
  uint8_t* deginc = nullptr; // k: the incumbent's degenerate flags
  int* running = nullptr;
  double* partials = nullptr;  // ntiles x k x DM (sums in LDS only)
  int32_t* pcnt = nullptr;     // ntiles x k
};

// bigmeans_fit for BF16 points with BM_PREC_BF16_MFMA (Alg. 1 with the
// sample-level K-means on the matrix cores): all samples are drawn up front;
// per sample the incumbent's degenerate slots are reseeded by the solver in
// seed-only mode, then each K-means round is the matrix-core assignment
// (labels equal to the FP32 path's), the batched kernel's FP64 accumulation
// and objective for those labels, and its update with the stop rules; the
// keep-the-best comparison runs on the host between samples.  *handled is
// false (and nothing is done) when the shape does not suit this form.
static bm_status fit_mfma_run(const void* X, int64_t n, int32_t d, int32_t k, int64_t s,
                              int32_t n_samples, uint64_t seed, const bm_options& o,
                              float* centroids, double* sse, int32_t* labels, uint8_t* degenerate,
                              bm_stats* stats, int grid_cap, bool* handled) {
  *handled = false;
  bm_status st = BM_OK;
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  SolverPlan sp;
  if ((st = plan_solver(d, k, s, n, o.grid, &sp)) != BM_OK) return st;
  if (grid_cap > 0 && sp.grid > grid_cap && (st = plan_solver(d, k, s, n, grid_cap, &sp)) != BM_OK)
    return st;
  const int T = n_samples;
  if (T > 65535 || sample_slots(n, s, d, T, sp.cand_cap) < T) return BM_OK;
  const int dm = padded_dim(d);
  size_t lds_max = 0;
  if ((st = max_lds_per_block(&lds_max)) != BM_OK) return st;
  const bool sums_lds = batch_assign_lds(d, k, true) + 1024 <= lds_max;
  if (!sums_lds && batch_assign_lds(d, k, false) + 1024 > lds_max) return BM_OK;
  const bool final_pass = sse || labels;
  int fgrid = 0;
  if (final_pass && plan_assign_mfma(X, n, d, k, &fgrid) != BM_OK) {
    clear_error();
    return BM_OK;
  }
  int bgrid = 0;
  if ((st = batch_assign_grid(d, k, sums_lds, &bgrid)) != BM_OK) return st;
  // accumulation for the matrix-core labels: a wavefront per row (wide rows)
  // when its FP64 sums fit in LDS, else the batched kernel; either way one
  // tile of rows per workgroup, and with the sums in LDS each workgroup writes
  // one partial block, added in workgroup order
  const bool wave_rows = labels_accum_lds(d, k) + 1024 <= lds_max;
  if (wave_rows) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return set_error(BM_EDEVICE, "cannot query the device");
    const int64_t want = (s + 511) / 512;
    bgrid = static_cast<int>(want < cus ? (want < 1 ? 1 : want) : cus);
  }
  const int64_t tile_rows64 = (s + bgrid - 1) / bgrid;
  const int kTile = static_cast<int>(tile_rows64);
  const int ntiles = static_cast<int>((s + kTile - 1) / kTile);
  const bool use_partials = wave_rows || sums_lds;
  // the sample buffers of this form, on the inner pool
  MfmaLloydBuffers m;
  {
    InnerScratch inner;
    char* base = nullptr;
    for (int round = 0; round < 2; ++round) {
      Layout L;
      L.base = base;
      m.p16 = L.take<uint16_t>(static_cast<size_t>(s) * d + 8);
      m.ppad = L.take<float>(dm == d ? 1 : static_cast<size_t>(s) * dm);
      m.lab = L.take<int32_t>(s);
      m.sv = L.take<BatchSolve>(1);
      m.tiles = L.take<int32_t>(ntiles);
      m.tile_f = L.take<double>(ntiles);
      m.sums = L.take<double>(static_cast<size_t>(k) * dm);
      m.cnt = L.take<int32_t>(k);
      m.c64 = L.take<double>(static_cast<size_t>(k) * d);
      m.cpad = L.take<float>(static_cast<size_t>(k) * dm);
      m.cw = L.take<float>(static_cast<size_t>(k) * d);
      m.degw = L.take<uint8_t>(k);
      m.deginc = L.take<uint8_t>(k);
      m.running = L.take<int>(1);
      m.bad = L.take<int>(1);
      m.partials = L.take<double>(use_partials ? static_cast<size_t>(bgrid) * k * dm : 1);
      m.pcnt = L.take<int32_t>(use_partials ? static_cast<size_t>(bgrid) * k : 1);
      if (round == 0) {
        base = static_cast<char*>(scratch_get(L.off + 256, stream, &st));
        if (!base) return st;
      }
    }
  }
  int mgrid = 0;
  if (plan_assign_mfma(m.p16, s, d, k, &mgrid) != BM_OK) {
    clear_error();
    return BM_OK;
  }
  *handled = true;

  SolverBuffers b;
  memset(&b.a, 0, sizeof b.a);
  const int mx_grid = fgrid > mgrid ? fgrid : mgrid;
  if ((st = prepare_solver(stream, n, s, d, k, T, sp.cand_cap, true, true, true, true, mx_grid, T,
                           &b)) != BM_OK)
    return st;
  EventSet<3> ev;
  BM_HIP(ev.create());
  BM_HIP(hipEventRecord(ev[0], stream));

  // (1) every sample's indices; FP32 rows too when the accumulation reads them
  // (otherwise a sample's FP32 rows are gathered only when it reseeds)
  SolverArgs a = b.a;
  a.X = X;
  a.n = n;
  a.s = s;
  a.d = d;
  a.k = k;
  a.x_bf16 = 1;
  a.T = T;
  a.seed = seed;
  a.t0 = o.t_start;
  a.max_iter = o.max_iter;
  a.tol = o.tol;
  a.stop_rule = o.stop_rule;
  a.trials = o.n_local_trials;
  a.cmp_rule = BM_CMP_FOPT;
  a.do_sample = 1;
  a.do_gather = wave_rows ? 0 : 1;
  a.init_incumbent = 1;
  a.init_forgy = o.init_method == BM_INIT_FORGY ? 1 : 0;
  a.sums_in_lds = sp.sums_in_lds;
  a.c64_in_lds = sp.c64_in_lds;
  a.cand_cap = sp.cand_cap;
  a.win_lo = sp.win_lo;
  a.win_hi = sp.win_hi;
  a.spin_limit = o.spin_limit ? o.spin_limit : kDefaultSpinLimit;
  a.sample_idx_out = o.sample_idx;
  using clk = std::chrono::steady_clock;
  auto since = [](clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  };
  double ms_sampling = 0.0, ms_seeding = 0.0, ms_lloyd = 0.0;
  auto tp = clk::now();
  const int pmode = g_presample_mode.load();
  if (pmode != 1) st = launch_presample(a, sp.lds, stream, pmode == 2);
  if (st == BM_OK) st = launch_solver(a, sp.grid, sp.lds, stream);
  if (st != BM_OK) return st;
  if ((st = check_solver_error(a, stream, nullptr)) != BM_OK) return st;
  ms_sampling += since(tp);
  float* const Pb = b.a.P;
  int32_t* const idxb = b.a.idx;

  // (2) the incumbent: the caller's buffer (NaN when fresh)
  const size_t cbytes = sizeof(float) * static_cast<size_t>(k) * d;
  std::vector<uint8_t> deg_inc(static_cast<size_t>(k), 1);
  double f_opt = __builtin_inf();
  if (o.resume) {
    memcpy(deg_inc.data(), degenerate, size_t(k));
    f_opt = o.f_opt_in;
  } else {
    BM_HIP(hipMemsetAsync(centroids, 0xFF, cbytes, stream));
  }
  MfmaStage* stg = nullptr;
  if (k > 256) return set_error(BM_EINVAL, "k = %d beyond the matrix-core fit's 256", k);
  if ((st = mfma_stage(&stg)) != BM_OK) return st;
  BM_HIP(hipMemcpyAsync(m.deginc, deg_inc.data(), size_t(k), hipMemcpyHostToDevice, stream));
  std::vector<int32_t> tiles(ntiles, 0);
  BM_HIP(hipMemcpyAsync(m.tiles, tiles.data(), sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, stream));
  int64_t replaced = 0, passes_total = 0, reseeded = 0, nd = 0;
  int64_t seed_counters[kNumCounters] = {};
  // per-sample phase boundaries on the stream: start, seeded, last round
  EventSet<3> pe;
  BM_HIP(pe.create());
  BatchSolve init;
  memset(&init, 0, sizeof init);
  init.row0 = 0;
  init.s = s;
  init.c0 = 0;
  init.k = k;
  init.tile0 = 0;
  init.ntiles = ntiles;
  init.status = kSolveRunning;
  init.iter = 1;
  init.f_prev = __builtin_inf();
  for (int tt = 0; tt < T; ++tt) {
    const uint32_t t = static_cast<uint32_t>(o.t_start + tt);
    float* P = Pb + static_cast<size_t>(tt) * s * d;
    BM_HIP(hipEventRecord(pe[0], stream));
    // the sample's solve starts from the incumbent
    if ((st = launch_solve_start(centroids, m.deginc, m.cw, m.degw, m.sv, init, m.sums, m.cnt, k, d,
                                 stream)) != BM_OK)
      return st;
    bool any_deg = false;
    for (int j = 0; j < k; ++j) any_deg = any_deg || deg_inc[j];
    if (any_deg) {  // reseed on this sample (K-means++ or Forgy, draws of sample t)
      if (wave_rows) {
        BM_HIP(hipMemsetAsync(m.bad, 0, sizeof(int), stream));
        if ((st = launch_gather_rows(X, 1, n, d, idxb + static_cast<size_t>(tt) * s, s, P, m.bad,
                                     stream)) != BM_OK)
          return st;
      }
      SolverArgs q = a;
      q.P = P;
      q.T = 1;
      q.t0 = static_cast<int32_t>(t);
      q.sbatch = 1;
      q.do_sample = 0;
      q.do_gather = 0;
      q.do_seed = 1;
      q.init_incumbent = 0;
      q.presampled = 0;
      q.sample_idx_out = nullptr;
      q.Cinc = m.cw;
      q.deg_inc = m.degw;
      BM_HIP(hipMemsetAsync(b.a.bar, 0, b.ctrl_bytes, stream));
      if ((st = launch_solver(q, sp.grid, sp.lds, stream)) != BM_OK) return st;
      BM_HIP(hipMemcpyAsync(stg->cnt, q.counters, sizeof stg->cnt, hipMemcpyDeviceToHost, stream));
      BM_HIP(hipMemcpyAsync(&stg->err, q.err, sizeof stg->err, hipMemcpyDeviceToHost, stream));
    }
    BM_HIP(hipEventRecord(pe[1], stream));
    // (3) K-means on the sample: matrix-core labels, FP64 sums and objective
    if ((st = launch_gather_rows_bf16(static_cast<const uint16_t*>(X), d,
                                      idxb + static_cast<size_t>(tt) * s, s, m.p16, stream)) != BM_OK)
      return st;
    const float* Pp = P;
    if (dm != d && !wave_rows) {
      if ((st = launch_pad_rows(P, m.ppad, s, d, stream)) != BM_OK) return st;
      Pp = m.ppad;
    }
    if ((st = launch_batch_init(m.cw, m.c64, m.cpad, k, d, stream)) != BM_OK) return st;
    // Rounds go out in groups of kRoundsPerSync between reads of the solve's
    // record: every kernel of a round returns at once when the solve is done,
    // so rounds queued past the end cost a few empty launches, less than a
    // host round trip per round.
    constexpr int kRoundsPerSync = 4;
    bool done = false, first_group = true;
    for (int round = 0; round <= o.max_iter && !done;) {
      for (int q = 0; q < kRoundsPerSync && round <= o.max_iter; ++q, ++round) {
        if ((st = launch_assign_mfma(m.p16, s, d, m.cw, m.degw, k, m.lab, nullptr, nullptr, nullptr,
                                     b.rechecked, mgrid, stream, &m.sv->status)) != BM_OK)
          return st;
        if (wave_rows) {
          if ((st = launch_labels_accum(m.p16, s, d, k, m.cw, m.lab, m.sv, m.partials, m.pcnt,
                                        m.tile_f, ntiles, stream)) != BM_OK)
            return st;
        } else if ((st = launch_batch_assign(Pp, d, m.cw, m.cpad, m.degw, m.sv, m.tiles, ntiles, kTile,
                                             k, sums_lds, m.sums, m.cnt, m.tile_f, nullptr, 0, ntiles,
                                             stream, m.lab, sums_lds ? m.partials : nullptr,
                                             sums_lds ? m.pcnt : nullptr)) != BM_OK) {
          return st;
        }
        if (use_partials &&
            (st = launch_batch_reduce(m.partials, m.pcnt, ntiles, k, d, m.sums, m.cnt, m.sv, stream)) != BM_OK)
          return st;
        if ((st = launch_batch_update(m.sv, 1, m.tile_f, m.sums, m.cnt, m.cw, m.cpad, m.c64, m.degw, d,
                                      o.max_iter, o.tol, o.stop_rule, m.running, stream, k)) != BM_OK)
          return st;
      }
      // the solve's record and flags after these rounds
      BM_HIP(hipEventRecord(pe[2], stream));
      BM_HIP(hipMemcpyAsync(&stg->hs, m.sv, sizeof stg->hs, hipMemcpyDeviceToHost, stream));
      BM_HIP(hipMemcpyAsync(stg->deg, m.degw, size_t(k), hipMemcpyDeviceToHost, stream));
      BM_HIP(hipStreamSynchronize(stream));
      if (first_group && any_deg) {
        if ((st = solver_error(stg->err)) != BM_OK) return st;
        reseeded += stg->cnt[kCntReseeded];
        nd += stg->cnt[kCntND];
        for (int c = 0; c < kNumCounters; ++c) seed_counters[c] += stg->cnt[c];
      }
      first_group = false;
      done = stg->hs.status == kSolveDone;
    }
    if (!done) return set_error(BM_EDEVICE, "sample K-means did not finish in max_iter + 1 rounds");
    const BatchSolve hs = stg->hs;
    if (any_deg) ms_seeding += elapsed_ms(pe[0], pe[1]);
    ms_lloyd += elapsed_ms(pe[1], pe[2]);
    passes_total += hs.passes;
    nd += hs.nd;
    if (o.sample_f) o.sample_f[tt] = hs.f;
    // (4) keep the best (Alg. 1)
    if (f_opt > hs.f) {
      BM_HIP(hipMemcpyAsync(centroids, m.cw, cbytes, hipMemcpyDeviceToDevice, stream));
      BM_HIP(hipMemcpyAsync(m.deginc, m.degw, size_t(k), hipMemcpyDeviceToDevice, stream));
      memcpy(deg_inc.data(), stg->deg, size_t(k));
      f_opt = hs.f;
      ++replaced;
    }
  }
  BM_HIP(hipEventRecord(ev[1], stream));
  // final assignment (Alg. 1 last step) on the matrix cores
  double sse_host = 0.0;
  unsigned long long nrecheck = 0;
  if (final_pass) {
    BM_HIP(hipMemcpyAsync(b.a.deg_inc, deg_inc.data(), size_t(k), hipMemcpyHostToDevice, stream));
    BM_HIP(hipMemsetAsync(b.rechecked, 0, sizeof(unsigned long long), stream));
    if ((st = launch_assign_mfma(static_cast<const uint16_t*>(X), n, d, centroids, b.a.deg_inc, k,
                                 labels, nullptr, b.partial, b.sse_dev, b.rechecked, fgrid,
                                 stream)) != BM_OK)
      return st;
    BM_HIP(hipMemcpyAsync(&sse_host, b.sse_dev, sizeof(double), hipMemcpyDeviceToHost, stream));
    BM_HIP(hipMemcpyAsync(&nrecheck, b.rechecked, sizeof nrecheck, hipMemcpyDeviceToHost, stream));
  }
  BM_HIP(hipEventRecord(ev[2], stream));
  BM_HIP(hipStreamSynchronize(stream));
  if (sse) *sse = sse_host;
  if (degenerate) memcpy(degenerate, deg_inc.data(), size_t(k));
  seed_counters[kCntPasses] = passes_total;
  seed_counters[kCntSamples] = T;
  memcpy(g_last_counters, seed_counters, sizeof seed_counters);
  if (stats) {
    memset(reinterpret_cast<char*>(stats) + sizeof(uint32_t), 0, sizeof(bm_stats) - sizeof(uint32_t));
    stats->samples = T;
    stats->replacements = static_cast<int32_t>(replaced);
    stats->grid = sp.grid;
    stats->lloyd_iters = passes_total;
    stats->reseeded = reseeded;
    stats->n_d = nd;
    stats->boundary_draws = seed_counters[kCntBoundary];
    stats->f_opt = f_opt;
    stats->ms_solver = elapsed_ms(ev[0], ev[1]);
    stats->ms_final = final_pass ? elapsed_ms(ev[1], ev[2]) : 0.0;
    stats->rechecked = static_cast<int64_t>(nrecheck);
    // host-timed phases of this form (each ends with a synchronisation)
    stats->ms_sampling = ms_sampling;
    stats->ms_seeding = ms_seeding;
    stats->ms_lloyd = ms_lloyd;
  }
  return BM_OK;
}

// The body of bigmeans_fit after validation.  The caller serialises access to
// the scratch pool in use (the shared pool under g_mu, or a serving slot's own
// pool).  grid_cap > 0 bounds the cooperative grid.
bm_status fit_run(const void* X, int64_t n, int32_t d, int32_t k, int64_t s, int32_t n_samples,
                  uint64_t seed, const bm_options& o, float* centroids, double* sse,
                  int32_t* labels, uint8_t* degenerate, bm_stats* stats, int grid_cap) {
  bm_status st = BM_OK;
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  // Host-side setup and launches of concurrent fits (serving slots) are
  // serialised; the device work they enqueue still overlaps.
  std::unique_lock<std::mutex> launch_lock(g_launch_mu);
  if (o.precision == BM_PREC_BF16_MFMA && o.x_dtype == BM_BF16 && o.compare_rule == BM_CMP_FOPT &&
      o.time_budget_ms <= 0.0 && o.final_mode == BM_FINAL_ASSIGN && g_mfma_lloyd.load() && !t_pool) {
    bool handled = false;
    st = fit_mfma_run(X, n, d, k, s, n_samples, seed, o, centroids, sse, labels, degenerate, stats,
                      grid_cap, &handled);
    if (handled || st != BM_OK) return st;
  }
  SolverPlan sp;
  if ((st = plan_solver(d, k, s, n, o.grid, &sp)) != BM_OK) return st;
  if (grid_cap > 0 && sp.grid > grid_cap &&
      (st = plan_solver(d, k, s, n, grid_cap, &sp)) != BM_OK)
    return st;

  const bool polish = o.final_mode == BM_FINAL_POLISH && (sse || labels);
  const bool final_pass = (sse || labels) && !polish;
  const bool final_mfma = final_pass && o.precision == BM_PREC_BF16_MFMA;
  int final_grid = final_pass ? assign_grid(n, d) : 0;
  if (final_mfma && (st = plan_assign_mfma(X, n, d, k, &final_grid)) != BM_OK) return st;
  // with a time budget the samples are drawn a few at a time (most of a
  // larger batch could go unused)
  const bool budget = o.time_budget_ms > 0.0;
  int sbatch = sample_slots(n, s, d, n_samples, sp.cand_cap);
  if (budget && sbatch > 2) sbatch = 2;
  uint64_t budget_ticks = 0;
  if (budget) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      return set_error(BM_EDEVICE, "cannot read the device wall-clock rate");
    const double ticks = o.time_budget_ms * static_cast<double>(khz);
    budget_ticks = ticks < 1.0 ? 1 : static_cast<uint64_t>(ticks);
  }
  SolverBuffers b;
  memset(&b.a, 0, sizeof b.a);
  if ((st = prepare_solver(stream, n, s, d, k, n_samples, sp.cand_cap, true, true, true, true,
                           final_grid, sbatch, &b)) != BM_OK)
    return st;
  SolverArgs& a = b.a;
  a.X = X;
  a.n = n;
  a.s = s;
  a.d = d;
  a.k = k;
  a.x_bf16 = o.x_dtype == BM_BF16;
  a.T = n_samples;
  a.seed = seed;
  a.t0 = o.t_start;
  a.max_iter = o.max_iter;
  a.tol = o.tol;
  a.stop_rule = o.stop_rule;
  a.trials = o.n_local_trials;
  a.cmp_rule = o.compare_rule;
  a.do_sample = 1;
  a.do_gather = 1;
  a.do_seed = 1;
  a.do_lloyd = 1;
  a.do_keep = 1;
  a.init_incumbent = o.resume ? 0 : 1;
  a.init_forgy = o.init_method == BM_INIT_FORGY ? 1 : 0;
  a.budget_ticks = budget_ticks;
  a.sums_in_lds = sp.sums_in_lds;
  a.c64_in_lds = sp.c64_in_lds;
  a.cand_cap = sp.cand_cap;
  a.win_lo = sp.win_lo;
  a.win_hi = sp.win_hi;
  a.spin_limit = o.spin_limit ? o.spin_limit : kDefaultSpinLimit;
  a.sample_idx_out = o.sample_idx;

  if (o.resume) {
    BM_HIP(hipMemcpyAsync(a.Cinc, centroids, sizeof(float) * size_t(k) * d, hipMemcpyDeviceToDevice, stream));
    BM_HIP(hipMemcpyAsync(a.deg_inc, degenerate, size_t(k), hipMemcpyHostToDevice, stream));
    BM_HIP(hipMemcpyAsync(a.f_opt, &o.f_opt_in, sizeof(double), hipMemcpyHostToDevice, stream));
  }

  EventSet<3> ev;
  BM_HIP(ev.create());
  BM_HIP(hipEventRecord(ev[0], stream));
  // every sample drawn up front by ordinary launches when they all have a slot
  const int pmode = g_presample_mode.load();
  if (pmode != 1 && !budget && a.sbatch == a.T && a.T <= 65535)
    st = launch_presample(a, sp.lds, stream, pmode == 2);
  if (st == BM_OK) st = launch_solver(a, sp.grid, sp.lds, stream);
  if (st != BM_OK) return st;
  BM_HIP(hipEventRecord(ev[1], stream));

  // final assignment (Alg. 1 last step) over all of X
  double sse_host = 0.0;
  bm_status fst = BM_OK;
  if (final_mfma) {
    fst = launch_assign_mfma(static_cast<const uint16_t*>(X), n, d, a.Cinc, a.deg_inc, k, labels,
                             nullptr, b.partial, b.sse_dev, b.rechecked, final_grid, stream);
  } else if (final_pass) {
    fst = launch_assign(X, a.x_bf16, n, d, a.Cinc, a.deg_inc, k, labels, nullptr, b.partial,
                        b.sse_dev, final_grid, stream);
  }
  BM_HIP(hipEventRecord(ev[2], stream));
  launch_lock.unlock();
  if (final_pass && fst == BM_OK)
    BM_HIP(hipMemcpyAsync(&sse_host, b.sse_dev, sizeof(double), hipMemcpyDeviceToHost, stream));

  BM_HIP(hipMemcpyAsync(centroids, a.Cinc, sizeof(float) * size_t(k) * d, hipMemcpyDeviceToDevice, stream));
  int64_t counters[kNumCounters];
  double fopt = 0.0;
  BM_HIP(hipMemcpyAsync(counters, a.counters, sizeof counters, hipMemcpyDeviceToHost, stream));
  BM_HIP(hipMemcpyAsync(&fopt, a.f_opt, sizeof fopt, hipMemcpyDeviceToHost, stream));
  unsigned long long nrecheck = 0;
  if (final_mfma)
    BM_HIP(hipMemcpyAsync(&nrecheck, b.rechecked, sizeof nrecheck, hipMemcpyDeviceToHost, stream));
  if (degenerate)
    BM_HIP(hipMemcpyAsync(degenerate, a.deg_inc, size_t(k), hipMemcpyDeviceToHost, stream));
  if (o.sample_f)
    BM_HIP(hipMemcpyAsync(o.sample_f, a.sample_f, sizeof(double) * n_samples, hipMemcpyDeviceToHost, stream));
  std::vector<uint8_t> deg_host(static_cast<size_t>(k));
  if (polish)
    BM_HIP(hipMemcpyAsync(deg_host.data(), a.deg_inc, size_t(k), hipMemcpyDeviceToHost, stream));
  int32_t code = 0;
  st = check_solver_error(a, stream, &code);
  memcpy(g_last_counters, counters, sizeof counters);
  const float ms_solver = elapsed_ms(ev[0], ev[1]);
  float ms_final = final_pass ? elapsed_ms(ev[1], ev[2]) : 0.f;
  if (st != BM_OK) return st;
  if (fst != BM_OK) return fst;
  int32_t polish_passes = 0;
  if (polish) {
    // Sec. 3.4: K-means on all of X from the Big-means centroids (in place in
    // the caller's buffer), one batched problem; its last assignment gives
    // the labels and the objective of the returned centroids
    const auto t0 = std::chrono::steady_clock::now();
    InnerScratch inner;
    const int64_t rows[1] = {n};
    const int32_t ks[1] = {k};
    double fp = 0.0;
    bm_status pst = batched_run(1, static_cast<const float*>(X), d, rows, ks, centroids,
                                deg_host.data(), o, labels, &fp, &polish_passes);
    if (pst != BM_OK) return pst;
    if (degenerate) memcpy(degenerate, deg_host.data(), size_t(k));
    sse_host = fp;
    ms_final = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (sse) *sse = sse_host;
  if (stats) {
    stats->samples = static_cast<int32_t>(counters[kCntSamples]);
    stats->replacements = static_cast<int32_t>(counters[kCntReplaced]);
    stats->grid = sp.grid;
    stats->lloyd_iters = counters[kCntPasses];
    stats->reseeded = counters[kCntReseeded];
    stats->n_d = counters[kCntND];
    stats->boundary_draws = counters[kCntBoundary];
    stats->f_opt = fopt;
    stats->ms_solver = ms_solver;
    stats->ms_final = ms_final;
    stats->rechecked = static_cast<int64_t>(nrecheck);
    stats->final_passes = polish_passes;
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0) {
      stats->ms_sampling = static_cast<double>(counters[kCntTicksSample]) / khz;
      stats->ms_seeding = static_cast<double>(counters[kCntTicksSeed]) / khz;
      stats->ms_lloyd = static_cast<double>(counters[kCntTicksLloyd]) / khz;
      stats->ms_lloyd_pass = static_cast<double>(counters[kCntTicksPass]) / khz;
      stats->ms_lloyd_post = static_cast<double>(counters[kCntTicksPost]) / khz;
      stats->ms_lloyd_wait = static_cast<double>(counters[kCntTicksBarrier]) / khz;
    }
  }
  return BM_OK;
}

}  // namespace bm

extern "C" {

bm_status bigmeans_fit(const void* X, int64_t n, int32_t d, int32_t k, int64_t s,
                       int32_t n_samples, uint64_t seed, const bm_options* opt_in,
                       float* centroids, double* sse, int32_t* labels, uint8_t* degenerate,
                       bm_stats* stats) {
  clear_error();
  bm_options o;
  bm_status st = fit_validate(X, n, d, k, s, n_samples, opt_in, centroids, degenerate, stats, &o);
  if (st != BM_OK) return st;
  std::lock_guard<std::mutex> lock(g_mu);
  return fit_run(X, n, d, k, s, n_samples, seed, o, centroids, sse, labels, degenerate, stats, 0);
}

bm_status kmeans_assign(const void* X, int64_t n, int32_t d, const float* C, const uint8_t* deg,
                        int32_t k, const bm_options* opt_in, int32_t* labels, float* min_d2,
                        double* sse) {
  clear_error();
  bm_options o;
  bm_status st = resolve(opt_in, &o);
  if (st != BM_OK) return st;
  if (n < 1 || n > 2147483647LL || d < 1 || k < 1)
    return set_error(BM_EINVAL, "bad sizes n=%lld d=%d k=%d", (long long)n, d, k);
  if (!X || !C) return set_error(BM_EINVAL, "X and C are required");
  if (deg) {
    int active = 0;
    for (int j = 0; j < k; ++j) active += deg[j] ? 0 : 1;
    if (!active) return set_error(BM_EINVAL, "every centroid is degenerate");
  }
  if (padded_dim(d) < 0) return set_error(BM_ENOTSUP, "d = %d exceeds the limit of 256", d);
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  const bool mfma = o.precision == BM_PREC_BF16_MFMA;
  std::lock_guard<std::mutex> lock(g_mu);
  int grid = assign_grid(n, d);
  if (mfma && (st = plan_assign_mfma(X, n, d, k, &grid)) != BM_OK) return st;
  uint8_t* deg_p = nullptr;
  double* partial_p = nullptr;
  double* sse_p = nullptr;
  unsigned long long* rechecked_p = nullptr;
  char* base = nullptr;
  for (int round = 0; round < 2; ++round) {
    Layout L;
    L.base = base;
    deg_p = L.take<uint8_t>(k);
    partial_p = L.take<double>(grid);
    sse_p = L.take<double>(1);
    rechecked_p = L.take<unsigned long long>(1);
    if (round == 0) {
      bm_status st2 = BM_OK;
      base = static_cast<char*>(scratch_get(L.off + 256, stream, &st2));
      if (!base) return st2;
    }
  }
  if (deg) BM_HIP(hipMemcpyAsync(deg_p, deg, size_t(k), hipMemcpyHostToDevice, stream));
  if (mfma) BM_HIP(hipMemsetAsync(rechecked_p, 0, sizeof(unsigned long long), stream));
  EventSet<2> ev;
  BM_HIP(ev.create());
  BM_HIP(hipEventRecord(ev[0], stream));
  if (mfma) {
    st = launch_assign_mfma(static_cast<const uint16_t*>(X), n, d, C, deg ? deg_p : nullptr, k,
                            labels, min_d2, partial_p, sse_p, rechecked_p, grid, stream);
  } else {
    st = launch_assign(X, o.x_dtype == BM_BF16, n, d, C, deg ? deg_p : nullptr, k, labels, min_d2,
                       partial_p, sse_p, grid, stream);
  }
  if (st == BM_OK && hipEventRecord(ev[1], stream) != hipSuccess)
    st = set_error(BM_EDEVICE, "hipEventRecord failed");
  if (st != BM_OK) return st;
  double v = 0.0;
  unsigned long long nrecheck = 0;
  BM_HIP(hipMemcpyAsync(&v, sse_p, sizeof v, hipMemcpyDeviceToHost, stream));
  if (mfma)
    BM_HIP(hipMemcpyAsync(&nrecheck, rechecked_p, sizeof nrecheck, hipMemcpyDeviceToHost, stream));
  const hipError_t sync = hipStreamSynchronize(stream);
  g_last_assign_ms = sync == hipSuccess ? elapsed_ms(ev[0], ev[1]) : 0.0;
  if (sync != hipSuccess)
    return set_error(BM_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(sync));
  g_last_rechecked = static_cast<int64_t>(nrecheck);
  if (sse) *sse = v;
  return BM_OK;
}

static bm_status run_solver_on_sample(const float* P, int64_t s, int32_t d, int32_t k, float* C,
                                      uint8_t* deg, uint64_t seed, uint32_t t, bool seed_only,
                                      const bm_options& o, int32_t* labels, double* f,
                                      int32_t* passes) {
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  std::lock_guard<std::mutex> lock(g_mu);
  SolverPlan sp;
  bm_status st = plan_solver(d, k, s, 2 * s, o.grid, &sp);
  if (st != BM_OK) return st;
  SolverBuffers b;
  memset(&b.a, 0, sizeof b.a);
  b.a.P = const_cast<float*>(P);
  b.a.Cinc = C;
  b.a.labels = labels;
  if ((st = prepare_solver(stream, s, s, d, k, 1, sp.cand_cap, false, true, labels == nullptr, false,
                           0, 1, &b)) != BM_OK)
    return st;
  SolverArgs& a = b.a;
  a.X = nullptr;
  a.n = s;
  a.s = s;
  a.d = d;
  a.k = k;
  a.T = 1;
  a.seed = seed;
  a.t0 = static_cast<int32_t>(t);
  a.max_iter = o.max_iter;
  a.tol = o.tol;
  a.stop_rule = o.stop_rule;
  a.trials = o.n_local_trials;
  a.cmp_rule = BM_CMP_FOPT;
  a.do_seed = seed_only ? 1 : 0;
  a.do_lloyd = seed_only ? 0 : 1;
  a.sums_in_lds = sp.sums_in_lds;
  a.c64_in_lds = sp.c64_in_lds;
  a.cand_cap = sp.cand_cap;
  a.win_lo = sp.win_lo;
  a.win_hi = sp.win_hi;
  a.spin_limit = o.spin_limit ? o.spin_limit : kDefaultSpinLimit;
  BM_HIP(hipMemcpyAsync(a.deg_inc, deg, size_t(k), hipMemcpyHostToDevice, stream));
  if ((st = launch_solver(a, sp.grid, sp.lds, stream)) != BM_OK) return st;
  int64_t counters[kNumCounters];
  double fv = 0.0;
  BM_HIP(hipMemcpyAsync(deg, a.deg_inc, size_t(k), hipMemcpyDeviceToHost, stream));
  BM_HIP(hipMemcpyAsync(counters, a.counters, sizeof counters, hipMemcpyDeviceToHost, stream));
  BM_HIP(hipMemcpyAsync(&fv, a.sample_f, sizeof fv, hipMemcpyDeviceToHost, stream));
  if ((st = check_solver_error(a, stream, nullptr)) != BM_OK) return st;
  if (f) *f = fv;
  if (passes) *passes = static_cast<int32_t>(counters[kCntPasses]);
  return BM_OK;
}

bm_status kmeanspp_seed(const float* P, int64_t s, int32_t d, int32_t k, float* C, uint8_t* deg,
                        uint64_t seed, uint64_t stream_id, const bm_options* opt_in) {
  clear_error();
  bm_options o;
  bm_status st = resolve(opt_in, &o);
  if (st != BM_OK) return st;
  if (s < 1 || s > 2147483647LL || d < 1 || k < 1)
    return set_error(BM_EINVAL, "bad sizes s=%lld d=%d k=%d", (long long)s, d, k);
  if (!P || !C || !deg) return set_error(BM_EINVAL, "P, C and deg are required");
  if (stream_id > 0xffffffffull) return set_error(BM_EINVAL, "stream_id must be < 2^32");
  return run_solver_on_sample(P, s, d, k, C, deg, seed, static_cast<uint32_t>(stream_id), true, o,
                              nullptr, nullptr, nullptr);
}

bm_status kmeans_lloyd(const float* P, int64_t s, int32_t d, int32_t k, float* C, uint8_t* deg,
                       const bm_options* opt_in, int32_t* labels, double* f, int32_t* passes) {
  clear_error();
  bm_options o;
  bm_status st = resolve(opt_in, &o);
  if (st != BM_OK) return st;
  if (s < 1 || s > 2147483647LL || d < 1 || k < 1)
    return set_error(BM_EINVAL, "bad sizes s=%lld d=%d k=%d", (long long)s, d, k);
  if (!P || !C || !deg) return set_error(BM_EINVAL, "P, C and deg are required");
  int active = 0;
  for (int j = 0; j < k; ++j) active += deg[j] ? 0 : 1;
  if (!active) return set_error(BM_EINVAL, "every centroid is degenerate");
  return run_solver_on_sample(P, s, d, k, C, deg, 0, 0, false, o, labels, f, passes);
}

bm_status bm_sample_indices(int64_t n, int64_t s, uint64_t seed, int32_t t, int32_t* idx,
                            const bm_options* opt_in) {
  clear_error();
  bm_options o;
  bm_status st = resolve(opt_in, &o);
  if (st != BM_OK) return st;
  if (n < 1 || n > 2147483647LL || s < 1 || s > n)
    return set_error(BM_EINVAL, "need 1 <= s <= n < 2^31 (s=%lld, n=%lld)", (long long)s, (long long)n);
  if (t < 0) return set_error(BM_EINVAL, "t must be >= 0");
  if (!idx) return set_error(BM_EINVAL, "idx is required");
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  std::lock_guard<std::mutex> lock(g_mu);
  SolverPlan sp;
  if ((st = plan_solver(1, 1, s, n, o.grid, &sp)) != BM_OK) return st;
  SolverBuffers b;
  memset(&b.a, 0, sizeof b.a);
  b.a.idx = idx;
  if ((st = prepare_solver(stream, n, s, 1, 1, 1, sp.cand_cap, false, false, true, true, 0, 1, &b)) != BM_OK)
    return st;
  SolverArgs& a = b.a;
  a.n = n;
  a.s = s;
  a.d = 1;
  a.k = 1;
  a.T = 1;
  a.seed = seed;
  a.t0 = t;
  a.max_iter = 1;
  a.trials = 1;
  a.do_sample = 1;
  a.cand_cap = sp.cand_cap;
  a.win_lo = sp.win_lo;
  a.win_hi = sp.win_hi;
  a.sums_in_lds = sp.sums_in_lds;
  a.c64_in_lds = sp.c64_in_lds;
  a.spin_limit = o.spin_limit ? o.spin_limit : kDefaultSpinLimit;
  if ((st = launch_solver(a, sp.grid, sp.lds, stream)) != BM_OK) return st;
  return check_solver_error(a, stream, nullptr);
}

bm_status bm_gather_rows(const void* X, int64_t n, int32_t d, const int32_t* idx, int64_t s,
                         float* P, const bm_options* opt_in) {
  clear_error();
  bm_options o;
  bm_status st = resolve(opt_in, &o);
  if (st != BM_OK) return st;
  if (n < 1 || n > 2147483647LL || d < 1 || s < 1)
    return set_error(BM_EINVAL, "bad sizes n=%lld d=%d s=%lld", (long long)n, d, (long long)s);
  if (!X || !idx || !P) return set_error(BM_EINVAL, "X, idx and P are required");
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  std::lock_guard<std::mutex> lock(g_mu);
  int* bad = static_cast<int*>(scratch_get(256, stream, &st));
  if (!bad) return st;
  BM_HIP(hipMemsetAsync(bad, 0, sizeof(int), stream));
  if ((st = launch_gather_rows(X, o.x_dtype == BM_BF16, n, d, idx, s, P, bad, stream)) != BM_OK)
    return st;
  int bad_h = 0;
  BM_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
  BM_HIP(hipStreamSynchronize(stream));
  if (bad_h) return set_error(BM_EINVAL, "an index is outside [0, n)");
  return BM_OK;
}

bm_status kmeans_lloyd_batched(int32_t n_solves, const float* P, int32_t d, const int64_t* s,
                               const int32_t* k, float* C, uint8_t* deg, const bm_options* opt_in,
                               int32_t* labels, double* f, int32_t* passes) {
  clear_error();
  bm_options o;
  bm_status st = resolve(opt_in, &o);
  if (st != BM_OK) return st;
  std::lock_guard<std::mutex> lock(g_mu);
  return batched_run(n_solves, P, d, s, k, C, deg, o, labels, f, passes);
}

// Rounds and rows per tile of the last kmeans_lloyd_batched on this thread
// (declared in include/bigmeans_debug.h, as the next one).
int32_t bm_debug_batch_info(int32_t* rounds, int32_t* tile_rows) {
  if (rounds) *rounds = g_last_batch_rounds;
  if (tile_rows) *tile_rows = g_last_batch_tile;
  return BM_OK;
}

// Device time (ms) of round i of the last kmeans_lloyd_batched (0 if out of range).
double bm_debug_batch_round_ms(int32_t i) {
  return (i >= 0 && static_cast<size_t>(i) < g_last_batch_ms.size()) ? g_last_batch_ms[i] : 0.0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Collective parallel Big-means (Sec. 3.6, third scheme) and the sample-size
// rule of thumb (Sec. 5), composed from the kernels above.

namespace bm {

// Device buffer owned for the duration of one call.
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  bm_status alloc(size_t bytes) {
    if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return set_error(BM_ENOMEM, "cannot allocate %zu bytes of device memory", bytes);
    }
    return BM_OK;
  }
};

// The body of bigmeans_fit_collective after validation; the caller holds g_mu.
static bm_status collective_run(const void* X, int64_t n, int32_t d, int32_t k, int64_t s, int32_t W,
                                int32_t R, uint64_t seed, const bm_options& o, float* centroids,
                                double* sse, int32_t* labels, uint8_t* degenerate, bm_stats* stats,
                                double* worker_f) {
  bm_status st = BM_OK;
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  SolverPlan sp;
  if ((st = plan_solver(d, k, s, n, o.grid, &sp)) != BM_OK) return st;
  if (sample_slots(n, s, d, W, sp.cand_cap) < W)
    return set_error(BM_ENOTSUP, "the %d samples of a round do not fit the sample buffers", W);
  const bool final_pass = sse || labels;
  const bool final_mfma = final_pass && o.precision == BM_PREC_BF16_MFMA;
  int final_grid = final_pass ? assign_grid(n, d) : 0;
  if (final_mfma && (st = plan_assign_mfma(X, n, d, k, &final_grid)) != BM_OK) return st;
  SolverBuffers b;
  memset(&b.a, 0, sizeof b.a);
  if ((st = prepare_solver(stream, n, s, d, k, W, sp.cand_cap, true, true, true, true, final_grid, W,
                           &b)) != BM_OK)
    return st;
  // the workers' centroids and flags, and the incumbent's flags on the device
  const size_t cbytes = sizeof(float) * static_cast<size_t>(k) * d;
  DevBuf cw, degw_d;
  if ((st = cw.alloc(cbytes * W)) != BM_OK) return st;
  if ((st = degw_d.alloc(static_cast<size_t>(k) * W)) != BM_OK) return st;
  float* Cw = static_cast<float*>(cw.p);
  uint8_t* Dw = static_cast<uint8_t*>(degw_d.p);
  std::vector<uint8_t> deg_inc(static_cast<size_t>(k), 1), degw(static_cast<size_t>(k) * W);
  std::vector<int64_t> s_arr(W, s);
  std::vector<int32_t> k_arr(W, k), passes(W);
  std::vector<double> fw(W);
  double f_opt = __builtin_inf();
  int64_t replaced = 0, lloyd_iters = 0, reseeded = 0, boundary = 0;
  float* const Pb = b.a.P;
  // the incumbent lives in the caller's buffer: all degenerate (NaN) at first
  BM_HIP(hipMemsetAsync(centroids, 0xFF, cbytes, stream));
  const int pmode = g_presample_mode.load();

  for (int32_t r = 0; r < R; ++r) {
    const uint32_t t0 = static_cast<uint32_t>(static_cast<int64_t>(r) * W);
    // (1) the round's W samples, t = r W .. r W + W - 1, rows into slots w
    SolverArgs a = b.a;
    a.X = X;
    a.n = n;
    a.s = s;
    a.d = d;
    a.k = k;
    a.x_bf16 = o.x_dtype == BM_BF16;
    a.T = W;
    a.seed = seed;
    a.t0 = static_cast<int32_t>(t0);
    a.max_iter = o.max_iter;
    a.tol = o.tol;
    a.stop_rule = o.stop_rule;
    a.trials = o.n_local_trials;
    a.cmp_rule = BM_CMP_FOPT;
    a.do_sample = 1;
    a.do_gather = 1;
    a.init_incumbent = 1;
    a.init_forgy = o.init_method == BM_INIT_FORGY ? 1 : 0;
    a.sums_in_lds = sp.sums_in_lds;
    a.c64_in_lds = sp.c64_in_lds;
    a.cand_cap = sp.cand_cap;
    a.win_lo = sp.win_lo;
    a.win_hi = sp.win_hi;
    a.spin_limit = o.spin_limit ? o.spin_limit : kDefaultSpinLimit;
    a.presampled = 0;
    BM_HIP(hipMemsetAsync(b.a.bar, 0, b.ctrl_bytes, stream));
    if (pmode != 1 && W <= 65535) st = launch_presample(a, sp.lds, stream, pmode == 2);
    if (st == BM_OK) st = launch_solver(a, sp.grid, sp.lds, stream);
    if (st != BM_OK) return st;
    if ((st = check_solver_error(a, stream, nullptr)) != BM_OK) return st;
    // (2) every worker starts from the incumbent; its degenerate slots are
    // reinitialised on its own sample with its own draws (t = r W + w)
    for (int32_t w = 0; w < W; ++w) {
      BM_HIP(hipMemcpyAsync(Cw + static_cast<size_t>(w) * k * d, centroids, cbytes,
                            hipMemcpyDeviceToDevice, stream));
      memcpy(degw.data() + static_cast<size_t>(w) * k, deg_inc.data(), size_t(k));
    }
    BM_HIP(hipMemcpyAsync(Dw, degw.data(), degw.size(), hipMemcpyHostToDevice, stream));
    bool any_deg = false;
    for (int j = 0; j < k; ++j) any_deg = any_deg || deg_inc[j];
    if (any_deg) {
      for (int32_t w = 0; w < W; ++w) {
        SolverArgs q = a;
        q.P = Pb + static_cast<size_t>(w) * s * d;
        q.T = 1;
        q.t0 = static_cast<int32_t>(t0 + w);
        q.sbatch = 1;
        q.do_sample = 0;
        q.do_gather = 0;
        q.do_seed = 1;
        q.init_incumbent = 0;
        q.presampled = 0;
        q.Cinc = Cw + static_cast<size_t>(w) * k * d;
        q.deg_inc = Dw + static_cast<size_t>(w) * k;
        BM_HIP(hipMemsetAsync(b.a.bar, 0, b.ctrl_bytes, stream));
        if ((st = launch_solver(q, sp.grid, sp.lds, stream)) != BM_OK) return st;
        int64_t cnt[kNumCounters];
        BM_HIP(hipMemcpyAsync(cnt, q.counters, sizeof cnt, hipMemcpyDeviceToHost, stream));
        if ((st = check_solver_error(q, stream, nullptr)) != BM_OK) return st;
        reseeded += cnt[kCntReseeded];
        boundary += cnt[kCntBoundary];
      }
      BM_HIP(hipMemcpyAsync(degw.data(), Dw, degw.size(), hipMemcpyDeviceToHost, stream));
      BM_HIP(hipStreamSynchronize(stream));
    }
    // (3) K-means of all workers at once (the batched kernels)
    {
      InnerScratch inner;
      if ((st = batched_run(W, Pb, d, s_arr.data(), k_arr.data(), Cw, degw.data(), o, nullptr,
                            fw.data(), passes.data())) != BM_OK)
        return st;
    }
    // (4) the round's best worker (ties to the lowest) against f_opt (Alg. 1)
    int32_t best = 0;
    for (int32_t w = 1; w < W; ++w)
      if (fw[w] < fw[best]) best = w;
    for (int32_t w = 0; w < W; ++w) {
      lloyd_iters += passes[w];
      if (worker_f) worker_f[static_cast<size_t>(r) * W + w] = fw[w];
    }
    if (f_opt > fw[best]) {
      BM_HIP(hipMemcpyAsync(centroids, Cw + static_cast<size_t>(best) * k * d, cbytes,
                            hipMemcpyDeviceToDevice, stream));
      memcpy(deg_inc.data(), degw.data() + static_cast<size_t>(best) * k, size_t(k));
      f_opt = fw[best];
      ++replaced;
    }
  }
  // final assignment (Alg. 1 last step)
  double sse_host = 0.0;
  if (final_pass) {
    BM_HIP(hipMemcpyAsync(b.a.deg_inc, deg_inc.data(), size_t(k), hipMemcpyHostToDevice, stream));
    if (final_mfma) {
      st = launch_assign_mfma(static_cast<const uint16_t*>(X), n, d, centroids, b.a.deg_inc, k,
                              labels, nullptr, b.partial, b.sse_dev, b.rechecked, final_grid,
                              stream);
    } else {
      st = launch_assign(X, o.x_dtype == BM_BF16, n, d, centroids, b.a.deg_inc, k, labels, nullptr,
                         b.partial, b.sse_dev, final_grid, stream);
    }
    if (st != BM_OK) return st;
    BM_HIP(hipMemcpyAsync(&sse_host, b.sse_dev, sizeof(double), hipMemcpyDeviceToHost, stream));
  }
  BM_HIP(hipStreamSynchronize(stream));
  if (sse) *sse = sse_host;
  if (degenerate) memcpy(degenerate, deg_inc.data(), size_t(k));
  if (stats) {
    memset(reinterpret_cast<char*>(stats) + sizeof(uint32_t), 0, sizeof(bm_stats) - sizeof(uint32_t));
    stats->samples = static_cast<int32_t>(static_cast<int64_t>(R) * W);
    stats->replacements = static_cast<int32_t>(replaced);
    stats->grid = sp.grid;
    stats->lloyd_iters = lloyd_iters;
    stats->reseeded = reseeded;
    stats->n_d = -1;  // the batched kernels do not count distance evaluations
    stats->boundary_draws = boundary;
    stats->f_opt = f_opt;
  }
  return BM_OK;
}

}  // namespace bm

extern "C" {

bm_status bigmeans_fit_collective(const void* X, int64_t n, int32_t d, int32_t k, int64_t s,
                                  int32_t n_workers, int32_t n_rounds, uint64_t seed,
                                  const bm_options* opt_in, float* centroids, double* sse,
                                  int32_t* labels, uint8_t* degenerate, bm_stats* stats,
                                  double* worker_f) {
  clear_error();
  if (n_workers < 1 || n_workers > 1024 || n_rounds < 1)
    return set_error(BM_EINVAL, "need 1 <= n_workers <= 1024 and n_rounds >= 1");
  const int64_t total = static_cast<int64_t>(n_workers) * n_rounds;
  if (total > 2147483647LL) return set_error(BM_EINVAL, "n_rounds x n_workers exceeds 2^31");
  bm_options o;
  bm_status st = fit_validate(X, n, d, k, s, static_cast<int32_t>(total), opt_in, centroids, nullptr,
                              stats, &o);
  if (st != BM_OK) return st;
  if (o.compare_rule != BM_CMP_FOPT)
    return set_error(BM_ENOTSUP, "the collective mode compares with f_opt (BM_CMP_FOPT) only");
  std::lock_guard<std::mutex> lock(g_mu);
  return collective_run(X, n, d, k, s, n_workers, n_rounds, seed, o, centroids, sse, labels,
                        degenerate, stats, worker_f);
}

bm_status bigmeans_sample_size_sweep(const void* X, int64_t n, int32_t d, int32_t k,
                                     int64_t s_min, int64_t s_max, int32_t n_samples,
                                     uint64_t seed, const bm_options* opt_in, float* centroids,
                                     double* sse, int32_t* labels, uint8_t* degenerate,
                                     int64_t* s_best, int64_t* s_tried, double* sse_tried,
                                     int32_t max_tried, int32_t* n_tried) {
  clear_error();
  if (!sse || !s_best) return set_error(BM_EINVAL, "sse and s_best are required");
  if (s_min > s_max) return set_error(BM_EINVAL, "need s_min <= s_max");
  bm_options o;
  bm_status st = fit_validate(X, n, d, k, s_min, n_samples, opt_in, centroids, nullptr, nullptr, &o);
  if (st != BM_OK) return st;
  if (o.final_mode != BM_FINAL_ASSIGN)
    return set_error(BM_EINVAL, "the sweep compares final assignments (final_mode BM_FINAL_ASSIGN)");
  o.resume = 0;
  o.t_start = 0;
  o.sample_idx = nullptr;
  o.sample_f = nullptr;
  if (s_max > n) s_max = n;
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  DevBuf ct, lt;
  const size_t cbytes = sizeof(float) * static_cast<size_t>(k) * d;
  if ((st = ct.alloc(cbytes)) != BM_OK) return st;
  if (labels && (st = lt.alloc(sizeof(int32_t) * static_cast<size_t>(n))) != BM_OK) return st;
  std::vector<uint8_t> degt(static_cast<size_t>(k));
  std::lock_guard<std::mutex> lock(g_mu);
  double best = __builtin_inf();
  int64_t bs = -1;
  int32_t m = 0;
  for (int64_t s = s_min;;) {
    double f = 0.0;
    st = fit_run(X, n, d, k, s, n_samples, seed, o, static_cast<float*>(ct.p), &f,
                 labels ? static_cast<int32_t*>(lt.p) : nullptr, degt.data(), nullptr, 0);
    if (st != BM_OK) return st;
    if (m < max_tried) {
      if (s_tried) s_tried[m] = s;
      if (sse_tried) sse_tried[m] = f;
    }
    ++m;
    if (!(f < best)) break;  // no improvement: the sweet spot is behind
    best = f;
    bs = s;
    BM_HIP(hipMemcpyAsync(centroids, ct.p, cbytes, hipMemcpyDeviceToDevice, stream));
    if (labels)
      BM_HIP(hipMemcpyAsync(labels, lt.p, sizeof(int32_t) * static_cast<size_t>(n),
                            hipMemcpyDeviceToDevice, stream));
    if (degenerate) memcpy(degenerate, degt.data(), size_t(k));
    if (s >= s_max) break;
    s = (s > s_max / 2) ? s_max : 2 * s;
  }
  BM_HIP(hipStreamSynchronize(stream));
  *sse = best;
  *s_best = bs;
  if (n_tried) *n_tried = m < max_tried ? m : max_tried;
  return BM_OK;
}

}  // extern "C"
