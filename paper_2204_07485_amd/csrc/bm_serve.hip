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
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string.h>
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

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }

  // Scratch bytes scratch_get() allocates for a request of `bytes`.
  static size_t pool_alloc(size_t bytes) { return bytes + bytes / 4 + (1u << 20); }

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
  c->slots.resize(cfg.slots);
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
  j->alloc = bm_ctx::pool_alloc(fit_scratch_bytes(J.n, J.d, J.k, J.s, J.n_samples,
                                                  J.sse != nullptr || J.labels != nullptr));
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
