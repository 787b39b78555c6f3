// bm_solver.hip -- the Big-means sample loop as one cooperative kernel.
//
// One launch runs Alg. 1's loop for T samples with all control on the device:
//   1. sample t: every point gets a Philox key; the s smallest (key, index)
//      pairs are found by an MSB radix select over 8-bit digits (histogram
//      passes until the window holding the s-th key is small, then a collect
//      pass and a bitonic sort in LDS), and emitted in index order while the
//      rows are gathered into the contiguous sample P (Sec. 3.1, 3.5);
//   2. C' <- C, then K-means++ on P for the degenerate slots of C' (Sec. 2,
//      greedy form of Sec. 5; Sec. 3.3), D^2 weights in FP64 by direct
//      differences, candidate located by an FP64 running sum;
//   3. K-means on P from C' (Sec. 2): fused assign + accumulate, FP32
//      distances by direct differences, FP64 sums in LDS flushed with FP64
//      atomics, one grid barrier per round;
//   4. keep the best (Alg. 1): replace the incumbent when the new sample
//      objective is strictly lower.
// Every workgroup makes the same control decisions from the same global
// reductions (fixed summation order), so all of them agree on every branch.
// Workgroup g owns a contiguous chunk of the sample rows and of the point
// pairs; per-workgroup partial results are combined after a grid barrier.
#include <math.h>

#include <type_traits>

#include <map>
#include <mutex>
#include <utility>

#include "bm_internal.h"
#include "bm_rng.h"

namespace bm {

namespace {

constexpr int kHistBins = 256;
constexpr int kCandStage = 4096;  // sampler candidates staged in LDS per workgroup

struct Lds {
  float* C;          // k x DM, padded with zeros past d
  int* act;          // active slots, ascending
  int* degf;         // degenerate flags
  int* tmpi;         // scan scratch
  double* tmpd;      // reduction scratch
  int* misc;         // [0] number of active slots, [1] chosen bucket, [2] hit flag, [6] last weighted row
  int64_t* misc64;   // [0] bucket count, [1] found row, [2] fallback row, [3] pick, [4..] draws
  double* miscd;     // [0] broadcast value, [1..] per-trial scratch
  double* c64;       // k x d FP64 means (when they fit)
  unsigned char* B;  // phase-local region
};

__device__ __forceinline__ int64_t imin64(int64_t x, int64_t y) { return x < y ? x : y; }

// Row stride (in doubles) of the per-cluster sums in LDS: odd, so the same
// coordinate of different clusters falls in different LDS banks.
__host__ __device__ __forceinline__ int sums_ld(int d) { return (d & 1) ? d : d + 1; }

// The LDS sums come in `reps` replicas (1, 2 or 4): lane l of a wavefront adds
// into replica l % reps, so lanes of one wavefront with the same label hit
// reps different words (same-address LDS atomics are serialised), and the
// replicas are added in a fixed order when the workgroup flushes.  Replica
// stride in doubles: odd, so a word's replicas fall in different banks.
__host__ __device__ __forceinline__ int sums_rstride(int k, int d) { return (k * sums_ld(d)) | 1; }

__host__ __device__ __forceinline__ size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

struct LdsPlan {
  size_t C, act, degf, tmpi, tmpd, misc, misc64, miscd, c64, B;
  size_t hist, selc, ckey, cidx, total_sampling;
  size_t sums, cntl, total_lloyd;
  size_t total;
};

// sums_reps: replicas of the FP64 cluster sums in LDS (0: the sums are
// accumulated in the global ring instead).
__host__ __device__ inline LdsPlan plan_lds(int dm, int k, int d, int sums_reps,
                                            bool c64_in_lds) {
  LdsPlan p;
  size_t o = 0;
  p.C = o; o = align16(o + sizeof(float) * size_t(k) * dm);
  p.act = o; o = align16(o + sizeof(int) * size_t(k));
  p.degf = o; o = align16(o + sizeof(int) * size_t(k));
  p.tmpi = o; o = align16(o + sizeof(int) * 32);
  p.tmpd = o; o = align16(o + sizeof(double) * 32);
  p.misc = o; o = align16(o + sizeof(int) * 8);
  p.misc64 = o; o = align16(o + sizeof(int64_t) * (4 + kMaxTrials));
  p.miscd = o; o = align16(o + sizeof(double) * (4 + 4 * kMaxTrials));
  p.c64 = o; o = align16(o + (c64_in_lds ? sizeof(double) * size_t(k) * d : 0));
  p.B = o;
  size_t b = 0;
  p.hist = b; b = align16(b + sizeof(unsigned int) * kHistBins);
  p.selc = b; b = align16(b + sizeof(unsigned int) * kMaxGrid);
  p.ckey = b; b = align16(b + sizeof(uint64_t) * kCandStage);
  p.cidx = b; b = align16(b + sizeof(int32_t) * kCandStage);
  // K-means++: scan staging (kBlock doubles) and the candidate rows
  const size_t seed_stage = sizeof(double) * kBlock + sizeof(float) * kMaxTrials * size_t(dm);
  if (b < seed_stage) b = seed_stage;
  p.total_sampling = b;
  b = 0;
  p.sums = b; b = align16(b + (sums_reps ? sizeof(double) * size_t(sums_reps) * sums_rstride(k, d) : 0));
  p.cntl = b; b = align16(b + sizeof(int) * size_t(k) * (sums_reps > 1 ? sums_reps : 1));
  p.total_lloyd = b;
  p.total = o + (p.total_sampling > p.total_lloyd ? p.total_sampling : p.total_lloyd);
  return p;
}

__device__ __forceinline__ Lds carve(unsigned char* base, const LdsPlan& p) {
  Lds L;
  L.C = reinterpret_cast<float*>(base + p.C);
  L.act = reinterpret_cast<int*>(base + p.act);
  L.degf = reinterpret_cast<int*>(base + p.degf);
  L.tmpi = reinterpret_cast<int*>(base + p.tmpi);
  L.tmpd = reinterpret_cast<double*>(base + p.tmpd);
  L.misc = reinterpret_cast<int*>(base + p.misc);
  L.misc64 = reinterpret_cast<int64_t*>(base + p.misc64);
  L.miscd = reinterpret_cast<double*>(base + p.miscd);
  L.c64 = reinterpret_cast<double*>(base + p.c64);
  L.B = base + p.B;
  return L;
}

static_assert(kMaxGrid <= kBarrierMaxGroups * kBarrierMaxGroups,
              "the grid barrier's groups must cover the largest grid");

__device__ __forceinline__ void set_err(const SolverArgs& a, int code) {
  atomicCAS(a.err, 0, code);
  __hip_atomic_store(&a.bar->abort.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool sync_grid(const SolverArgs& a) {
  const bool ok = grid_barrier(a.bar, gridDim.x, a.spin_limit);
  if (!ok && threadIdx.x == 0) atomicCAS(a.err, 0, kErrBarrier);
  return ok;
}

// Sum of G per-workgroup partials p[g * stride] (G <= 2 * kBlock), loaded in
// parallel and combined in a fixed order, so every workgroup gets the same bits.
__device__ __forceinline__ double grid_partials_sum(const double* p, int G, int stride,
                                                    double* tmp) {
  const int g0 = 2 * threadIdx.x;
  double v = 0.0;
  if (g0 < G) v = p[static_cast<size_t>(g0) * stride];
  if (g0 + 1 < G) v += p[static_cast<size_t>(g0 + 1) * stride];
  return block_sum_f64<kBlock>(v, tmp);
}

// Rebuild the ascending list of active slots from the flags (whole block):
// a block-wide exclusive scan of the "active" flags gives each slot its place.
__device__ __forceinline__ void rebuild_active(Lds& L, int k) {
  __syncthreads();
  int base = 0;
  for (int j0 = 0; j0 < k; j0 += kBlock) {
    const int j = j0 + threadIdx.x;
    const int f = (j < k && !L.degf[j]) ? 1 : 0;
    int tot = 0;
    const int ex = block_exclusive_scan<kBlock, int>(f, L.tmpi, tot);
    if (f) L.act[base + ex] = j;
    base += tot;
  }
  if (threadIdx.x == 0) L.misc[0] = base;
  __syncthreads();
}

// ---------------------------------------------------------------------------
// 1. Sampling.

__device__ __forceinline__ bool key_in_window(uint64_t key, uint64_t pre, int nbits) {
  return nbits == 0 || (key >> (64 - nbits)) == pre;
}
__device__ __forceinline__ bool pair_le(uint64_t k, int64_t i, uint64_t tk, int64_t ti) {
  return k < tk || (k == tk && i <= ti);
}

// Buffers of one sample slot.  Samples are drawn in batches of a.sbatch
// (they depend only on (seed, t)); slot b holds the b-th sample of a batch.
// Bytes between the code arrays of two slots (16-byte aligned slots, so the
// two codes of a point pair are one aligned 16-bit store).
__host__ __device__ __forceinline__ size_t code_stride(int64_t n) {
  return (static_cast<size_t>(n) + 15) & ~size_t(15);
}

struct SBuf {
  float* P;              // s x d gathered rows (null when rows are not gathered)
  int32_t* idx;          // s sampled indices
  uint8_t* selcode;      // n: key below (1), inside (2), above (0) the window
  uint64_t* cand_key;    // cand_cap
  int32_t* cand_idx;     // cand_cap
  uint32_t* cand_count;  // 1
  uint32_t* wg_lo;       // kMaxGrid
  uint32_t* wg_off;      // kMaxGrid
  uint64_t* thr;         // 2: threshold key, index
};

__device__ __forceinline__ SBuf slot_bufs(const SolverArgs& a, float* Pb, int32_t* idxb, int b) {
  SBuf q;
  q.P = Pb ? Pb + static_cast<size_t>(b) * a.s * a.d : nullptr;
  q.idx = idxb + static_cast<size_t>(b) * a.s;
  q.selcode = a.selcode + static_cast<size_t>(b) * code_stride(a.n);
  q.cand_key = a.cand_key + static_cast<size_t>(b) * a.cand_cap;
  q.cand_idx = a.cand_idx + static_cast<size_t>(b) * a.cand_cap;
  q.cand_count = a.cand_count + b;
  q.wg_lo = a.wg_lo + static_cast<size_t>(b) * kMaxGrid;
  q.wg_off = a.wg_off + static_cast<size_t>(b) * kMaxGrid;
  q.thr = a.thr + 2 * static_cast<size_t>(b);
  return q;
}

// Append (key, index) to this workgroup's candidate buffer in LDS (one LDS
// atomic per wavefront); entries beyond the buffer go straight to the global
// list.  flush_candidates moves the buffer to the global list with a single
// global atomic per workgroup.
__device__ __forceinline__ void append_candidate(const SolverArgs& a, const SBuf& sb, const LdsPlan& pl,
                                                 Lds& L, bool pred, uint64_t key, int64_t i) {
  const unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int leader = __builtin_ctzll(mask);
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(reinterpret_cast<unsigned int*>(&L.misc[4]),
                                       static_cast<unsigned int>(__popcll(mask)));
  base = __shfl(base, leader, kWave);
  if (pred) {
    const unsigned int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
    if (slot < static_cast<unsigned int>(kCandStage)) {
      reinterpret_cast<uint64_t*>(L.B + pl.ckey)[slot] = key;
      reinterpret_cast<int32_t*>(L.B + pl.cidx)[slot] = static_cast<int32_t>(i);
    } else {
      const unsigned int gs = atomicAdd(sb.cand_count, 1u);
      if (gs < static_cast<unsigned int>(a.cand_cap)) {
        sb.cand_key[gs] = key;
        sb.cand_idx[gs] = static_cast<int32_t>(i);
      }
    }
  }
}

__device__ __forceinline__ void flush_candidates(const SolverArgs& a, const SBuf& sb, const LdsPlan& pl,
                                                 Lds& L) {
  __syncthreads();
  const unsigned int cnt = static_cast<unsigned int>(L.misc[4]);
  const unsigned int nl = cnt < static_cast<unsigned int>(kCandStage) ? cnt : kCandStage;
  if (threadIdx.x == 0) L.misc[5] = nl ? static_cast<int>(atomicAdd(sb.cand_count, nl)) : 0;
  __syncthreads();
  const unsigned int gb = static_cast<unsigned int>(L.misc[5]);
  const uint64_t* ck = reinterpret_cast<const uint64_t*>(L.B + pl.ckey);
  const int32_t* ci = reinterpret_cast<const int32_t*>(L.B + pl.cidx);
  for (unsigned int r = threadIdx.x; r < nl; r += kBlock) {
    if (gb + r < static_cast<unsigned int>(a.cand_cap)) {
      sb.cand_key[gb + r] = ck[r];
      sb.cand_idx[gb + r] = ci[r];
    }
  }
  __syncthreads();  // the LDS stage is reused by the next collect pass
}

// Write sampled point i at position pos: index, and its row gathered into P
// (the whole row is loaded into registers first, so its loads overlap).
template <int DM>
__device__ __forceinline__ void emit_point(const SolverArgs& a, const SBuf& sb, int tt, int64_t pos,
                                           int64_t i) {
  if (pos < 0 || pos >= a.s) {  // inconsistent bookkeeping: never write out of bounds
    atomicCAS(a.err, 0, kErrSelect);
    return;
  }
  sb.idx[pos] = static_cast<int32_t>(i);
  if (a.sample_idx_out) a.sample_idx_out[static_cast<size_t>(tt) * a.s + pos] = static_cast<int32_t>(i);
  if (a.do_gather) {
    const int d = a.d;
    float x[DM];
    if (a.x_bf16)
      load_row_bf16<DM>(static_cast<const uint16_t*>(a.X) + static_cast<size_t>(i) * d, d, x);
    else
      load_row_f32<DM>(static_cast<const float*>(a.X) + static_cast<size_t>(i) * d, d, x);
    float* dst = sb.P + static_cast<size_t>(pos) * d;
    if ((d & 3) == 0) {
#pragma unroll
      for (int q = 0; q < DM / 4; ++q)
        if (4 * q < d)
          reinterpret_cast<float4*>(dst)[q] = make_float4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
    } else {
#pragma unroll
      for (int t = 0; t < DM; ++t)
        if (t < d) dst[t] = x[t];
    }
  }
}

// One workgroup: the need-th smallest (key, index) pair among the m collected
// candidates of a sample (exact MSB radix select over 8-bit digits), then the
// output offset of every workgroup.  Every key below the window is selected,
// so workgroup g emits wg_lo[g] plus its candidates that do not exceed the
// threshold pair.
__device__ __forceinline__ bool select_threshold(const SolverArgs& a, const SBuf& sb, const LdsPlan& pl,
                                                 Lds& L, int64_t below, int64_t m, int64_t ppw,
                                                 int G_ = 0) {
  const int tid = threadIdx.x;
  const int G = G_ > 0 ? G_ : static_cast<int>(gridDim.x);  // workgroups that collected
  unsigned int* hist = reinterpret_cast<unsigned int*>(L.B + pl.hist);
  unsigned int* selc = reinterpret_cast<unsigned int*>(L.B + pl.selc);
  const int64_t need = a.s - below;
  if (m > a.cand_cap || need < 1 || need > m) {
    if (tid == 0) set_err(a, kErrSelect);
    return false;
  }
  // candidates read from LDS when they fit the stage, else from global memory
  const bool staged = m <= kCandStage;
  const uint64_t* ckey = staged ? reinterpret_cast<const uint64_t*>(L.B + pl.ckey) : sb.cand_key;
  const int32_t* cidx = staged ? reinterpret_cast<const int32_t*>(L.B + pl.cidx) : sb.cand_idx;
  if (staged) {
    uint64_t* sk = reinterpret_cast<uint64_t*>(L.B + pl.ckey);
    int32_t* si = reinterpret_cast<int32_t*>(L.B + pl.cidx);
#pragma unroll 4
    for (int64_t r = tid; r < m; r += kBlock) {
      sk[r] = sb.cand_key[r];
      si[r] = sb.cand_idx[r];
    }
    __syncthreads();
  }
  uint64_t pre = 0;
  int nbits = 0;
  int64_t rem = need;  // rank inside the current prefix class
  int64_t cnt = m;
  while (cnt > 1 && nbits < 64) {
    for (int b = tid; b < kHistBins; b += kBlock) hist[b] = 0u;
    __syncthreads();
    const int shift = 56 - nbits;
    for (int64_t r = tid; r < m; r += kBlock) {
      const uint64_t key = ckey[r];
      if (key_in_window(key, pre, nbits)) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (tid == 0) L.misc[1] = -1;
    const int hb = (tid < kHistBins) ? static_cast<int>(hist[tid]) : 0;
    int tot = 0;
    const int ex = block_exclusive_scan<kBlock, int>(hb, L.tmpi, tot);
    if (tid < kHistBins && ex < rem && rem <= static_cast<int64_t>(ex) + hb) {
      L.misc[1] = tid;
      L.misc64[0] = ex;
      L.misc64[1] = hb;
    }
    __syncthreads();
    if (L.misc[1] < 0) {
      if (tid == 0) set_err(a, kErrSelect);
      return false;
    }
    rem -= L.misc64[0];
    pre = (pre << 8) | static_cast<uint64_t>(L.misc[1]);
    nbits += 8;
    cnt = L.misc64[1];
    __syncthreads();
  }
  // the threshold is the rem-th smallest index among the candidates whose
  // key has prefix `pre` (one candidate, or equal 64-bit keys)
  if (tid == 0) L.misc64[2] = -1;
  __syncthreads();
  for (int64_t r = tid; r < m; r += kBlock) {
    const uint64_t key = ckey[r];
    if (!key_in_window(key, pre, nbits)) continue;
    const int32_t idx = cidx[r];
    int64_t rank = 0;
    if (cnt > 1) {
      for (int64_t r2 = 0; r2 < m; ++r2)
        if (key_in_window(ckey[r2], pre, nbits) && cidx[r2] < idx) ++rank;
    }
    if (rank == rem - 1) {
      L.misc64[2] = idx;
      L.misc64[3] = static_cast<int64_t>(key);
    }
  }
  for (int gg = tid; gg < G; gg += kBlock) selc[gg] = 0u;
  __syncthreads();
  if (L.misc64[2] < 0) {
    if (tid == 0) set_err(a, kErrSelect);
    return false;
  }
  const uint64_t tk = static_cast<uint64_t>(L.misc64[3]);
  const int64_t ti = L.misc64[2];
  for (int64_t r = tid; r < m; r += kBlock) {
    const uint64_t key = ckey[r];
    const int64_t idx = cidx[r];
    if (pair_le(key, idx, tk, ti)) atomicAdd(&selc[static_cast<int>((idx >> 1) / ppw)], 1u);
  }
  __syncthreads();
  // output offset of every workgroup: exclusive scan of (selected candidates
  // + keys below the window), two workgroups per thread
  for (int gg = tid; gg < G; gg += kBlock) selc[gg] += sb.wg_lo[gg];
  __syncthreads();
  const int g0 = 2 * tid;
  const int v0 = (g0 < G) ? static_cast<int>(selc[g0]) : 0;
  const int v1 = (g0 + 1 < G) ? static_cast<int>(selc[g0 + 1]) : 0;
  int total = 0;
  const int ex = block_exclusive_scan<kBlock, int>(v0 + v1, L.tmpi, total);
  if (g0 < G) sb.wg_off[g0] = static_cast<uint32_t>(ex);
  if (g0 + 1 < G) sb.wg_off[g0 + 1] = static_cast<uint32_t>(ex + v0);
  if (tid == 0) {
    sb.thr[0] = tk;
    sb.thr[1] = static_cast<uint64_t>(ti);
    if (total != a.s) set_err(a, kErrSelect);
    L.misc[2] = (total == a.s) ? 1 : 0;
  }
  __syncthreads();
  return L.misc[2] != 0;
}

// Collect pass over this workgroup's point pairs: count the keys below
// [lo, hi] (inclusive) into wg_lo[g], append the keys inside to the candidate
// list, and record per point whether its key is below (1), inside (2) or
// above (0) the window.  Each thread takes a contiguous run of pairs.
__device__ __forceinline__ void collect_pass(const SolverArgs& a, const SBuf& sb, const LdsPlan& pl,
                                             Lds& L, uint32_t t, int64_t p0, int64_t p1, uint64_t lo,
                                             uint64_t hi, int g_ = -1) {
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const int64_t per = (p1 - p0 + kBlock - 1) / kBlock;
  const int64_t q0 = p0 + tid * per;
  const int64_t q1 = imin64(p1, q0 + per);
  if (tid == 0) L.misc[4] = 0;
  __syncthreads();
  int lo_count = 0;
  for (int64_t step = 0; step < per; ++step) {  // uniform trip count for the ballots
    const int64_t p = q0 + step;
    const bool v0 = p < q1;
    const bool v1 = v0 && (2 * p + 1 < n);
    uint64_t k0 = 0, k1 = 0;
    if (v0) sample_key_pair(a.seed, t, static_cast<uint64_t>(p), k0, k1);
    const int c0 = !v0 ? 0 : (k0 < lo ? 1 : (k0 <= hi ? 2 : 0));
    const int c1 = !v1 ? 0 : (k1 < lo ? 1 : (k1 <= hi ? 2 : 0));
    lo_count += (c0 == 1) + (c1 == 1);
    if (v1) {
      reinterpret_cast<uint16_t*>(sb.selcode)[p] = static_cast<uint16_t>(c0 | (c1 << 8));
    } else if (v0) {
      sb.selcode[2 * p] = static_cast<uint8_t>(c0);
    }
    append_candidate(a, sb, pl, L, c0 == 2, k0, 2 * p);
    append_candidate(a, sb, pl, L, c1 == 2, k1, 2 * p + 1);
  }
  flush_candidates(a, sb, pl, L);
  const int wg_lo = block_sum_i32<kBlock>(lo_count, L.tmpi);
  if (tid == 0) sb.wg_lo[g_ >= 0 ? g_ : static_cast<int>(blockIdx.x)] = static_cast<uint32_t>(wg_lo);
}

// Number of keys below the window over all workgroups (fixed order).
__device__ __forceinline__ int64_t keys_below(const SBuf& sb, Lds& L, int G_ = 0) {
  const int G = G_ > 0 ? G_ : static_cast<int>(gridDim.x);
  const int g0 = 2 * threadIdx.x;
  int v = 0;
  if (g0 < G) v += static_cast<int>(sb.wg_lo[g0]);
  if (g0 + 1 < G) v += static_cast<int>(sb.wg_lo[g0 + 1]);
  return block_sum_i32<kBlock>(v, L.tmpi);
}

// Exact selection for a sample whose predicted window missed the threshold
// (rare): MSB histogram passes over all keys narrow an exact window, then a
// collect pass and the selection by workgroup 0.  All workgroups call it.
__device__ __forceinline__ bool exact_select(const SolverArgs& a, const SBuf& sb, const LdsPlan& pl,
                                             Lds& L, uint32_t t, int64_t p0, int64_t p1, int64_t ppw,
                                             int64_t& hist_passes) {
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int64_t n = a.n;
  unsigned int* hist = reinterpret_cast<unsigned int*>(L.B + pl.hist);
  uint64_t pre = 0;
  int nbits = 0;
  int64_t blw = 0;
  int64_t mm = n;
  while (mm > a.cand_cap) {
    if (nbits >= 64) {
      if (tid == 0) set_err(a, kErrSelect);
      return false;
    }
    unsigned int* Hcur = a.hist + (hist_passes % 3) * kHistBins;
    unsigned int* Hnext = a.hist + ((hist_passes + 1) % 3) * kHistBins;
    for (int b = tid; b < kHistBins; b += kBlock) hist[b] = 0u;
    if (g == 0)
      for (int b = tid; b < kHistBins; b += kBlock) Hnext[b] = 0u;
    __syncthreads();
    const int shift = 56 - nbits;
    for (int64_t p = p0 + tid; p < p1; p += kBlock) {
      uint64_t k0, k1;
      sample_key_pair(a.seed, t, static_cast<uint64_t>(p), k0, k1);
      if (key_in_window(k0, pre, nbits)) atomicAdd(&hist[(k0 >> shift) & 255u], 1u);
      if (2 * p + 1 < n && key_in_window(k1, pre, nbits))
        atomicAdd(&hist[(k1 >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int b = tid; b < kHistBins; b += kBlock) {
      const unsigned int v2 = hist[b];
      if (v2) atomicAdd(&Hcur[b], v2);
    }
    if (!sync_grid(a)) return false;
    const int64_t need = a.s - blw;
    if (tid == 0) L.misc[1] = -1;
    const int hb = (tid < kHistBins) ? static_cast<int>(Hcur[tid]) : 0;
    int tot = 0;
    const int ex = block_exclusive_scan<kBlock, int>(hb, L.tmpi, tot);
    if (tid < kHistBins && ex < need && need <= static_cast<int64_t>(ex) + hb) {
      L.misc[1] = tid;
      L.misc64[0] = ex;
      L.misc64[1] = hb;
    }
    __syncthreads();
    if (L.misc[1] < 0) {
      if (tid == 0) set_err(a, kErrSelect);
      return false;
    }
    blw += L.misc64[0];
    pre = (pre << 8) | static_cast<uint64_t>(L.misc[1]);
    nbits += 8;
    mm = L.misc64[1];
    ++hist_passes;
    __syncthreads();
  }
  const uint64_t lo = nbits ? pre << (64 - nbits) : 0ull;
  const uint64_t hi = nbits ? lo | (~0ull >> nbits) : ~0ull;
  collect_pass(a, sb, pl, L, t, p0, p1, lo, hi);
  if (!sync_grid(a)) return false;
  if (g == 0) {
    const int64_t got = __hip_atomic_load(sb.cand_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (got != mm) {
      if (tid == 0) set_err(a, kErrSelect);
      return false;
    }
    if (!select_threshold(a, sb, pl, L, blw, mm, ppw)) return false;
    if (tid == 0) __hip_atomic_store(sb.cand_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return sync_grid(a);
}

// Emit sample slot sb in index order and gather its rows: each thread takes a
// contiguous run of pairs, counts its selected points from the codes (a key
// inside the window is recomputed and compared with the threshold pair), and
// writes them at its offset from one block-wide scan.  No barrier.
template <int DM>
__device__ __forceinline__ void emit_sample(const SolverArgs& a, const SBuf& sb, Lds& L, uint32_t t,
                                            int tt, int64_t p0, int64_t p1, int g_ = -1) {
  const int tid = threadIdx.x;
  const int g = g_ >= 0 ? g_ : static_cast<int>(blockIdx.x);
  const int64_t n = a.n;
  const uint64_t tk = sb.thr[0];
  const int64_t ti = static_cast<int64_t>(sb.thr[1]);
  const int64_t per = (p1 - p0 + kBlock - 1) / kBlock;
  const int64_t q0 = p0 + tid * per;
  const int64_t q1 = imin64(p1, q0 + per);
  auto selected = [&](int64_t i, int code) -> bool {
    if (code != 2) return code == 1;
    uint64_t ke, ko;
    sample_key_pair(a.seed, t, static_cast<uint64_t>(i >> 1), ke, ko);
    return pair_le((i & 1) ? ko : ke, i, tk, ti);
  };
  const uint16_t* code2 = reinterpret_cast<const uint16_t*>(sb.selcode);
  auto codes_of = [&](int64_t p) -> int {  // both codes of pair p (odd n: last pair has one)
    return (2 * p + 1 < n) ? static_cast<int>(code2[p]) : static_cast<int>(sb.selcode[2 * p]);
  };
  // selection bits of this thread's points (up to 128), decided once
  uint64_t bits_lo = 0, bits_hi = 0;
  const bool fits = per <= 64;
  int mine = 0;
  if (fits) {
#pragma unroll 4
    for (int64_t p = q0; p < q1; ++p) {
      const int c = codes_of(p);
      const int j = static_cast<int>(2 * (p - q0));
      const uint64_t b = (selected(2 * p, c & 255) ? 1ull : 0ull) |
                         ((2 * p + 1 < n && selected(2 * p + 1, c >> 8)) ? 2ull : 0ull);
      if (j < 64) bits_lo |= b << j;
      else bits_hi |= b << (j - 64);
    }
    mine = __popcll(bits_lo) + __popcll(bits_hi);
  } else {
    for (int64_t p = q0; p < q1; ++p) {
      const int c = codes_of(p);
      mine += selected(2 * p, c & 255) ? 1 : 0;
      if (2 * p + 1 < n) mine += selected(2 * p + 1, c >> 8) ? 1 : 0;
    }
  }
  int total = 0;
  const int excl = block_exclusive_scan<kBlock, int>(mine, L.tmpi, total);
  int64_t pos = static_cast<int64_t>(sb.wg_off[g]) + excl;
  if (fits) {
    while (bits_lo) {
      const int j = __builtin_ctzll(bits_lo);
      bits_lo &= bits_lo - 1;
      emit_point<DM>(a, sb, tt, pos++, 2 * q0 + j);
    }
    while (bits_hi) {
      const int j = __builtin_ctzll(bits_hi);
      bits_hi &= bits_hi - 1;
      emit_point<DM>(a, sb, tt, pos++, 2 * q0 + 64 + j);
    }
  } else {
    for (int64_t p = q0; p < q1; ++p) {
      const int c = codes_of(p);
      if (selected(2 * p, c & 255)) emit_point<DM>(a, sb, tt, pos++, 2 * p);
      if (2 * p + 1 < n && selected(2 * p + 1, c >> 8)) emit_point<DM>(a, sb, tt, pos++, 2 * p + 1);
    }
  }
}

// Samples tt0 .. tt0 + nb - 1 of this call into slots 0 .. nb - 1: the s
// smallest (key, index) pairs of each, emitted in index order with their rows
// gathered.  The key window [win_lo, win_hi] predicted from the order
// statistics of uniform keys (the s-th smallest of n lies within 8 standard
// deviations of s/n of the key range, plus a margin) almost always holds the
// threshold, so one collect pass per sample suffices; a miss takes the exact
// histogram path for that sample.  One barrier after collecting all samples,
// the thresholds selected in parallel (workgroup g takes samples g, g + G,
// ...), one barrier, then every sample emitted and one barrier: three grid
// barriers per batch.
template <int DM>
__device__ __forceinline__ bool sample_batch(const SolverArgs& a, const LdsPlan& pl, Lds& L, float* Pb,
                                             int32_t* idxb, int tt0, int nb, int64_t& hist_passes) {
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int G = gridDim.x;
  const int64_t npairs = (a.n + 1) >> 1;
  const int64_t ppw = (npairs + G - 1) / G;
  const int64_t p0 = imin64(npairs, static_cast<int64_t>(g) * ppw);
  const int64_t p1 = imin64(npairs, p0 + ppw);

  const uint64_t s0 = wall_clock64();
  for (int b = 0; b < nb; ++b)
    collect_pass(a, slot_bufs(a, Pb, idxb, b), pl, L, static_cast<uint32_t>(a.t0 + tt0 + b), p0, p1,
                 a.win_lo, a.win_hi);
  const uint64_t s1 = wall_clock64();
  if (!sync_grid(a)) return false;
  const uint64_t s2 = wall_clock64();
  if (g == 0 && tid == 0) {
    a.counters[kCntTicksCollect] += static_cast<int64_t>(s1 - s0);
    a.counters[kCntTicksCollectWait] += static_cast<int64_t>(s2 - s1);
  }
  for (int b = g; b < nb; b += G) {
    const SBuf sb = slot_bufs(a, Pb, idxb, b);
    const int64_t below = keys_below(sb, L);
    const int64_t m = __hip_atomic_load(sb.cand_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool hit = m <= a.cand_cap && below < a.s && a.s <= below + m;
    if (hit && !select_threshold(a, sb, pl, L, below, m, ppw)) return false;
    if (tid == 0) {
      a.smiss[b] = hit ? 0 : 1;
      __hip_atomic_store(sb.cand_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
  const uint64_t s3 = wall_clock64();
  if (!sync_grid(a)) return false;
  if (g == 0 && tid == 0) a.counters[kCntTicksSelect] += static_cast<int64_t>(s3 - s2);
  for (int b = 0; b < nb; ++b) {
    if (__hip_atomic_load(&a.smiss[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &&
        !exact_select(a, slot_bufs(a, Pb, idxb, b), pl, L, static_cast<uint32_t>(a.t0 + tt0 + b), p0,
                      p1, ppw, hist_passes))
      return false;
  }
  const uint64_t s4 = wall_clock64();
  for (int b = 0; b < nb; ++b)
    emit_sample<DM>(a, slot_bufs(a, Pb, idxb, b), L, static_cast<uint32_t>(a.t0 + tt0 + b), tt0 + b,
                    p0, p1);
  if (g == 0 && tid == 0) a.counters[kCntTicksEmit] += static_cast<int64_t>(wall_clock64() - s4);
  return sync_grid(a);
}

// Sample rows a thread keeps in registers across Lloyd rounds (rows
// r0 + tid + q * kBlock), used when the workgroup's chunk fits: every grid
// barrier ends with an acquire fence that drops the L2's copy of the sample,
// so re-reading it would cost a memory round trip per round.
template <int DM>
struct RowCache {
  static constexpr int kRows = DM <= 16 ? 1 : 0;
  float x[kRows > 0 ? kRows : 1][DM];
};

// ---------------------------------------------------------------------------
// 2. K-means++ reseeding of the degenerate slots.
//
// The D^2 weights are FP64 direct differences of the FP32 values, formed in
// dimension order with FMAs, so they are the same numbers the FP64 definition
// gives.  The running sum that inverts a draw is taken over workgroup chunks
// (a fixed-order scan of per-workgroup sums) and then inside the owning chunk.

// FP64 squared distances of the sample row at p to `trials` candidate rows
// (LDS, DM wide, zero padded), each accumulated with FMAs in dimension order
// as dist2_f64_row does on a loaded row, so the values are the same; the row
// is read 16 coordinates at a time instead of being held in registers.
template <int DM>
__device__ __forceinline__ void dist2_f64_candidates(const float* __restrict__ p, int d,
                                                     const float* __restrict__ cand, int trials,
                                                     double (&out)[kMaxTrials]) {
#pragma unroll
  for (int l = 0; l < kMaxTrials; ++l) out[l] = 0.0;
#pragma unroll
  for (int t0 = 0; t0 < DM; t0 += 16) {
    float xc[16];
    if ((d & 3) == 0) {
#pragma unroll
      for (int u = 0; u < 16; u += 4) {
        if (t0 + u < d) {
          const float4 v = *reinterpret_cast<const float4*>(p + t0 + u);
          xc[u] = v.x;
          xc[u + 1] = v.y;
          xc[u + 2] = v.z;
          xc[u + 3] = v.w;
        } else {
          xc[u] = xc[u + 1] = xc[u + 2] = xc[u + 3] = 0.f;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < 16; ++u) xc[u] = (t0 + u < d) ? p[t0 + u] : 0.f;
    }
#pragma unroll
    for (int l = 0; l < kMaxTrials; ++l) {
      if (l < trials) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          if (t0 + u < DM) {  // DM need not be a multiple of 16 (e.g. 72)
            const double e = static_cast<double>(xc[u]) - static_cast<double>(cand[l * DM + t0 + u]);
            out[l] = __builtin_fma(e, e, out[l]);
          }
        }
      }
    }
  }
}

// Smallest FP64 squared distance of the sample row at p to the active slots
// act[0 .. na-1] of C (LDS, DM wide): the same dimension-order FMA chain as
// dist2_f64_row for every slot, run for kMinBatch slots at once over 8
// coordinates at a time, so the row is streamed rather than held and the
// chains are independent.
constexpr int kMinBatch = 8;
template <int DM>
__device__ __forceinline__ double min_dist2_f64_stream(const float* __restrict__ p, int d,
                                                       const float* __restrict__ C,
                                                       const int* __restrict__ act, int na) {
  double best = __builtin_inf();
  for (int a0 = 0; a0 < na; a0 += kMinBatch) {
    double acc[kMinBatch];
    int off[kMinBatch];
#pragma unroll
    for (int u = 0; u < kMinBatch; ++u) {
      acc[u] = 0.0;
      off[u] = act[a0 + u < na ? a0 + u : na - 1] * DM;
    }
#pragma unroll 1
    for (int t0 = 0; t0 < DM; t0 += 8) {
      float xc[8];
      if ((d & 3) == 0) {
#pragma unroll
        for (int u = 0; u < 8; u += 4) {
          if (t0 + u < d) {
            const float4 v = *reinterpret_cast<const float4*>(p + t0 + u);
            xc[u] = v.x;
            xc[u + 1] = v.y;
            xc[u + 2] = v.z;
            xc[u + 3] = v.w;
          } else {
            xc[u] = xc[u + 1] = xc[u + 2] = xc[u + 3] = 0.f;
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) xc[u] = (t0 + u < d) ? p[t0 + u] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kMinBatch; ++u) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          if (t0 + v < DM) {  // DM is a multiple of 4, not always of 8 (72 is)
            const double e = static_cast<double>(xc[v]) - static_cast<double>(C[off[u] + t0 + v]);
            acc[u] = __builtin_fma(e, e, acc[u]);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kMinBatch; ++u)
      if (a0 + u < na && acc[u] < best) best = acc[u];
  }
  return best;
}

constexpr int kLocRows = 4;

// Workgroup minimum (maximum) of `value` over the threads whose `pred` holds,
// for values that increase with the thread index: in each wavefront the
// lowest (highest) such lane holds the wavefront's extreme and alone updates
// *dst (LDS), so the word takes one atomic per wavefront instead of one per
// thread.  Called by every lane of the wavefront.
__device__ __forceinline__ void wave_min_first(bool pred, int value, int* dst) {
  const unsigned long long m = __ballot(pred);
  if (m && static_cast<int>(threadIdx.x & (kWave - 1)) == __builtin_ctzll(m)) atomicMin(dst, value);
}
__device__ __forceinline__ void wave_max_last(bool pred, int value, int* dst) {
  const unsigned long long m = __ballot(pred);
  if (m && static_cast<int>(threadIdx.x & (kWave - 1)) == 63 - __builtin_clzll(m)) atomicMax(dst, value);
}

// A D^2 draw within this distance of a row boundary may fall on the other
// side of it when W and the running sum are added one row at a time in row
// order: for nonnegative terms, any order of summation is within about
// s units of rounding of W of the exact sums, the two targets u W differ by
// as much again, and the row-order sums likewise (4 s plus a margin).
__device__ __forceinline__ double draw_tol(int64_t s, double W) {
  return (4.0 * static_cast<double>(s) + 64.0) * 0x1p-53 * W;
}

// Lane j's double, read into every lane (j uniform).
__device__ __forceinline__ double lane_f64(double v, int j) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b), j));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), j));
  return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// The D^2 draw of K-means++ (Sec. 2) with W and the running sum added one row
// at a time in row order: the first row whose running sum exceeds unit * W;
// when rounding leaves none, the last row with weight; -1 when every weight is
// zero.  Run by one whole wavefront (every lane gets the result): rows are
// loaded 64 at a time and added lane by lane.  Used for the rare draws that
// the chunked sums leave within draw_tol of a boundary.
__device__ int64_t seq_draw(const double* __restrict__ w, int64_t s, double unit) {
  const int lane = threadIdx.x & (kWave - 1);
  double W = 0.0;
  for (int64_t b = 0; b < s; b += kWave) {
    const double v = (b + lane < s) ? w[b + lane] : 0.0;  // zeros past s add nothing
#pragma unroll 8
    for (int j = 0; j < kWave; ++j) W += lane_f64(v, j);
  }
  const double target = unit * W;
  double run = 0.0;
  for (int64_t b = 0; b < s; b += kWave) {
    const double v = (b + lane < s) ? w[b + lane] : 0.0;
    int hit = -1;
#pragma unroll 8
    for (int j = 0; j < kWave; ++j) {
      run += lane_f64(v, j);
      if (hit < 0 && run > target) hit = j;
    }
    if (hit >= 0) return b + hit;  // a padding zero never first exceeds the target
  }
  for (int64_t b = ((s - 1) / kWave) * kWave; b >= 0; b -= kWave) {
    const double v = (b + lane < s) ? w[b + lane] : 0.0;
    const unsigned long long m = __ballot(v > 0.0);
    if (m) return b + 63 - __builtin_clzll(m);
  }
  return -1;
}

// The row of chunk [o0, o1) whose running weight sum (from `base`, rows in
// index order) first exceeds `target`; every workgroup calls it with the same
// arguments and gets the same row.  Thread tid holds the weights of its run of
// rpt consecutive rows (when rpt <= kLocRows, loaded by the caller), one
// block-wide scan orders the runs, and the thread whose run holds the target
// walks it.  A target beyond the chunk's total (rounding) takes the chunk's
// last row with weight.  Returns the row and sets *near when the target lies
// within tol of the row's boundaries.  Longer runs are read from memory.
__device__ __forceinline__ void chunk_run(int64_t o0, int64_t o1, int64_t* i0, int* nr) {
  const int64_t rpt = (o1 - o0 + kBlock - 1) / kBlock;
  const int64_t a = o0 + threadIdx.x * rpt < o1 ? o0 + threadIdx.x * rpt : o1;
  const int64_t b = a + rpt < o1 ? a + rpt : o1;
  *i0 = a;
  *nr = static_cast<int>(b - a);
}

__device__ __forceinline__ void load_run(const double* __restrict__ w, int64_t o0, int64_t o1,
                                         double (&wv)[kLocRows]) {
  int64_t i0;
  int nr;
  chunk_run(o0, o1, &i0, &nr);
#pragma unroll
  for (int q = 0; q < kLocRows; ++q) wv[q] = q < nr ? w[i0 + q] : 0.0;
}

// REG: the run's weights are wv (rpt <= kLocRows); otherwise they are read
// from w.
template <bool REG>
__device__ __forceinline__ int64_t locate_in_chunk(const double (&wv)[kLocRows], const double* __restrict__ w,
                                                   int64_t o0, int64_t o1, double base, double target,
                                                   double tol, Lds& L, bool* near) {
  const int tid = threadIdx.x;
  int64_t i0;
  int nr;
  chunk_run(o0, o1, &i0, &nr);
  auto wt = [&](int q) { return REG ? wv[q < kLocRows ? q : 0] : w[i0 + q]; };
  const int nq = REG ? kLocRows : nr;
  double local = 0.0;
#pragma unroll
  for (int q = 0; q < nq; ++q)
    if (q < nr) local += wt(q);
  double tot = 0.0;
  const double incl = block_inclusive_scan_f64<kBlock>(local, L.tmpd, tot);
  double* incl_l = reinterpret_cast<double*>(L.B);  // kBlock doubles
  incl_l[tid] = incl;
  if (tid == 0) {
    L.misc[2] = 0x7fffffff;
    L.misc[6] = -1;
  }
  __syncthreads();
  const double v0 = base + (tid > 0 ? incl_l[tid - 1] : 0.0);
  wave_min_first(nr > 0 && v0 + local > target, tid, &L.misc[2]);
  int last = -1;  // last row with weight, for a target beyond the chunk's sum
#pragma unroll
  for (int q = 0; q < nq; ++q)
    if (q < nr && wt(q) > 0.0) last = q;
  // runs start at increasing rows, so the last weighted row is the highest lane's
  wave_max_last(last >= 0, static_cast<int>(i0 - o0) + last, &L.misc[6]);
  __syncthreads();
  if (tid == L.misc[2]) {
    double run = v0;
    int64_t pick = i0 + nr - 1;
    int nb = 0;
    bool found = false;
#pragma unroll
    for (int q = 0; q < nq; ++q) {
      if (q < nr && !found) {
        const double prev = run;
        run += wt(q);
        if (run > target) {
          pick = i0 + q;
          nb = ((run - target) < tol || (target - prev) < tol) ? 1 : 0;
          found = true;
        }
      }
    }
    L.misc64[1] = pick;
    L.misc64[3] = nb;
  }
  __syncthreads();
  int64_t pick;
  if (L.misc[2] != 0x7fffffff) {
    pick = L.misc64[1];
    *near = L.misc64[3] != 0;
  } else {
    pick = L.misc[6] >= 0 ? o0 + L.misc[6] : -1;
    *near = true;
  }
  __syncthreads();
  return pick;
}

// LEAN (the reseeding kernel): the D^2 pass streams the rows over batches of
// slots, and every workgroup locates the draws itself (no barrier); the
// persistent solver keeps the owning workgroup's search and a barrier, which
// need fewer registers there.
template <int DM, bool LEAN>
__device__ __forceinline__ bool reseed_phase(const SolverArgs& a, Lds& L, uint32_t t, int64_t r0, int64_t r1,
                             bool cached, const RowCache<DM>& rc, int64_t& nd, int64_t& nres) {
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int G = gridDim.x;
  const int d = a.d;
  const int k = a.k;
  const int64_t s = a.s;
  const int trials = a.trials;
  uint64_t q = 0;
  double* tgt = L.miscd + 4;                 // per-trial target
  double* basev = L.miscd + 4 + kMaxTrials;  // per-trial chunk base
  int* owner = L.tmpi + 16;                  // per-trial owning workgroup (tmpi has 32)
  double* incl_l = reinterpret_cast<double*>(L.B);                            // kBlock doubles
  float* cand_rows = reinterpret_cast<float*>(L.B + sizeof(double) * kBlock);  // trials x DM
  const int64_t tiles = (r1 - r0 + kBlock - 1) / kBlock;
  // with cached rows the chunk is a single tile and the weight stays in a register
  double w_reg = 0.0;
  auto row = [&](int64_t tile, float (&x)[DM]) {
    if (cached) {
#pragma unroll
      for (int tdim = 0; tdim < DM; ++tdim) x[tdim] = rc.x[0][tdim];
    } else {
      load_row_f32<DM>(a.P + static_cast<size_t>(r0 + tile * kBlock + tid) * d, d, x);
    }
  };
  auto get_w = [&](int64_t tile, int64_t i) { return cached ? w_reg : a.w[i]; };
  // the weights also go to a.w in cached mode: a draw's target may lie in
  // another workgroup's chunk, and a draw near a boundary reads them all
  auto set_w = [&](int64_t i, double v) {
    if (cached) w_reg = v;
    a.w[i] = v;
  };

  // phase ticks of workgroup 0, kept in registers and added to the counters
  // once at the end
  uint64_t tk = wall_clock64();
  uint64_t ticks[4] = {0, 0, 0, 0};
  auto tick = [&](int c) {
    if (!LEAN) return;
    const uint64_t now = wall_clock64();
    ticks[c - kCntTicksSeedInit] += now - tk;
    tk = now;
  };
  if (L.misc[0] > 0) {
    const int na = L.misc[0];
    double part = 0.0;
    for (int64_t tile = 0; tile < tiles; ++tile) {
      const int64_t i = r0 + tile * kBlock + tid;
      if (i >= r1) continue;
      double best = __builtin_inf();
      if (cached || !LEAN) {
        float x[DM];
        row(tile, x);
        for (int aa = 0; aa < na; ++aa) {
          const double dd = dist2_f64_row<DM>(x, L.C + L.act[aa] * DM);
          if (dd < best) best = dd;
        }
      } else {
        best = min_dist2_f64_stream<DM>(a.P + static_cast<size_t>(i) * d, d, L.C, L.act, na);
      }
      set_w(i, best);
      part += best;
    }
    const double ws = block_sum_f64<kBlock>(part, L.tmpd);
    if (tid == 0) a.wsum[g] = ws;
    nd += s * na;
    if (!sync_grid(a)) return false;
    tick(kCntTicksSeedInit);
  }

  for (int j = 0; j < k; ++j) {
    if (!L.degf[j]) continue;
    const int na = L.misc[0];
    int64_t pick = -1;
    int picked = -1;  // which candidate won, when the potentials were computed
    if (na == 0) {
      pick = static_cast<int64_t>(below_from_word(seed_draw(a.seed, t, q), static_cast<uint64_t>(s)));
      ++q;
    } else {
      // W and, per draw, the chunk holding the target: inclusive scan of the
      // per-workgroup weight sums (two chunks per thread, fixed order); chunk g
      // starts at E_g, the scan value before it
      {
        const int g0 = 2 * tid;
        const double w0 = (g0 < G) ? a.wsum[g0] : 0.0;
        const double w1 = (g0 + 1 < G) ? a.wsum[g0 + 1] : 0.0;
        double tot = 0.0;
        const double incl = block_inclusive_scan_f64<kBlock>(w0 + w1, L.tmpd, tot);
        incl_l[tid] = incl;
        if (tid < kMaxTrials) { owner[tid] = 0x7fffffff; L.tmpi[24 + tid] = -1; }
        __syncthreads();
        const double e0 = tid > 0 ? incl_l[tid - 1] : 0.0;
        const double e1 = e0 + w0;
        for (int l = 0; l < trials; ++l) {
          const double target = unit_from_word(seed_draw(a.seed, t, q + l)) * tot;
          // first chunk whose end passes the target, and the last chunk with
          // weight (thread tid holds chunks 2 tid and 2 tid + 1)
          const bool h0 = g0 < G && e0 + w0 > target;
          const bool h1 = g0 + 1 < G && e1 + w1 > target;
          wave_min_first(h0 || h1, h0 ? g0 : g0 + 1, &owner[l]);
          const bool p1 = g0 + 1 < G && w1 > 0.0;
          const bool p0 = g0 < G && w0 > 0.0;
          wave_max_last(p0 || p1, p1 ? g0 + 1 : g0, &L.tmpi[24 + l]);
          if (tid == 0) tgt[l] = target;
        }
        __syncthreads();
        if (tid == 0) {
          for (int l = 0; l < trials; ++l)
            if (owner[l] == 0x7fffffff) owner[l] = L.tmpi[24 + l];  // rounding fallback
        }
        __syncthreads();
        for (int l = 0; l < trials; ++l) {
          if (g0 == owner[l]) basev[l] = e0;
          if (g0 + 1 == owner[l]) basev[l] = e1;
        }
        if (tid == 0) L.miscd[0] = tot;
        __syncthreads();
      }
      const double W = L.miscd[0];
      if (W == 0.0) break;  // every remaining D^2 is zero: leave the slots degenerate
      q += trials;
      int64_t cands[kMaxTrials];
      bool valid = true;
      if constexpr (LEAN) {
        // every workgroup locates each draw in the chunk that holds it (the
        // weights of the last update are visible since its barrier); the next
        // draw's weights load while one is located
        const int64_t rpw = (s + G - 1) / G;
        const bool reg = (rpw + kBlock - 1) / kBlock <= kLocRows;
        auto chunk_of = [&](int l, int64_t* o0, int64_t* o1) {
          *o0 = imin64(s, static_cast<int64_t>(owner[l]) * rpw);
          *o1 = imin64(s, *o0 + rpw);
        };
        double wv[kLocRows], wn[kLocRows];
        {
          int64_t o0, o1;
          chunk_of(0, &o0, &o1);
          if (reg) load_run(a.w, o0, o1, wv);
        }
        int64_t* cand_l = L.misc64 + 4;  // per-draw candidate rows
#pragma unroll 1
        for (int l = 0; l < trials; ++l) {
          int64_t o0, o1;
          if (reg && l + 1 < trials) {
            chunk_of(l + 1, &o0, &o1);
            load_run(a.w, o0, o1, wn);
          }
          chunk_of(l, &o0, &o1);
          bool near = false;
          const double tol = draw_tol(s, W);
          const int64_t c = reg ? locate_in_chunk<true>(wv, a.w, o0, o1, basev[l], tgt[l], tol, L, &near)
                                : locate_in_chunk<false>(wv, a.w, o0, o1, basev[l], tgt[l], tol, L, &near);
          if (near || a.exact_draws) {
            // near a boundary: the draw as the row-order sums take it
            if (tid < kWave) {
              const int64_t r = seq_draw(a.w, s, unit_from_word(seed_draw(a.seed, t, q - trials + l)));
              if (tid == 0) cand_l[l] = r;
            }
            if (g == 0 && tid == 0)
              atomicAdd(reinterpret_cast<unsigned long long*>(&a.counters[kCntBoundary]), 1ull);
          } else if (tid == 0) {
            cand_l[l] = c;
          }
#pragma unroll
          for (int q = 0; q < kLocRows; ++q) wv[q] = wn[q];
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < kMaxTrials; ++l) {
          cands[l] = l < trials ? cand_l[l] : 0;
          valid = valid && (l >= trials || (cands[l] >= 0 && cands[l] < s));
        }
        tick(kCntTicksSeedLocate);
        if (!valid) {
          if (tid == 0) set_err(a, kErrSeed);
          return false;
        }
      } else {
        for (int l = 0; l < trials; ++l) {
          if (owner[l] != g) continue;
          const double target = tgt[l];
          const double tol = draw_tol(s, W);
          double run = basev[l];
          if (tid == 0) { L.misc64[1] = -1; L.misc64[3] = 0; }
          __syncthreads();
          for (int64_t tile = 0; tile < tiles; ++tile) {
            const int64_t i = r0 + tile * kBlock + tid;
            const double wi = (i < r1) ? get_w(tile, i) : 0.0;
            double tot = 0.0;
            const double incl = block_inclusive_scan_f64<kBlock>(wi, L.tmpd, tot);
            const double v = run + incl;
            const bool hit = (i < r1) && (v > target);
            // first hitting row of the tile: minimum over hitting threads
            if (tid == 0) L.misc[2] = 0x7fffffff;
            __syncthreads();
            wave_min_first(hit, tid, &L.misc[2]);
            __syncthreads();
            const int first = L.misc[2];
            if (first != 0x7fffffff) {
              if (tid == first) {
                L.misc64[1] = i;
                const double prev = v - wi;
                L.misc64[3] = ((v - target) < tol || (target - prev) < tol) ? 1 : 0;
              }
              __syncthreads();
              break;
            }
            run += tot;
          }
          __syncthreads();
          if (L.misc64[1] < 0) {
            // rounding left the target beyond this chunk: last row with weight
            if (tid == 0) L.misc[2] = -1;
            __syncthreads();
            for (int64_t tile = 0; tile < tiles; ++tile) {
              const int64_t i = r0 + tile * kBlock + tid;
              if (i < r1 && get_w(tile, i) > 0.0) atomicMax(&L.misc[2], static_cast<int>(i - r0));
            }
            __syncthreads();
            if (tid == 0) {
              L.misc64[1] = (L.misc[2] >= 0) ? r0 + L.misc[2] : -1;
              L.misc64[3] = 1;
            }
            __syncthreads();
          }
          if (L.misc64[3] || a.exact_draws) {
            // near a boundary: the draw as the row-order sums take it
            if (tid < kWave) {
              const int64_t r = seq_draw(a.w, s, unit_from_word(seed_draw(a.seed, t, q - trials + l)));
              if (tid == 0) L.misc64[1] = r;
            }
            if (tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&a.counters[kCntBoundary]), 1ull);
            __syncthreads();
          }
          if (tid == 0) {
            a.cand[l] = L.misc64[1];
            if (L.misc64[1] < 0) set_err(a, kErrSeed);
          }
          __syncthreads();
        }
        if (!sync_grid(a)) return false;
#pragma unroll
        for (int l = 0; l < kMaxTrials; ++l) {
          cands[l] = (l < trials) ? a.cand[l] : 0;
          valid = valid && cands[l] >= 0 && cands[l] < s;
        }
      }
      if (!valid) {
        if (tid == 0) set_err(a, kErrSeed);
        return false;
      }
      if (trials == 1) {
        pick = cands[0];
      } else {
        // candidate rows into LDS, then the potentials sum_i min(D_i^2, |p_i - c|^2)
        for (int e = tid; e < trials * DM; e += kBlock) {
          const int l = e / DM;
          const int tdim = e - l * DM;
          int64_t c = cands[0];
#pragma unroll
          for (int l2 = 1; l2 < kMaxTrials; ++l2)
            if (l2 == l) c = cands[l2];
          cand_rows[e] = (tdim < d) ? a.P[static_cast<size_t>(c) * d + tdim] : 0.f;
        }
        __syncthreads();
        double ph[kMaxTrials];
#pragma unroll
        for (int l = 0; l < kMaxTrials; ++l) ph[l] = 0.0;
        for (int64_t tile = 0; tile < tiles; ++tile) {
          const int64_t i = r0 + tile * kBlock + tid;
          if (i >= r1) continue;
          double dd[kMaxTrials];
          if (cached || DM < 64) {
            float x[DM];
            row(tile, x);
#pragma unroll
            for (int l = 0; l < kMaxTrials; ++l)
              dd[l] = (l < trials) ? dist2_f64_row<DM>(x, cand_rows + l * DM) : 0.0;
          } else {  // wide rows: stream them rather than hold them
            dist2_f64_candidates<DM>(a.P + static_cast<size_t>(i) * d, d, cand_rows, trials, dd);
          }
          const double wi = get_w(tile, i);
#pragma unroll
          for (int l = 0; l < kMaxTrials; ++l) {
            if (l < trials) {
              ph[l] += dd[l] < wi ? dd[l] : wi;
              // streamed rows keep the distance for the D^2 update below
              if (!cached) a.dcache[static_cast<size_t>(l) * s + i] = dd[l];
            }
          }
        }
#pragma unroll
        for (int l = 0; l < kMaxTrials; ++l) {
          if (l < trials) {
            const double v = block_sum_f64<kBlock>(ph[l], L.tmpd);
            if (tid == 0) a.phi_part[g * kMaxTrials + l] = v;
          }
        }
        nd += s * trials;
        if (!sync_grid(a)) return false;
        tick(kCntTicksSeedPot);
        int best = 0;
        double best_phi = __builtin_inf();
        for (int l = 0; l < trials; ++l) {
          const double phi = grid_partials_sum(a.phi_part + l, G, kMaxTrials, L.tmpd);
          if (phi < best_phi) { best_phi = phi; best = l; }
        }
        pick = cands[0];
#pragma unroll
        for (int l = 1; l < kMaxTrials; ++l)
          if (l == best) pick = cands[l];
        picked = best;
      }
    }
    if (pick < 0 || pick >= s) {  // no valid candidate: stop (error already raised)
      if (tid == 0) set_err(a, kErrSeed);
      return false;
    }
    // place centroid j at P[pick]
    for (int tdim = tid; tdim < DM; tdim += kBlock)
      L.C[j * DM + tdim] = (tdim < d) ? a.P[static_cast<size_t>(pick) * d + tdim] : 0.f;
    __syncthreads();
    if (tid == 0) L.degf[j] = 0;
    // update D^2 over this workgroup's rows
    double part = 0.0;
    const float* cj = L.C + j * DM;
    // a streamed row's distance to the winning candidate was kept by the
    // potentials pass: the same FP64 arithmetic on the same FP32 values (the
    // candidate is the row P[pick]), so it is read instead of recomputed
    const bool reuse = !cached && picked >= 0;
    for (int64_t tile = 0; tile < tiles; ++tile) {
      const int64_t i = r0 + tile * kBlock + tid;
      if (i >= r1) continue;
      double dd;
      if (reuse) {
        dd = a.dcache[static_cast<size_t>(picked) * s + i];
      } else {
        float x[DM];
        row(tile, x);
        dd = dist2_f64_row<DM>(x, cj);
      }
      const double wold = get_w(tile, i);
      const double wi = (na == 0) ? dd : (dd < wold ? dd : wold);
      set_w(i, wi);
      part += wi;
    }
    const double ws = block_sum_f64<kBlock>(part, L.tmpd);
    if (tid == 0) a.wsum[g] = ws;
    nd += s;
    nres += 1;
    rebuild_active(L, k);
    if (!sync_grid(a)) return false;
    tick(kCntTicksSeedUpdate);
  }
  if (LEAN && g == 0 && tid == 0)
    for (int c = 0; c < 4; ++c) a.counters[kCntTicksSeedInit + c] += static_cast<int64_t>(ticks[c]);
  return true;
}

// ---------------------------------------------------------------------------
// 3. K-means on the sample.

// SUMS_LDS: sums_dst is the workgroup's LDS copy (otherwise the global ring);
// a compile-time choice, so the accumulation compiles to LDS or global
// atomics instead of generic ones.
template <int DM, bool SUMS_LDS>
__device__ __forceinline__ void assign_row(const SolverArgs& a, Lds& L, const float (&x)[DM],
                                           int64_t i, int na, bool accumulate, double* sums_dst,
                                           int ld, int* cnt_l, double& sse) {
  int bj;
  float bd;
  // every slot in index order: a degenerate slot holds NaN and never compares
  // smaller, and the strict comparison keeps the lowest index on exact ties
  bj = L.act[0];
  bd = __builtin_inff();
  int j = 0;
  if (DM <= 32) {  // four slots at a time (their chains overlap), compared in index order
    for (; j + 4 <= a.k; j += 4) {
      float v[4];
      dist2_f32_x4<DM>(x, L.C + j * DM, L.C + (j + 1) * DM, L.C + (j + 2) * DM, L.C + (j + 3) * DM, v);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (v[u] < bd) {
          bd = v[u];
          bj = j + u;
        }
      }
    }
  }
  for (; j < a.k; ++j) {
    const float v = dist2_f32<DM>(x, L.C + j * DM);
    if (v < bd) {
      bd = v;
      bj = j;
    }
  }
  if (a.labels) a.labels[i] = bj;
  sse += dist2_f64_row<DM>(x, L.C + bj * DM);
  if (accumulate) {
    atomicAdd(&cnt_l[bj], 1);
    double* dst = sums_dst + bj * ld;
#pragma unroll
    for (int tdim = 0; tdim < DM; ++tdim)
      if (tdim < a.d) unsafeAtomicAdd(dst + tdim, static_cast<double>(x[tdim]));
  }
}

// One assignment pass over this workgroup's rows, optionally accumulating the
// cluster sums and counts into ring slot (pass % 3).  Ends with a grid
// barrier; the per-workgroup objectives are left in sse_part[pass % 2].
template <int DM>
__device__ __forceinline__ bool assign_pass(const SolverArgs& a, const LdsPlan& pl, Lds& L, uint32_t pass,
                            int64_t r0, int64_t r1, bool accumulate, bool cached,
                            const RowCache<DM>& rc) {
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int d = a.d;
  const int k = a.k;
  const int kd = k * d;
  const int na = L.misc[0];
  // this workgroup's replica of ring slot (pass % 3)
  const int rep = g % kReplicas;
  double* ring = a.sums + (static_cast<size_t>(pass % 3) * kReplicas + rep) * kd;
  int32_t* cring = a.cnt + (static_cast<size_t>(pass % 3) * kReplicas + rep) * k;
  double* sums_l = reinterpret_cast<double*>(L.B + pl.sums);
  int* cnt_l = reinterpret_cast<int*>(L.B + pl.cntl);
  const uint64_t a0 = wall_clock64();

  if (g == 0) {  // clear the ring slot (all replicas) the next pass accumulates into
    double* nring = a.sums + static_cast<size_t>((pass + 1) % 3) * kReplicas * kd;
    int32_t* ncring = a.cnt + static_cast<size_t>((pass + 1) % 3) * kReplicas * k;
    for (int e = tid; e < kReplicas * kd; e += kBlock) nring[e] = 0.0;
    for (int j = tid; j < kReplicas * k; j += kBlock) ncring[j] = 0;
  }
  const int ld = a.sums_in_lds ? sums_ld(d) : d;
  const int reps = a.sums_in_lds > 1 ? a.sums_in_lds : 1;  // LDS replicas
  const int rstride = sums_rstride(k, d);
  const int rep_l = tid & (reps - 1);                        // this lane's replica
  int* cnt_rep = cnt_l + rep_l * k;
  if (accumulate) {
    if (a.sums_in_lds)
      for (int e = tid; e < reps * rstride; e += kBlock) sums_l[e] = 0.0;
    for (int j = tid; j < reps * k; j += kBlock) cnt_l[j] = 0;
    __syncthreads();
  }
  const uint64_t a1 = wall_clock64();
  double sse = 0.0;
  auto rows = [&](auto sums_lds_tag, double* sums_dst) {
    constexpr bool kL = decltype(sums_lds_tag)::value;
    if (cached) {
#pragma unroll
      for (int q = 0; q < RowCache<DM>::kRows; ++q) {
        const int64_t i = r0 + tid + static_cast<int64_t>(q) * kBlock;
        if (i < r1) assign_row<DM, kL>(a, L, rc.x[q], i, na, accumulate, sums_dst, ld, cnt_rep, sse);
      }
    } else {
      for (int64_t i = r0 + tid; i < r1; i += kBlock) {
        float x[DM];
        load_row_f32<DM>(a.P + static_cast<size_t>(i) * d, d, x);
        assign_row<DM, kL>(a, L, x, i, na, accumulate, sums_dst, ld, cnt_rep, sse);
      }
    }
  };
  if (a.sums_in_lds) rows(std::true_type{}, sums_l + static_cast<size_t>(rep_l) * rstride);
  else rows(std::false_type{}, ring);
  const uint64_t a2 = wall_clock64();
  // this workgroup's objective: wavefront sums, then thread 0 adds them in
  // order (the barrier also completes every row's LDS accumulation before
  // the flush; tmpd is next written after the grid barrier)
  {
    const int lane = tid & (kWave - 1);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) sse += __shfl_down(sse, o, kWave);
    if (lane == 0) L.tmpd[tid / kWave] = sse;
  }
  __syncthreads();
  const uint64_t f0 = wall_clock64();
  if (accumulate) {
    auto count = [&](int j) {
      int c = 0;
      for (int r = 0; r < reps; ++r) c += cnt_l[r * k + j];
      return c;
    };
    if (a.sums_in_lds) {
      for (int e = tid; e < kd; e += kBlock) {
        const int j = e / d;
        if (!count(j)) continue;
        const int q = j * ld + (e - j * d);
        double v = sums_l[q];
        for (int r = 1; r < reps; ++r) v += sums_l[r * rstride + q];  // fixed order
        unsafeAtomicAdd(&ring[e], v);
      }
    }
    for (int j = tid; j < k; j += kBlock) {
      const int c = count(j);
      if (c) atomicAdd(&cring[j], c);
    }
  }
  if (tid == 0) {
    double wsse = 0.0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) wsse += L.tmpd[w];
    a.sse_part[(pass & 1u) * kMaxGrid + g] = wsse;
  }
  const uint64_t b0 = wall_clock64();
  const bool ok = sync_grid(a);
  if (g == 0 && tid == 0) {
    a.counters[kCntTicksAssign] += static_cast<int64_t>(f0 - a0);
    a.counters[kCntTicksAssignInit] += static_cast<int64_t>(a1 - a0);
    a.counters[kCntTicksAssignRows] += static_cast<int64_t>(a2 - a1);
    a.counters[kCntTicksAssignSum] += static_cast<int64_t>(f0 - a2);
    a.counters[kCntTicksFlush] += static_cast<int64_t>(b0 - f0);
    a.counters[kCntTicksBarrier] += static_cast<int64_t>(wall_clock64() - b0);
  }
  return ok;
}

// After the barrier of pass `used`: read the objective partials, the cluster
// sums and the counts in one round of loads (sums staged in the idle LDS sums
// area when it exists), then return the objective of the pass.
__device__ __forceinline__ double gather_pass(const SolverArgs& a, const LdsPlan& pl, Lds& L, uint32_t used) {
  const int tid = threadIdx.x;
  const int k = a.k;
  const int kd = k * a.d;
  const int G = gridDim.x;
  const double* part = a.sse_part + (used & 1u) * kMaxGrid;
  // the objective: wavefront 0 adds the per-workgroup partials (lane l takes
  // l, l + 64, ... in order, then a shuffle tree: a fixed order, so every
  // workgroup gets the same bits); the first two per lane load with the sums
  const int lane = tid & (kWave - 1);
  double p0 = 0.0, p1 = 0.0;
  if (tid < kWave) {
    if (lane < G) p0 = part[lane];
    if (lane + kWave < G) p1 = part[lane + kWave];
  }
  const double* ring = a.sums + static_cast<size_t>(used % 3) * kReplicas * kd;
  const int32_t* cring = a.cnt + static_cast<size_t>(used % 3) * kReplicas * k;
  int* cnt_l = reinterpret_cast<int*>(L.B + pl.cntl);
  if (a.sums_in_lds) {
    double* stage = reinterpret_cast<double*>(L.B + pl.sums);
    const int d = a.d;
    const int ld = sums_ld(d);
    for (int e = tid; e < kd; e += kBlock) {
      double r[kReplicas];
#pragma unroll
      for (int q = 0; q < kReplicas; ++q) r[q] = ring[static_cast<size_t>(q) * kd + e];
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < kReplicas; ++q) v += r[q];  // fixed order
      const int j = e / d;
      stage[j * ld + (e - j * d)] = v;
    }
  }
  for (int j = tid; j < k; j += kBlock) {
    int c = 0;
#pragma unroll
    for (int q = 0; q < kReplicas; ++q) c += cring[static_cast<size_t>(q) * k + j];
    cnt_l[j] = c;
  }
  if (tid < kWave) {
    double v = p0 + p1;
    for (int g = lane + 2 * kWave; g < G; g += kWave) v += part[g];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    if (tid == 0) L.miscd[2] = v;
  }
  __syncthreads();  // the staged sums, the counts and the objective
  return L.miscd[2];
}

// New centroids from the gathered sums: the mean of each non-empty cluster as
// an FP64 sum / count (kept as FP64 means, rounded to FP32 for the distance
// kernels); an empty cluster turns degenerate.  Returns the largest Euclidean
// move of a surviving centroid, measured between FP64 means.  Every workgroup
// computes the same values.  The FP64 means live in LDS when they fit,
// otherwise in c64[it % 2] (every workgroup writes the same bits; the
// previous means are read from the other half).
template <int DM, bool C64_LDS>
__device__ __forceinline__ double update_centroids(const SolverArgs& a, const LdsPlan& pl, Lds& L, uint32_t used,
                                   int it) {
  const int tid = threadIdx.x;
  const int d = a.d;
  const int k = a.k;
  const double* ring = a.sums + static_cast<size_t>(used % 3) * kReplicas * k * d;
  const double* c_old = C64_LDS ? L.c64 : a.c64 + static_cast<size_t>((it + 1) & 1) * k * d;
  double* c_new = C64_LDS ? L.c64 : a.c64 + static_cast<size_t>(it & 1) * k * d;
  const int* cnt_l = reinterpret_cast<const int*>(L.B + pl.cntl);
  // staged sums, overwritten in place by the squared coordinate moves
  double* dsq = a.sums_in_lds ? reinterpret_cast<double*>(L.B + pl.sums) : nullptr;
  const int ld = sums_ld(d);
  // only the shift stop rule reads the largest move
  const bool need_shift = a.stop_rule == BM_STOP_SHIFT;
  if (tid == 0) L.misc[3] = 0;
  if (dsq) {
    for (int e = tid; e < k * d; e += kBlock) {
      const int j = e / d;
      const int c = cnt_l[j];
      if (L.degf[j] || c == 0) continue;
      const int q = j * ld + (e - j * d);
      const double mean = dsq[q] / static_cast<double>(c);
      if (need_shift) {
        const double diff = mean - c_old[e];
        dsq[q] = __dmul_rn(diff, diff);
      }
      c_new[e] = mean;
      L.C[j * DM + (e - j * d)] = static_cast<float>(mean);
    }
  }
  __syncthreads();
  double local = 0.0;
  for (int j = tid; j < k; j += kBlock) {
    if (L.degf[j]) continue;
    const int c = cnt_l[j];
    float* cj = L.C + j * DM;
    if (c == 0) {
      L.degf[j] = 1;
      L.misc[3] = 1;
      for (int tdim = 0; tdim < d; ++tdim) cj[tdim] = __builtin_nanf("");
      continue;
    }
    double moved = 0.0;
    if (dsq) {
      if (need_shift)
        for (int tdim = 0; tdim < d; ++tdim) moved = __dadd_rn(moved, dsq[j * ld + tdim]);
    } else {
      for (int tdim = 0; tdim < d; ++tdim) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < kReplicas; ++q) sum += ring[static_cast<size_t>(q) * k * d + j * d + tdim];
        const double mean = sum / static_cast<double>(c);
        const double diff = mean - c_old[j * d + tdim];
        moved = __dadd_rn(moved, __dmul_rn(diff, diff));
        c_new[j * d + tdim] = mean;
        cj[tdim] = static_cast<float>(mean);
      }
    }
    moved = sqrt(moved);
    local = moved > local ? moved : local;
  }
  if (!need_shift) {
    __syncthreads();
    // (the next pass reads the new centroids and slots after its own barrier)
    if (L.misc[3]) rebuild_active(L, k);  // a cluster emptied this round
    return 0.0;
  }
  // block max (exact, order-free)
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const double y = __shfl_down(local, o, kWave);
    local = y > local ? y : local;
  }
  __syncthreads();
  if (lane == 0) L.tmpd[wave] = local;
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int w = 0; w < kWavesPerBlock; ++w) mx = L.tmpd[w] > mx ? L.tmpd[w] : mx;
    L.miscd[1] = mx;
  }
  __syncthreads();
  if (L.misc[3]) rebuild_active(L, k);  // a cluster emptied this round
  const double shift = L.miscd[1];
  __syncthreads();
  return shift;
}

template <int DM>
__device__ __forceinline__ bool lloyd_phase(const SolverArgs& a, const LdsPlan& pl, Lds& L, uint32_t& pass,
                            int64_t r0, int64_t r1, bool cached, const RowCache<DM>& rc,
                            double& f_out, int& passes_out, int64_t& nd, uint64_t& tk_pass,
                            uint64_t& tk_post) {
  double f_prev = __builtin_inf();
  double f = 0.0;
  int passes = 0;
  bool by_objective = false;
  const int d = a.d;
  // FP64 means start as the FP32 start centroids
  for (int e = threadIdx.x; e < a.k * d; e += kBlock) {
    const int j = e / d;
    const double v = static_cast<double>(L.C[j * DM + (e - j * d)]);
    if (a.c64_in_lds) L.c64[e] = v;
    else a.c64[e] = v;
  }
  for (int it = 1; it <= a.max_iter; ++it) {
    const int na = L.misc[0];
    const uint64_t c0t = wall_clock64();
    if (!assign_pass<DM>(a, pl, L, pass, r0, r1, true, cached, rc)) return false;
    const uint64_t c1t = wall_clock64();
    const uint32_t used = pass++;
    ++passes;
    nd += a.s * na;
    f = gather_pass(a, pl, L, used);
    if (a.stop_rule == BM_STOP_REL_OBJ && it > 1 && (f_prev - f) <= a.tol * f_prev) {
      by_objective = true;
      break;
    }
    const double shift = a.c64_in_lds ? update_centroids<DM, true>(a, pl, L, used, it)
                                      : update_centroids<DM, false>(a, pl, L, used, it);
    const uint64_t c2t = wall_clock64();
    tk_pass += c1t - c0t;
    tk_post += c2t - c1t;
    f_prev = f;
    if (a.stop_rule == BM_STOP_SHIFT && shift < a.tol) break;
  }
  if (!by_objective) {
    const int na = L.misc[0];
    if (!assign_pass<DM>(a, pl, L, pass, r0, r1, false, cached, rc)) return false;
    f = gather_pass(a, pl, L, pass);
    ++pass;
    ++passes;
    nd += a.s * na;
  }
  f_out = f;
  passes_out = passes;
  return true;
}

// Another initialisation of the degenerate slots (Sec. 3.3 allows other
// strategies than K-means++): each degenerate slot, ascending, takes the
// sample row at a uniformly drawn index (draw q of sample t of the K-means++
// stream; independent draws, so two slots may take the same row and the later
// one then empties).  Every workgroup draws the same indices; no distances and
// no grid barrier are needed.
template <int DM>
__device__ __forceinline__ void forgy_phase(const SolverArgs& a, Lds& L, uint32_t t, int64_t& nres) {
  const int d = a.d;
  const int k = a.k;
  uint64_t q = 0;
  for (int j = 0; j < k; ++j) {
    if (!L.degf[j]) continue;
    const int64_t pick =
        static_cast<int64_t>(below_from_word(seed_draw(a.seed, t, q), static_cast<uint64_t>(a.s)));
    ++q;
    for (int tdim = threadIdx.x; tdim < DM; tdim += kBlock)
      L.C[j * DM + tdim] = (tdim < d) ? a.P[static_cast<size_t>(pick) * d + tdim] : 0.f;
    __syncthreads();
    if (threadIdx.x == 0) L.degf[j] = 0;
    __syncthreads();
    nres += 1;
  }
  rebuild_active(L, k);
}

// ---------------------------------------------------------------------------

// The incumbent into LDS; a degenerate slot is filled with NaN so that no
// distance to it compares smaller in the assignment scans.
template <int DM>
__device__ __forceinline__ void load_incumbent(const SolverArgs& a, Lds& L) {
  const int d = a.d;
  const int k = a.k;
  for (int e = threadIdx.x; e < k * DM; e += kBlock) {
    const int j = e / DM;
    const int tdim = e - j * DM;
    L.C[e] = (tdim < d) ? (a.deg_inc[j] ? __builtin_nanf("") : a.Cinc[j * d + tdim]) : 0.f;
  }
  for (int j = threadIdx.x; j < k; j += kBlock) L.degf[j] = a.deg_inc[j] ? 1 : 0;
  rebuild_active(L, k);
}

template <int DM>
__device__ __forceinline__ void store_incumbent(const SolverArgs& a, Lds& L, double f) {
  const int d = a.d;
  const int k = a.k;
  for (int e = threadIdx.x; e < k * d; e += kBlock) {
    const int j = e / d;
    const int tdim = e - j * d;
    a.Cinc[e] = L.degf[j] ? __builtin_nanf("") : L.C[j * DM + tdim];
  }
  for (int j = threadIdx.x; j < k; j += kBlock) a.deg_inc[j] = static_cast<uint8_t>(L.degf[j]);
  if (threadIdx.x == 0) *a.f_opt = f;
}

}  // namespace

template <int DM>
__global__ void __launch_bounds__(kBlock) solver_kernel(SolverArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const LdsPlan pl = plan_lds(DM, a.k, a.d, a.sums_in_lds, a.c64_in_lds != 0);
  Lds L = carve(lds_raw, pl);
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int G = gridDim.x;
  const int64_t rpw = (a.s + G - 1) / G;
  const int64_t r0 = imin64(a.s, static_cast<int64_t>(g) * rpw);
  const int64_t r1 = imin64(a.s, r0 + rpw);

  int64_t c_passes = 0, c_reseeded = 0, c_replaced = 0, c_nd = 0, c_samples = 0, c_hist = 0;
  uint64_t c_tsample = 0, c_tseed = 0, c_tlloyd = 0, c_tpass = 0, c_tpost = 0;
  uint32_t pass = 0;
  bool ok = true;

  if (a.init_incumbent && g == 0) {
    for (int e = tid; e < a.k * a.d; e += kBlock) a.Cinc[e] = __builtin_nanf("");
    for (int j = tid; j < a.k; j += kBlock) a.deg_inc[j] = 1;
    if (tid == 0) *a.f_opt = __builtin_inf();
  }
  if (a.init_incumbent) ok = sync_grid(a);

  // samples are drawn a.sbatch at a time into slots; the phases below read
  // the current sample's rows through a.P
  float* const Pb = a.P;
  int32_t* const idxb = a.idx;
  bool stored = false;  // the previous sample replaced the incumbent (grid-uniform)
  const uint64_t clk_launch = wall_clock64();
  // every sample was drawn before this launch (presample_* kernels) unless a
  // predicted window missed; then the samples are drawn here as usual
  const bool presampled =
      a.presampled && __hip_atomic_load(a.presample_miss, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
  for (int tt = 0; ok && tt < a.T; ++tt) {
    const uint32_t t = static_cast<uint32_t>(a.t0 + tt);
    const int slot = tt % a.sbatch;
    if (a.budget_ticks && tt > 0) {
      // time budget (the CPU-time stop condition of Sec. 5): workgroup 0
      // reads its clock, and every workgroup takes its decision after a
      // barrier, so all stop before the same sample
      if (g == 0 && tid == 0)
        __hip_atomic_store(a.stop_flag, (wall_clock64() - clk_launch) >= a.budget_ticks ? 1 : 0,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ok = sync_grid(a);
      if (!ok) break;
      if (__hip_atomic_load(a.stop_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      // the flag is written again before the next sample; no workgroup reads
      // it until that sample's barrier
    }
    uint64_t clk0 = wall_clock64();
    if (a.do_sample && slot == 0 && !presampled) {
      const int nb = a.T - tt < a.sbatch ? a.T - tt : a.sbatch;
      ok = sample_batch<DM>(a, pl, L, Pb, idxb, tt, nb, c_hist);
      if (!ok) break;
    } else if (stored) {
      // workgroup 0 wrote the incumbent at the end of the previous sample;
      // every workgroup reads it below, so wait for that write to land
      ok = sync_grid(a);
      if (!ok) break;
    }
    if (Pb) a.P = Pb + static_cast<size_t>(slot) * a.s * a.d;
    a.idx = idxb + static_cast<size_t>(slot) * a.s;
    uint64_t clk1 = wall_clock64();
    c_tsample += clk1 - clk0;
    load_incumbent<DM>(a, L);
    // this workgroup's sample rows stay in registers for the whole sample
    // when the chunk is a single tile
    // (only when a sample exists and a phase that reads it will run)
    RowCache<DM> rc;
    const bool uses_rows = a.P != nullptr && (a.do_seed || a.do_lloyd || a.do_keep);
    const bool cached = uses_rows && RowCache<DM>::kRows > 0 && (r1 - r0) <= kBlock;
    if (cached) {
      const int64_t i = r0 + tid;
      if (i < r1) load_row_f32<DM>(a.P + static_cast<size_t>(i) * a.d, a.d, rc.x[0]);
    }
    double f_ref = 0.0;
    if (a.do_keep) {
      if (a.cmp_rule == BM_CMP_RESAMPLE) {
        if (L.misc[0] > 0) {
          ok = assign_pass<DM>(a, pl, L, pass, r0, r1, false, cached, rc);
          if (!ok) break;
          f_ref = gather_pass(a, pl, L, pass);
          ++pass;
        } else {
          f_ref = __builtin_inf();
        }
      } else {
        f_ref = *a.f_opt;
      }
    }
    clk0 = wall_clock64();
    if (a.do_seed && L.misc[0] < a.k) {
      if (a.init_forgy) {
        forgy_phase<DM>(a, L, t, c_reseeded);
      } else {
        ok = reseed_phase<DM, false>(a, L, t, r0, r1, cached, rc, c_nd, c_reseeded);
        if (!ok) break;
      }
    }
    clk1 = wall_clock64();
    c_tseed += clk1 - clk0;
    double f = 0.0;
    int passes = 0;
    if (a.do_lloyd) {
      ok = lloyd_phase<DM>(a, pl, L, pass, r0, r1, cached, rc, f, passes, c_nd, c_tpass, c_tpost);
      if (!ok) break;
      c_passes += passes;
    }
    c_tlloyd += wall_clock64() - clk1;
    if (a.do_keep) {
      stored = f_ref > f;
      if (stored) {
        if (g == 0) store_incumbent<DM>(a, L, f);
        ++c_replaced;
      }
    } else {
      stored = true;
      if (g == 0) store_incumbent<DM>(a, L, f);
    }
    if (g == 0 && tid == 0 && a.sample_f) a.sample_f[tt] = f;
    ++c_samples;
  }
  if (g == 0 && tid == 0) {
    a.counters[kCntPasses] = c_passes;
    a.counters[kCntReseeded] = c_reseeded;
    a.counters[kCntReplaced] = c_replaced;
    a.counters[kCntND] = c_nd;
    a.counters[kCntSamples] = c_samples;
    a.counters[kCntSelectPasses] = c_hist;
    a.counters[kCntTicksSample] = static_cast<int64_t>(c_tsample);
    a.counters[kCntTicksSeed] = static_cast<int64_t>(c_tseed);
    a.counters[kCntTicksLloyd] = static_cast<int64_t>(c_tlloyd);
    a.counters[kCntTicksPass] = static_cast<int64_t>(c_tpass);
    a.counters[kCntTicksPost] = static_cast<int64_t>(c_tpost);
  }
}

// The reseeding step alone (one sample already in a.P, no Lloyd, no
// keep-the-best): the solver's K-means++ (or Forgy) phase on the incumbent,
// whose result replaces the incumbent.  A kernel of its own, so its registers
// are not sized by the other phases.
template <int DM>
__global__ void __launch_bounds__(kBlock) seed_kernel(SolverArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const LdsPlan pl = plan_lds(DM, a.k, a.d, a.sums_in_lds, a.c64_in_lds != 0);
  Lds L = carve(lds_raw, pl);
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int G = gridDim.x;
  const int64_t rpw = (a.s + G - 1) / G;
  const int64_t r0 = imin64(a.s, static_cast<int64_t>(g) * rpw);
  const int64_t r1 = imin64(a.s, r0 + rpw);
  const uint32_t t = static_cast<uint32_t>(a.t0);
  int64_t c_reseeded = 0, c_nd = 0;
  const uint64_t clk0 = wall_clock64();
  load_incumbent<DM>(a, L);
  RowCache<DM> rc;
  const bool cached = RowCache<DM>::kRows > 0 && (r1 - r0) <= kBlock;
  if (cached) {
    const int64_t i = r0 + tid;
    if (i < r1) load_row_f32<DM>(a.P + static_cast<size_t>(i) * a.d, a.d, rc.x[0]);
  }
  bool ok = true;
  if (L.misc[0] < a.k) {
    if (a.init_forgy) forgy_phase<DM>(a, L, t, c_reseeded);
    else ok = reseed_phase<DM, true>(a, L, t, r0, r1, cached, rc, c_nd, c_reseeded);
  }
  if (!ok) return;
  if (g == 0) store_incumbent<DM>(a, L, 0.0);
  if (g == 0 && tid == 0) {
    a.counters[kCntReseeded] = c_reseeded;
    a.counters[kCntND] = c_nd;
    a.counters[kCntSamples] = 1;
    a.counters[kCntTicksSeed] = static_cast<int64_t>(wall_clock64() - clk0);
    if (a.sample_f) a.sample_f[0] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Presampling: every sample of a fit drawn before the persistent solver starts,
// by three ordinary launches over the whole device (a sample depends only on
// (seed, t)), when all of a fit's samples fit the sample buffers.  Workgroup
// (g, b) takes chunk g of the point pairs of sample b; the selection is the
// solver's own (collect, threshold select, emit in index order), with `gp`
// chunks in place of the solver's workgroups, so the samples are the same.  A
// sample whose predicted window misses raises *presample_miss, and the solver
// then draws every sample itself.

template <int DM>
__global__ void __launch_bounds__(kBlock) presample_collect_kernel(SolverArgs a, int gp) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const LdsPlan pl = plan_lds(DM, a.k, a.d, a.sums_in_lds, a.c64_in_lds != 0);
  Lds L = carve(lds_raw, pl);
  const int g = blockIdx.x, b = blockIdx.y;
  const int64_t npairs = (a.n + 1) >> 1;
  const int64_t ppw = (npairs + gp - 1) / gp;
  const int64_t p0 = imin64(npairs, static_cast<int64_t>(g) * ppw);
  const int64_t p1 = imin64(npairs, p0 + ppw);
  collect_pass(a, slot_bufs(a, a.P, a.idx, b), pl, L, static_cast<uint32_t>(a.t0 + b), p0, p1, a.win_lo,
               a.win_hi, g);
}

template <int DM>
__global__ void __launch_bounds__(kBlock) presample_select_kernel(SolverArgs a, int gp) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const LdsPlan pl = plan_lds(DM, a.k, a.d, a.sums_in_lds, a.c64_in_lds != 0);
  Lds L = carve(lds_raw, pl);
  const int b = blockIdx.x;
  const int64_t npairs = (a.n + 1) >> 1;
  const int64_t ppw = (npairs + gp - 1) / gp;
  const SBuf sb = slot_bufs(a, a.P, a.idx, b);
  const int64_t below = keys_below(sb, L, gp);
  const int64_t m = __hip_atomic_load(sb.cand_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const bool hit = m <= a.cand_cap && below < a.s && a.s <= below + m;
  if (hit) {
    (void)select_threshold(a, sb, pl, L, below, m, ppw, gp);  // an inconsistency sets the error
  } else if (threadIdx.x == 0) {
    __hip_atomic_store(a.presample_miss, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(sb.cand_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int DM>
__global__ void __launch_bounds__(kBlock) presample_emit_kernel(SolverArgs a, int gp) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  if (__hip_atomic_load(a.presample_miss, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const LdsPlan pl = plan_lds(DM, a.k, a.d, a.sums_in_lds, a.c64_in_lds != 0);
  Lds L = carve(lds_raw, pl);
  const int g = blockIdx.x, b = blockIdx.y;
  const int64_t npairs = (a.n + 1) >> 1;
  const int64_t ppw = (npairs + gp - 1) / gp;
  const int64_t p0 = imin64(npairs, static_cast<int64_t>(g) * ppw);
  const int64_t p1 = imin64(npairs, p0 + ppw);
  emit_sample<DM>(a, slot_bufs(a, a.P, a.idx, b), L, static_cast<uint32_t>(a.t0 + b), b, p0, p1, g);
}

// Rows of every presampled sample (wide rows): one wavefront per row, lanes
// over the coordinates, so reads and writes are coalesced; the emit pass then
// writes only the indices.  Nothing is done after a predicted-window miss (the
// solver draws and gathers the samples itself).
template <bool BF16>
__global__ void __launch_bounds__(kBlock) presample_gather_kernel(SolverArgs a) {
  if (__hip_atomic_load(a.presample_miss, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t rows = static_cast<int64_t>(a.T) * a.s;
  const int64_t w0 = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kWave;
  const int64_t wstride = static_cast<int64_t>(gridDim.x) * kBlock / kWave;
  const int d = a.d;
  for (int64_t r = w0; r < rows; r += wstride) {
    const int64_t src = a.idx[r];
    if (src < 0 || src >= a.n) continue;  // never read outside X
    float* dst = a.P + static_cast<size_t>(r) * d;
    for (int t = lane; t < d; t += kWave) {
      float v;
      if (BF16)
        v = bf16_bits_to_float(static_cast<const uint16_t*>(a.X)[static_cast<size_t>(src) * d + t]);
      else
        v = static_cast<const float*>(a.X)[static_cast<size_t>(src) * d + t];
      dst[t] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Host side.

int padded_dim(int d) {
  if (d <= 4) return 4;
  if (d <= 8) return 8;
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  if (d <= 64) return 64;
  if (d <= 72) return 72;
  if (d <= 128) return 128;
  if (d <= 256) return 256;
  return -1;
}

size_t solver_lds_bytes(int dm, int k, int d, int sums_reps, bool c64_in_lds) {
  return plan_lds(dm, k, d, sums_reps, c64_in_lds).total;
}

static const void* seed_fn(int dm) {
  switch (dm) {
    case 4: return reinterpret_cast<const void*>(&seed_kernel<4>);
    case 8: return reinterpret_cast<const void*>(&seed_kernel<8>);
    case 16: return reinterpret_cast<const void*>(&seed_kernel<16>);
    case 32: return reinterpret_cast<const void*>(&seed_kernel<32>);
    case 64: return reinterpret_cast<const void*>(&seed_kernel<64>);
    case 72: return reinterpret_cast<const void*>(&seed_kernel<72>);
    case 128: return reinterpret_cast<const void*>(&seed_kernel<128>);
    case 256: return reinterpret_cast<const void*>(&seed_kernel<256>);
    default: return nullptr;
  }
}

static const void* solver_fn(int dm) {
  switch (dm) {
    case 4: return reinterpret_cast<const void*>(&solver_kernel<4>);
    case 8: return reinterpret_cast<const void*>(&solver_kernel<8>);
    case 16: return reinterpret_cast<const void*>(&solver_kernel<16>);
    case 32: return reinterpret_cast<const void*>(&solver_kernel<32>);
    case 64: return reinterpret_cast<const void*>(&solver_kernel<64>);
    case 72: return reinterpret_cast<const void*>(&solver_kernel<72>);
    case 128: return reinterpret_cast<const void*>(&solver_kernel<128>);
    case 256: return reinterpret_cast<const void*>(&solver_kernel<256>);
    default: return nullptr;
  }
}

bm_status max_lds_per_block(size_t* bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(BM_EDEVICE, "hipGetDevice failed");
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return set_error(BM_EDEVICE, "cannot query LDS size");
  *bytes = static_cast<size_t>(v);
  return BM_OK;
}

bm_status reserve_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return BM_OK;
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> reserved;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(BM_EDEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = reserved[{dev, fn}];
  if (cur >= bytes) return BM_OK;
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(bytes));
  if (e != hipSuccess)
    return set_error(BM_ENOTSUP, "cannot reserve %zu B of LDS: %s", bytes, hipGetErrorString(e));
  cur = bytes;
  return BM_OK;
}

bm_status solver_max_grid(int dm, size_t lds, int* max_grid) {
  const void* fn = solver_fn(dm);
  if (!fn) return set_error(BM_ENOTSUP, "no solver for padded dimension %d", dm);
  int dev = 0, cus = 0, coop = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess)
    return set_error(BM_EDEVICE, "cannot query device attributes");
  if (!coop) return set_error(BM_ENOTSUP, "device lacks cooperative launch");
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds) != hipSuccess)
    return set_error(BM_EDEVICE, "occupancy query failed");
  if (per_cu < 1) return set_error(BM_ENOTSUP, "solver does not fit one workgroup per CU (LDS %zu B)", lds);
  int g = per_cu * cus;
  if (g > kMaxGrid) g = kMaxGrid;
  *max_grid = g;
  return BM_OK;
}

bm_status launch_solver(const SolverArgs& a, int grid, size_t lds, hipStream_t stream) {
  // every buffer a requested phase touches must exist
  const bool rows = a.do_seed || a.do_lloyd || a.do_keep || a.do_gather;
  if ((rows && !a.P) || (a.do_gather && !a.X) || a.sbatch < 1 || (!a.do_sample && a.sbatch != 1) ||
      (a.do_sample && (!a.idx || !a.cand_key || !a.selcode || !a.cand_idx || !a.wg_lo ||
                       !a.wg_off || !a.thr || !a.hist || !a.cand_count || !a.smiss)) ||
      (rows && (!a.w || !a.dcache)) || !a.Cinc || !a.deg_inc || !a.f_opt || !a.c64 || !a.sums ||
      !a.cnt || !a.sse_part || !a.wsum || !a.phi_part || !a.cand || !a.counters || !a.bar ||
      !a.err || !a.sample_f || (a.budget_ticks && !a.stop_flag) || grid < 1 || grid > kMaxGrid)
    return set_error(BM_EINVAL, "solver launch with a missing buffer or bad grid %d", grid);
  const int dm = padded_dim(a.d);
  // the reseeding step alone runs on its own kernel
  const bool seed_only = a.do_seed && !a.do_lloyd && !a.do_keep && !a.do_sample && !a.do_gather &&
                         a.T == 1 && !a.init_incumbent && !a.budget_ticks;
  const void* fn = seed_only ? seed_fn(dm) : solver_fn(dm);
  if (!fn) return set_error(BM_ENOTSUP, "dimension %d exceeds the solver's limit of 256", a.d);
  if (bm_status sr = reserve_lds(fn, lds)) return sr;
  SolverArgs copy = a;
  copy.exact_draws = exact_draws_forced() ? 1 : 0;
  void* args[] = {&copy};
  const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args,
                                                  static_cast<unsigned int>(lds), stream);
  if (e != hipSuccess)
    return set_error(BM_EDEVICE, "cooperative launch failed (grid %d, LDS %zu B): %s", grid, lds,
                     hipGetErrorString(e));
  return BM_OK;
}

// Draw all a.T samples into their slots before the solver (see the
// presample kernels); the caller has checked a.sbatch == a.T.
bm_status launch_presample(SolverArgs& a, size_t lds, hipStream_t stream, bool force_miss) {
  const int dm = padded_dim(a.d);
  const void* fc = nullptr;
  const void* fs = nullptr;
  const void* fe = nullptr;
  switch (dm) {
#define BM_PRE(D)                                                        \
  case D:                                                                \
    fc = reinterpret_cast<const void*>(&presample_collect_kernel<D>);    \
    fs = reinterpret_cast<const void*>(&presample_select_kernel<D>);     \
    fe = reinterpret_cast<const void*>(&presample_emit_kernel<D>);       \
    break;
    BM_PRE(4) BM_PRE(8) BM_PRE(16) BM_PRE(32) BM_PRE(64) BM_PRE(72) BM_PRE(128) BM_PRE(256)
#undef BM_PRE
    default: return set_error(BM_ENOTSUP, "dimension %d exceeds the solver's limit of 256", a.d);
  }
  if (a.sbatch != a.T || a.T < 1 || a.T > 65535 || !a.presample_miss)
    return set_error(BM_EINVAL, "presampling needs every sample in its own slot");
  const int64_t npairs = (a.n + 1) >> 1;
  int64_t gp = (npairs + 4095) / 4096;  // ~8 pairs per thread
  if (gp < 1) gp = 1;
  if (gp > kMaxGrid) gp = kMaxGrid;
  for (const void* f : {fc, fs, fe})
    if (bm_status sr = reserve_lds(f, lds)) return sr;
  SolverArgs copy = a;
  // wide rows are gathered by a separate coalesced pass after the emit
  const bool coop_gather = a.do_gather && a.d >= 32 && a.P && a.idx;
  if (coop_gather) copy.do_gather = 0;
  int g32 = static_cast<int>(gp);
  void* args[] = {&copy, &g32};
  hipError_t e = hipLaunchKernel(fc, dim3(g32, a.T), dim3(kBlock), args, lds, stream);
  if (e == hipSuccess) e = hipLaunchKernel(fs, dim3(a.T), dim3(kBlock), args, lds, stream);
  if (e == hipSuccess && force_miss) e = hipMemsetAsync(a.presample_miss, 1, 1, stream);  // test hook
  if (e == hipSuccess) e = hipLaunchKernel(fe, dim3(g32, a.T), dim3(kBlock), args, lds, stream);
  if (e == hipSuccess && coop_gather) {
    const int64_t rows = static_cast<int64_t>(a.T) * a.s;
    int64_t blocks = (rows * kWave + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    void* gargs[] = {&copy};
    const void* fg = a.x_bf16 ? reinterpret_cast<const void*>(&presample_gather_kernel<true>)
                              : reinterpret_cast<const void*>(&presample_gather_kernel<false>);
    e = hipLaunchKernel(fg, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), gargs, 0, stream);
  }
  if (e != hipSuccess) return set_error(BM_EDEVICE, "presample launch failed: %s", hipGetErrorString(e));
  a.presampled = 1;
  return BM_OK;
}

}  // namespace bm

namespace bm {

// Key window that holds the s-th smallest of n independent uniform 64-bit
// keys with overwhelming probability: its rank is s on average with standard
// deviation sqrt(s (1 - s/n)); the window spans 8 deviations plus 64 ranks on
// either side, mapped to key values.  The candidate list holds the expected
// window count with ample slack; a miss falls back to exact histogram passes.
int sample_slots(int64_t n, int64_t s, int d, int T, int64_t cand_cap) {
  const double per = 4.0 * static_cast<double>(s) * d + 4.0 * s + static_cast<double>(n) +
                     12.0 * cand_cap + 8.0 * kMaxGrid + 64.0;
  double b = floor(kSampleBatchBytes / per);
  if (b > T) b = T;
  if (b < 1) b = 1;
  return static_cast<int>(b);
}

void sampler_window(int64_t n, int64_t s, uint64_t* lo, uint64_t* hi, int64_t* cap) {
  const double nn = static_cast<double>(n), ss = static_cast<double>(s);
  const double sigma = sqrt(ss * (1.0 - ss / nn));
  const double delta = 8.0 * sigma + 64.0;
  const double lo_rank = ss - delta, hi_rank = ss + delta;
  *lo = lo_rank <= 0.0 ? 0ull : static_cast<uint64_t>(ldexp(lo_rank / nn, 64));
  *hi = hi_rank >= nn ? ~0ull : static_cast<uint64_t>(ldexp(hi_rank / nn, 64));
  const double expect = 2.0 * delta + 1.0;
  double c = expect + 8.0 * sqrt(expect) + 4096.0;
  if (c > nn) c = nn;
  *cap = static_cast<int64_t>(c);
}

}  // namespace bm
