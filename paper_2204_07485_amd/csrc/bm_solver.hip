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

#include "bm_internal.h"
#include "bm_rng.h"

namespace bm {

namespace {

constexpr int kHistBins = 256;

struct Lds {
  float* C;          // k x DM, padded with zeros past d
  int* act;          // active slots, ascending
  int* degf;         // degenerate flags
  int* tmpi;         // scan scratch
  double* tmpd;      // reduction scratch
  int* misc;         // [0] number of active slots, [1] chosen bucket, [2] hit flag
  int64_t* misc64;   // [0] bucket count, [1] found row, [2] fallback row, [3] pick
  double* miscd;     // [0] broadcast value, [1..] per-trial scratch
  unsigned char* B;  // phase-local region
};

__device__ __forceinline__ int64_t imin64(int64_t x, int64_t y) { return x < y ? x : y; }

__host__ __device__ __forceinline__ size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

struct LdsPlan {
  size_t C, act, degf, tmpi, tmpd, misc, misc64, miscd, B;
  size_t hist, skey, sidx, selc, total_sampling;
  size_t sums, cntl, total_lloyd;
  size_t total;
};

__host__ __device__ inline LdsPlan plan_lds(int dm, int k, int d, int cand_cap, bool sums_in_lds) {
  LdsPlan p;
  size_t o = 0;
  p.C = o; o = align16(o + sizeof(float) * size_t(k) * dm);
  p.act = o; o = align16(o + sizeof(int) * size_t(k));
  p.degf = o; o = align16(o + sizeof(int) * size_t(k));
  p.tmpi = o; o = align16(o + sizeof(int) * 32);
  p.tmpd = o; o = align16(o + sizeof(double) * 32);
  p.misc = o; o = align16(o + sizeof(int) * 8);
  p.misc64 = o; o = align16(o + sizeof(int64_t) * 8);
  p.miscd = o; o = align16(o + sizeof(double) * (4 + 4 * kMaxTrials));
  p.B = o;
  size_t b = 0;
  p.hist = b; b = align16(b + sizeof(unsigned int) * kHistBins);
  p.skey = b; b = align16(b + sizeof(uint64_t) * size_t(cand_cap));
  p.sidx = b; b = align16(b + sizeof(int32_t) * size_t(cand_cap));
  p.selc = b; b = align16(b + sizeof(unsigned int) * kMaxGrid);
  p.total_sampling = b;
  b = 0;
  p.sums = b; b = align16(b + (sums_in_lds ? sizeof(double) * size_t(k) * d : 0));
  p.cntl = b; b = align16(b + sizeof(int) * size_t(k));
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
  L.B = base + p.B;
  return L;
}

__device__ __forceinline__ void set_err(const SolverArgs& a, int code) {
  atomicCAS(a.err, 0, code);
  __hip_atomic_store(&a.bar->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool sync_grid(const SolverArgs& a) {
  const bool ok = grid_barrier(a.bar, gridDim.x, a.spin_limit);
  if (!ok && threadIdx.x == 0) atomicCAS(a.err, 0, kErrBarrier);
  return ok;
}

// Rebuild the ascending list of active slots from the flags (whole block).
__device__ __forceinline__ void rebuild_active(Lds& L, int k) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int na = 0;
    for (int j = 0; j < k; ++j)
      if (!L.degf[j]) L.act[na++] = j;
    L.misc[0] = na;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// 1. Sampling.

__device__ __forceinline__ bool key_in_window(uint64_t key, uint64_t pre, int nbits) {
  return nbits == 0 || (key >> (64 - nbits)) == pre;
}
__device__ __forceinline__ bool key_below_window(uint64_t key, uint64_t pre, int nbits) {
  return nbits != 0 && (key >> (64 - nbits)) < pre;
}
__device__ __forceinline__ bool pair_le(uint64_t k, int64_t i, uint64_t tk, int64_t ti) {
  return k < tk || (k == tk && i <= ti);
}

// Append (key, index) to the candidate list with one atomic per wavefront.
__device__ __forceinline__ void append_candidate(const SolverArgs& a, bool pred, uint64_t key,
                                                 int64_t i) {
  const unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int leader = __builtin_ctzll(mask);
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(a.cand_count, static_cast<unsigned int>(__popcll(mask)));
  base = __shfl(base, leader, kWave);
  if (pred) {
    const unsigned int rank = __popcll(mask & ((1ull << lane) - 1ull));
    const unsigned int slot = base + rank;
    if (slot < static_cast<unsigned int>(a.cand_cap)) {
      a.cand_key[slot] = key;
      a.cand_idx[slot] = static_cast<int32_t>(i);
    }
  }
}

__device__ __forceinline__ void emit_point(const SolverArgs& a, int tt, int64_t pos, int64_t i) {
  if (pos < 0 || pos >= a.s) {  // inconsistent bookkeeping: never write out of bounds
    atomicCAS(a.err, 0, kErrSelect);
    return;
  }
  a.idx[pos] = static_cast<int32_t>(i);
  if (a.sample_idx_out) a.sample_idx_out[static_cast<size_t>(tt) * a.s + pos] = static_cast<int32_t>(i);
  if (a.do_gather) {
    const int d = a.d;
    float* dst = a.P + static_cast<size_t>(pos) * d;
    if (a.x_bf16) {
      const uint16_t* src = static_cast<const uint16_t*>(a.X) + static_cast<size_t>(i) * d;
      for (int t = 0; t < d; ++t) dst[t] = bf16_bits_to_float(src[t]);
    } else {
      const float* src = static_cast<const float*>(a.X) + static_cast<size_t>(i) * d;
      for (int t = 0; t < d; ++t) dst[t] = src[t];
    }
  }
}

// WG 0: sort the collected window, fix the threshold pair and the output
// offset of every workgroup.
__device__ bool select_threshold(const SolverArgs& a, const LdsPlan& pl, Lds& L, int64_t below,
                                 int64_t m, int64_t ppw) {
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  uint64_t* skey = reinterpret_cast<uint64_t*>(L.B + pl.skey);
  int32_t* sidx = reinterpret_cast<int32_t*>(L.B + pl.sidx);
  unsigned int* selc = reinterpret_cast<unsigned int*>(L.B + pl.selc);

  const unsigned int got = __hip_atomic_load(a.cand_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int64_t need = a.s - below;
  if (static_cast<int64_t>(got) != m || m > a.cand_cap || need < 1 || need > m) {
    if (tid == 0) set_err(a, kErrSelect);
    return false;
  }
  int n2 = 2;
  while (n2 < m) n2 <<= 1;
  for (int r = tid; r < n2; r += kBlock) {
    if (r < m) {
      skey[r] = a.cand_key[r];
      sidx[r] = a.cand_idx[r];
    } else {
      skey[r] = ~0ull;
      sidx[r] = 0x7fffffff;
    }
  }
  for (int gg = tid; gg < G; gg += kBlock) selc[gg] = 0u;
  __syncthreads();
  // bitonic sort by (key, index), ascending
  for (int kk = 2; kk <= n2; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int r = tid; r < n2; r += kBlock) {
        const int partner = r ^ jj;
        if (partner > r) {
          const bool up = (r & kk) == 0;
          const uint64_t ka = skey[r], kb = skey[partner];
          const int32_t ia = sidx[r], ib = sidx[partner];
          const bool a_gt_b = ka > kb || (ka == kb && ia > ib);
          if (a_gt_b == up) {
            skey[r] = kb; skey[partner] = ka;
            sidx[r] = ib; sidx[partner] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int64_t r = tid; r < need; r += kBlock) {
    const int64_t i = sidx[r];
    const int owner = static_cast<int>((i >> 1) / ppw);
    atomicAdd(&selc[owner], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    a.thr[0] = skey[need - 1];
    a.thr[1] = static_cast<uint64_t>(sidx[need - 1]);
    int64_t run = 0;
    for (int gg = 0; gg < G; ++gg) {
      a.wg_off[gg] = static_cast<uint32_t>(run);
      run += static_cast<int64_t>(selc[gg]) + a.wg_lo[gg];
    }
    __hip_atomic_store(a.cand_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (run != a.s) set_err(a, kErrSelect);
    L.misc[2] = (run == a.s) ? 1 : 0;
  }
  __syncthreads();
  return L.misc[2] != 0;
}

__device__ bool sample_phase(const SolverArgs& a, const LdsPlan& pl, Lds& L, uint32_t t, int tt,
                             int64_t& hist_passes) {
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int G = gridDim.x;
  const int64_t n = a.n;
  const int64_t npairs = (n + 1) >> 1;
  const int64_t ppw = (npairs + G - 1) / G;
  const int64_t p0 = imin64(npairs, static_cast<int64_t>(g) * ppw);
  const int64_t p1 = imin64(npairs, p0 + ppw);
  unsigned int* hist = reinterpret_cast<unsigned int*>(L.B + pl.hist);

  uint64_t pre = 0;
  int nbits = 0;
  int64_t below = 0;
  int64_t m = n;
  while (m > a.cand_cap) {
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
      const unsigned int v = hist[b];
      if (v) atomicAdd(&Hcur[b], v);
    }
    if (!sync_grid(a)) return false;
    if (tid == 0) {
      const int64_t need = a.s - below;
      int64_t cum = 0;
      int b = 0;
      for (; b < kHistBins; ++b) {
        const int64_t h = Hcur[b];
        if (cum + h >= need) break;
        cum += h;
      }
      if (b == kHistBins) b = kHistBins - 1;  // inconsistent counts; caught below
      L.misc[1] = b;
      L.misc64[0] = cum;
      L.misc64[1] = Hcur[b];
    }
    __syncthreads();
    below += L.misc64[0];
    pre = (pre << 8) | static_cast<uint64_t>(L.misc[1]);
    nbits += 8;
    m = L.misc64[1];
    ++hist_passes;
    __syncthreads();
  }

  // collect the window; count keys below it
  int lo_count = 0;
  const int64_t span = p1 - p0;
  const int64_t tiles = (span + kBlock - 1) / kBlock;
  for (int64_t tile = 0; tile < tiles; ++tile) {
    const int64_t p = p0 + tile * kBlock + tid;
    const bool v0 = p < p1;
    const bool v1 = v0 && (2 * p + 1 < n);
    uint64_t k0 = 0, k1 = 0;
    if (v0) sample_key_pair(a.seed, t, static_cast<uint64_t>(p), k0, k1);
    lo_count += (v0 && key_below_window(k0, pre, nbits)) ? 1 : 0;
    lo_count += (v1 && key_below_window(k1, pre, nbits)) ? 1 : 0;
    append_candidate(a, v0 && key_in_window(k0, pre, nbits), k0, 2 * p);
    append_candidate(a, v1 && key_in_window(k1, pre, nbits), k1, 2 * p + 1);
  }
  const int wg_lo = block_sum_i32<kBlock>(lo_count, L.tmpi);
  if (tid == 0) a.wg_lo[g] = static_cast<uint32_t>(wg_lo);
  if (!sync_grid(a)) return false;

  if (g == 0) {
    if (!select_threshold(a, pl, L, below, m, ppw)) return false;
  }
  if (!sync_grid(a)) return false;

  // emit in index order and gather
  const uint64_t tk = a.thr[0];
  const int64_t ti = static_cast<int64_t>(a.thr[1]);
  int64_t base = a.wg_off[g];
  for (int64_t tile = 0; tile < tiles; ++tile) {
    const int64_t p = p0 + tile * kBlock + tid;
    const bool v0 = p < p1;
    const bool v1 = v0 && (2 * p + 1 < n);
    uint64_t k0 = 0, k1 = 0;
    if (v0) sample_key_pair(a.seed, t, static_cast<uint64_t>(p), k0, k1);
    const int s0 = (v0 && pair_le(k0, 2 * p, tk, ti)) ? 1 : 0;
    const int s1 = (v1 && pair_le(k1, 2 * p + 1, tk, ti)) ? 1 : 0;
    int total = 0;
    const int excl = block_exclusive_scan<kBlock, int>(s0 + s1, L.tmpi, total);
    const int64_t pos = base + excl;
    if (s0) emit_point(a, tt, pos, 2 * p);
    if (s1) emit_point(a, tt, pos + s0, 2 * p + 1);
    base += total;
  }
  return sync_grid(a);
}

// ---------------------------------------------------------------------------
// 2. K-means++ reseeding of the degenerate slots.

template <int DM>
__device__ bool reseed_phase(const SolverArgs& a, Lds& L, uint32_t t, int64_t r0, int64_t r1,
                             int64_t& nd, int64_t& nres, int64_t& nbound) {
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

  if (L.misc[0] > 0) {
    const int na = L.misc[0];
    double part = 0.0;
    for (int64_t i = r0 + tid; i < r1; i += kBlock) {
      const float* p = a.P + static_cast<size_t>(i) * d;
      double best = __builtin_inf();
      for (int aa = 0; aa < na; ++aa) {
        const double dd = dist2_f64(p, L.C + L.act[aa] * DM, d);
        if (dd < best) best = dd;
      }
      a.w[i] = best;
      part += best;
    }
    const double ws = block_sum_f64<kBlock>(part, L.tmpd);
    if (tid == 0) a.wsum[g] = ws;
    nd += s * na;
    if (!sync_grid(a)) return false;
  }

  for (int j = 0; j < k; ++j) {
    if (!L.degf[j]) continue;
    const int na = L.misc[0];
    int64_t pick = -1;
    if (na == 0) {
      pick = static_cast<int64_t>(below_from_word(seed_draw(a.seed, t, q), static_cast<uint64_t>(s)));
      ++q;
    } else {
      if (tid == 0) {
        double W = 0.0;
        for (int gg = 0; gg < G; ++gg) W += a.wsum[gg];
        L.miscd[0] = W;
        for (int l = 0; l < trials; ++l) {
          const double target = unit_from_word(seed_draw(a.seed, t, q + l)) * W;
          double E = 0.0;
          int own = -1;
          for (int gg = 0; gg < G; ++gg) {
            const double wsg = a.wsum[gg];
            if (E + wsg > target) { own = gg; break; }
            E += wsg;
          }
          if (own < 0) {  // rounding: fall back to the last chunk with weight
            E = 0.0;
            double Elast = 0.0;
            for (int gg = 0; gg < G; ++gg) {
              if (a.wsum[gg] > 0.0) { own = gg; Elast = E; }
              E += a.wsum[gg];
            }
            E = Elast;
          }
          tgt[l] = target;
          basev[l] = E;
          owner[l] = own;
        }
      }
      __syncthreads();
      const double W = L.miscd[0];
      if (W == 0.0) break;  // every remaining D^2 is zero: leave the slots degenerate
      q += trials;
      for (int l = 0; l < trials; ++l) {
        if (owner[l] != g) continue;
        const double target = tgt[l];
        double run = basev[l];
        if (tid == 0) { L.misc64[1] = -1; L.misc64[2] = -1; }
        __syncthreads();
        const int64_t tiles = (r1 - r0 + kBlock - 1) / kBlock;
        for (int64_t tile = 0; tile < tiles; ++tile) {
          const int64_t i = r0 + tile * kBlock + tid;
          const double wi = (i < r1) ? a.w[i] : 0.0;
          double tot = 0.0;
          const double incl = block_inclusive_scan_f64<kBlock>(wi, L.tmpd, tot);
          const double v = run + incl;
          const bool hit = (i < r1) && (v > target);
          // first hitting row of the tile: minimum over hitting threads
          if (tid == 0) L.misc[2] = 0x7fffffff;
          __syncthreads();
          if (hit) atomicMin(&L.misc[2], tid);
          __syncthreads();
          const int first = L.misc[2];
          if (first != 0x7fffffff) {
            if (tid == first) {
              L.misc64[1] = i;
              const double prev = v - wi;
              L.misc64[3] = ((v - target) < 1e-12 * W || (target - prev) < 1e-12 * W) ? 1 : 0;
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
          for (int64_t i = r0 + tid; i < r1; i += kBlock)
            if (a.w[i] > 0.0) atomicMax(&L.misc[2], static_cast<int>(i - r0));
          __syncthreads();
          if (tid == 0) {
            L.misc64[1] = (L.misc[2] >= 0) ? r0 + L.misc[2] : -1;
            L.misc64[3] = 1;
          }
          __syncthreads();
        }
        if (tid == 0) {
          a.cand[l] = L.misc64[1];
          if (L.misc64[3]) atomicAdd(reinterpret_cast<unsigned long long*>(&a.counters[kCntBoundary]), 1ull);
          if (L.misc64[1] < 0) set_err(a, kErrSeed);
        }
        __syncthreads();
      }
      if (!sync_grid(a)) return false;
      if (trials == 1) {
        pick = a.cand[0];
      } else {
        int64_t cands[kMaxTrials];
        double ph[kMaxTrials];
        bool valid = true;
#pragma unroll
        for (int l = 0; l < kMaxTrials; ++l) {
          cands[l] = (l < trials) ? a.cand[l] : 0;
          valid = valid && cands[l] >= 0 && cands[l] < s;
          ph[l] = 0.0;
        }
        if (!valid) {
          if (tid == 0) set_err(a, kErrSeed);
          return false;
        }
        for (int64_t i = r0 + tid; i < r1; i += kBlock) {
          const float* p = a.P + static_cast<size_t>(i) * d;
          const double wi = a.w[i];
#pragma unroll
          for (int l = 0; l < kMaxTrials; ++l) {
            if (l < trials) {
              const double dd = dist2_f64(p, a.P + static_cast<size_t>(cands[l]) * d, d);
              ph[l] += dd < wi ? dd : wi;
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
        if (tid == 0) {
          int best = 0;
          double best_phi = __builtin_inf();
          for (int l = 0; l < trials; ++l) {
            double phi = 0.0;
            for (int gg = 0; gg < G; ++gg) phi += a.phi_part[gg * kMaxTrials + l];
            if (phi < best_phi) { best_phi = phi; best = l; }
          }
          L.misc64[4] = a.cand[best];
        }
        __syncthreads();
        pick = L.misc64[4];
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
    for (int64_t i = r0 + tid; i < r1; i += kBlock) {
      const double dd = dist2_f64(a.P + static_cast<size_t>(i) * d, cj, d);
      const double wi = (na == 0) ? dd : (dd < a.w[i] ? dd : a.w[i]);
      a.w[i] = wi;
      part += wi;
    }
    const double ws = block_sum_f64<kBlock>(part, L.tmpd);
    if (tid == 0) a.wsum[g] = ws;
    nd += s;
    nres += 1;
    rebuild_active(L, k);
    if (!sync_grid(a)) return false;
  }
  (void)nbound;
  return true;
}

// ---------------------------------------------------------------------------
// 3. K-means on the sample.

// One assignment pass over this workgroup's rows, optionally accumulating the
// cluster sums and counts into sums ring slot (pass % 3); ends with a grid
// barrier and returns the objective of the current centroids on P.
template <int DM>
__device__ bool assign_pass(const SolverArgs& a, const LdsPlan& pl, Lds& L, uint32_t pass,
                            int64_t r0, int64_t r1, bool accumulate, double& f_out) {
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int G = gridDim.x;
  const int d = a.d;
  const int k = a.k;
  const int kd = k * d;
  const int na = L.misc[0];
  double* ring = a.sums + static_cast<size_t>(pass % 3) * kd;
  int32_t* cring = a.cnt + static_cast<size_t>(pass % 3) * k;
  double* sums_l = reinterpret_cast<double*>(L.B + pl.sums);
  int* cnt_l = reinterpret_cast<int*>(L.B + pl.cntl);

  if (g == 0) {  // clear the ring slot the next pass accumulates into
    double* nring = a.sums + static_cast<size_t>((pass + 1) % 3) * kd;
    int32_t* ncring = a.cnt + static_cast<size_t>((pass + 1) % 3) * k;
    for (int e = tid; e < kd; e += kBlock) nring[e] = 0.0;
    for (int j = tid; j < k; j += kBlock) ncring[j] = 0;
  }
  if (accumulate) {
    if (a.sums_in_lds)
      for (int e = tid; e < kd; e += kBlock) sums_l[e] = 0.0;
    for (int j = tid; j < k; j += kBlock) cnt_l[j] = 0;
    __syncthreads();
  }
  double sse = 0.0;
  for (int64_t i = r0 + tid; i < r1; i += kBlock) {
    float x[DM];
    load_row_f32<DM>(a.P + static_cast<size_t>(i) * d, d, x);
    int bj;
    float bd;
    nearest_f32<DM>(x, L.C, L.act, na, bj, bd);
    a.labels[i] = bj;
    sse += dist2_f64_row<DM>(x, L.C + bj * DM);
    if (accumulate) {
      atomicAdd(&cnt_l[bj], 1);
      double* dst = a.sums_in_lds ? sums_l + bj * d : ring + bj * d;
#pragma unroll
      for (int tdim = 0; tdim < DM; ++tdim)
        if (tdim < d) unsafeAtomicAdd(dst + tdim, static_cast<double>(x[tdim]));
    }
  }
  const double wsse = block_sum_f64<kBlock>(sse, L.tmpd);
  if (accumulate) {
    if (a.sums_in_lds) {
      for (int e = tid; e < kd; e += kBlock)
        if (cnt_l[e / d]) unsafeAtomicAdd(&ring[e], sums_l[e]);
    }
    for (int j = tid; j < k; j += kBlock)
      if (cnt_l[j]) atomicAdd(&cring[j], cnt_l[j]);
  }
  if (tid == 0) a.sse_part[(pass & 1u) * kMaxGrid + g] = wsse;
  if (!sync_grid(a)) return false;
  if (tid == 0) {
    double f = 0.0;
    for (int gg = 0; gg < G; ++gg) f += a.sse_part[(pass & 1u) * kMaxGrid + gg];
    L.miscd[0] = f;
  }
  __syncthreads();
  f_out = L.miscd[0];
  __syncthreads();
  return true;
}

// New centroids from ring slot `used`: the mean of each non-empty cluster
// as an FP64 sum / count (kept in c64, rounded to FP32 for the distance
// kernels); an empty cluster turns degenerate.  Returns the largest Euclidean
// move of a surviving centroid, measured between FP64 means.  Every workgroup
// computes the same values and writes the same bits into c64[it % 2]; the
// previous means are read from the other half.
template <int DM>
__device__ double update_centroids(const SolverArgs& a, Lds& L, uint32_t used, int it) {
  const int tid = threadIdx.x;
  const int d = a.d;
  const int k = a.k;
  const double* ring = a.sums + static_cast<size_t>(used % 3) * k * d;
  const int32_t* cring = a.cnt + static_cast<size_t>(used % 3) * k;
  const double* c_old = a.c64 + static_cast<size_t>((it + 1) & 1) * k * d;
  double* c_new = a.c64 + static_cast<size_t>(it & 1) * k * d;
  double local = 0.0;
  for (int j = tid; j < k; j += kBlock) {
    if (L.degf[j]) continue;
    const int c = cring[j];
    float* cj = L.C + j * DM;
    if (c == 0) {
      L.degf[j] = 1;
      for (int tdim = 0; tdim < d; ++tdim) cj[tdim] = __builtin_nanf("");
      continue;
    }
    double moved = 0.0;
    for (int tdim = 0; tdim < d; ++tdim) {
      const double mean = ring[j * d + tdim] / static_cast<double>(c);
      const double diff = mean - c_old[j * d + tdim];
      moved = __dadd_rn(moved, __dmul_rn(diff, diff));
      c_new[j * d + tdim] = mean;
      cj[tdim] = static_cast<float>(mean);
    }
    moved = sqrt(moved);
    local = moved > local ? moved : local;
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
  rebuild_active(L, k);
  const double shift = L.miscd[1];
  __syncthreads();
  return shift;
}

template <int DM>
__device__ bool lloyd_phase(const SolverArgs& a, const LdsPlan& pl, Lds& L, uint32_t& pass,
                            int64_t r0, int64_t r1, double& f_out, int& passes_out, int64_t& nd) {
  double f_prev = __builtin_inf();
  double f = 0.0;
  int passes = 0;
  bool by_objective = false;
  // FP64 means start as the FP32 start centroids (identical writes from every
  // workgroup; first read after the next grid barrier)
  for (int e = threadIdx.x; e < a.k * a.d; e += kBlock) {
    const int j = e / a.d;
    a.c64[e] = static_cast<double>(L.C[j * DM + (e - j * a.d)]);
  }
  for (int it = 1; it <= a.max_iter; ++it) {
    const int na = L.misc[0];
    if (!assign_pass<DM>(a, pl, L, pass, r0, r1, true, f)) return false;
    const uint32_t used = pass++;
    ++passes;
    nd += a.s * na;
    if (a.stop_rule == BM_STOP_REL_OBJ && it > 1 && (f_prev - f) <= a.tol * f_prev) {
      by_objective = true;
      break;
    }
    const double shift = update_centroids<DM>(a, L, used, it);
    f_prev = f;
    if (a.stop_rule == BM_STOP_SHIFT && shift < a.tol) break;
  }
  if (!by_objective) {
    const int na = L.misc[0];
    if (!assign_pass<DM>(a, pl, L, pass, r0, r1, false, f)) return false;
    ++pass;
    ++passes;
    nd += a.s * na;
  }
  f_out = f;
  passes_out = passes;
  return true;
}

// ---------------------------------------------------------------------------

template <int DM>
__device__ void load_incumbent(const SolverArgs& a, Lds& L) {
  const int d = a.d;
  const int k = a.k;
  for (int e = threadIdx.x; e < k * DM; e += kBlock) {
    const int j = e / DM;
    const int tdim = e - j * DM;
    L.C[e] = (tdim < d) ? a.Cinc[j * d + tdim] : 0.f;
  }
  for (int j = threadIdx.x; j < k; j += kBlock) L.degf[j] = a.deg_inc[j] ? 1 : 0;
  rebuild_active(L, k);
}

template <int DM>
__device__ void store_incumbent(const SolverArgs& a, Lds& L, double f) {
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
  const LdsPlan pl = plan_lds(DM, a.k, a.d, a.cand_cap, a.sums_in_lds != 0);
  Lds L = carve(lds_raw, pl);
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int G = gridDim.x;
  const int64_t rpw = (a.s + G - 1) / G;
  const int64_t r0 = imin64(a.s, static_cast<int64_t>(g) * rpw);
  const int64_t r1 = imin64(a.s, r0 + rpw);

  int64_t c_passes = 0, c_reseeded = 0, c_replaced = 0, c_nd = 0, c_samples = 0, c_hist = 0;
  int64_t c_bound = 0;
  uint32_t pass = 0;
  bool ok = true;

  if (a.init_incumbent && g == 0) {
    for (int e = tid; e < a.k * a.d; e += kBlock) a.Cinc[e] = __builtin_nanf("");
    for (int j = tid; j < a.k; j += kBlock) a.deg_inc[j] = 1;
    if (tid == 0) *a.f_opt = __builtin_inf();
  }
  if (a.init_incumbent) ok = sync_grid(a);

  for (int tt = 0; ok && tt < a.T; ++tt) {
    const uint32_t t = static_cast<uint32_t>(a.t0 + tt);
    if (a.do_sample) {
      ok = sample_phase(a, pl, L, t, tt, c_hist);
      if (!ok) break;
    }
    load_incumbent<DM>(a, L);
    double f_ref = 0.0;
    if (a.do_keep) {
      if (a.cmp_rule == BM_CMP_RESAMPLE) {
        if (L.misc[0] > 0) {
          ok = assign_pass<DM>(a, pl, L, pass, r0, r1, false, f_ref);
          ++pass;
          if (!ok) break;
        } else {
          f_ref = __builtin_inf();
        }
      } else {
        f_ref = *a.f_opt;
      }
    }
    if (a.do_seed && L.misc[0] < a.k) {
      ok = reseed_phase<DM>(a, L, t, r0, r1, c_nd, c_reseeded, c_bound);
      if (!ok) break;
    }
    double f = 0.0;
    int passes = 0;
    if (a.do_lloyd) {
      ok = lloyd_phase<DM>(a, pl, L, pass, r0, r1, f, passes, c_nd);
      if (!ok) break;
      c_passes += passes;
    }
    if (a.do_keep) {
      if (f_ref > f) {
        if (g == 0) store_incumbent<DM>(a, L, f);
        ++c_replaced;
      }
    } else if (g == 0) {
      store_incumbent<DM>(a, L, f);
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

size_t solver_lds_bytes(int dm, int k, int d, int grid, int cand_cap, bool sums_in_lds) {
  (void)grid;
  return plan_lds(dm, k, d, cand_cap, sums_in_lds).total;
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
  const int dm = padded_dim(a.d);
  const void* fn = solver_fn(dm);
  if (!fn) return set_error(BM_ENOTSUP, "dimension %d exceeds the solver's limit of 256", a.d);
  if (lds > 65536) {
    const hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                              static_cast<int>(lds));
    if (ea != hipSuccess)
      return set_error(BM_ENOTSUP, "cannot reserve %zu B of LDS: %s", lds, hipGetErrorString(ea));
  }
  SolverArgs copy = a;
  void* args[] = {&copy};
  const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args,
                                                  static_cast<unsigned int>(lds), stream);
  if (e != hipSuccess)
    return set_error(BM_EDEVICE, "cooperative launch failed (grid %d, LDS %zu B): %s", grid, lds,
                     hipGetErrorString(e));
  return BM_OK;
}

}  // namespace bm
