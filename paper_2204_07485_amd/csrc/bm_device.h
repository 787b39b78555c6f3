// bm_device.h -- device building blocks shared by the library's kernels:
// a bounded grid barrier for cooperative launches, block-wide scans and
// reductions for 64-wide wavefronts, and the direct-difference distances.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bm {

constexpr int kWave = 64;
constexpr int kBlock = 512;                 // solver workgroup: 8 wavefronts
constexpr int kWavesPerBlock = kBlock / kWave;

// ---------------------------------------------------------------------------
// Grid barrier for a cooperative launch (every workgroup is resident).
//
// Two-level arrival: the G workgroups form about sqrt(G) groups of
// consecutive workgroups, each with its own arrival counter; the last arriver
// of a group arrives at the top counter, and the last of those publishes the
// next generation to one word per group, which that group's members poll.
// Every word sits in a cache line of its own, so no line takes more than
// about sqrt(G) of the same-address atomics or pollers: same-address device
// atomics are serialized where device coherence is kept, which made a single
// counter cost time linear in G.
//
// Ordering: a workgroup publishes its writes with one agent-scope release
// fence before arriving; a group's last arriver takes an acquire-release
// fence before forwarding the group to the top counter; the final arriver
// acquires, resets the top counter and release-stores the generation words;
// a waiter polls with relaxed loads (no cache maintenance per poll) and takes
// one agent-scope acquire fence after the wait.  Counters are reset by the
// arriver that completes them, before the release that lets their group
// arrive again.  A waiter that polls more than spin_limit times raises
// `abort`, and every later barrier returns false at once, so a logic error
// ends the kernel instead of hanging it.
struct alignas(128) BarrierWord {
  unsigned int v;
  unsigned int pad[31];
};
constexpr int kBarrierMaxGroups = 64;  // groups of ceil(sqrt(G)) for G <= 4096

struct GridBarrier {
  BarrierWord top;                        // groups whose members have all arrived
  BarrierWord abort;                      // nonzero: every barrier fails at once
  BarrierWord arrive[kBarrierMaxGroups];  // arrivals per group
  BarrierWord gen[kBarrierMaxGroups];     // generation, one copy per group
};

__device__ __forceinline__ unsigned int barrier_group_size(unsigned int nblocks) {
  unsigned int s = static_cast<unsigned int>(__builtin_sqrtf(static_cast<float>(nblocks)));
  while (s * s < nblocks) ++s;
  while (s > 1 && (s - 1) * (s - 1) >= nblocks) --s;
  return s;  // ceil(sqrt(nblocks))
}

__device__ __forceinline__ bool grid_barrier(GridBarrier* b, unsigned int nblocks,
                                             unsigned int spin_limit) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned int S = barrier_group_size(nblocks);
    const unsigned int grp = blockIdx.x / S;
    unsigned int* my_gen = &b->gen[grp].v;
    // the abort flag and this group's generation are loaded together (one
    // round trip); the generation cannot move before this workgroup arrives
    const unsigned int aborted = __hip_atomic_load(&b->abort.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned int g = __hip_atomic_load(my_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (aborted) {
      ok = 0;
    } else {
      const unsigned int gsize = (nblocks - grp * S) < S ? (nblocks - grp * S) : S;
      const unsigned int ngroups = (nblocks + S - 1) / S;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      bool wait = true;
      const unsigned int prev =
          __hip_atomic_fetch_add(&b->arrive[grp].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (prev == gsize - 1) {
        // the group is complete: reset its counter, then forward it
        __hip_atomic_store(&b->arrive[grp].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        const unsigned int prev2 =
            __hip_atomic_fetch_add(&b->top.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev2 == ngroups - 1) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          __hip_atomic_store(&b->top.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          for (unsigned int q = 0; q < ngroups; ++q)
            __hip_atomic_store(&b->gen[q].v, g + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          wait = false;
        }
      }
      if (wait) {
        unsigned int polls = 0;
        while (__hip_atomic_load(my_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
          if ((polls & 15u) == 15u &&
              __hip_atomic_load(&b->abort.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = 0;
            break;
          }
          if (++polls > spin_limit) {
            __hip_atomic_store(&b->abort.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// ---------------------------------------------------------------------------
// Block-wide primitives for blockDim.x == BLOCK (a multiple of 64).  `tmp` is
// LDS scratch of at least BLOCK/64 + 1 elements; every thread must call.

template <int BLOCK, typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* tmp, T& total) {
  constexpr int NW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  T incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const T y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) tmp[wave] = incl;
  __syncthreads();
  // every thread runs the same in-order pass over the wavefront totals
  T run = T(0), before = T(0);
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w == wave) before = run;
    run += tmp[w];
  }
  const T excl = incl - v + before;
  total = run;
  __syncthreads();  // tmp may be reused at once
  return excl;
}

// Inclusive scan in FP64 with a fixed combination order (wave tree, then
// waves in order).
template <int BLOCK>
__device__ __forceinline__ double block_inclusive_scan_f64(double v, double* tmp, double& total) {
  constexpr int NW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  double incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) tmp[wave] = incl;
  __syncthreads();
  // every thread runs the same in-order pass over the wavefront totals
  double run = 0.0, before = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w == wave) before = run;
    run += tmp[w];
  }
  const double out = incl + before;
  total = run;
  __syncthreads();  // tmp may be reused at once
  return out;
}

// Sum over the block in a fixed order; the result is returned to every thread.
template <int BLOCK>
__device__ __forceinline__ double block_sum_f64(double v, double* tmp) {
  constexpr int NW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  if (lane == 0) tmp[wave] = v;
  __syncthreads();
  // every thread adds the wavefront sums in the same order (same bits)
  double run = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) run += tmp[w];
  __syncthreads();  // tmp may be reused at once
  return run;
}

template <int BLOCK>
__device__ __forceinline__ int block_sum_i32(int v, int* tmp) {
  constexpr int NW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  if (lane == 0) tmp[wave] = v;
  __syncthreads();
  int run = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) run += tmp[w];
  __syncthreads();  // tmp may be reused at once
  return run;
}

// ---------------------------------------------------------------------------
// Element loads: FP32, or BF16 bit patterns widened exactly to FP32.
__device__ __forceinline__ float bf16_bits_to_float(uint16_t h) {
  return __uint_as_float(static_cast<unsigned int>(h) << 16);
}

// Load row `r` (d elements) into registers x[DM], zero-filled past d.
template <int DM>
__device__ __forceinline__ void load_row_f32(const float* __restrict__ r, int d, float (&x)[DM]) {
  if ((d & 3) == 0) {
    const float4* r4 = reinterpret_cast<const float4*>(r);
#pragma unroll
    for (int q = 0; q < DM / 4; ++q) {
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (4 * q < d) v = r4[q];
      x[4 * q + 0] = v.x;
      x[4 * q + 1] = v.y;
      x[4 * q + 2] = v.z;
      x[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int t = 0; t < DM; ++t) x[t] = (t < d) ? r[t] : 0.f;
  }
}

template <int DM>
__device__ __forceinline__ void load_row_bf16(const uint16_t* __restrict__ r, int d,
                                              float (&x)[DM]) {
#pragma unroll
  for (int t = 0; t < DM; ++t) x[t] = (t < d) ? bf16_bits_to_float(r[t]) : 0.f;
}

// Squared distance in FP32 by direct differences, FMA in dimension order,
// against a centroid row padded with zeros to DM (the padding adds exact 0).
template <int DM>
__device__ __forceinline__ float dist2_f32(const float (&x)[DM], const float* __restrict__ c) {
  float acc = 0.f;
#pragma unroll
  for (int t = 0; t < DM; t += 4) {
    const float4 cv = *reinterpret_cast<const float4*>(c + t);
    float e = x[t + 0] - cv.x;
    acc = __builtin_fmaf(e, e, acc);
    e = x[t + 1] - cv.y;
    acc = __builtin_fmaf(e, e, acc);
    e = x[t + 2] - cv.z;
    acc = __builtin_fmaf(e, e, acc);
    e = x[t + 3] - cv.w;
    acc = __builtin_fmaf(e, e, acc);
  }
  return acc;
}

// dist2_f32 for four centroid rows at once: four independent FMA chains,
// each with exactly dist2_f32's arithmetic and order, interleaved so that
// their latencies overlap.
template <int DM>
__device__ __forceinline__ void dist2_f32_x4(const float (&x)[DM], const float* __restrict__ c0,
                                             const float* __restrict__ c1, const float* __restrict__ c2,
                                             const float* __restrict__ c3, float (&out)[4]) {
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
  for (int t = 0; t < DM; t += 4) {
    const float4 v0 = *reinterpret_cast<const float4*>(c0 + t);
    const float4 v1 = *reinterpret_cast<const float4*>(c1 + t);
    const float4 v2 = *reinterpret_cast<const float4*>(c2 + t);
    const float4 v3 = *reinterpret_cast<const float4*>(c3 + t);
    const float w0[4] = {v0.x, v0.y, v0.z, v0.w};
    const float w1[4] = {v1.x, v1.y, v1.z, v1.w};
    const float w2[4] = {v2.x, v2.y, v2.z, v2.w};
    const float w3[4] = {v3.x, v3.y, v3.z, v3.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float e0 = x[t + q] - w0[q];
      const float e1 = x[t + q] - w1[q];
      const float e2 = x[t + q] - w2[q];
      const float e3 = x[t + q] - w3[q];
      a0 = __builtin_fmaf(e0, e0, a0);
      a1 = __builtin_fmaf(e1, e1, a1);
      a2 = __builtin_fmaf(e2, e2, a2);
      a3 = __builtin_fmaf(e3, e3, a3);
    }
  }
  out[0] = a0;
  out[1] = a1;
  out[2] = a2;
  out[3] = a3;
}

// Nearest active centroid: `act` lists the na active slots in ascending order,
// so a strict comparison keeps the lowest index on exact ties.
template <int DM>
__device__ __forceinline__ void nearest_f32(const float (&x)[DM], const float* __restrict__ Cl,
                                            const int* __restrict__ act, int na, int& best_j,
                                            float& best_d) {
  // a row whose distances are all NaN or +inf still gets a valid slot
  best_j = na > 0 ? act[0] : -1;
  best_d = __builtin_inff();
  for (int a = 0; a < na; ++a) {
    const int j = act[a];
    const float v = dist2_f32<DM>(x, Cl + j * DM);
    if (v < best_d) {
      best_d = v;
      best_j = j;
    }
  }
}

// nearest_f32 with four active slots' chains at a time (dist2_f32_x4),
// compared in ascending slot order: the same distances and the same winner.
template <int DM>
__device__ __forceinline__ void nearest_f32_x4(const float (&x)[DM], const float* __restrict__ Cl,
                                               const int* __restrict__ act, int na, int& best_j,
                                               float& best_d) {
  best_j = na > 0 ? act[0] : -1;
  best_d = __builtin_inff();
  int a = 0;
  for (; a + 4 <= na; a += 4) {
    const int j0 = act[a], j1 = act[a + 1], j2 = act[a + 2], j3 = act[a + 3];
    float v[4];
    dist2_f32_x4<DM>(x, Cl + j0 * DM, Cl + j1 * DM, Cl + j2 * DM, Cl + j3 * DM, v);
    const int jj[4] = {j0, j1, j2, j3};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (v[u] < best_d) {
        best_d = v[u];
        best_j = jj[u];
      }
    }
  }
  for (; a < na; ++a) {
    const int j = act[a];
    const float v = dist2_f32<DM>(x, Cl + j * DM);
    if (v < best_d) {
      best_d = v;
      best_j = j;
    }
  }
}

// The same nearest-centroid search with the centroid rows read through the
// scalar data cache into SGPRs: every lane compares its row with the same
// centroid, so the values are wavefront-uniform and the inner loop is two
// VALU operations per coordinate with an SGPR operand, no LDS traffic.
// Cpad holds the centroids zero-padded to DM columns (read only during the
// kernel); `act` (LDS) lists the na active slots ascending.  Identical
// arithmetic to nearest_f32.
typedef const float __attribute__((address_space(4))) scalar_f32;

template <int DM>
__device__ __forceinline__ void nearest_f32_sgpr(const float (&x)[DM], const float* __restrict__ Cpad,
                                                 const int* __restrict__ act, int na, int& best_j,
                                                 float& best_d) {
  // a row whose distances are all NaN or +inf still gets a valid slot
  best_j = na > 0 ? __builtin_amdgcn_readfirstlane(act[0]) : -1;
  best_d = __builtin_inff();
  for (int a = 0; a < na; ++a) {
    const int j = __builtin_amdgcn_readfirstlane(act[a]);
    const scalar_f32* c = (const scalar_f32*)(Cpad) + static_cast<size_t>(j) * DM;
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < DM; ++t) {
      const float e = x[t] - c[t];
      acc = __builtin_fmaf(e, e, acc);
      // keep the scalar loads of one 16-column chunk from being hoisted
      // above the previous chunk (bounded SGPR use)
      if ((t & 15) == 15) __builtin_amdgcn_sched_barrier(0);
    }
    if (acc < best_d) {
      best_d = acc;
      best_j = j;
    }
  }
}

// Squared distance in FP64 of a register row to a padded LDS row (the
// objective of the chosen centroid; padding contributes exact zeros).
template <int DM>
__device__ __forceinline__ double dist2_f64_row(const float (&x)[DM], const float* __restrict__ c) {
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < DM; ++t) {
    const double e = static_cast<double>(x[t]) - static_cast<double>(c[t]);
    acc = __builtin_fma(e, e, acc);
  }
  return acc;
}

// Squared distance in FP64 by direct differences of FP32 values, FMA in
// dimension order (used where the result steers a random draw).
__device__ __forceinline__ double dist2_f64(const float* __restrict__ a,
                                            const float* __restrict__ b, int d) {
  double acc = 0.0;
  for (int t = 0; t < d; ++t) {
    const double e = static_cast<double>(a[t]) - static_cast<double>(b[t]);
    acc = __builtin_fma(e, e, acc);
  }
  return acc;
}

}  // namespace bm
