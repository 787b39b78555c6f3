// bm_assign_mfma32.hip -- the assignment step (Sec. 2) and objective (Eq. (1))
// for FP32 points on the matrix cores, returning exactly the labels of the
// FP32 direct-difference path (the final pass and kmeans_assign for FP32 X).
//
// For a point x the nearest centroid minimises e(c) = |c|^2 - 2 x.c.  x.c comes
// from v_mfma_f32_16x16x4_f32 (FP32 operands, FP32 accumulation, d products
// in an order of the instruction's choosing), |c|^2 is an FP64 sum rounded to
// FP32.  With u = 2^-24, any summation order of d products (rounded or not)
// is within (d + 1) u' sum |x_t c_t| <= (d + 1) u' |x| |c| of x.c, and the two
// FP32 roundings of |c|^2 and of the subtraction add at most
// u (|c|^2 + |c|^2 + 2 |x| |c|) (u' = u / (1 - (d + 1) u)).  So every computed
// e(c) is within
//     E = (2 d + 8) u |x| cmax + 3 u cmax^2        (cmax = max |c|)
// of the exact value, and the FP32 direct-difference distance the FP32 path
// computes is within F = (d + 3) u (|x| + cmax)^2 of the exact squared
// distance.  Every centroid whose e exceeds the smallest by more than
// B = 2 (E + F) loses to the matrix-core winner in the FP32 path too, so when
// the runner-up is beyond B the winner is the FP32 path's label.  Otherwise
// (rare: ties and near-ties) the point's four lanes recompute the FP32 path's
// distance to every active centroid, in the FP32 kernel's arithmetic and
// order, and take the smallest (lowest index on exact ties).  The bound is
// applied with a 2 % margin and padded norms.
//
// The objective term of a point is its FP64 squared distance to the chosen
// centroid (each of the point's four lanes adds its coordinates' FP64 squared
// differences, the four parts are added), as the FP32 kernel's up to the
// association of the FP64 sum.
//
// Tiling: a wavefront takes 16 kNT points per step and runs every 16-centroid
// tile over them; d is covered in 16-column chunks, each four instructions
// with K = 4.  Lane l holds point l % 16 of a tile and reads its columns
// 16 q + 4 (l / 16) .. + 3 of chunk q as one 16-byte load, so a point's chunk
// is 64 contiguous bytes over its four lanes; instruction kk of chunk q takes
// column 16 q + 4 (l / 16) + kk of lane l, and the centroid operand (LDS,
// stored in the instruction's lane layout) the same column, so each
// instruction's K index is the same column on both sides.  Lane l holds the
// products of centroid rows 4 (l / 16) .. + 3 of each tile with its point; a
// point's best and runner-up are merged over its four lanes.
#include "bm_internal.h"

namespace bm {

namespace {

typedef float f32x4v __attribute__((ext_vector_type(4)));

constexpr int kMaxCT32 = 8;  // centroid tiles (k <= 128)

struct Mfma32Lds {
  size_t atile, c32, cnorm, act, total;
  int ct, kp, ldc;
};

__host__ __device__ inline Mfma32Lds mfma32_lds_plan(int nq, int k) {
  Mfma32Lds p;
  p.ct = (k + 15) / 16;
  p.kp = 16 * p.ct;
  p.ldc = 16 * nq + 4;  // FP32 centroid row stride in floats (16-byte rows, skewed banks)
  p.atile = 0;
  p.c32 = p.atile + sizeof(float) * 64 * 4 * static_cast<size_t>(nq) * p.ct;
  p.cnorm = p.c32 + sizeof(float) * static_cast<size_t>(p.kp) * p.ldc;
  p.act = p.cnorm + sizeof(float) * p.kp;
  p.total = p.act + sizeof(int) * p.kp;
  return p;
}

template <int NQ>
constexpr int nt32_for() { return NQ <= 8 ? 2 : 1; }
constexpr int kMfma32Block = 512;

// Chunk q of point i for this lane: columns 16 q + 4 grp .. + 3.  Rows past n
// read row n - 1 and columns past d read as zeros, so every address is in
// bounds.  VEC: d % 4 == 0 and X 16-byte aligned.
template <int NQ, bool VEC>
__device__ __forceinline__ void load_point(const float* __restrict__ X, int64_t n, int d, int64_t i,
                                           int grp, float4 (&b)[NQ]) {
  const float* row = X + static_cast<size_t>(i < n ? i : n - 1) * d;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t0 = 16 * q + 4 * grp;
    if (VEC) {
      const bool in = t0 < d;
      const float4 v = *reinterpret_cast<const float4*>(row + (in ? t0 : 0));
      b[q] = in ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      float e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + u;
        const float v = row[t < d ? t : d - 1];
        e[u] = t < d ? v : 0.f;
      }
      b[q] = make_float4(e[0], e[1], e[2], e[3]);
    }
  }
}

__device__ __forceinline__ float f4_at(const float4& v, int u) {
  return u == 0 ? v.x : u == 1 ? v.y : u == 2 ? v.z : v.w;
}

// The FP32 path's squared distance of row xr (d columns, global) to the FP32
// centroid row cr (LDS): FMA chain in dimension order, as the FP32 kernel's
// (its zero padding adds exact zeros).
template <bool VEC>
__device__ __forceinline__ float fp32_row_dist(const float* __restrict__ xr, int d,
                                               const float* __restrict__ cr) {
  float acc = 0.f;
  int t = 0;
  if (VEC) {
    for (; t + 4 <= d; t += 4) {
      const float4 v = *reinterpret_cast<const float4*>(xr + t);
      float e = v.x - cr[t];
      acc = __builtin_fmaf(e, e, acc);
      e = v.y - cr[t + 1];
      acc = __builtin_fmaf(e, e, acc);
      e = v.z - cr[t + 2];
      acc = __builtin_fmaf(e, e, acc);
      e = v.w - cr[t + 3];
      acc = __builtin_fmaf(e, e, acc);
    }
  }
  for (; t < d; ++t) {
    const float e = xr[t] - cr[t];
    acc = __builtin_fmaf(e, e, acc);
  }
  return acc;
}

__device__ __forceinline__ double quad_sum64(double v) {
  v += __shfl_xor(v, 16, kWave);
  v += __shfl_xor(v, 32, kWave);
  return v;
}

template <int NQ, bool VEC>
__global__ void __launch_bounds__(kMfma32Block)
    assign_mfma32_kernel(const float* __restrict__ X, int64_t n, int d, const float* __restrict__ C,
                         const uint8_t* __restrict__ deg, int k, int32_t* __restrict__ labels,
                         float* __restrict__ min_d2, double* __restrict__ partial,
                         unsigned long long* __restrict__ rechecked) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const Mfma32Lds P = mfma32_lds_plan(NQ, k);
  const int CT = P.ct;
  const int ldc = P.ldc;
  float* atile = reinterpret_cast<float*>(lds_raw + P.atile);
  float* c32 = reinterpret_cast<float*>(lds_raw + P.c32);
  float* cnorm = reinterpret_cast<float*>(lds_raw + P.cnorm);
  int* act = reinterpret_cast<int*>(lds_raw + P.act);
  constexpr int kWaves = kMfma32Block / kWave;
  constexpr int kNT = nt32_for<NQ>();
  __shared__ float s_cmax;
  __shared__ double s_tmp[kWaves + 1];
  const int tid = threadIdx.x;

  // FP32 centroids (zero rows for inactive or padding slots)
  for (int e = tid; e < P.kp * 16 * NQ; e += kMfma32Block) {
    const int m = e / (16 * NQ);
    const int t = e - m * (16 * NQ);
    const bool live = m < k && !(deg && deg[m]);
    c32[m * ldc + t] = (live && t < d) ? C[static_cast<size_t>(m) * d + t] : 0.f;
  }
  __syncthreads();
  // the A operands in the instruction's lane layout: instruction (ct, q, kk),
  // lane l -> centroid 16 ct + l % 16, column 16 q + 4 (l / 16) + kk
  for (int e = tid; e < CT * NQ * 4 * 64; e += kMfma32Block) {
    const int lane = e & 63;
    const int ins = e >> 6;  // (ct * NQ + q) * 4 + kk
    const int kk = ins & 3;
    const int q = (ins >> 2) % NQ;
    const int ct = (ins >> 2) / NQ;
    atile[e] = c32[(16 * ct + (lane & 15)) * ldc + 16 * q + 4 * (lane >> 4) + kk];
  }
  // |c|^2 (FP64 sum rounded to FP32) and the activity flags
  for (int m = tid; m < P.kp; m += kMfma32Block) {
    const bool live = m < k && !(deg && deg[m]);
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
      const double c = c32[m * ldc + t];
      acc += c * c;
    }
    cnorm[m] = live ? static_cast<float>(acc) : __builtin_inff();
    act[m] = live ? 1 : 0;
  }
  __syncthreads();
  if (tid < kWave) {  // largest centroid norm, padded upwards
    float v = 0.f;
    for (int m = tid; m < P.kp; m += kWave)
      if (act[m]) v = fmaxf(v, sqrtf(cnorm[m]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    if (tid == 0) s_cmax = v * 1.0001f;
  }
  __syncthreads();
  const float cmax = s_cmax;
  const float dd = static_cast<float>(d);
  const float kE1 = (2.f * dd + 8.f) * 0x1.0p-24f;
  const float kE2 = 3.f * 0x1.0p-24f * cmax * cmax;
  const float kF = (dd + 3.f) * 0x1.0p-24f;

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int col = lane & 15;
  const int grp = lane >> 4;
  const int64_t steps = (n + 16 * kNT - 1) / (16 * kNT);
  const int64_t wstride = static_cast<int64_t>(gridDim.x) * kWaves;
  double sse = 0.0;
  unsigned long long nrecheck = 0;

  int64_t step = static_cast<int64_t>(blockIdx.x) * kWaves + wave;
  float4 b[kNT][NQ];
  if (step < steps) {
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt)
      load_point<NQ, VEC>(X, n, d, step * (16 * kNT) + 16 * nt + col, grp, b[nt]);
  }
  for (; step < steps; step += wstride) {
    // the next step's points are loaded while this one is processed
    const int64_t nstep = step + wstride < steps ? step + wstride : step;
    float4 bn[kNT][NQ];
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt)
      load_point<NQ, VEC>(X, n, d, nstep * (16 * kNT) + 16 * nt + col, grp, bn[nt]);

    float b1[kNT], b2[kNT];
    int j1[kNT];
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt) {
      b1[nt] = __builtin_inff();
      b2[nt] = __builtin_inff();
      j1[nt] = -1;
    }
    for (int ct = 0; ct < CT; ++ct) {
      f32x4v acc[kNT];
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt) acc[nt] = f32x4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const float a = atile[((ct * NQ + q) * 4 + kk) * 64 + lane];
#pragma unroll
          for (int nt = 0; nt < kNT; ++nt)
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, f4_at(b[nt][q], kk), acc[nt], 0, 0, 0);
        }
      }
      const float4 cn = *reinterpret_cast<const float4*>(cnorm + 16 * ct + 4 * grp);
      const float cnq[4] = {cn.x, cn.y, cn.z, cn.w};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 16 * ct + 4 * grp + r;
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
          // keep b1 <= b2 the two smallest; the median of three is the new
          // runner-up, and j1 moves only on a strict improvement (ascending m)
          const float e = __builtin_fmaf(-2.0f, acc[nt][r], cnq[r]);
          const bool lt = e < b1[nt];
          j1[nt] = lt ? m : j1[nt];
          b2[nt] = __builtin_amdgcn_fmed3f(b1[nt], b2[nt], e);
          b1[nt] = lt ? e : b1[nt];
        }
      }
    }
    // merge best / runner-up over the four lanes of each point, the winner's
    // FP64 distance and |x|^2, and the decision to recheck
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt) {
      const int64_t i = step * (16 * kNT) + 16 * nt + col;
      const bool valid = i < n;
#pragma unroll
      for (int off = 16; off <= 32; off <<= 1) {
        const float ob1 = __shfl_xor(b1[nt], off, kWave);
        const float ob2 = __shfl_xor(b2[nt], off, kWave);
        const int oj1 = __shfl_xor(j1[nt], off, kWave);
        const bool other = ob1 < b1[nt] ||
                           (ob1 == b1[nt] && static_cast<unsigned>(oj1) < static_cast<unsigned>(j1[nt]));
        b2[nt] = other ? fminf(b1[nt], ob2) : fminf(b2[nt], ob1);
        b1[nt] = other ? ob1 : b1[nt];
        j1[nt] = other ? oj1 : j1[nt];
      }
      int w = j1[nt];
      // this lane's share of |x|^2 (FP32, for the error bound only)
      float xx = 0.f;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) xx = __builtin_fmaf(f4_at(b[nt][q], u), f4_at(b[nt][q], u), xx);
      xx += __shfl_xor(xx, 16, kWave);
      xx += __shfl_xor(xx, 32, kWave);
      const float xn = sqrtf(xx) * 1.001f;
      const float band = 2.02f * (kE1 * xn * cmax + kE2 + kF * (xn + cmax) * (xn + cmax));
      // NaN-safe: anything but a clear margin is rechecked
      const bool rchk = valid && !(b2[nt] - b1[nt] > band);
      if (__ballot(rchk)) {
        // the FP32 path's distance to every active centroid: lane grp takes
        // rows 4 grp .. + 3 of each tile (ascending), the four lanes merge;
        // the FP32 path's rule is the smallest distance, NaN never winning
        // and the lowest index on ties (the first active slot when nothing
        // is below +inf), i.e. the smallest (key, index) with key(NaN) = +inf
        const float* xr = X + static_cast<size_t>(valid ? i : 0) * d;
        float best = __builtin_inff();
        int bj = -1;
        if (rchk) {
          for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int m = 16 * ct + 4 * grp + r;
              if (act[m]) {
                const float v = fp32_row_dist<VEC>(xr, d, c32 + m * ldc);
                const float key = v == v ? v : __builtin_inff();
                if (bj < 0 || key < best) {
                  best = key;
                  bj = m;
                }
              }
            }
          }
        }
#pragma unroll
        for (int off = 16; off <= 32; off <<= 1) {
          const float ob = __shfl_xor(best, off, kWave);
          const int oj = __shfl_xor(bj, off, kWave);
          if (oj >= 0 && (bj < 0 || ob < best ||
                          (ob == best && static_cast<unsigned>(oj) < static_cast<unsigned>(bj)))) {
            best = ob;
            bj = oj;
          }
        }
        if (rchk) {
          w = bj;
          if (grp == 0) ++nrecheck;
        }
      }
      // the winner's FP64 squared distance: this lane's columns, then the four parts
      double part = 0.0;
      const float* cw = c32 + (w >= 0 ? w : 0) * ldc;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const float4 cv = *reinterpret_cast<const float4*>(cw + 16 * q + 4 * grp);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double e = static_cast<double>(f4_at(b[nt][q], u)) - static_cast<double>(f4_at(cv, u));
          part = __builtin_fma(e, e, part);
        }
      }
      part = quad_sum64(part);
      if (valid && grp == 0) {
        const double pv = w >= 0 ? part : __builtin_nan("");
        if (labels) labels[i] = w;
        if (min_d2) min_d2[i] = static_cast<float>(pv);
        sse += pv;
      }
    }
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
      for (int q = 0; q < NQ; ++q) b[nt][q] = bn[nt][q];
  }
  if (rechecked && nrecheck) atomicAdd(rechecked, nrecheck);
  const double bsum = block_sum_f64<kMfma32Block>(sse, s_tmp);
  // the partials are added in workgroup order by sum_partials_kernel, launched
  // after this kernel (no fence and atomic per workgroup)
  if (tid == 0) partial[blockIdx.x] = bsum;
}

// The batched Lloyd assignment (the work list, solve states and accumulation
// of batch_assign_kernel in bm_batch.hip) with the labels from the matrix
// cores: rows are the zero-padded copies (row stride dm = padded d), a
// workgroup stages each solve's centroids (FP32 rows, the lane-layout operand
// tiles, norms and flags) when its tile list reaches the solve, and for every
// labelled row the point's four lanes add their coordinates' FP64 values to
// the solve's cluster sums and their FP64 squared differences to the tile's
// objective, so sums, counts and objectives are those of the VALU kernel up
// to the association of FP64 sums.
constexpr int kBM32Block = 256;

template <int NQ, bool SUMS_LDS>
__global__ void __launch_bounds__(kBM32Block)
    batch_assign_mfma32_kernel(const float* __restrict__ Pp, int dm, int d, const float* __restrict__ C,
                               const uint8_t* __restrict__ deg, const BatchSolve* __restrict__ sv,
                               const int32_t* __restrict__ tile_solve, int ntiles, int tile_rows,
                               int kmax, double* __restrict__ sums, int32_t* __restrict__ cnt,
                               double* __restrict__ tile_f, int32_t* __restrict__ labels, int dry) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const Mfma32Lds P = mfma32_lds_plan(NQ, kmax);
  const int ldc = P.ldc;
  const int lds_ld = dm + 1;  // cluster-sum row stride in LDS (odd)
  float* atile = reinterpret_cast<float*>(lds_raw + P.atile);
  float* c32 = reinterpret_cast<float*>(lds_raw + P.c32);
  float* cnorm = reinterpret_cast<float*>(lds_raw + P.cnorm);
  int* act = reinterpret_cast<int*>(lds_raw + P.act);
  int* cnt_l = act + P.kp;
  double* sums_l = reinterpret_cast<double*>(lds_raw + ((P.total + sizeof(int) * P.kp + 15) & ~size_t(15)));
  constexpr int kWaves = kBM32Block / kWave;
  constexpr int kNT = nt32_for<NQ>();
  __shared__ int s_j, s_k, s_c0, s_status, s_tile0;
  __shared__ int64_t s_row0, s_s;
  __shared__ float s_cmax;
  __shared__ double s_tmp[kWaves + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int col = lane & 15;
  const int grp = lane >> 4;
  const float dd = static_cast<float>(d);
  const float kE1 = (2.f * dd + 8.f) * 0x1.0p-24f;
  const float kF = (dd + 3.f) * 0x1.0p-24f;

  int cur = -1;          // solve whose centroids are staged
  bool cur_acc = false;  // ... and whose sums are being accumulated
  int cur_k = 0, cur_c0 = 0;
  auto flush = [&]() {  // this workgroup's LDS sums and counts of solve `cur`
    __syncthreads();
    if (SUMS_LDS) {
      for (int e = tid; e < cur_k * d; e += kBM32Block) {
        const int j = e / d;
        const int t = e - j * d;
        if (cnt_l[j]) unsafeAtomicAdd(&sums[static_cast<size_t>(cur_c0 + j) * dm + t], sums_l[j * lds_ld + t]);
      }
    }
    for (int j = tid; j < cur_k; j += kBM32Block)
      if (cnt_l[j]) atomicAdd(&cnt[cur_c0 + j], cnt_l[j]);
    __syncthreads();
  };

  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    if (tid == 0) {
      const int j = tile_solve[t];
      const BatchSolve S = sv[j];
      s_j = j;
      s_k = S.k;
      s_c0 = S.c0;
      s_status = S.status;
      s_tile0 = S.tile0;
      s_row0 = S.row0;
      s_s = S.s;
    }
    __syncthreads();
    const int status = s_status;
    if (status == kSolveDone) {
      __syncthreads();
      continue;
    }
    const int k = s_k;
    const int c0 = s_c0;
    const int CT = (k + 15) / 16;
    const bool accumulate = status == kSolveRunning && !dry;
    if (s_j != cur) {
      if (cur_acc) flush();
      cur = s_j;
      cur_acc = accumulate;
      cur_k = k;
      cur_c0 = c0;
      const int kp = 16 * CT;
      for (int e = tid; e < kp * 16 * NQ; e += kBM32Block) {
        const int m = e / (16 * NQ);
        const int tt = e - m * (16 * NQ);
        const bool live = m < k && !deg[c0 + m];
        c32[m * ldc + tt] = (live && tt < d) ? C[static_cast<size_t>(c0 + m) * d + tt] : 0.f;
      }
      for (int j = tid; j < kp; j += kBM32Block) cnt_l[j] = 0;
      if (SUMS_LDS && accumulate)
        for (int e = tid; e < k * lds_ld; e += kBM32Block) sums_l[e] = 0.0;
      __syncthreads();
      for (int e = tid; e < CT * NQ * 4 * 64; e += kBM32Block) {
        const int ln = e & 63;
        const int ins = e >> 6;
        const int kk = ins & 3;
        const int q = (ins >> 2) % NQ;
        const int ct = (ins >> 2) / NQ;
        atile[e] = c32[(16 * ct + (ln & 15)) * ldc + 16 * q + 4 * (ln >> 4) + kk];
      }
      for (int m = tid; m < kp; m += kBM32Block) {
        const bool live = m < k && !deg[c0 + m];
        double acc = 0.0;
        for (int tt = 0; tt < d; ++tt) {
          const double c = c32[m * ldc + tt];
          acc += c * c;
        }
        cnorm[m] = live ? static_cast<float>(acc) : __builtin_inff();
        act[m] = live ? 1 : 0;
      }
      __syncthreads();
      if (tid < kWave) {
        float v = 0.f;
        for (int m = tid; m < kp; m += kWave)
          if (act[m]) v = fmaxf(v, sqrtf(cnorm[m]));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
        if (tid == 0) s_cmax = v * 1.0001f;
      }
      __syncthreads();
    }
    const float cmax = s_cmax;
    const float kE2 = 3.f * 0x1.0p-24f * cmax * cmax;
    const int64_t r0 = s_row0 + static_cast<int64_t>(t - s_tile0) * tile_rows;
    const int64_t rend = s_row0 + s_s;
    const int64_t r1 = r0 + tile_rows < rend ? r0 + tile_rows : rend;
    const int64_t nsteps = (r1 - r0 + 16 * kNT - 1) / (16 * kNT);
    double* sums_dst = SUMS_LDS ? sums_l : sums + static_cast<size_t>(c0) * dm;
    const int sld = SUMS_LDS ? lds_ld : dm;
    double f = 0.0;
    for (int64_t step = wave; step < nsteps; step += kWaves) {
      float4 b[kNT][NQ];
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt) {
        const int64_t i = r0 + step * (16 * kNT) + 16 * nt + col;
        const float* row = Pp + static_cast<size_t>(i < r1 ? i : r1 - 1) * dm;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int t0 = 16 * q + 4 * grp;
          const bool in = t0 < dm;  // rows are dm wide (a multiple of 4), zero padded past d
          const float4 v = *reinterpret_cast<const float4*>(row + (in ? t0 : 0));
          b[nt][q] = in ? v : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
      float b1[kNT], b2[kNT];
      int j1[kNT];
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt) {
        b1[nt] = __builtin_inff();
        b2[nt] = __builtin_inff();
        j1[nt] = -1;
      }
      for (int ct = 0; ct < CT; ++ct) {
        f32x4v acc[kNT];
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) acc[nt] = f32x4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const float a = atile[((ct * NQ + q) * 4 + kk) * 64 + lane];
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt)
              acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, f4_at(b[nt][q], kk), acc[nt], 0, 0, 0);
          }
        }
        const float4 cn = *reinterpret_cast<const float4*>(cnorm + 16 * ct + 4 * grp);
        const float cnq[4] = {cn.x, cn.y, cn.z, cn.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = 16 * ct + 4 * grp + r;
#pragma unroll
          for (int nt = 0; nt < kNT; ++nt) {
            const float e = __builtin_fmaf(-2.0f, acc[nt][r], cnq[r]);
            const bool lt = e < b1[nt];
            j1[nt] = lt ? m : j1[nt];
            b2[nt] = __builtin_amdgcn_fmed3f(b1[nt], b2[nt], e);
            b1[nt] = lt ? e : b1[nt];
          }
        }
      }
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt) {
        const int64_t i = r0 + step * (16 * kNT) + 16 * nt + col;
        const bool valid = i < r1;
#pragma unroll
        for (int off = 16; off <= 32; off <<= 1) {
          const float ob1 = __shfl_xor(b1[nt], off, kWave);
          const float ob2 = __shfl_xor(b2[nt], off, kWave);
          const int oj1 = __shfl_xor(j1[nt], off, kWave);
          const bool other = ob1 < b1[nt] ||
                             (ob1 == b1[nt] && static_cast<unsigned>(oj1) < static_cast<unsigned>(j1[nt]));
          b2[nt] = other ? fminf(b1[nt], ob2) : fminf(b2[nt], ob1);
          b1[nt] = other ? ob1 : b1[nt];
          j1[nt] = other ? oj1 : j1[nt];
        }
        int w = j1[nt];
        float xx = 0.f;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int u = 0; u < 4; ++u) xx = __builtin_fmaf(f4_at(b[nt][q], u), f4_at(b[nt][q], u), xx);
        xx += __shfl_xor(xx, 16, kWave);
        xx += __shfl_xor(xx, 32, kWave);
        const float xn = sqrtf(xx) * 1.001f;
        const float band = 2.02f * (kE1 * xn * cmax + kE2 + kF * (xn + cmax) * (xn + cmax));
        const bool rchk = valid && !(b2[nt] - b1[nt] > band);
        if (__ballot(rchk)) {
          // the FP32 path's distance to every active centroid (see the
          // full-data kernel above)
          const float* xr = Pp + static_cast<size_t>(valid ? i : r0) * dm;
          float best = __builtin_inff();
          int bj = -1;
          if (rchk) {
            for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int m = 16 * ct + 4 * grp + r;
                if (act[m]) {
                  const float v = fp32_row_dist<true>(xr, d, c32 + m * ldc);
                  const float key = v == v ? v : __builtin_inff();
                  if (bj < 0 || key < best) {
                    best = key;
                    bj = m;
                  }
                }
              }
            }
          }
#pragma unroll
          for (int off = 16; off <= 32; off <<= 1) {
            const float ob = __shfl_xor(best, off, kWave);
            const int oj = __shfl_xor(bj, off, kWave);
            if (oj >= 0 && (bj < 0 || ob < best ||
                            (ob == best && static_cast<unsigned>(oj) < static_cast<unsigned>(bj)))) {
              best = ob;
              bj = oj;
            }
          }
          if (rchk) w = bj;
        }
        if (valid && w >= 0) {
          if (labels && !dry && grp == 0) labels[i] = w;
          // the winner's FP64 squared distance (this lane's columns) and,
          // when accumulating, the FP64 cluster sums and the count
          const float* cw = c32 + w * ldc;
          double part = 0.0;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const float4 cv = *reinterpret_cast<const float4*>(cw + 16 * q + 4 * grp);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int tc = 16 * q + 4 * grp + u;
              const double xv = static_cast<double>(f4_at(b[nt][q], u));
              const double e = xv - static_cast<double>(f4_at(cv, u));
              part = __builtin_fma(e, e, part);
              if (accumulate && tc < d) unsafeAtomicAdd(sums_dst + w * sld + tc, xv);
            }
          }
          f += part;
          if (accumulate && grp == 0) atomicAdd(&cnt_l[w], 1);
        }
      }
    }
    const double ft = block_sum_f64<kBM32Block>(f, s_tmp);
    if (tid == 0) tile_f[t] = ft;
    __syncthreads();
  }
  if (cur_acc) flush();
}

int mfma32_nq(int d) {
  return d <= 16 ? 1 : d <= 32 ? 2 : d <= 64 ? 4 : d <= 80 ? 5 : d <= 128 ? 8 : 16;
}

template <int NQ>
const void* mfma32_fn(bool vec) {
  return vec ? reinterpret_cast<const void*>(&assign_mfma32_kernel<NQ, true>)
             : reinterpret_cast<const void*>(&assign_mfma32_kernel<NQ, false>);
}

const void* pick_mfma32(int nq, bool vec) {
  switch (nq) {
    case 1: return mfma32_fn<1>(vec);
    case 2: return mfma32_fn<2>(vec);
    case 4: return mfma32_fn<4>(vec);
    case 5: return mfma32_fn<5>(vec);
    case 8: return mfma32_fn<8>(vec);
    case 16: return mfma32_fn<16>(vec);
    default: return nullptr;
  }
}

bool mfma32_vec(const void* X, int d) {
  return (d & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
}

}  // namespace

bm_status plan_assign_mfma32(const void* X, int64_t n, int d, int k, int* grid) {
  if (d < 1 || d > 256)
    return set_error(BM_ENOTSUP, "FP32 MFMA assignment supports 1 <= d <= 256 (d = %d)", d);
  if (k < 1 || k > 16 * kMaxCT32)
    return set_error(BM_ENOTSUP, "FP32 MFMA assignment supports k <= %d (k = %d)", 16 * kMaxCT32, k);
  const int nq = mfma32_nq(d);
  const size_t lds = mfma32_lds_plan(nq, k).total;
  size_t lds_max = 0;
  bm_status st = max_lds_per_block(&lds_max);
  if (st != BM_OK) return st;
  if (lds + 1024 > lds_max)
    return set_error(BM_ENOTSUP, "k*d = %d*%d centroids do not fit in LDS for FP32 MFMA", k, d);
  const bool vec = mfma32_vec(X, d);
  const void* fn = pick_mfma32(nq, vec);
  if (bm_status sr = reserve_lds(fn, lds)) return sr;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kMfma32Block, lds) != hipSuccess)
    return set_error(BM_EDEVICE, "cannot query the device for the FP32 MFMA assignment plan");
  if (per_cu < 1 || cus < 1) return set_error(BM_ENOTSUP, "FP32 MFMA assignment kernel cannot be resident");
  const int pts = 16 * (nq <= 8 ? 2 : 1) * (kMfma32Block / kWave);  // points per workgroup step
  const int64_t want = (n + pts - 1) / pts;
  const int64_t cap = static_cast<int64_t>(cus) * per_cu;
  const int64_t g = want < cap ? want : cap;
  *grid = static_cast<int>(g < 1 ? 1 : g);
  return BM_OK;
}

bm_status launch_assign_mfma32(const float* X, int64_t n, int d, const float* C, const uint8_t* deg_dev,
                               int k, int32_t* labels, float* min_d2, double* partial,
                               double* sse_dev, unsigned long long* rechecked, int grid,
                               hipStream_t stream) {
  const int nq = mfma32_nq(d);
  if (grid < 1 || n < 1 || d < 1 || d > 256 || k < 1 || k > 16 * kMaxCT32)
    return set_error(BM_EINVAL, "FP32 MFMA assignment: bad plan");
  const void* fn = pick_mfma32(nq, mfma32_vec(X, d));
  const size_t lds = mfma32_lds_plan(nq, k).total;
  void* args[] = {const_cast<float**>(&X), &n, &d, const_cast<float**>(&C),
                  const_cast<uint8_t**>(&deg_dev), &k, &labels, &min_d2, &partial, &rechecked};
  const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kMfma32Block), args, lds, stream);
  if (e != hipSuccess)
    return set_error(BM_EDEVICE, "FP32 MFMA assign launch failed: %s", hipGetErrorString(e));
  return launch_sum_partials(partial, grid, sse_dev, stream);
}

size_t batch_assign_mfma32_lds(int d, int kmax, bool sums_lds) {
  if (d < 1 || d > 256 || kmax < 1 || kmax > 16 * kMaxCT32) return ~size_t(0);
  const Mfma32Lds P = mfma32_lds_plan(mfma32_nq(d), kmax);
  size_t b = (P.total + sizeof(int) * P.kp + 15) & ~size_t(15);
  if (sums_lds) b += sizeof(double) * static_cast<size_t>(kmax) * (padded_dim(d) + 1);
  return b;
}

namespace {
template <int NQ, bool SUMS_LDS>
const void* bm32_fn() {
  return reinterpret_cast<const void*>(&batch_assign_mfma32_kernel<NQ, SUMS_LDS>);
}
template <bool SUMS_LDS>
const void* pick_bm32(int nq) {
  switch (nq) {
    case 1: return bm32_fn<1, SUMS_LDS>();
    case 2: return bm32_fn<2, SUMS_LDS>();
    case 4: return bm32_fn<4, SUMS_LDS>();
    case 5: return bm32_fn<5, SUMS_LDS>();
    case 8: return bm32_fn<8, SUMS_LDS>();
    case 16: return bm32_fn<16, SUMS_LDS>();
    default: return nullptr;
  }
}
}  // namespace

bm_status launch_batch_assign_mfma32(const float* Pp, int d, const float* C, const uint8_t* deg,
                                     const BatchSolve* sv, const int32_t* tile_solve, int ntiles,
                                     int tile_rows, int kmax, bool sums_lds, double* sums,
                                     int32_t* cnt, double* tile_f, int32_t* labels, int dry,
                                     hipStream_t stream) {
  const int nq = mfma32_nq(d);
  const void* fn = sums_lds ? pick_bm32<true>(nq) : pick_bm32<false>(nq);
  const size_t lds = batch_assign_mfma32_lds(d, kmax, sums_lds);
  if (!fn || lds == ~size_t(0)) return set_error(BM_EINVAL, "batched FP32 MFMA assignment: bad plan");
  static_assert(kBM32Block == 256, "one workgroup size for the plan below");
  if (bm_status sr = reserve_lds(fn, lds)) return sr;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBM32Block, lds) != hipSuccess || per_cu < 1)
    return set_error(BM_EDEVICE, "cannot plan the batched FP32 MFMA assignment");
  int grid = cus * per_cu;
  if (grid > ntiles) grid = ntiles;
  if (grid < 1) return BM_OK;
  int dm = padded_dim(d);
  void* args[] = {const_cast<float**>(&Pp), &dm, &d, const_cast<float**>(&C), const_cast<uint8_t**>(&deg),
                  const_cast<BatchSolve**>(&sv), const_cast<int32_t**>(&tile_solve), &ntiles, &tile_rows,
                  &kmax, &sums, &cnt, &tile_f, &labels, &dry};
  const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kBM32Block), args, lds, stream);
  if (e != hipSuccess)
    return set_error(BM_EDEVICE, "batched FP32 MFMA assign launch failed: %s", hipGetErrorString(e));
  return BM_OK;
}

}  // namespace bm
