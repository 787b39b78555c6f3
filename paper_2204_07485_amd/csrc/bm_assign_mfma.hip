// bm_assign_mfma.hip -- the assignment step (Sec. 2) and objective (Eq. (1))
// for BF16 points on the matrix cores, returning exactly the labels of the
// FP32 direct-difference path.
//
// For a point x the nearest centroid minimises e(c) = |c|^2 - 2 x.c.  x is BF16
// (exact); every FP32 centroid is split into two BF16 parts (round to
// nearest each), c = c_hi + c_lo + r with |r| <= 2^-16 |c| per coordinate, and
// x.c_hi + x.c_lo comes from v_mfma_f32_16x16x32_bf16 (exact BF16 products,
// FP32 accumulation).  Counting at most 2d + 2 KS + 6 roundings of 2^-23 on
// any product's path through the accumulation (serial or tree order inside the
// instruction, 2 KS chained instructions), |c_hi| + |c_lo| <= 1.008 |c|,
// 2 |x.r| <= 2^-15 |x| |c|, and the FP32 rounding of |c|^2 and of the final
// subtraction, the error of every computed e(c) for d <= 256 is below
//     E = ((4.05 d + 64) 2^-23 + 2^-15) |x| cmax + 2^-22 cmax^2   (cmax = max |c|)
// and the FP32 direct-difference distance the FP32 path computes is within
//     F = (d + 3) 2^-24 (|x| + cmax)^2
// of the exact squared distance.  So every centroid whose e exceeds the
// smallest by more than B = 2 (E + F) loses to the MFMA winner in the FP32 path
// too, and when the runner-up is beyond B the MFMA winner is the FP32 path's
// label.  Otherwise (rare: ties and near-ties) the wavefront recomputes the
// FP32 path's distance for the candidates within B of the minimum, in the same
// arithmetic and order as the FP32 kernel, and takes the smallest (lowest index
// on exact ties).
//
// The objective term of a point is its squared distance to the chosen
// centroid by direct differences: FP32 sums of 8 squared FP32 differences
// (relative error below 10 2^-24 each), added in FP64, so every term and the
// objective are within 6e-7 relative of the exact values.
//
// Tiling: a wavefront takes 32 points (two 16-point MFMA tiles) at a time and
// runs every 16-centroid tile over both, so each centroid operand read from
// LDS serves 32 points; the next 32 points' operands are loaded while these
// are processed.  The split centroids sit in LDS in the exact register layout
// of the instruction's A operand (16 bytes per lane, conflict-free); the points
// are the B operand, 16 bytes per lane straight from X.  Lane l holds point
// l % 16 of a tile and centroid rows 4 (l / 16) .. + 3 of every centroid tile;
// a point's best and runner-up are merged over its 4 lanes.
#include "bm_internal.h"

namespace bm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxCT = 8;  // centroid tiles (k <= 128)

union Pack8 {
  uint4 u;
  bf16x8 v;
  uint16_t h[8];
};

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// Element q of a packed group of 8 BF16 values, widened exactly to FP32.
__device__ __forceinline__ float bf16_at(const Pack8& p, int q) {
  const uint32_t w = (q & 1) ? (reinterpret_cast<const uint32_t*>(&p.u)[q >> 1] & 0xFFFF0000u)
                             : (reinterpret_cast<const uint32_t*>(&p.u)[q >> 1] << 16);
  return __uint_as_float(w);
}

// LDS layout of one workgroup (byte offsets); shared with the host sizing.
struct MfmaLds {
  size_t atile, c32, cnorm, act, total;
  int ct, kp, ldc;
};

__host__ __device__ inline MfmaLds mfma_lds_plan(int ks, int k) {
  MfmaLds p;
  p.ct = (k + 15) / 16;
  p.kp = 16 * p.ct;
  p.ldc = 32 * ks + 4;  // FP32 centroid row stride in floats (16-byte aligned, skewed banks)
  p.atile = 0;
  p.c32 = p.atile + sizeof(uint4) * 2 * 64 * static_cast<size_t>(ks) * p.ct;
  p.cnorm = p.c32 + sizeof(float) * static_cast<size_t>(p.kp) * p.ldc;
  p.act = p.cnorm + sizeof(float) * p.kp;
  p.total = p.act + sizeof(int) * p.kp;
  return p;
}

// B operand of one 16-point tile: columns 32 ks + 8 grp .. + 7 of row i.
// Rows past n read row n - 1 and columns past d read as zeros, so every
// address is in bounds and no lane branches.  VEC: d % 8 == 0 and X 16-byte
// aligned.
template <int KS, bool VEC>
__device__ __forceinline__ void load_tile_b(const uint16_t* __restrict__ X, int64_t n, int d,
                                            int64_t i, int grp, Pack8 (&b)[KS]) {
  const uint16_t* row = X + static_cast<size_t>(i < n ? i : n - 1) * d;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int t0 = 32 * ks + 8 * grp;
    if (VEC) {
      const bool in = t0 < d;
      const uint4 v = *reinterpret_cast<const uint4*>(row + (in ? t0 : 0));
      b[ks].u.x = in ? v.x : 0u;
      b[ks].u.y = in ? v.y : 0u;
      b[ks].u.z = in ? v.z : 0u;
      b[ks].u.w = in ? v.w : 0u;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int t = t0 + q;
        const uint16_t v = row[t < d ? t : d - 1];
        b[ks].h[q] = t < d ? v : static_cast<uint16_t>(0);
      }
    }
  }
}

// FP32 direct-difference squared distance in dimension order, bit-identical to
// the FP32 assignment kernel's (its zero padding adds exact zeros).
template <bool VEC>
__device__ __forceinline__ float fp32_path_dist(const uint16_t* __restrict__ xr, int d,
                                                const float* __restrict__ cr) {
  float acc = 0.f;
  int t = 0;
  if (VEC) {
    for (; t + 8 <= d; t += 8) {
      Pack8 p;
      p.u = *reinterpret_cast<const uint4*>(xr + t);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float e = bf16_at(p, q) - cr[t + q];
        acc = __builtin_fmaf(e, e, acc);
      }
    }
  }
  for (; t < d; ++t) {
    const float e = bf16_bits_to_float(xr[t]) - cr[t];
    acc = __builtin_fmaf(e, e, acc);
  }
  return acc;
}

template <int KS>
__device__ __forceinline__ f32x4 centroid_tile_dot(const uint4* __restrict__ atile, int ct, int lane,
                                                   const Pack8 (&b)[KS]) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    Pack8 ah, al;
    ah.u = atile[((ct * KS + ks) * 2 + 0) * 64 + lane];
    al.u = atile[((ct * KS + ks) * 2 + 1) * 64 + lane];
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah.v, b[ks].v, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al.v, b[ks].v, acc, 0, 0, 0);
  }
  return acc;
}

// This lane's share (its 8 KS columns) of a point's squared distance to an
// FP32 centroid row: FP32 sums of 8 squared differences, added in FP64; the
// four lanes of the point add their shares.  Also this lane's share of |x|^2
// (FP32, for the error bound only).
template <int KS>
__device__ __forceinline__ double dist_share(const Pack8 (&b)[KS], const float* __restrict__ cr,
                                             int grp, float& xx) {
  double part = 0.0;
  xx = 0.f;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const float4 c0 = *reinterpret_cast<const float4*>(cr + 32 * ks + 8 * grp);
    const float4 c1 = *reinterpret_cast<const float4*>(cr + 32 * ks + 8 * grp + 4);
    const float c[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
    float g = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float x = bf16_at(b[ks], q);
      const float e = x - c[q];  // padding columns give exact zeros
      g = __builtin_fmaf(e, e, g);
      xx = __builtin_fmaf(x, x, xx);
    }
    part += static_cast<double>(g);
  }
  return part;
}

__device__ __forceinline__ double quad_sum(double v) {
  v += __shfl_xor(v, 16, kWave);
  v += __shfl_xor(v, 32, kWave);
  return v;
}

// 16-point tiles per wavefront step: two (centroid operands shared by 32
// points) while the B operands of both, and of the next step, fit in 128
// VGPRs, with workgroups of 16 wavefronts; otherwise (d > 128, or element-wise
// loads, which hold a register per element) one tile and 8 wavefronts.
template <int KS, bool VEC>
constexpr bool wide_for() { return VEC && KS < 8; }
template <int KS, bool VEC>
constexpr int nt_for() { return wide_for<KS, VEC>() ? 2 : 1; }
template <int KS, bool VEC>
constexpr int block_for() { return wide_for<KS, VEC>() ? 1024 : 512; }

template <int KS, bool VEC>
__global__ void __launch_bounds__((block_for<KS, VEC>()))
    assign_mfma_kernel(const uint16_t* __restrict__ X, int64_t n, int d,
                       const float* __restrict__ C, const uint8_t* __restrict__ deg, int k,
                       int32_t* __restrict__ labels, float* __restrict__ min_d2,
                       double* __restrict__ partial, unsigned long long* __restrict__ rechecked,
                       const int32_t* __restrict__ stop) {
  if (stop && *stop == kSolveDone) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const MfmaLds P = mfma_lds_plan(KS, k);
  const int CT = P.ct;
  const int ldc = P.ldc;
  uint4* atile = reinterpret_cast<uint4*>(lds_raw + P.atile);
  float* c32 = reinterpret_cast<float*>(lds_raw + P.c32);
  float* cnorm = reinterpret_cast<float*>(lds_raw + P.cnorm);
  int* act = reinterpret_cast<int*>(lds_raw + P.act);
  constexpr int kMfmaBlock = block_for<KS, VEC>();
  constexpr int kMfmaWaves = kMfmaBlock / kWave;
  constexpr int kNT = nt_for<KS, VEC>();
  __shared__ float s_cmax;
  __shared__ double s_tmp[kMfmaWaves + 1];
  const int tid = threadIdx.x;

  // FP32 centroids (zero rows for inactive or padding slots)
  for (int e = tid; e < P.kp * 32 * KS; e += kMfmaBlock) {
    const int m = e / (32 * KS);
    const int t = e - m * (32 * KS);
    const bool live = m < k && !(deg && deg[m]);
    c32[m * ldc + t] = (live && t < d) ? C[static_cast<size_t>(m) * d + t] : 0.f;
  }
  __syncthreads();
  // split into BF16 hi + lo parts, in the A-operand lane layout
  for (int e = tid; e < CT * KS * 64; e += kMfmaBlock) {
    const int lane = e & 63;
    const int ks = (e >> 6) % KS;
    const int ct = (e >> 6) / KS;
    const float* src = c32 + (16 * ct + (lane & 15)) * ldc + 32 * ks + 8 * (lane >> 4);
    Pack8 hi, lo;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float c = src[q];
      const uint16_t h = f32_to_bf16_rne(c);
      hi.h[q] = h;
      lo.h[q] = f32_to_bf16_rne(c - bf16_bits_to_float(h));  // c - hi is exact in FP32
    }
    atile[((ct * KS + ks) * 2 + 0) * 64 + lane] = hi.u;
    atile[((ct * KS + ks) * 2 + 1) * 64 + lane] = lo.u;
  }
  // |c|^2 (FP64 sum rounded to FP32) and the activity flags
  for (int m = tid; m < P.kp; m += kMfmaBlock) {
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
  const float kE1 = (4.05f * dd + 64.f) * 0x1.0p-23f + 0x1.0p-15f;
  const float kE2 = 0x1.0p-22f * cmax * cmax;
  const float kF = (dd + 3.f) * 0x1.0p-24f;

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int col = lane & 15;
  const int grp = lane >> 4;
  const int64_t steps = (n + 16 * kNT - 1) / (16 * kNT);
  const int64_t wstride = static_cast<int64_t>(gridDim.x) * kMfmaWaves;
  double sse = 0.0;
  unsigned long long nrecheck = 0;

  // With 16-byte loads the next step's operands are in flight during this
  // one; element-wise loads hold one register per element, so they are
  // issued at the start of their own step instead.
  int64_t step = static_cast<int64_t>(blockIdx.x) * kMfmaWaves + wave;
  Pack8 b[kNT][KS];
  if (VEC && step < steps) {
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt)
      load_tile_b<KS, VEC>(X, n, d, step * (16 * kNT) + 16 * nt + col, grp, b[nt]);
  }
  for (; step < steps; step += wstride) {
    const int64_t nstep = VEC ? (step + wstride < steps ? step + wstride : step) : step;
    Pack8 bn[kNT][KS];
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt)
      load_tile_b<KS, VEC>(X, n, d, nstep * (16 * kNT) + 16 * nt + col, grp, VEC ? bn[nt] : b[nt]);

    float b1[kNT], b2[kNT];
    int j1[kNT];
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt) {
      b1[nt] = __builtin_inff();
      b2[nt] = __builtin_inff();
      j1[nt] = -1;
    }
    for (int ct = 0; ct < CT; ++ct) {
      f32x4 acc[kNT];
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        Pack8 ah, al;
        ah.u = atile[((ct * KS + ks) * 2 + 0) * 64 + lane];
        al.u = atile[((ct * KS + ks) * 2 + 1) * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah.v, b[nt][ks].v, acc[nt], 0, 0, 0);
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al.v, b[nt][ks].v, acc[nt], 0, 0, 0);
        }
      }
      const float4 cn = *reinterpret_cast<const float4*>(cnorm + 16 * ct + 4 * grp);
      const float cnq[4] = {cn.x, cn.y, cn.z, cn.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = 16 * ct + 4 * grp + q;
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
          // keep b1 <= b2 the two smallest; the median of three is the new
          // runner-up, and j1 moves only on a strict improvement (ascending m)
          const float e = __builtin_fmaf(-2.0f, acc[nt][q], cnq[q]);
          const bool lt = e < b1[nt];
          j1[nt] = lt ? m : j1[nt];
          b2[nt] = __builtin_amdgcn_fmed3f(b1[nt], b2[nt], e);
          b1[nt] = lt ? e : b1[nt];
        }
      }
    }
    // epilogue: merge best / runner-up over the four lanes of each point, the
    // winner's distance, the error band, and the decision to recheck
    int win[kNT];
    bool rchk[kNT];
    float lim[kNT];
    double part[kNT];
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt) {
      const bool valid = step * (16 * kNT) + 16 * nt + col < n;
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
      const int w = j1[nt];
      float xx;
      part[nt] = quad_sum(dist_share<KS>(b[nt], c32 + (w >= 0 ? w : 0) * ldc, grp, xx));
      xx += __shfl_xor(xx, 16, kWave);
      xx += __shfl_xor(xx, 32, kWave);
      const float xn = sqrtf(xx) * 1.001f;
      const float band = 2.02f * (kE1 * xn * cmax + kE2 + kF * (xn + cmax) * (xn + cmax));
      // NaN-safe: anything but a clear margin is rechecked
      rchk[nt] = valid && !(b2[nt] - b1[nt] > band);
      lim[nt] = b1[nt] + 1.5f * band;  // extra half band covers the rounding of the sum
      win[nt] = w;
    }
    // rare: recompute e(c) for the tile (operands reloaded, so they need not
    // stay in registers), then the FP32 path's distance of every candidate
    // within the band of the minimum
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt) {
      if (!__ballot(rchk[nt])) continue;
      const int64_t i = step * (16 * kNT) + 16 * nt + col;
      Pack8 br[KS];
      load_tile_b<KS, VEC>(X, n, d, i, grp, br);
      float best = __builtin_inff();
      int bj = -1;
      const uint16_t* xr = X + static_cast<size_t>(rchk[nt] ? i : 0) * d;
      for (int ct = 0; ct < CT; ++ct) {
        const f32x4 acc = centroid_tile_dot<KS>(atile, ct, lane, br);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int m = 16 * ct + 4 * grp + q;
          const float e = __builtin_fmaf(-2.0f, acc[q], cnorm[m]);
          if (rchk[nt] && act[m] && e <= lim[nt]) {
            const float v = fp32_path_dist<VEC>(xr, d, c32 + m * ldc);
            if (v < best) {
              best = v;
              bj = m;
            }
          }
        }
      }
#pragma unroll
      for (int off = 16; off <= 32; off <<= 1) {
        const float ob = __shfl_xor(best, off, kWave);
        const int oj = __shfl_xor(bj, off, kWave);
        if (ob < best || (ob == best && static_cast<unsigned>(oj) < static_cast<unsigned>(bj))) {
          best = ob;
          bj = oj;
        }
      }
      const bool moved = rchk[nt] && bj != win[nt];
      if (__ballot(moved)) {
        float xx_unused;
        const double pv = quad_sum(dist_share<KS>(br, c32 + (bj >= 0 ? bj : 0) * ldc, grp, xx_unused));
        if (moved) part[nt] = pv;
      }
      if (rchk[nt]) {
        win[nt] = bj;
        if (grp == 0) ++nrecheck;
      }
    }
#pragma unroll
    for (int nt = 0; nt < kNT; ++nt) {
      const int64_t i = step * (16 * kNT) + 16 * nt + col;
      if (i < n && grp == 0) {
        const double pv = win[nt] >= 0 ? part[nt] : __builtin_nan("");
        if (labels) labels[i] = win[nt];
        if (min_d2) min_d2[i] = static_cast<float>(pv);
        sse += pv;
      }
    }
    if (VEC) {
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) b[nt][ks] = bn[nt][ks];
    }
  }
  if (rechecked && nrecheck) atomicAdd(rechecked, nrecheck);
  if (!partial) return;
  const double bsum = block_sum_f64<kMfmaBlock>(sse, s_tmp);
  // the partials are added in workgroup order by sum_partials_kernel, launched
  // after this kernel (no fence and atomic per workgroup)
  if (tid == 0) partial[blockIdx.x] = bsum;
}

int mfma_ks(int d) { return d <= 32 ? 1 : d <= 64 ? 2 : d <= 128 ? 4 : 8; }

template <int KS>
const void* mfma_fn(bool vec) {
  return vec ? reinterpret_cast<const void*>(&assign_mfma_kernel<KS, true>)
             : reinterpret_cast<const void*>(&assign_mfma_kernel<KS, false>);
}

const void* pick_mfma(int ks, bool vec) {
  switch (ks) {
    case 1: return mfma_fn<1>(vec);
    case 2: return mfma_fn<2>(vec);
    case 4: return mfma_fn<4>(vec);
    case 8: return mfma_fn<8>(vec);
    default: return nullptr;
  }
}

int mfma_block(int ks, bool vec) { return (vec && ks < 8) ? block_for<1, true>() : block_for<8, true>(); }
int mfma_nt(int ks, bool vec) { return (vec && ks < 8) ? nt_for<1, true>() : nt_for<8, true>(); }

bool mfma_vec(const void* X, int d) {
  return (d & 7) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
}

}  // namespace

bm_status plan_assign_mfma(const void* X, int64_t n, int d, int k, int* grid) {
  if (d < 1 || d > 256)
    return set_error(BM_ENOTSUP, "BF16 MFMA assignment supports 1 <= d <= 256 (d = %d)", d);
  if (k < 1 || k > 16 * kMaxCT)
    return set_error(BM_ENOTSUP, "BF16 MFMA assignment supports k <= %d (k = %d)", 16 * kMaxCT, k);
  const int ks = mfma_ks(d);
  const size_t lds = mfma_lds_plan(ks, k).total;
  size_t lds_max = 0;
  bm_status st = max_lds_per_block(&lds_max);
  if (st != BM_OK) return st;
  if (lds + 1024 > lds_max)
    return set_error(BM_ENOTSUP, "k*d = %d*%d split centroids do not fit in LDS for BF16 MFMA", k, d);
  const void* fn = pick_mfma(ks, mfma_vec(X, d));
  if (bm_status sr = reserve_lds(fn, lds)) return sr;
  int dev = 0, cus = 0, per_cu = 0;
  const bool vec = mfma_vec(X, d);
  const int block = mfma_block(ks, vec);
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess)
    return set_error(BM_EDEVICE, "cannot query the device for the MFMA assignment plan");
  if (per_cu < 1 || cus < 1) return set_error(BM_ENOTSUP, "MFMA assignment kernel cannot be resident");
  const int pts = 16 * mfma_nt(ks, vec) * (block / kWave);  // points per workgroup step
  const int64_t want = (n + pts - 1) / pts;
  const int64_t cap = static_cast<int64_t>(cus) * per_cu;
  const int64_t g = want < cap ? want : cap;
  *grid = static_cast<int>(g < 1 ? 1 : g);
  return BM_OK;
}

bm_status launch_assign_mfma(const uint16_t* X, int64_t n, int d, const float* C,
                             const uint8_t* deg_dev, int k, int32_t* labels, float* min_d2,
                             double* partial, double* sse_dev, unsigned long long* rechecked,
                             int grid, hipStream_t stream, const int32_t* stop) {
  const int ks = mfma_ks(d);
  if (grid < 1 || n < 1 || d < 1 || d > 256 || k < 1 || k > 16 * kMaxCT)
    return set_error(BM_EINVAL, "MFMA assignment: bad plan");
  const void* fn = pick_mfma(ks, mfma_vec(X, d));
  const size_t lds = mfma_lds_plan(ks, k).total;
  void* args[] = {const_cast<uint16_t**>(&X), &n, &d, const_cast<float**>(&C),
                  const_cast<uint8_t**>(&deg_dev), &k, &labels, &min_d2, &partial,
                  &rechecked, const_cast<int32_t**>(&stop)};
  const hipError_t e =
      hipLaunchKernel(fn, dim3(grid), dim3(mfma_block(ks, mfma_vec(X, d))), args, lds, stream);
  if (e != hipSuccess)
    return set_error(BM_EDEVICE, "MFMA assign launch failed: %s", hipGetErrorString(e));
  return partial ? launch_sum_partials(partial, grid, sse_dev, stream) : BM_OK;
}

}  // namespace bm
