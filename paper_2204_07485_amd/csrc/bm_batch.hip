// bm_batch.hip -- K-means (Lloyd, Sec. 2) on many independent problems at
// once: the batched form of the local search that parallel Big-means workers
// run on their own samples (Sec. 3.6), one assignment + update round of every
// unfinished problem per graph launch.
//
// Problems ("solves") are concatenated: solve j owns rows row0 .. row0 + s - 1
// of P and centroid rows c0 .. c0 + k - 1 of C.  A round is two kernels:
//   batch_assign  -- a grid-stride loop over a work list of row tiles (a tile
//                    never spans two solves): stage the tile's solve's
//                    centroids in LDS, assign each row to its nearest active
//                    centroid (FP32 direct differences in dimension order,
//                    exact ties to the lowest index, the same arithmetic as the
//                    single-problem kernels), write its FP64 distance into the
//                    tile's objective partial, and accumulate FP64 cluster sums
//                    and counts (LDS, then one atomic per centroid coordinate);
//   batch_update  -- one workgroup per solve: add its tile partials in tile
//                    order (the objective), then take the stop decisions of
//                    the single-problem Lloyd in the same order: relative
//                    objective rule before the update, new FP64 means (empty
//                    clusters turn degenerate, Sec. 3.3), shift rule and the
//                    iteration cap after it, and one last assignment pass when
//                    the loop ends without the objective rule.
// Finished solves' tiles return at once, so late rounds cost little.
#include "bm_internal.h"

namespace bm {

namespace {

constexpr int kBatchBlock = 256;

// Cluster sums are kept DM wide (the zero padding of the rows adds exact
// zeros), so the unrolled accumulation needs no per-column guard; in LDS the
// row stride is DM + 1 (odd, spreading rows over the banks).
template <int DM>
__device__ __forceinline__ constexpr int batch_sums_ld() { return DM + 1; }

template <int DM, bool SUMS_LDS>
__global__ void __launch_bounds__(kBatchBlock)
    batch_assign_kernel(const float* __restrict__ Pp, int d, const float* __restrict__ C,
                        const float* __restrict__ Cpad, const uint8_t* __restrict__ deg,
                        const BatchSolve* __restrict__ sv,
                        const int32_t* __restrict__ tile_solve, int ntiles, int tile_rows,
                        double* __restrict__ sums, int32_t* __restrict__ cnt,
                        double* __restrict__ tile_f, int32_t* __restrict__ labels, int dry,
                        const int32_t* __restrict__ labels_in) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int s_k, s_na, s_c0, s_status, s_tile0;
  __shared__ int64_t s_row0, s_s;
  __shared__ double s_tmp[kBatchBlock / kWave + 1];
  const int tid = threadIdx.x;

  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    if (tid == 0) {
      const int j = tile_solve[t];
      const BatchSolve S = sv[j];
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
    const bool accumulate = status == kSolveRunning && !dry;
    float* Cl = reinterpret_cast<float*>(lds_raw);
    int* act = reinterpret_cast<int*>(lds_raw + sizeof(float) * static_cast<size_t>(k) * DM);
    int* cnt_l = act + k;
    double* sums_l = reinterpret_cast<double*>(
        lds_raw + ((sizeof(float) * static_cast<size_t>(k) * DM + sizeof(int) * 2 * k + 15) & ~size_t(15)));
    constexpr int ld = batch_sums_ld<DM>();
    for (int e = tid; e < k * DM; e += kBatchBlock) {
      const int j = e / DM;
      const int tdim = e - j * DM;
      Cl[e] = (tdim < d) ? C[static_cast<size_t>(c0 + j) * d + tdim] : 0.f;
    }
    for (int j = tid; j < k; j += kBatchBlock) {
      act[j] = deg[c0 + j] ? 1 : 0;
      cnt_l[j] = 0;
    }
    if (SUMS_LDS && accumulate)
      for (int e = tid; e < k * ld; e += kBatchBlock) sums_l[e] = 0.0;
    __syncthreads();
    if (tid == 0) {  // compact the active slots in place, ascending
      int na = 0;
      for (int j = 0; j < k; ++j)
        if (!act[j]) act[na++] = j;
      s_na = na;
    }
    __syncthreads();
    const int na = s_na;
    const int64_t r0 = s_row0 + static_cast<int64_t>(t - s_tile0) * tile_rows;
    const int64_t rend = s_row0 + s_s;
    const int64_t r1 = r0 + tile_rows < rend ? r0 + tile_rows : rend;
    double f = 0.0;
    for (int64_t i = r0 + tid; i < r1; i += kBatchBlock) {
      float x[DM];
      {  // rows are DM wide and zero padded: 16-byte loads, no column guard
        const float4* r4 = reinterpret_cast<const float4*>(Pp + static_cast<size_t>(i) * DM);
#pragma unroll
        for (int q = 0; q < DM / 4; ++q) {
          const float4 v = r4[q];
          x[4 * q + 0] = v.x;
          x[4 * q + 1] = v.y;
          x[4 * q + 2] = v.z;
          x[4 * q + 3] = v.w;
        }
      }
      int bj;
      float bd;
      if (labels_in) {
        // labels computed elsewhere for these centroids (the matrix-core
        // assignment, which returns the labels of this kernel's FP32 search)
        bj = labels_in[i];
      } else {
        nearest_f32_sgpr<DM>(x, Cpad + static_cast<size_t>(c0) * DM, act, na, bj, bd);
      }
      if (bj < 0) continue;  // no active centroid: nothing to assign or add
      if (labels && !dry) labels[i] = bj;
      const float* cw = Cl + bj * DM;
      if (accumulate) {
        // FP64 distance of the winner (dimension order, as dist2_f64_row) fused
        // with the accumulation, so each widened coordinate is used at once
        atomicAdd(&cnt_l[bj], 1);
        double* dst = SUMS_LDS ? sums_l + bj * ld : sums + static_cast<size_t>(c0 + bj) * DM;
        double acc = 0.0;
#pragma unroll
        for (int tdim = 0; tdim < DM; ++tdim) {
          const double xv = static_cast<double>(x[tdim]);
          const double e = xv - static_cast<double>(cw[tdim]);
          acc = __builtin_fma(e, e, acc);
          unsafeAtomicAdd(dst + tdim, xv);
        }
        f += acc;
      } else {
        f += dist2_f64_row<DM>(x, cw);
      }
    }
    const double ft = block_sum_f64<kBatchBlock>(f, s_tmp);
    if (tid == 0) tile_f[t] = ft;
    if (accumulate) {
      __syncthreads();
      if (SUMS_LDS) {
        for (int e = tid; e < k * d; e += kBatchBlock) {
          const int j = e / d;
          const int tdim = e - j * d;
          if (cnt_l[j])
            unsafeAtomicAdd(&sums[static_cast<size_t>(c0 + j) * DM + tdim], sums_l[j * ld + tdim]);
        }
      }
      for (int j = tid; j < k; j += kBatchBlock)
        if (cnt_l[j]) atomicAdd(&cnt[c0 + j], cnt_l[j]);
    }
    __syncthreads();
  }
}

// One workgroup per solve (see the file comment).  sums and counts of the
// solve are cleared after use, ready for the next round.
__global__ void __launch_bounds__(kBatchBlock)
    batch_update_kernel(BatchSolve* __restrict__ sv, const double* __restrict__ tile_f,
                        double* __restrict__ sums, int32_t* __restrict__ cnt, float* __restrict__ C,
                        float* __restrict__ Cpad, int dm, double* __restrict__ C64,
                        uint8_t* __restrict__ deg, int d, int max_iter, double tol, int stop_rule,
                        int* __restrict__ running) {
  __shared__ double s_tmp[kBatchBlock / kWave + 1];
  __shared__ double s_max[kBatchBlock / kWave];
  __shared__ int s_done;
  const int tid = threadIdx.x;
  BatchSolve* S = sv + blockIdx.x;
  const int status = S->status;
  if (status == kSolveDone) return;
  // objective: tile partials in tile order
  double v = 0.0;
  for (int q = tid; q < S->ntiles; q += kBatchBlock) v += tile_f[S->tile0 + q];
  const double f = block_sum_f64<kBatchBlock>(v, s_tmp);
  const int k = S->k;
  const int c0 = S->c0;
  if (tid == 0) {
    int active = 0;  // the slots this round's assignment searched
    for (int j = 0; j < k; ++j) active += deg[c0 + j] ? 0 : 1;
    S->nd += S->s * active;
    S->passes += 1;
    int done = 0;
    if (status == kSolveFinal) {
      done = 1;
    } else if (stop_rule == BM_STOP_REL_OBJ && S->iter > 1 && (S->f_prev - f) <= tol * S->f_prev) {
      done = 1;
    }
    if (done) {
      S->f = f;
      S->status = kSolveDone;
    }
    s_done = done;
  }
  __syncthreads();
  if (s_done) {
    // the last assignment of a solve stopped by the objective rule filled its
    // sums; leave them cleared like every other round
    for (int e = tid; e < k * dm; e += kBatchBlock) sums[static_cast<size_t>(c0) * dm + e] = 0.0;
    for (int j = tid; j < k; j += kBatchBlock) cnt[c0 + j] = 0;
    return;
  }
  // update: FP64 means, squared moves summed in dimension order per centroid
  double local = 0.0;
  for (int j = tid; j < k; j += kBatchBlock) {
    const size_t row = static_cast<size_t>(c0 + j);
    if (deg[row]) continue;
    const int c = cnt[row];
    float* cj = C + row * d;
    double* cj64 = C64 + row * d;
    double* sj = sums + row * dm;
    if (c == 0) {
      deg[row] = 1;
      for (int tdim = 0; tdim < d; ++tdim) cj[tdim] = __builtin_nanf("");
      continue;
    }
    double moved = 0.0;
    for (int tdim = 0; tdim < d; ++tdim) {
      const double mean = sj[tdim] / static_cast<double>(c);
      const double diff = mean - cj64[tdim];
      moved = __dadd_rn(moved, __dmul_rn(diff, diff));
      cj64[tdim] = mean;
      cj[tdim] = static_cast<float>(mean);
      Cpad[row * dm + tdim] = static_cast<float>(mean);
    }
    for (int tdim = 0; tdim < dm; ++tdim) sj[tdim] = 0.0;
    cnt[row] = 0;
    moved = sqrt(moved);
    local = moved > local ? moved : local;
  }
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const double y = __shfl_down(local, o, kWave);
    local = y > local ? y : local;
  }
  if (lane == 0) s_max[wave] = local;
  __syncthreads();
  if (tid == 0) {
    double shift = 0.0;
    for (int w = 0; w < kBatchBlock / kWave; ++w) shift = s_max[w] > shift ? s_max[w] : shift;
    const int it = S->iter;
    S->f_prev = f;
    if ((stop_rule == BM_STOP_SHIFT && shift < tol) || it >= max_iter) {
      S->status = kSolveFinal;
    } else {
      S->iter = it + 1;
    }
    atomicAdd(running, 1);
  }
}

// Seed the FP64 means and the zero-padded FP32 copy from the start centroids
// (rows x d).
__global__ void batch_init_kernel(const float* __restrict__ C, double* __restrict__ C64,
                                  float* __restrict__ Cpad, int64_t rows, int d, int dm) {
  const int64_t n = rows * dm;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = e / dm;
    const int t = static_cast<int>(e - r * dm);
    const float v = t < d ? C[r * d + t] : 0.f;
    Cpad[e] = v;
    if (t < d) C64[r * d + t] = static_cast<double>(v);
  }
}

// Copy rows (d wide) into rows DM wide, zero padded.
__global__ void pad_rows_kernel(const float* __restrict__ P, float* __restrict__ Pp, int64_t rows,
                                int d, int dm) {
  const int64_t n = rows * dm;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = e / dm;
    const int t = static_cast<int>(e - r * dm);
    Pp[e] = t < d ? P[r * d + t] : 0.f;
  }
}

// Gather rows of X (FP32 or BF16 widened exactly) into P: one wavefront per row.
template <bool BF16>
__global__ void gather_rows_kernel(const void* __restrict__ X, int64_t n, int d,
                                   const int32_t* __restrict__ idx, int64_t s, float* __restrict__ P,
                                   int* __restrict__ bad) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t w0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t wstride = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t r = w0; r < s; r += wstride) {
    const int64_t src = idx[r];
    if (src < 0 || src >= n) {
      if (lane == 0) atomicExch(bad, 1);
      continue;
    }
    for (int t = lane; t < d; t += kWave) {
      float v;
      if (BF16)
        v = bf16_bits_to_float(static_cast<const uint16_t*>(X)[static_cast<size_t>(src) * d + t]);
      else
        v = static_cast<const float*>(X)[static_cast<size_t>(src) * d + t];
      P[static_cast<size_t>(r) * d + t] = v;
    }
  }
}

// Gather BF16 rows of X (bit copies): one wavefront per row; idx is trusted
// (it comes from the sampler).
__global__ void gather_rows_bf16_kernel(const uint16_t* __restrict__ X, int d,
                                        const int32_t* __restrict__ idx, int64_t s,
                                        uint16_t* __restrict__ P) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t w0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t wstride = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t r = w0; r < s; r += wstride) {
    const int64_t src = idx[r];
    for (int t = lane; t < d; t += kWave) P[static_cast<size_t>(r) * d + t] = X[static_cast<size_t>(src) * d + t];
  }
}

template <int DM, bool SUMS_LDS>
const void* batch_assign_fn() {
  return reinterpret_cast<const void*>(&batch_assign_kernel<DM, SUMS_LDS>);
}

template <bool SUMS_LDS>
const void* pick_batch_assign(int dm) {
  switch (dm) {
    case 4: return batch_assign_fn<4, SUMS_LDS>();
    case 8: return batch_assign_fn<8, SUMS_LDS>();
    case 16: return batch_assign_fn<16, SUMS_LDS>();
    case 32: return batch_assign_fn<32, SUMS_LDS>();
    case 64: return batch_assign_fn<64, SUMS_LDS>();
    case 72: return batch_assign_fn<72, SUMS_LDS>();
    case 128: return batch_assign_fn<128, SUMS_LDS>();
    case 256: return batch_assign_fn<256, SUMS_LDS>();
    default: return nullptr;
  }
}

}  // namespace

size_t batch_assign_lds(int d, int kmax, bool sums_lds) {
  const int dm = padded_dim(d);
  size_t b = (sizeof(float) * static_cast<size_t>(kmax) * dm + sizeof(int) * 2 * kmax + 15) & ~size_t(15);
  if (sums_lds) b += sizeof(double) * static_cast<size_t>(kmax) * (dm + 1);
  return b;
}

bm_status batch_assign_grid(int d, int kmax, bool sums_lds, int* grid) {
  const void* fn = sums_lds ? pick_batch_assign<true>(padded_dim(d)) : pick_batch_assign<false>(padded_dim(d));
  if (!fn) return set_error(BM_ENOTSUP, "d = %d exceeds the limit of 256", d);
  const size_t lds = batch_assign_lds(d, kmax, sums_lds);
  if (lds > 65536 &&
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
    return set_error(BM_ENOTSUP, "cannot reserve %zu B of LDS for the batched assignment", lds);
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBatchBlock, lds) != hipSuccess)
    return set_error(BM_EDEVICE, "cannot query the device for the batched assignment");
  if (per_cu < 1) return set_error(BM_ENOTSUP, "batched assignment kernel cannot be resident");
  *grid = cus * per_cu;
  return BM_OK;
}

bm_status launch_batch_assign(const float* Pp, int d, const float* C, const float* Cpad,
                              const uint8_t* deg, const BatchSolve* sv, const int32_t* tile_solve,
                              int ntiles, int tile_rows, int kmax, bool sums_lds, double* sums,
                              int32_t* cnt, double* tile_f, int32_t* labels, int dry, int grid,
                              hipStream_t stream, const int32_t* labels_in) {
  const void* fn = sums_lds ? pick_batch_assign<true>(padded_dim(d)) : pick_batch_assign<false>(padded_dim(d));
  if (!fn || grid < 1) return set_error(BM_EINVAL, "batched assignment: bad plan");
  const size_t lds = batch_assign_lds(d, kmax, sums_lds);
  void* args[] = {const_cast<float**>(&Pp), &d, const_cast<float**>(&C), const_cast<float**>(&Cpad),
                  const_cast<uint8_t**>(&deg), const_cast<BatchSolve**>(&sv), const_cast<int32_t**>(&tile_solve), &ntiles,
                  &tile_rows, &sums, &cnt, &tile_f, &labels, &dry, const_cast<int32_t**>(&labels_in)};
  const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kBatchBlock), args, lds, stream);
  if (e != hipSuccess)
    return set_error(BM_EDEVICE, "batched assignment launch failed: %s", hipGetErrorString(e));
  return BM_OK;
}

bm_status launch_batch_update(BatchSolve* sv, int n_solves, const double* tile_f, double* sums,
                              int32_t* cnt, float* C, float* Cpad, double* C64, uint8_t* deg, int d,
                              int max_iter, double tol, int stop_rule, int* running,
                              hipStream_t stream) {
  const int dm = padded_dim(d);
  hipLaunchKernelGGL(batch_update_kernel, dim3(n_solves), dim3(kBatchBlock), 0, stream, sv, tile_f,
                     sums, cnt, C, Cpad, dm, C64, deg, d, max_iter, tol, stop_rule, running);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return set_error(BM_EDEVICE, "batched update launch failed: %s", hipGetErrorString(e));
  return BM_OK;
}

bm_status launch_batch_init(const float* C, double* C64, float* Cpad, int64_t rows, int d,
                            hipStream_t stream) {
  const int dm = padded_dim(d);
  const int64_t blocks = (rows * dm + 255) / 256;
  hipLaunchKernelGGL(batch_init_kernel,
                     dim3(static_cast<unsigned>(blocks < 1024 ? (blocks < 1 ? 1 : blocks) : 1024)),
                     dim3(256), 0, stream, C, C64, Cpad, rows, d, dm);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BM_EDEVICE, "batch init launch failed: %s", hipGetErrorString(e));
  return BM_OK;
}

bm_status launch_pad_rows(const float* P, float* Pp, int64_t rows, int d, hipStream_t stream) {
  const int dm = padded_dim(d);
  int64_t blocks = (rows * dm + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(pad_rows_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, P, Pp,
                     rows, d, dm);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BM_EDEVICE, "pad launch failed: %s", hipGetErrorString(e));
  return BM_OK;
}

bm_status launch_gather_rows(const void* X, int x_bf16, int64_t n, int d, const int32_t* idx,
                             int64_t s, float* P, int* bad, hipStream_t stream) {
  const int64_t waves = s;
  int64_t blocks = (waves * kWave + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  if (x_bf16)
    hipLaunchKernelGGL(gather_rows_kernel<true>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                       stream, X, n, d, idx, s, P, bad);
  else
    hipLaunchKernelGGL(gather_rows_kernel<false>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                       stream, X, n, d, idx, s, P, bad);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BM_EDEVICE, "gather launch failed: %s", hipGetErrorString(e));
  return BM_OK;
}

bm_status launch_gather_rows_bf16(const uint16_t* X, int d, const int32_t* idx, int64_t s,
                                  uint16_t* P, hipStream_t stream) {
  int64_t blocks = (s * kWave + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(gather_rows_bf16_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                     X, d, idx, s, P);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BM_EDEVICE, "BF16 gather launch failed: %s", hipGetErrorString(e));
  return BM_OK;
}

}  // namespace bm
