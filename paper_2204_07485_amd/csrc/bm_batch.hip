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
                        const int32_t* __restrict__ labels_in, double* __restrict__ partials,
                        int32_t* __restrict__ pcnt, int tpc) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int s_j, s_k, s_na, s_c0, s_status, s_tile0;
  __shared__ int64_t s_row0, s_s;
  __shared__ double s_tmp[kBatchBlock / kWave + 1];
  const int tid = threadIdx.x;
  constexpr int ld = batch_sums_ld<DM>();
  float* Cl = reinterpret_cast<float*>(lds_raw);

  // Chunks of tpc consecutive tiles, grid-strided over the workgroups:
  // consecutive tiles mostly belong to one solve, whose cluster sums stay in
  // LDS until the solve changes (a flush per chunk rather than per tile),
  // while late rounds with few running solves still spread over many
  // workgroups.
  int cur = -1;            // solve whose state is in LDS
  bool cur_acc = false;    // ... and whose sums are being accumulated
  int cur_k = 0, cur_c0 = 0;
  // flush this workgroup's sums and counts of solve `cur`
  auto flush = [&]() {
    int* act = reinterpret_cast<int*>(lds_raw + sizeof(float) * static_cast<size_t>(cur_k) * DM);
    int* cnt_l = act + cur_k;
    double* sums_l = reinterpret_cast<double*>(
        lds_raw + ((sizeof(float) * static_cast<size_t>(cur_k) * DM + sizeof(int) * 2 * cur_k + 15) & ~size_t(15)));
    __syncthreads();
    if (partials) {
      // one solve, one block of partial sums per workgroup: plain stores,
      // added in workgroup order by batch_reduce_kernel
      double* pb = partials + static_cast<size_t>(blockIdx.x) * cur_k * DM;
      for (int e = tid; e < cur_k * DM; e += kBatchBlock) {
        const int j = e / DM;
        pb[e] = SUMS_LDS ? sums_l[j * ld + (e - j * DM)] : 0.0;
      }
      for (int j = tid; j < cur_k; j += kBatchBlock) pcnt[static_cast<size_t>(blockIdx.x) * cur_k + j] = cnt_l[j];
    } else {
      if (SUMS_LDS) {
        for (int e = tid; e < cur_k * d; e += kBatchBlock) {
          const int j = e / d;
          const int tdim = e - j * d;
          if (cnt_l[j])
            unsafeAtomicAdd(&sums[static_cast<size_t>(cur_c0 + j) * DM + tdim], sums_l[j * ld + tdim]);
        }
      }
      for (int j = tid; j < cur_k; j += kBatchBlock)
        if (cnt_l[j]) atomicAdd(&cnt[cur_c0 + j], cnt_l[j]);
    }
    __syncthreads();
  };

  for (int64_t chunk = blockIdx.x; chunk * tpc < ntiles; chunk += gridDim.x) {
  const int64_t tend = (chunk + 1) * tpc < ntiles ? (chunk + 1) * tpc : ntiles;
  for (int64_t t = chunk * tpc; t < tend; ++t) {
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
    const bool accumulate = status == kSolveRunning && !dry;
    int* act = reinterpret_cast<int*>(lds_raw + sizeof(float) * static_cast<size_t>(k) * DM);
    int* cnt_l = act + k;
    double* sums_l = reinterpret_cast<double*>(
        lds_raw + ((sizeof(float) * static_cast<size_t>(k) * DM + sizeof(int) * 2 * k + 15) & ~size_t(15)));
    if (s_j != cur) {
      if (cur_acc) flush();
      cur = s_j;
      cur_acc = accumulate;
      cur_k = k;
      cur_c0 = c0;
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
    }
    const int na = s_na;
    const int64_t r0 = s_row0 + static_cast<int64_t>(t - s_tile0) * tile_rows;
    const int64_t rend = s_row0 + s_s;
    const int64_t r1 = r0 + tile_rows < rend ? r0 + tile_rows : rend;
    double f = 0.0;
    // rows are DM wide and zero padded: 16-byte loads, no column guard; up to
    // 32 columns the next row's loads are in flight while a row is processed
    constexpr bool kAhead = DM <= 32;
    auto load = [&](int64_t i, float (&x)[DM]) {
      const float4* r4 = reinterpret_cast<const float4*>(Pp + static_cast<size_t>(i) * DM);
#pragma unroll
      for (int q = 0; q < DM / 4; ++q) {
        const float4 v = r4[q];
        x[4 * q + 0] = v.x;
        x[4 * q + 1] = v.y;
        x[4 * q + 2] = v.z;
        x[4 * q + 3] = v.w;
      }
    };
    float x[DM];
    if (kAhead && r0 + tid < r1) load(r0 + tid, x);
    for (int64_t i = r0 + tid; i < r1; i += kBatchBlock) {
      float xn[kAhead ? DM : 1];
      const bool more = kAhead && i + kBatchBlock < r1;
      if constexpr (kAhead) {
        if (more) load(i + kBatchBlock, xn);
      } else {
        load(i, x);
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
      if (bj >= 0) {  // else no active centroid: nothing to assign or add
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
      if constexpr (kAhead) {
        if (more) {
#pragma unroll
          for (int t2 = 0; t2 < DM; ++t2) x[t2] = xn[t2];
        }
      }
    }
    const double ft = block_sum_f64<kBatchBlock>(f, s_tmp);
    if (tid == 0) tile_f[t] = ft;
    __syncthreads();
  }
  }
  if (cur_acc) flush();
  else if (partials && cur < 0 && sv[0].status == kSolveRunning && !dry) {
    // no tile here: this workgroup's partial block is zero
    const int k = sv[0].k;
    for (int e = tid; e < k * DM; e += kBatchBlock) partials[static_cast<size_t>(blockIdx.x) * k * DM + e] = 0.0;
    for (int j = tid; j < k; j += kBatchBlock) pcnt[static_cast<size_t>(blockIdx.x) * k + j] = 0;
  }
}

// One solve's partial sums and counts, one block per workgroup of the
// assignment kernel (partials: nparts x n, n = k x DM, then pcnt: nparts x k),
// added in a fixed order: workgroup b takes 64 consecutive elements; its
// wavefront w adds the parts of its contiguous share w cp .. (w + 1) cp - 1
// in part order (kRedUnroll coalesced loads in flight), and the wavefront sums
// are added in wavefront order.  Nothing to add unless the solve is running.
constexpr int kReduceBlock = 1024;
constexpr int kRedUnroll = 8;
__global__ void __launch_bounds__(kReduceBlock)
    batch_reduce_kernel(const double* __restrict__ partials, const int32_t* __restrict__ pcnt,
                        int nparts, int k, int dm, double* __restrict__ sums,
                        int32_t* __restrict__ cnt, const BatchSolve* __restrict__ sv) {
  constexpr int kWaves = kReduceBlock / kWave;
  __shared__ double s_part[kWaves][kWave];
  __shared__ int s_cpart[kWaves][kWave];
  if (sv[0].status != kSolveRunning) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int cp = (nparts + kWaves - 1) / kWaves;
  const int w0 = wave * cp < nparts ? wave * cp : nparts;
  const int w1 = w0 + cp < nparts ? w0 + cp : nparts;
  const int64_t n = static_cast<int64_t>(k) * dm;
  const int64_t nblk_sums = (n + kWave - 1) / kWave;
  const int64_t nblk = nblk_sums + (k + kWave - 1) / kWave;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    if (b < nblk_sums) {
      const int64_t e = b * kWave + lane;
      const int64_t ec = e < n ? e : n - 1;
      double v = 0.0;
      int w = w0;
      for (; w + kRedUnroll <= w1; w += kRedUnroll) {
        double t[kRedUnroll];
#pragma unroll
        for (int u = 0; u < kRedUnroll; ++u) t[u] = partials[static_cast<size_t>(w + u) * n + ec];
#pragma unroll
        for (int u = 0; u < kRedUnroll; ++u) v += t[u];
      }
      for (; w < w1; ++w) v += partials[static_cast<size_t>(w) * n + ec];
      s_part[wave][lane] = v;
      __syncthreads();
      if (wave == 0 && e < n) {
        double t = s_part[0][lane];
        for (int q = 1; q < kWaves; ++q) t += s_part[q][lane];
        sums[e] = t;
      }
    } else {
      const int64_t j = (b - nblk_sums) * kWave + lane;
      const int64_t jc = j < k ? j : k - 1;
      int c = 0;
      for (int w = w0; w < w1; ++w) c += pcnt[static_cast<size_t>(w) * k + jc];
      s_cpart[wave][lane] = c;
      __syncthreads();
      if (wave == 0 && j < k) {
        int t = 0;
        for (int q = 0; q < kWaves; ++q) t += s_cpart[q][lane];
        cnt[j] = t;
      }
    }
    __syncthreads();
  }
}

// The accumulation of one solve for labels computed elsewhere (the
// matrix-core assignment), BF16 rows: LPR lanes per row, each with 8
// consecutive columns (one 16-byte load when rows are 16-byte aligned, else 8
// element loads), so a wavefront instruction covers 64 / LPR rows and a batch
// kAccUnroll instructions; the next batch's loads are in flight while one is
// added.  Nothing in the loop branches: rows past the range repeat the last
// row with no weight.  FP64 sums sit in LDS column-permuted (column 8 g + q of
// a centroid at q LPR + g), so for each q the lanes of a row add to
// consecutive addresses; the FP32 centroids sit row-major for the objective
// (two 16-byte LDS reads per lane and row).  Each workgroup takes a
// contiguous range of rows and writes one partial block of sums and counts
// (k x DM in column order, added by batch_reduce_kernel) and its objective
// partial: the FP64 squared distance of every row to its centroid.
constexpr int kAccBlock = 1024;
constexpr int kAccUnroll = 2;

__host__ __device__ constexpr int accum_lpr(int d) {
  return d <= 8 ? 1 : d <= 16 ? 2 : d <= 32 ? 4 : d <= 64 ? 8 : d <= 128 ? 16 : 32;
}

union AccPack {
  uint4 u;
  uint16_t h[8];
};

__device__ __forceinline__ float acc_bf16_at(const AccPack& p, int q) {
  const uint32_t w = (q & 1) ? (reinterpret_cast<const uint32_t*>(&p.u)[q >> 1] & 0xFFFF0000u)
                             : (reinterpret_cast<const uint32_t*>(&p.u)[q >> 1] << 16);
  return __uint_as_float(w);
}

template <int LPR, bool VEC>
__global__ void __launch_bounds__(kAccBlock)
    labels_accum_kernel(const uint16_t* __restrict__ P, int64_t s, int d, int dm, int k,
                        const float* __restrict__ C, int c_vec, const int32_t* __restrict__ labels,
                        const BatchSolve* __restrict__ sv, double* __restrict__ partials,
                        int32_t* __restrict__ pcnt, double* __restrict__ tile_f) {
  constexpr int RPI = kWave / LPR;        // rows per wavefront instruction
  constexpr int RPB = RPI * kAccUnroll;   // rows per batch
  constexpr int DMP = 8 * LPR;            // LDS row stride (>= DM)
  constexpr int kWaves = kAccBlock / kWave;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* sums_l = reinterpret_cast<double*>(lds_raw);                           // k x DMP, permuted
  float* c_l = reinterpret_cast<float*>(sums_l + static_cast<size_t>(k) * DMP);  // k x DMP
  int* cnt_l = reinterpret_cast<int*>(c_l + static_cast<size_t>(k) * DMP);
  __shared__ double s_tmp[kWaves + 1];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int status = sv[0].status;
  if (status == kSolveDone) return;
  const bool accumulate = status == kSolveRunning;
  if (accumulate) {
    double2* z = reinterpret_cast<double2*>(sums_l);
    for (int e = tid; e < k * DMP / 2; e += kAccBlock) z[e] = make_double2(0.0, 0.0);
    for (int j = tid; j < k; j += kAccBlock) cnt_l[j] = 0;
  }
  constexpr int Q4 = DMP / 4;
  for (int e = tid; e < k * Q4; e += kAccBlock) {
    const int j = e / Q4;
    const int t = 4 * (e - j * Q4);
    const float* cr = C + static_cast<size_t>(j) * d;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (c_vec) {
      if (t < d) v = *reinterpret_cast<const float4*>(cr + t);
    } else {
      v.x = t + 0 < d ? cr[t + 0] : 0.f;
      v.y = t + 1 < d ? cr[t + 1] : 0.f;
      v.z = t + 2 < d ? cr[t + 2] : 0.f;
      v.w = t + 3 < d ? cr[t + 3] : 0.f;
    }
    reinterpret_cast<float4*>(c_l)[e] = v;
  }
  __syncthreads();
  const int64_t per = (s + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t r1 = r0 + per < s ? r0 + per : s;
  const int g = lane % LPR;
  const int sub = lane / LPR;
  const int t0 = 8 * g;
  const bool colv = t0 < d;
  double f = 0.0;
  AccPack x[kAccUnroll];
  int jl[kAccUnroll];
  bool live[kAccUnroll];
  auto load = [&](int64_t base, AccPack (&xo)[kAccUnroll], int (&jo)[kAccUnroll],
                  bool (&lo)[kAccUnroll]) {
#pragma unroll
    for (int u = 0; u < kAccUnroll; ++u) {
      const int64_t row = base + u * RPI + sub;
      const int64_t rc = row < r1 ? row : r1 - 1;
      const int j = labels[rc];
      lo[u] = row < r1 && j >= 0;
      jo[u] = j >= 0 ? j : 0;
      const uint16_t* pr = P + static_cast<size_t>(rc) * d;
      if (VEC) {
        const uint4 v = *reinterpret_cast<const uint4*>(pr + (colv ? t0 : 0));
        xo[u].u = colv ? v : make_uint4(0u, 0u, 0u, 0u);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int t = t0 + q;
          const uint16_t h = pr[t < d ? t : 0];
          xo[u].h[q] = t < d ? h : static_cast<uint16_t>(0);
        }
      }
    }
  };
  int64_t b0 = r0 + static_cast<int64_t>(wave) * RPB;
  if (b0 < r1) load(b0, x, jl, live);
  for (; b0 < r1; b0 += static_cast<int64_t>(kWaves) * RPB) {
    const int64_t nb0 = b0 + static_cast<int64_t>(kWaves) * RPB;
    AccPack xn[kAccUnroll];
    int jn[kAccUnroll];
    bool ln[kAccUnroll];
    if (nb0 < r1) load(nb0, xn, jn, ln);
#pragma unroll
    for (int u = 0; u < kAccUnroll; ++u) {
      const int j = jl[u];
      const float4 c0 = *reinterpret_cast<const float4*>(c_l + j * DMP + t0);
      const float4 c1 = *reinterpret_cast<const float4*>(c_l + j * DMP + t0 + 4);
      const float cc[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
      double* dst = sums_l + j * DMP + g;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        // padding columns hold zeros on both sides: they add exact zeros
        const double xd = live[u] ? static_cast<double>(acc_bf16_at(x[u], q)) : 0.0;
        const double e = live[u] ? xd - static_cast<double>(cc[q]) : 0.0;
        f = __builtin_fma(e, e, f);
        if (accumulate) unsafeAtomicAdd(dst + q * LPR, xd);
      }
      if (accumulate && g == 0 && live[u]) atomicAdd(&cnt_l[j], 1);
    }
    if (nb0 < r1) {
#pragma unroll
      for (int u = 0; u < kAccUnroll; ++u) {
        x[u] = xn[u];
        jl[u] = jn[u];
        live[u] = ln[u];
      }
    }
  }
  const double ft = block_sum_f64<kAccBlock>(f, s_tmp);
  if (tid == 0) tile_f[blockIdx.x] = ft;
  if (accumulate) {
    __syncthreads();
    double* pb = partials + static_cast<size_t>(blockIdx.x) * k * dm;
    for (int e = tid; e < k * DMP; e += kAccBlock) {
      const int j = e / DMP;
      const int p = e - j * DMP;
      const int q = p / LPR;
      const int t = 8 * (p - q * LPR) + q;
      if (t < dm) pb[static_cast<size_t>(j) * dm + t] = sums_l[e];
    }
    for (int j = tid; j < k; j += kAccBlock) pcnt[static_cast<size_t>(blockIdx.x) * k + j] = cnt_l[j];
  }
}

// One workgroup per solve (see the file comment).  sums and counts of the
// solve are cleared after use, ready for the next round.
constexpr int kUpdBlock = 1024;
__global__ void __launch_bounds__(kUpdBlock)
    batch_update_kernel(BatchSolve* __restrict__ sv, const double* __restrict__ tile_f,
                        double* __restrict__ sums, int32_t* __restrict__ cnt, float* __restrict__ C,
                        float* __restrict__ Cpad, int dm, double* __restrict__ C64,
                        uint8_t* __restrict__ deg, int d, int max_iter, double tol, int stop_rule,
                        int* __restrict__ running) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* dsq = reinterpret_cast<double*>(lds_raw);  // k x (d | 1): squared coordinate moves
  __shared__ double s_tmp[kUpdBlock / kWave + 1];
  __shared__ double s_max[kUpdBlock / kWave];
  __shared__ int s_done;
  const int tid = threadIdx.x;
  BatchSolve* S = sv + blockIdx.x;
  const int status = S->status;
  if (status == kSolveDone) return;
  // objective: tile partials in tile order
  double v = 0.0;
  for (int q = tid; q < S->ntiles; q += kUpdBlock) v += tile_f[S->tile0 + q];
  const double f = block_sum_f64<kUpdBlock>(v, s_tmp);
  const int k = S->k;
  const int c0 = S->c0;
  int act_part = 0;  // the slots this round's assignment searched
  for (int j = tid; j < k; j += kUpdBlock) act_part += deg[c0 + j] ? 0 : 1;
  const int active = static_cast<int>(block_sum_f64<kUpdBlock>(static_cast<double>(act_part), s_tmp));
  if (tid == 0) {
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
    for (int e = tid; e < k * dm; e += kUpdBlock) sums[static_cast<size_t>(c0) * dm + e] = 0.0;
    for (int j = tid; j < k; j += kUpdBlock) cnt[c0 + j] = 0;
    return;
  }
  // update, in three parallel steps: (A) every coordinate's FP64 mean and
  // squared move (into LDS), (B) per centroid the move summed in
  // dimension order, empty clusters turning degenerate, (C) sums and counts
  // cleared for the next round.  Loads are issued in groups so that their
  // latencies overlap.
  const int64_t kd = static_cast<int64_t>(k) * d;
  const int ldq = d | 1;  // odd row stride: the centroids of a wavefront in distinct banks
  constexpr int kGroup = 4;
  for (int64_t e0 = tid; e0 < kd; e0 += static_cast<int64_t>(kUpdBlock) * kGroup) {
    double sm[kGroup], old[kGroup];
    int cc[kGroup];
#pragma unroll
    for (int q = 0; q < kGroup; ++q) {
      const int64_t e = e0 + static_cast<int64_t>(q) * kUpdBlock;
      cc[q] = 0;
      if (e < kd) {
        const int64_t j = e / d;
        const size_t row = static_cast<size_t>(c0 + j);
        const int tdim = static_cast<int>(e - j * d);
        cc[q] = deg[row] ? 0 : cnt[row];
        sm[q] = sums[row * dm + tdim];
        old[q] = C64[row * d + tdim];
      }
    }
#pragma unroll
    for (int q = 0; q < kGroup; ++q) {
      const int64_t e = e0 + static_cast<int64_t>(q) * kUpdBlock;
      if (e < kd && cc[q] > 0) {
        const int64_t j = e / d;
        const size_t row = static_cast<size_t>(c0 + j);
        const int tdim = static_cast<int>(e - j * d);
        const double mean = sm[q] / static_cast<double>(cc[q]);
        const double diff = mean - old[q];
        dsq[j * ldq + tdim] = __dmul_rn(diff, diff);
        C64[row * d + tdim] = mean;
        C[row * d + tdim] = static_cast<float>(mean);
        Cpad[row * dm + tdim] = static_cast<float>(mean);
      }
    }
  }
  __syncthreads();
  double local = 0.0;
  for (int j = tid; j < k; j += kUpdBlock) {
    const size_t row = static_cast<size_t>(c0 + j);
    if (deg[row]) continue;
    if (cnt[row] == 0) {
      deg[row] = 1;
      float* cj = C + row * d;
      for (int tdim = 0; tdim < d; ++tdim) cj[tdim] = __builtin_nanf("");
      continue;
    }
    const double* sj = dsq + static_cast<size_t>(j) * ldq;
    double moved = 0.0;
    for (int tdim = 0; tdim < d; ++tdim) moved = __dadd_rn(moved, sj[tdim]);
    moved = sqrt(moved);
    local = moved > local ? moved : local;
  }
  __syncthreads();
  for (int64_t e = tid; e < static_cast<int64_t>(k) * dm; e += kUpdBlock)
    sums[static_cast<size_t>(c0) * dm + e] = 0.0;
  for (int j = tid; j < k; j += kUpdBlock) cnt[c0 + j] = 0;
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
    for (int w = 0; w < kUpdBlock / kWave; ++w) shift = s_max[w] > shift ? s_max[w] : shift;
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

// Start of one solve (the matrix-core fit's sample): working centroids and
// flags from the incumbent, the solve record, cleared sums and counts; one
// launch in place of a copy, two transfers and two fills.
__global__ void solve_start_kernel(const float* __restrict__ Cinc, const uint8_t* __restrict__ deginc,
                                   float* __restrict__ cw, uint8_t* __restrict__ degw,
                                   BatchSolve* __restrict__ sv, BatchSolve init,
                                   double* __restrict__ sums, int32_t* __restrict__ cnt, int k, int d,
                                   int dm) {
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = tid; e < static_cast<int64_t>(k) * d; e += stride) cw[e] = Cinc[e];
  for (int64_t e = tid; e < static_cast<int64_t>(k) * dm; e += stride) sums[e] = 0.0;
  for (int64_t j = tid; j < k; j += stride) {
    degw[j] = deginc[j];
    cnt[j] = 0;
  }
  if (tid == 0) *sv = init;
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
  if (bm_status sr = reserve_lds(fn, lds)) return sr;
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
                              hipStream_t stream, const int32_t* labels_in, double* partials,
                              int32_t* pcnt) {
  // rows at least 8 wide and up to 128 centroids per solve with kmax d >= 256:
  // labels from the matrix cores (the same labels, sums, counts and
  // objectives up to FP64 association), when its larger LDS plan fits
  if (!labels_in && !partials && d >= 8 && kmax >= 8 && kmax <= 128 && kmax * d >= 256 &&
      fp32_mfma_enabled()) {
    size_t lds_max = 0;
    if (max_lds_per_block(&lds_max) == BM_OK && batch_assign_mfma32_lds(d, kmax, sums_lds) + 1024 <= lds_max)
      return launch_batch_assign_mfma32(Pp, d, C, deg, sv, tile_solve, ntiles, tile_rows, kmax, sums_lds,
                                        sums, cnt, tile_f, labels, dry, stream);
    clear_error();
  }
  const void* fn = sums_lds ? pick_batch_assign<true>(padded_dim(d)) : pick_batch_assign<false>(padded_dim(d));
  if (!fn || grid < 1) return set_error(BM_EINVAL, "batched assignment: bad plan");
  if (partials && ntiles > grid)
    return set_error(BM_EINVAL, "batched assignment: partial blocks need a tile per workgroup");
  const size_t lds = batch_assign_lds(d, kmax, sums_lds);
  // one tile per chunk: longer chunks (fewer flushes) measured slower on the
  // batched workload, whose late rounds have few running solves
  int tpc = 1;
  void* args[] = {const_cast<float**>(&Pp), &d, const_cast<float**>(&C), const_cast<float**>(&Cpad),
                  const_cast<uint8_t**>(&deg), const_cast<BatchSolve**>(&sv), const_cast<int32_t**>(&tile_solve), &ntiles,
                  &tile_rows, &sums, &cnt, &tile_f, &labels, &dry, const_cast<int32_t**>(&labels_in),
                  &partials, &pcnt, &tpc};
  const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kBatchBlock), args, lds, stream);
  if (e != hipSuccess)
    return set_error(BM_EDEVICE, "batched assignment launch failed: %s", hipGetErrorString(e));
  return BM_OK;
}

bm_status launch_batch_reduce(const double* partials, const int32_t* pcnt, int nparts, int k, int d,
                              double* sums, int32_t* cnt, const BatchSolve* sv, hipStream_t stream) {
  const int dm = padded_dim(d);
  const int64_t n = static_cast<int64_t>(k) * dm;
  int64_t blocks = (n + kWave - 1) / kWave + (k + kWave - 1) / kWave;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(batch_reduce_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kReduceBlock), 0,
                     stream, partials, pcnt, nparts, k, dm, sums, cnt, sv);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BM_EDEVICE, "batched reduce launch failed: %s", hipGetErrorString(e));
  return BM_OK;
}

bm_status launch_batch_update(BatchSolve* sv, int n_solves, const double* tile_f, double* sums,
                              int32_t* cnt, float* C, float* Cpad, double* C64, uint8_t* deg, int d,
                              int max_iter, double tol, int stop_rule, int* running,
                              hipStream_t stream, int kmax) {
  const int dm = padded_dim(d);
  const size_t lds = sizeof(double) * static_cast<size_t>(kmax) * (d | 1);
  if (bm_status sr = reserve_lds(reinterpret_cast<const void*>(&batch_update_kernel), lds)) return sr;
  hipLaunchKernelGGL(batch_update_kernel, dim3(n_solves), dim3(kUpdBlock), lds, stream, sv, tile_f,
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

bm_status launch_solve_start(const float* Cinc, const uint8_t* deginc, float* cw, uint8_t* degw,
                             BatchSolve* sv, const BatchSolve& init, double* sums, int32_t* cnt, int k,
                             int d, hipStream_t stream) {
  const int dm = padded_dim(d);
  int64_t blocks = (static_cast<int64_t>(k) * dm + 255) / 256;
  if (blocks > 256) blocks = 256;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(solve_start_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, Cinc,
                     deginc, cw, degw, sv, init, sums, cnt, k, d, dm);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BM_EDEVICE, "solve start launch failed: %s", hipGetErrorString(e));
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

size_t labels_accum_lds(int d, int k) {
  if (d < 1 || d > 256) return ~size_t(0);
  return (sizeof(double) + sizeof(float)) * static_cast<size_t>(k) * 8 * accum_lpr(d) +
         sizeof(int) * static_cast<size_t>(k);
}

namespace {
template <int LPR>
const void* accum_fn(bool vec) {
  return vec ? reinterpret_cast<const void*>(&labels_accum_kernel<LPR, true>)
             : reinterpret_cast<const void*>(&labels_accum_kernel<LPR, false>);
}
}  // namespace

bm_status launch_labels_accum(const uint16_t* P, int64_t s, int d, int k, const float* C,
                              const int32_t* labels, const BatchSolve* sv, double* partials,
                              int32_t* pcnt, double* tile_f, int grid, hipStream_t stream) {
  if (s < 1 || d < 1 || d > 256 || k < 1 || grid < 1 || grid > s)
    return set_error(BM_EINVAL, "accumulation: bad plan");
  const bool vec = (d & 7) == 0 && (reinterpret_cast<uintptr_t>(P) & 15) == 0;
  const void* fn = nullptr;
  switch (accum_lpr(d)) {
    case 1: fn = accum_fn<1>(vec); break;
    case 2: fn = accum_fn<2>(vec); break;
    case 4: fn = accum_fn<4>(vec); break;
    case 8: fn = accum_fn<8>(vec); break;
    case 16: fn = accum_fn<16>(vec); break;
    default: fn = accum_fn<32>(vec); break;
  }
  const size_t lds = labels_accum_lds(d, k);
  if (bm_status sr = reserve_lds(fn, lds)) return sr;
  int dm = padded_dim(d);
  int c_vec = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0;
  void* args[] = {const_cast<uint16_t**>(&P), &s, &d, &dm, &k, const_cast<float**>(&C), &c_vec,
                  const_cast<int32_t**>(&labels), const_cast<BatchSolve**>(&sv), &partials, &pcnt,
                  &tile_f};
  const hipError_t le = hipLaunchKernel(fn, dim3(grid), dim3(kAccBlock), args, lds, stream);
  if (le != hipSuccess)
    return set_error(BM_EDEVICE, "accumulation launch failed: %s", hipGetErrorString(le));
  return BM_OK;
}

}  // namespace bm
