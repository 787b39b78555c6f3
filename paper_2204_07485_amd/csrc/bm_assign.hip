// bm_assign.hip -- the final assignment pass of Big-means (Alg. 1 / Sec. 3.4)
// and the kmeans_assign entry point: every row of X goes to its nearest
// non-degenerate centroid, and the objective of Eq. (1) is summed in FP64.
//
// A grid of a few workgroups per CU streams X once from HBM (each thread owns
// whole rows, held in registers, and for rows up to 64 wide loads its next row
// while it processes one); the centroids sit in LDS, padded with zeros to a
// multiple of 4 columns so the inner loop reads them as broadcast 16-byte LDS
// loads (four centroid chains at a time), or, for unpadded rows up to 32 wide,
// come through the scalar cache as SGPR operands.  The nearest centroid is chosen with FP32 direct
// differences (FMA chain in dimension order; exact ties to the lowest index);
// the chosen distance is then recomputed in FP64 for the objective.  Each workgroup
// writes its FP64 partial objective and one more launch adds the partials in
// workgroup order, so the result does not depend on timing (a fence and a
// counter per workgroup to find the last one cost more than that launch).
#include "bm_internal.h"

namespace bm {

namespace {

constexpr int kAssignBlock = 256;

template <int DM, bool BF16>
__global__ void __launch_bounds__(kAssignBlock)
    assign_kernel(const void* __restrict__ Xv, int64_t n, int d, const float* __restrict__ C,
                  const uint8_t* __restrict__ deg, int k, int32_t* __restrict__ labels,
                  float* __restrict__ min_d2, double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* Cl = reinterpret_cast<float*>(lds_raw);
  int* act = reinterpret_cast<int*>(lds_raw + sizeof(float) * static_cast<size_t>(k) * DM);
  __shared__ int s_na;
  __shared__ double s_tmp[kAssignBlock / kWave + 1];

  const int tid = threadIdx.x;
  for (int e = tid; e < k * DM; e += kAssignBlock) {
    const int j = e / DM;
    const int t = e - j * DM;
    Cl[e] = (t < d) ? C[static_cast<size_t>(j) * d + t] : 0.f;
  }
  for (int j = tid; j < k; j += kAssignBlock) act[j] = (deg && deg[j]) ? 1 : 0;
  __syncthreads();
  if (tid == 0) {  // compact the active slots in place, ascending
    int na = 0;
    for (int j = 0; j < k; ++j)
      if (!act[j]) act[na++] = j;
    s_na = na;
  }
  __syncthreads();
  const int na = s_na;

  double sse = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kAssignBlock;
  // with no active centroid (a failed fit) the outputs are left untouched
  const int64_t n_rows = na > 0 ? n : 0;
  // the next row's loads are in flight while a row is processed (rows up to
  // 64 wide; wider ones would double too many registers)
  constexpr bool kAhead = DM <= 64;
  auto load = [&](int64_t i, float (&x)[DM]) {
    if (BF16) {
      load_row_bf16<DM>(static_cast<const uint16_t*>(Xv) + static_cast<size_t>(i) * d, d, x);
    } else {
      load_row_f32<DM>(static_cast<const float*>(Xv) + static_cast<size_t>(i) * d, d, x);
    }
  };
  int64_t i = static_cast<int64_t>(blockIdx.x) * kAssignBlock + tid;
  float x[DM];
  if (kAhead && i < n_rows) load(i, x);
  for (; i < n_rows; i += stride) {
    float xn[kAhead ? DM : 1];
    const bool more = kAhead && i + stride < n_rows;
    if constexpr (kAhead) {
      if (more) load(i + stride, xn);
    } else {
      load(i, x);
    }
    int bj;
    float bd;
    // unpadded rows (d == DM): the centroid values come through the scalar
    // cache as SGPR operands, sparing the LDS bandwidth of 64 broadcast lanes
    if (DM <= 32 && d == DM) nearest_f32_sgpr<DM>(x, C, act, na, bj, bd);
    else if (DM <= 32) nearest_f32_x4<DM>(x, Cl, act, na, bj, bd);
    else nearest_f32<DM>(x, Cl, act, na, bj, bd);
    const double exact = dist2_f64_row<DM>(x, Cl + bj * DM);
    if (labels) labels[i] = bj;
    if (min_d2) min_d2[i] = static_cast<float>(exact);
    sse += exact;
    if constexpr (kAhead) {
      if (more) {
#pragma unroll
        for (int t = 0; t < DM; ++t) x[t] = xn[t];
      }
    }
  }
  const double bsum = block_sum_f64<kAssignBlock>(sse, s_tmp);
  // the partials are added in workgroup order by sum_partials_kernel, launched
  // after this kernel (no fence and atomic per workgroup)
  if (tid == 0) partial[blockIdx.x] = bsum;
}

template <int DM>
const void* assign_fn(bool bf16) {
  return bf16 ? reinterpret_cast<const void*>(&assign_kernel<DM, true>)
              : reinterpret_cast<const void*>(&assign_kernel<DM, false>);
}

const void* pick_assign(int dm, bool bf16) {
  switch (dm) {
    case 4: return assign_fn<4>(bf16);
    case 8: return assign_fn<8>(bf16);
    case 16: return assign_fn<16>(bf16);
    case 32: return assign_fn<32>(bf16);
    case 64: return assign_fn<64>(bf16);
    case 72: return assign_fn<72>(bf16);
    case 128: return assign_fn<128>(bf16);
    case 256: return assign_fn<256>(bf16);
    default: return nullptr;
  }
}

}  // namespace

int assign_grid(int64_t n, int d) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // rows up to 64 wide: four workgroups per CU, each thread takes several
  // rows and the next row's loads overlap the current row's distances;
  // wider rows: eight
  const int64_t want = (n + kAssignBlock - 1) / kAssignBlock;
  const int64_t cap = static_cast<int64_t>(cus) * (padded_dim(d) <= 64 ? 4 : 8);
  int64_t g = want < cap ? want : cap;
  return static_cast<int>(g < 1 ? 1 : g);
}

bm_status launch_assign(const void* X, int x_bf16, int64_t n, int d, const float* C,
                        const uint8_t* deg_dev, int k, int32_t* labels, float* min_d2,
                        double* partial, double* sse_dev, int grid, hipStream_t stream) {
  // FP32 rows at least 8 wide against at least 8 centroids with k d >= 256
  // (below that the VALU scan is as fast): the matrix-core form (the same
  // labels, see bm_assign_mfma32.hip), on at most `grid` workgroups (the
  // caller's partial buffer)
  if (!x_bf16 && d >= 8 && k >= 8 && k * d >= 256 && fp32_mfma_enabled()) {
    int mgrid = 0;
    if (plan_assign_mfma32(X, n, d, k, &mgrid) == BM_OK) {
      return launch_assign_mfma32(static_cast<const float*>(X), n, d, C, deg_dev, k, labels, min_d2,
                                  partial, sse_dev, nullptr, mgrid < grid ? mgrid : grid, stream);
    }
    clear_error();  // too large for its LDS plan: the VALU form below
  }
  const int dm = padded_dim(d);
  const void* fn = pick_assign(dm, x_bf16 != 0);
  if (!fn) return set_error(BM_ENOTSUP, "dimension %d exceeds the assign kernel's limit of 256", d);
  const size_t lds = sizeof(float) * static_cast<size_t>(k) * dm + sizeof(int) * static_cast<size_t>(k);
  size_t lds_max = 0;
  bm_status st = max_lds_per_block(&lds_max);
  if (st != BM_OK) return st;
  if (lds + 1024 > lds_max)
    return set_error(BM_ENOTSUP, "k*d = %d*%d centroids do not fit in LDS", k, d);
  if (bm_status sr = reserve_lds(fn, lds)) return sr;
  void* args[] = {const_cast<void**>(&X), &n, &d, const_cast<float**>(&C),
                  const_cast<uint8_t**>(&deg_dev), &k, &labels, &min_d2, &partial};
  const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kAssignBlock), args, lds, stream);
  if (e != hipSuccess)
    return set_error(BM_EDEVICE, "assign launch failed: %s", hipGetErrorString(e));
  return launch_sum_partials(partial, grid, sse_dev, stream);
}

namespace {
// The objective: the workgroups' FP64 partials added in a fixed order (one
// workgroup; each thread adds a strided subset, then a fixed tree).
constexpr int kSumBlock = 256;
__global__ void __launch_bounds__(kSumBlock)
    sum_partials_kernel(const double* __restrict__ partial, int np, double* __restrict__ out) {
  __shared__ double s_tmp[kSumBlock / kWave + 1];
  double v = 0.0;
  for (int g = threadIdx.x; g < np; g += kSumBlock) v += partial[g];
  const double total = block_sum_f64<kSumBlock>(v, s_tmp);
  if (threadIdx.x == 0) *out = total;
}
}  // namespace

bm_status launch_sum_partials(const double* partial, int np, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kSumBlock), 0, stream, partial, np, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BM_EDEVICE, "objective sum launch failed: %s", hipGetErrorString(e));
  return BM_OK;
}

}  // namespace bm
