// bm_noalloc.hip -- kmeans_assign_noalloc: the assignment step and objective
// of kmeans_assign (Sec. 2, Eq. (1)) for callers that cannot allocate device
// memory.  Its scratch (the degenerate flags, per-workgroup partial
// objectives, the objective and the recheck count) lives in a fixed static
// device array instead of the library's
// growing pool; the kernels are the ones kmeans_assign launches.
//
// The array is a host-side stand-in in host code: its device address is taken
// once per device with hipGetSymbolAddress (with that device current) and
// only that address is ever handed to kernels or copies.
#include <mutex>

#include "bm_internal.h"

namespace bm {

namespace {

constexpr size_t kNoAllocScratchBytes = 64 * 1024;  // fixed per device, held until exit
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_noalloc_mu;             // calls on every device are serialised
void* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of this device's copy of `scratch` (set up on first use).
bm_status scratch_address(int dev, unsigned char** out) {
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(BM_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_dev[dev]);
  return BM_OK;
}

// Clears the recheck count (a kernel rather than a memset, so the call is
// safe inside a caller's graph capture).
__global__ void noalloc_clear_kernel(unsigned long long* rechecked) {
  if (threadIdx.x == 0) *rechecked = 0ull;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

}  // namespace bm

using namespace bm;

extern "C" bm_status kmeans_assign_noalloc(const void* X, int64_t n, int32_t d, const float* C,
                                           const uint8_t* deg, int32_t k, const bm_options* opt_in,
                                           int32_t* labels, float* min_d2, double* sse) {
  clear_error();
  bm_options o;
  bm_status st = resolve_options(opt_in, &o);
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
  const bool mfma = o.precision == BM_PREC_BF16_MFMA;
  hipStream_t stream = static_cast<hipStream_t>(o.stream);

  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return set_error(BM_EDEVICE, "no current HIP device");
  unsigned char* base = nullptr;
  if ((st = scratch_address(dev, &base)) != BM_OK) return st;

  int grid = assign_grid(n, d);
  if (mfma && (st = plan_assign_mfma(X, n, d, k, &grid)) != BM_OK) return st;
  // layout: flags | partials | objective | recheck count
  const size_t off_deg = 0;
  const size_t off_part = align256(off_deg + static_cast<size_t>(k));
  const size_t off_sse = align256(off_part + sizeof(double) * static_cast<size_t>(grid));
  const size_t off_rechk = off_sse + 64;
  const size_t need = off_rechk + 64;
  if (need > kNoAllocScratchBytes)
    return set_error(BM_EINVAL,
                     "kmeans_assign_noalloc needs %zu B of scratch for k=%d and %d workgroups; "
                     "its fixed scratch holds %zu B", need, k, grid, kNoAllocScratchBytes);
  uint8_t* deg_p = base + off_deg;
  double* partial_p = reinterpret_cast<double*>(base + off_part);
  double* sse_p = reinterpret_cast<double*>(base + off_sse);
  unsigned long long* rechecked_p = reinterpret_cast<unsigned long long*>(base + off_rechk);

  if (deg) {
    const hipError_t e = hipMemcpyAsync(deg_p, deg, size_t(k), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return set_error(BM_EDEVICE, "flag copy failed: %s", hipGetErrorString(e));
  }
  hipLaunchKernelGGL(noalloc_clear_kernel, dim3(1), dim3(64), 0, stream, rechecked_p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BM_EDEVICE, "clear launch failed: %s", hipGetErrorString(e));
  if (mfma) {
    st = launch_assign_mfma(static_cast<const uint16_t*>(X), n, d, C, deg ? deg_p : nullptr, k,
                            labels, min_d2, partial_p, sse_p, rechecked_p, grid, stream);
  } else {
    st = launch_assign(X, o.x_dtype == BM_BF16, n, d, C, deg ? deg_p : nullptr, k, labels, min_d2,
                       partial_p, sse_p, grid, stream);
  }
  if (st != BM_OK) return st;
  double v = 0.0;
  e = hipMemcpyAsync(&v, sse_p, sizeof v, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return set_error(BM_EDEVICE, "kmeans_assign_noalloc: %s", hipGetErrorString(e));
  if (sse) *sse = v;
  return BM_OK;
}
