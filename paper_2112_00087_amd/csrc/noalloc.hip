// Allocation-free variant of the complex dot product, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops).  The reduction's partial sums live in a file-scope device array of
// fixed size instead of a buffer the library allocates; the result goes to
// device memory, so the call neither allocates nor synchronises.
#include <mutex>

#include "ops.h"

namespace {

// reduce_grid() caps a reduction at 1024 blocks of partial sums (re, im):
// 16 KiB covers every n.
constexpr int kScratchBlocks = 1024;
__device__ __align__(256) double scratch[2 * kScratchBlocks];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
// Device address of `scratch` on each device (each GPU holds its own copy of
// the array).  In host code the array's name is only a host-side stand-in:
// kernels receive these addresses, never `scratch` itself.
double* g_scratch[kMaxDevices] = {};

}  // namespace

// Looks up the device address of `scratch` on `device`, which must be the
// current device.  Done once per device, at context creation.
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return hz_fail(HZ_ERR_INVALID, "device %d beyond the %d the allocation-free calls support", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return HZ_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return hz_fail(HZ_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  g_scratch[device] = static_cast<double*>(p);
  return HZ_OK;
}

extern "C" int hz_dotc_noalloc(hz_ctx ctx, int64_t n, const hz_c128* a_dev, const hz_c128* b_dev,
                               hz_c128* out_dev) {
  try {
    if (!ctx) return hz_fail(HZ_ERR_INVALID, "ctx is NULL");
    if (!a_dev || !b_dev || !out_dev || n < 0) return hz_fail(HZ_ERR_INVALID, "bad arguments");
    int dev = -1;
    HZ_HIP(hipGetDevice(&dev));
    if (dev != ctx->device) HZ_HIP(hipSetDevice(ctx->device));
    if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_scratch[ctx->device])
      HZ_TRY(noalloc_setup(ctx->device));
    if (reduce_grid(n) > kScratchBlocks)
      return hz_fail(HZ_ERR_INVALID, "n = %lld needs %d partial sums, more than the %d of the static scratch",
                     static_cast<long long>(n), reduce_grid(n), kScratchBlocks);
    return op_dotc_into(ctx->stream, n, reinterpret_cast<const z_t*>(a_dev), reinterpret_cast<const z_t*>(b_dev),
                        g_scratch[ctx->device], reinterpret_cast<double*>(out_dev));
  } catch (...) {
    return hz_fail(HZ_ERR_INVALID, "unexpected exception in the library");
  }
}
