// The display of a spectrum grid for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same work as
// wdd_display, with its scratch in a fixed device array instead of a stream-ordered
// allocation.
#include <hip/hip_runtime.h>

#include <mutex>

#include "wdd_internal.h"

namespace {

// Two 1024 x 1024 complex grids and the twiddles of two sides of up to 4096 values.
constexpr int64_t kNoAllocMaxCells = (int64_t)1 << 20;
constexpr size_t kScratchFloats = ((size_t)2 * kNoAllocMaxCells + 2 * wdd::kDisplayMaxSide) * 2;

// Each GPU the library runs on holds one copy of this array until the process ends.  Host
// code never uses its name as an address: the device address comes from
// hipGetSymbolAddress, per device (scratch_ptr).
__device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device with that device
// current.
wdd_status scratch_ptr(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return wdd::fail(WDD_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return wdd::fail(WDD_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return wdd::fail(WDD_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return WDD_OK;
}

}  // namespace

extern "C" {

wdd_status wdd_display_noalloc(const float* spectrum, int32_t sy, int32_t sx, float* out, void* hip_stream) {
  wdd_status st = wdd::check_display_args(spectrum, sy, sx, out);
  if (st != WDD_OK) return st;
  if ((int64_t)sy * sx > kNoAllocMaxCells)
    return wdd::fail(WDD_EINVAL, "grid %d x %d exceeds the %lld cells of the fixed scratch", sy, sx,
                     (long long)kNoAllocMaxCells);
  if (wdd::display_scratch_floats(sy, sx) > kScratchFloats)
    return wdd::fail(WDD_EINVAL, "grid %d x %d exceeds the fixed scratch", sy, sx);
  float* scr = nullptr;
  if ((st = scratch_ptr(&scr)) != WDD_OK) return st;
  return wdd::display_grid(spectrum, sy, sx, out, scr, hip_stream);
}

}  // extern "C"
