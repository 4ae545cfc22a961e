// Device scratch of the no-allocation estimator entry point.
//
// The array lives in the library's code object: each device the library is
// loaded on holds its own copy, from module load until the process ends.
// Host code never uses the array's name as an address (in host code it is
// a stand-in, not device memory); it resolves the device address with
// hipGetSymbolAddress, once per device with that device current, and hands
// that pointer to the kernels.  Every call on one device shares the array:
// calls that overlap on a device race (they must be serialized by the
// caller), and the array keeps the last call's contents (the estimator
// writes every value before reading it, so nothing needs clearing).
#include <mutex>

#include "internal.hpp"

namespace tlrqmc {

namespace {

constexpr int64_t kNoAllocBytes = int64_t{256} << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

int64_t noalloc_scratch_bytes() { return kNoAllocBytes; }

int noalloc_resolve(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(TLRQMC_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> g(g_mu);
  if (g_ptr[device]) return TLRQMC_OK;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return fail(TLRQMC_EDEVICE, "hipGetDevice failed");
  if (hipSetDevice(device) != hipSuccess) return fail(TLRQMC_EDEVICE, "hipSetDevice(%d) failed", device);
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  (void)hipSetDevice(cur);
  if (e != hipSuccess || !p)
    return fail(TLRQMC_EDEVICE, "hipGetSymbolAddress of the no-allocation scratch failed on device %d: %s", device,
                hipGetErrorString(e));
  g_ptr[device] = p;
  return TLRQMC_OK;
}

void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  return g_ptr[device];
}

}  // namespace tlrqmc
