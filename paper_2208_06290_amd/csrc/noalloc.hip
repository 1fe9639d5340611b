// Fixed device scratch for the allocation-free solve entry point
// (hodlr_solve_noalloc): a file-scope device array that the code object
// brings with it, so the call needs no device allocation of its own.  Each
// GPU that loads the library holds one copy until the process ends.  Host
// code never passes the array's name to a kernel (in host code it is only a
// stand-in for the symbol); it passes the device address looked up here once
// per device with hipGetSymbolAddress.
#include <mutex>

#include "internal.h"

namespace hodlr {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t scratch_capacity() { return kScratchBytes; }

hipError_t scratch_device_ptr(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace hodlr
