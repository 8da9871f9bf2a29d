// The allocation-free workspace: one static device array that
// tn_contract_grid_static contracts in, so that callers which may not
// allocate (code under stream capture, tight serving loops, harnesses that
// forbid hipMalloc) still get the library's contraction path.
//
// Host code never passes the array's name to a kernel or a copy: in host code
// that name is a host-side stand-in, not a device address.  Its address on
// each device is looked up once with hipGetSymbolAddress (with that device
// current) and only that address is used.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "exec.hpp"

namespace tn {
namespace {

constexpr size_t kScratchBytes = TN_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_lookup_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

tn_status static_scratch(void** ptr, size_t* bytes, std::string& err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return TN_EDEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device index " + std::to_string(dev) + " beyond the static workspace table";
    return TN_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_lookup_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return TN_EDEVICE;
    }
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  *bytes = kScratchBytes;
  return TN_OK;
}

}  // namespace tn
