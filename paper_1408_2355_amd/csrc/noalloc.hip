// Work area of the allocation-free entry point (sp_solve_async_noalloc): one
// file-scope device array, present on every device the library is loaded on
// until the process ends.  Host code never passes the array's name to a
// kernel (in host code it is a stand-in, not a device address): the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current, and is kept per device.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "internal.h"

namespace sp {

namespace {
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;  // device -> address of its copy of scratch
}  // namespace

Arena noalloc_scratch() {
  int dev = 0;
  SP_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      throw Error(SP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    it = g_scratch_ptr.emplace(dev, static_cast<char*>(ptr)).first;
  }
  Arena a;
  a.base = it->second;
  a.size = kScratchBytes;
  a.what = "sp_solve_async_noalloc scratch";
  return a;
}

}  // namespace sp
