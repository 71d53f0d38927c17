// Library-owned device workspace for filter_backward_noalloc: a file-scope device array,
// one copy per GPU, held until the process ends. Host code never passes the array's name
// to a kernel (on the host it is a stand-in, not a device address): the first call on a
// device resolves that device's copy with hipGetSymbolAddress, and every launch gets the
// resolved pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.hpp"

namespace ramlt {

namespace {

__device__ __align__(256) unsigned char scratch[kNoallocWorkspaceBytes];

constexpr int kMaxScratchDevices = 64;
std::once_flag g_once[kMaxScratchDevices];
void *g_ptr[kMaxScratchDevices];
hipError_t g_err[kMaxScratchDevices];

}  // namespace

hipError_t noalloc_workspace(void **ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  // once per device, with that device current (it is: hipGetDevice returned it)
  std::call_once(g_once[dev], [dev] {
    void *p = nullptr;
    g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[dev] = g_err[dev] == hipSuccess ? p : nullptr;
  });
  if (g_err[dev] != hipSuccess) return g_err[dev];
  *ptr = g_ptr[dev];
  return hipSuccess;
}

}  // namespace ramlt
