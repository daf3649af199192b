// The library's own device scratch for callers that cannot allocate (code
// under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
// a fixed array in the code object, one copy per GPU, held until the process
// ends.  gsr_render_forward_noalloc runs the forward with its workspace here.
//
// In host code the array's name is only a stand-in for the symbol, not a
// device address; the address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress (with that device current) and used
// everywhere host code passes the memory on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace gsr {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t scratch_address(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

}  // namespace gsr
