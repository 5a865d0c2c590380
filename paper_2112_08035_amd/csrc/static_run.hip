// static_run.hip -- the fixed device scratch of smcrt_run_ex_static: a
// file-scope device array each GPU holds from the library's first use on it
// until the process ends, so a run needs no device allocation.  Host code
// never passes the array's name to a kernel (in host code it is a host-side
// stand-in, not a device address): its address on each device is looked up
// once, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.h"

namespace smcrt {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices || !out) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

// the job record travels as a kernel argument (copied when the launch is
// queued), so no host buffer has to outlive the call
__global__ void write_job_kernel(WalkArgs a, WalkArgs* __restrict__ dst) { *dst = a; }

hipError_t launch_write_job(const WalkArgs& a, WalkArgs* dst, hipStream_t stream) {
  if (!dst) return hipErrorInvalidValue;
  hipLaunchKernelGGL(write_job_kernel, dim3(1), dim3(1), 0, stream, a, dst);
  return hipGetLastError();
}

}  // namespace smcrt
