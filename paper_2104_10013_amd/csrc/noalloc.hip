// Static device scratch for the allocation-free loss-and-gradient entry point.
//
// The array below holds, for ddp_loss_and_grad_static, what the handle's own
// buffers hold for ddp_loss_and_grad: the work counters of the persistent
// train launches (first kStaticCounterBytes) and the per-workgroup activation
// stash slots (the rest).  It lives in this translation unit only, so a
// process that never calls that entry point never loads it.  Each device the
// library runs on gets its own copy when this module is first used there and
// keeps it until the process ends.
//
// Host code never passes the array's name to a kernel: on the host that name
// is a stand-in, not a device address.  static_scratch() looks up the address
// with hipGetSymbolAddress once per device (that device current) and every
// launch takes that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace ddp {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// counters of the train launches start at zero (a fill kernel, not a memset,
// so the call can be captured into a graph)
__global__ void k_zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t static_scratch(int device, void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes the device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace ddp
