// Device memory of the allocation-free run (cc_run_static in cc.h): one
// file-scope array per device that holds every buffer such a run needs beyond
// the caller's inputs and outputs -- the packed operation and transaction
// descriptors, the pending list between passes, the ingest owner words and
// the ingest results.  The array lives as long as the process.
//
// Host code never passes `scratch` itself to a kernel: in host code the name
// is a host-side stand-in, not the device address.  static_scratch_address()
// returns the device address of the current device's copy, which the context
// keeps (resolved once per device, at cc_init).
#include <mutex>

#include "device.h"

namespace cce {

static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

// Every device holds its own copy of `scratch` at its own address: resolved
// once per device (with that device current) and kept for the process.
hipError_t static_scratch_address(int device, void **ptr) {
  static std::mutex mu;
  static void *addr[STATIC_MAX_DEVICES] = {};
  *ptr = nullptr;
  if (device < 0 || device >= STATIC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

// Clears n 64-bit words (the caller's read-value array before a run); a fill
// kernel instead of hipMemsetAsync, so that the clear is an ordinary kernel
// node wherever the stream goes.
__global__ void __launch_bounds__(256) fill_zero_kernel(int64_t *p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

hipError_t launch_fill_zero(hipStream_t s, int64_t *p, uint64_t n) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace cce
