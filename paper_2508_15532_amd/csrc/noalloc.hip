// Scratch of the allocation-free step entry point (rt_step_noalloc).
//
// The array below is the library's only device memory that is not allocated
// at run time: a file-scope static device array that every device holds from
// the moment the code object is loaded until the process ends.  In host code
// its name is a host-side stand-in, never a device address, so host code
// resolves the address once per device with hipGetSymbolAddress (with that
// device current) and afterwards uses only the resolved pointer: as kernel
// arguments, for fills and copies.  All calls on one device share the array;
// calls that overlap on one device race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx.hpp"

namespace rt {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* noalloc_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace rt
