// Working memory of bddc_solve_noalloc: a fixed device array, so that a solve
// allocates nothing (for callers that cannot allocate device memory).
//
// The per-column PCG state of a solve (iterates, residuals, search
// directions, partial sums, scalars, the condensed load) normally lives in
// an arena of the handle that grows with the number of right-hand sides.
// The no-allocation variant lays the same state out in `scratch` instead.
// Host code never passes `scratch` itself to a kernel (on the host the name
// stands for a host-side shadow, not for device memory): its device address
// is looked up once per device with hipGetSymbolAddress and kept here.
#include <algorithm>
#include <mutex>
#include <string>

#include "common.hpp"
#include "kernels.hpp"

namespace bddc {

static __device__ __align__(256) unsigned char scratch[BDDC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

__global__ void __launch_bounds__(kNT) k_zero_words(uint64_t* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (size_t)gridDim.x * kNT) p[i] = 0;
}

}  // namespace

// Device address of the scratch array on the current device (looked up on
// the first call for that device, with that device current).
void* noalloc_scratch() {
  int dev = 0;
  BDDC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(BDDC_EUNSUPPORTED, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(BDDC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Zero the first `bytes` (a multiple of 8) of a device buffer with a kernel
// (no memset node, so the call may sit in a captured stream).
void launch_zero_bytes(hipStream_t st, void* p, size_t bytes) {
  const size_t n = bytes / 8;
  if (n == 0) return;
  const unsigned blocks = (unsigned)std::min<size_t>(1024, (n + kNT - 1) / kNT);
  launch_kernel(k_zero_words, dim3(blocks), dim3(kNT), 0, st, static_cast<uint64_t*>(p), n);
}

}  // namespace bddc
