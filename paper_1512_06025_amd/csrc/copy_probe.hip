// Plain streaming copy (16-byte vector loads and stores, grid-stride), used
// to measure the HBM bandwidth a simple kernel reaches on the device and to
// calibrate the FETCH_SIZE / WRITE_SIZE counters against a known byte count.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bb_launch.hpp"

namespace bbdg {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Each thread moves 4 chunks of 16 bytes (4 loads in flight before the stores).
__global__ __launch_bounds__(256) void copy_probe_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                        int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  u32x4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + 256 * k;
    if (i < n) v[k] = __builtin_nontemporal_load(src + i);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + 256 * k;
    if (i < n) __builtin_nontemporal_store(v[k], dst + i);
  }
}

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t stream) {
  const int64_t n = (int64_t)(bytes / 16);
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 1023) / 1024;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  hipLaunchKernelGGL(copy_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (const u32x4*)src, (u32x4*)dst, n);
  return hipGetLastError();
}

}  // namespace bbdg
