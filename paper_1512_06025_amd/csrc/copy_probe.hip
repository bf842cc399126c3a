// Plain streaming copy (16-byte vector loads and stores, grid-stride), used
// to measure the HBM bandwidth a simple kernel reaches on the device and to
// calibrate the FETCH_SIZE / WRITE_SIZE counters against a known byte count.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bb_launch.hpp"

namespace bbdg {

__global__ __launch_bounds__(256) void copy_probe_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                        int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t stream) {
  const int64_t n = (int64_t)(bytes / 16);
  if (n <= 0) return hipSuccess;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return hipErrorInvalidDevice;
  int64_t blocks = (n + 255) / 256;
  const int64_t cap = (int64_t)cus * 16;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(copy_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (const uint4*)src, (uint4*)dst, n);
  return hipGetLastError();
}

}  // namespace bbdg
