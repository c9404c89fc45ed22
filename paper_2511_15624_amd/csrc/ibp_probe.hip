// Streaming-read bandwidth probe: the load pattern of the library's HBM-bound
// sweeps (float4 nontemporal loads, eight in flight per lane; 2048 blocks x 256
// threads, each block streaming a contiguous range) with a trivial sum, so that
// a caller can measure the read rate those sweeps can reach on this device.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ibp_devfun.h"
#include "ibp_kernels.h"

namespace ibp {

constexpr int kProbeBlocks = 2048;

__global__ __launch_bounds__(256) void read_probe(const float4* __restrict__ src, int64_t n, float* partial) {
  // block b streams its own contiguous range, 256 lanes x 8 float4 per step
  const int64_t per = (n + kProbeBlocks - 1) / kProbeBlocks;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = min(n, b0 + per);
  float acc = 0.0f;
  int64_t i = b0 + threadIdx.x;
  for (; i + 7 * 256 < b1; i += 8 * 256) {
    float4 x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = ld_stream(src + i + u * 256);
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (x[u].x + x[u].y) + (x[u].z + x[u].w);
  }
  for (; i < b1; i += 256) {
    const float4 x = ld_stream(src + i);
    acc += (x.x + x.y) + (x.z + x.w);
  }
  __shared__ float sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int m = 128; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m) sh[threadIdx.x] += sh[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

hipError_t launch_read_probe(const float4* src, int64_t n, float* partial, hipStream_t s) {
  hipLaunchKernelGGL(read_probe, dim3(kProbeBlocks), dim3(256), 0, s, src, n, partial);
  return hipGetLastError();
}

}  // namespace ibp
