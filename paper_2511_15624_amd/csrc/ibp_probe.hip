// Calibration probes.  Streaming-read bandwidth: the load pattern of the
// library's HBM-bound sweeps (float4 nontemporal loads, eight in flight per
// lane; 2048 blocks x 256 threads, each block streaming a contiguous range)
// with a trivial sum, so that a caller can measure the read rate those sweeps
// can reach on this device.  Float32 FMA issue rate: eight independent FMA
// chains per lane on the same grid (eight waves per SIMD), with every operand
// in a vector register or one in a scalar register, so that a caller can
// measure the vector-ALU rate the ALU-bound sweeps are priced against.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ibp_devfun.h"
#include "ibp_kernels.h"
#include "ibp_lanes.h"

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

// a <- a b + c per chain (b = 0.5, c = 1 from the caller: every chain reaches
// the fixed point 2 exactly after a few dozen steps); SCALAR = 1 reads b from
// its scalar register, SCALAR = 0 from a vector copy.
template <int SCALAR>
__global__ __launch_bounds__(256) void alu_probe(float* out, int64_t iters, float b, float c) {
  const float vb = vcopy(b), vc = vcopy(c);
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = 1.0f + 0.125f * j;
  // 32 FMAs between loop branches
  int64_t it = 0;
  for (; it + 4 <= iters; it += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] = fmaf(a[j], SCALAR ? b : vb, vc);
  }
  for (; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = fmaf(a[j], SCALAR ? b : vb, vc);
  }
  float t = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) t += a[j];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = t;
}

hipError_t launch_alu_probe(float* out, int64_t iters, int scalar, hipStream_t s) {
  if (scalar)
    hipLaunchKernelGGL(alu_probe<1>, dim3(kProbeBlocks), dim3(256), 0, s, out, iters, 0.5f, 1.0f);
  else
    hipLaunchKernelGGL(alu_probe<0>, dim3(kProbeBlocks), dim3(256), 0, s, out, iters, 0.5f, 1.0f);
  return hipGetLastError();
}

}  // namespace ibp
