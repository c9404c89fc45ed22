// Device-side helpers shared by the forward, batched and backward kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "ibp_device.h"

namespace ibp {

__device__ __forceinline__ float next_up_f32(float f) {
  if (!(f < INFINITY)) return f;  // +inf or NaN
  if (f == 0.0f) return __int_as_float(1);
  int b = __float_as_int(f);
  return __int_as_float(f > 0.0f ? b + 1 : b - 1);
}

// Smallest float32 >= x.
__device__ __forceinline__ float ru32(double x) {
  float f = (float)x;
  return ((double)f < x) ? next_up_f32(f) : f;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
}

// Block-wide sum over 256 threads (4 waves); every thread gets the result.
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}

// Streaming load of a float4 that is read exactly once (nontemporal hint: the
// line is not kept in the caches).
typedef float vf4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_stream(const float4* p) {
  const vf4_t t = __builtin_nontemporal_load(reinterpret_cast<const vf4_t*>(p));
  return make_float4(t.x, t.y, t.z, t.w);
}

template <typename T>
__device__ __forceinline__ T* ws_ptr(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

__device__ __forceinline__ void k3_elem(float lam, float cc, float rk, float cl, float h, float g,
                                        float& phi, float& plo) {
  const float C = fmaf(lam, cc, cl);
  const float A = fmaf(fabsf(lam), rk, h);
  const float B = fmaf(fabsf(lam), rk, g);
  phi = fmaxf(fabsf(C) + A, 0.0f);
  plo = fmaxf(fabsf(C) - B, 0.0f);
}

// Two outages x four lines, summed in float32 (depth 3) and added in float64.
__device__ __forceinline__ void k3_pair(const float4& x0, const int4& d0, const float4& x1,
                                        const int4& d1, const float4& c4, const float4& h4,
                                        const float4& g4, double& acc_hi, double& acc_lo) {
  const float cc0 = __int_as_float(d0.y), rk0 = __int_as_float(d0.z);
  const float cc1 = __int_as_float(d1.y), rk1 = __int_as_float(d1.z);
  float a0, a1, a2, a3, b0, b1, b2, b3, e0, e1, e2, e3, f0, f1, f2, f3;
  k3_elem(x0.x, cc0, rk0, c4.x, h4.x, g4.x, a0, b0);
  k3_elem(x0.y, cc0, rk0, c4.y, h4.y, g4.y, a1, b1);
  k3_elem(x0.z, cc0, rk0, c4.z, h4.z, g4.z, a2, b2);
  k3_elem(x0.w, cc0, rk0, c4.w, h4.w, g4.w, a3, b3);
  k3_elem(x1.x, cc1, rk1, c4.x, h4.x, g4.x, e0, f0);
  k3_elem(x1.y, cc1, rk1, c4.y, h4.y, g4.y, e1, f1);
  k3_elem(x1.z, cc1, rk1, c4.z, h4.z, g4.z, e2, f2);
  k3_elem(x1.w, cc1, rk1, c4.w, h4.w, g4.w, e3, f3);
  acc_hi += (double)(((a0 + a1) + (a2 + a3)) + ((e0 + e1) + (e2 + e3)));
  acc_lo += (double)(((b0 + b1) + (b2 + b3)) + ((f0 + f1) + (f2 + f3)));
}

__device__ __forceinline__ float add_ru(float a, float b) { return next_up_f32(a + b); }


}  // namespace ibp
