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

// DPP move of a float64 (both 32-bit halves with the same control); lanes of
// rows outside ROWS receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes of a wave (every lane active), returned to every lane.
// Within each row of 16 lanes: quad permutations [1,0,3,2] and [2,3,0,1], then
// the half-row and row mirrors leave the row sum in every lane; the row
// broadcasts of lane 15 (into rows 1 and 3) and lane 31 (into rows 2 and 3)
// then leave the total in lane 63, which is read back as a wave-uniform value.
// No LDS traffic, unlike a butterfly of lane shuffles.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_f64<0x140, 0xF>(v);  // row_mirror
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Maximum over the 64 lanes of a wave (every lane active), the same DPP
// pattern as wave_sum; lanes outside a row mask receive 0, which is neutral.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
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

// SIDES: 3 both penalty bounds, 1 the lower bound only (f_hi), 2 the upper
// bound only (f_lo); the side not computed is 0.
template <int SIDES = 3>
__device__ __forceinline__ void k3_elem(float lam, float cc, float rk, float cl, float h, float g,
                                        float& phi, float& plo) {
  const float C = fmaf(lam, cc, cl);
  phi = 0.0f;
  plo = 0.0f;
  if (SIDES & 2) {
    const float A = fmaf(fabsf(lam), rk, h);
    phi = fmaxf(fabsf(C) + A, 0.0f);
  }
  if (SIDES & 1) {
    const float B = fmaf(fabsf(lam), rk, g);
    plo = fmaxf(fabsf(C) - B, 0.0f);
  }
}

// Two outages x four lines, summed in float32 (depth 3) and added in float64.
template <int SIDES = 3>
__device__ __forceinline__ void k3_pair(const float4& x0, const int4& d0, const float4& x1,
                                        const int4& d1, const float4& c4, const float4& h4,
                                        const float4& g4, double& acc_hi, double& acc_lo) {
  const float cc0 = __int_as_float(d0.y), rk0 = __int_as_float(d0.z);
  const float cc1 = __int_as_float(d1.y), rk1 = __int_as_float(d1.z);
  float a0, a1, a2, a3, b0, b1, b2, b3, e0, e1, e2, e3, f0, f1, f2, f3;
  k3_elem<SIDES>(x0.x, cc0, rk0, c4.x, h4.x, g4.x, a0, b0);
  k3_elem<SIDES>(x0.y, cc0, rk0, c4.y, h4.y, g4.y, a1, b1);
  k3_elem<SIDES>(x0.z, cc0, rk0, c4.z, h4.z, g4.z, a2, b2);
  k3_elem<SIDES>(x0.w, cc0, rk0, c4.w, h4.w, g4.w, a3, b3);
  k3_elem<SIDES>(x1.x, cc1, rk1, c4.x, h4.x, g4.x, e0, f0);
  k3_elem<SIDES>(x1.y, cc1, rk1, c4.y, h4.y, g4.y, e1, f1);
  k3_elem<SIDES>(x1.z, cc1, rk1, c4.z, h4.z, g4.z, e2, f2);
  k3_elem<SIDES>(x1.w, cc1, rk1, c4.w, h4.w, g4.w, e3, f3);
  if (SIDES & 2) acc_hi += (double)(((a0 + a1) + (a2 + a3)) + ((e0 + e1) + (e2 + e3)));
  if (SIDES & 1) acc_lo += (double)(((b0 + b1) + (b2 + b3)) + ((f0 + f1) + (f2 + f3)));
}

__device__ __forceinline__ float add_ru(float a, float b) { return next_up_f32(a + b); }

// IBP of one piecewise-linear curve over x in [c - r, c + r] (Sec. III-B,
// eqs. (single ReLU) and (combined ReLUs)): F*_0 = 0 and
// F*_i = min(F*_{i-1} + a_i max(x - b_i, 0), U_i), node by node as in eq. (IBP):
// the affine node has centre a_i (c - b_i) and radius |a_i| r, the ReLU and the
// cap are monotone (applied to both ends), the sum adds the two intervals.
// float64 round-to-nearest; err bounds the distance of both computed ends from
// the exact ones: with T = sum |a_i| (|c| + |b_i| + r) and Um = max finite |U_i|,
// every intermediate is below T + Um in magnitude and each segment adds at most
// 4u |a_i| (|c| + |b_i| + r) + u (T + Um), so err <= (n + 4) u (T + Um).
__device__ __forceinline__ void curve_ibp(const double4* __restrict__ seg, int s0, int s1, double c, double r,
                                          double& lo, double& hi, double& err) {
#pragma clang fp contract(off)
  lo = 0.0;
  hi = 0.0;
  double T = 0.0, Um = 0.0;
  for (int s = s0; s < s1; ++s) {
    const double4 q = seg[s];
    const double cy = q.x * (c - q.y);
    const double ry = fabs(q.x) * r;
    lo = fmin(lo + fmax(cy - ry, 0.0), q.z);
    hi = fmin(hi + fmax(cy + ry, 0.0), q.z);
    T += fabs(q.x) * (fabs(c) + fabs(q.y) + r);
    Um = fmax(Um, q.w);
  }
  err = ((s1 - s0) + 5) * kU64 * 1.01 * (T + Um);
}

// Derivatives of the two ends of curve_ibp with respect to c and r (forward
// mode): (lc, lr) of the lower end, (hc, hr) of the upper end.  max(z, 0)
// passes the derivative iff z > 0; min(p, U) passes it iff p <= U.  No
// multiply-add contraction, so that z = a (c - b) -+ |a| r is rounded as
// written and an exact kink (z = 0, e.g. lo = b) is taken as such.
__device__ __forceinline__ void curve_ibp_tangents(const double4* __restrict__ seg, int s0, int s1, double c,
                                                   double r, double& lc, double& lr, double& hc, double& hr) {
#pragma clang fp contract(off)
  double lo = 0.0, hi = 0.0;
  lc = lr = hc = hr = 0.0;
  for (int s = s0; s < s1; ++s) {
    const double4 q = seg[s];
    const double cy = q.x * (c - q.y);
    const double ry = fabs(q.x) * r;
    const double zl = cy - ry, zh = cy + ry;
    const double pl = lo + fmax(zl, 0.0), ph = hi + fmax(zh, 0.0);
    double plc = lc, plr = lr, phc = hc, phr = hr;
    if (zl > 0.0) {
      plc += q.x;
      plr -= fabs(q.x);
    }
    if (zh > 0.0) {
      phc += q.x;
      phr += fabs(q.x);
    }
    if (pl <= q.z) {
      lo = pl;
      lc = plc;
      lr = plr;
    } else {
      lo = q.z;
      lc = lr = 0.0;
    }
    if (ph <= q.z) {
      hi = ph;
      hc = phc;
      hr = phr;
    } else {
      hi = q.z;
      hc = hr = 0.0;
    }
  }
}


}  // namespace ibp
