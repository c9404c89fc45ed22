// Lane exchanges for the halving reductions of the backward and relaxation
// sweeps (gfx950).  A halving step pairs lane t with lane t ^ m: one lane of
// the pair keeps register a and sends b, the other keeps b and sends a, and
// both add what they receive, so n registers shrink to n / 2 per step.
//
// For m = 32 and m = 16 one v_permlane32_swap / v_permlane16_swap moves the
// two sent halves at once (no selects, no LDS crossbar); for m = 8, 2, 1 the
// partner's value comes from a DPP row move; m = 4 uses a lane shuffle.
// Every step adds the same two values as the plain shuffle butterfly, so
// the sums are bitwise those of that butterfly.
#pragma once

#include <hip/hip_runtime.h>

namespace ibp {

// Lanes with bit 5 clear: a + a of lane t + 32; lanes with bit 5 set: b of
// lane t - 32 + b.
__device__ __forceinline__ float halve32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The same for bit 4 (lane t +- 16).
__device__ __forceinline__ float halve16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ double halve32(double a, double b) {
  const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
  const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  const double r0 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double r1 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return r0 + r1;
}

__device__ __forceinline__ double halve16(double a, double b) {
  const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
  const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  const double r0 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double r1 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return r0 + r1;
}

// A wave-uniform value held in a scalar register, copied into a vector
// register.  On gfx950 a float32 VALU instruction that reads a scalar
// register issues at half the rate of one whose operands are all vector
// registers or constants (8 independent chains per lane, 8 waves per SIMD:
// about 4.7 against 2.7 cycles per wave instruction), so a record value that
// many instructions read is moved once.  The move is written out so that the
// compiler cannot fold the scalar register back into its users; `s` must be
// uniform across the wave (a scalar-loaded record).
__device__ __forceinline__ float vcopy(float s) {
  float v;
  __asm__("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
  return v;
}

// DPP moves within a row of 16 lanes: lane t receives lane t ^ 8 (row
// rotation by 8), t ^ 2 (quad permutation [2,3,0,1]) or t ^ 1 ([1,0,3,2]).
constexpr int kDppXor8 = 0x128;
constexpr int kDppXor2 = 0x4E;
constexpr int kDppXor1 = 0xB1;

template <int CTRL>
__device__ __forceinline__ float lane_xor(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double lane_xor(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The outage factors are finite except the outaged line's own entry, which
// the network builder stores as the positive quiet NaN.  As signed integers,
// positive NaNs and +inf lie above FLT_MAX and every negative float below it,
// so one integer min maps that entry to FLT_MAX and leaves the others as they
// are (fminf would first canonicalise its operand: two instructions).
__device__ __forceinline__ float finite_factor(float lam) {
  return __int_as_float(min(__float_as_int(lam), 0x7f7fffff));
}

}  // namespace ibp
