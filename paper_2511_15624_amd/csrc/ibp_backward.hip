// Backward kernels: vector-Jacobian product of the IBP bounds with respect to
// the box endpoints.
//
// The map differentiated is the IBP of Sec. III-C through the graph of the
// Appendix, eq. (ibp_f), without the outward padding: with (c, r) the centre
// and radius of a flow interval and fmax its limit, the penalties
//   P_hi = max(|c| + r - fmax, 0)  (enters f_lo with weight -zeta)
//   P_lo = max(|c| - r - fmax, 0)  (enters f_hi with weight -zeta)
// have dP_hi/dc = sign(c) [t_hi > 0], dP_hi/dr = [t_hi > 0],
//      dP_lo/dc = sign(c) [t_lo > 0], dP_lo/dr = -[t_lo > 0]
// (sign(0) = 0; a max is active only when its argument is > 0).  Post-outage
// flows C = c_l + Lam c_c, R = r_l + |Lam| r_c (Sec. II-C, eq. ctg flow
// simplified per line) send dC to c_l and Lam dC to c_c, dR to r_l and |Lam| dR
// to r_c.  Line gradients go to injections through Phi^T and |Phi|^T
// (Sec. II-A, eq. line flow ptdf), injections to inputs through N_g, -N_d, and
// d lo = (d c - d r)/2, d hi = (d c + d r)/2.
//
//   K5   outage sweep: streams the outage factors once; per-line sums stay in
//        registers, per-outage sums are reduced across the wave by a halving
//        butterfly (32 values in 32 exchanges).
//   K5r  per line: base-case penalty gradient plus the K5 partials.
//   K6   per bus: transposed PTDF products.
//   K7   per input: endpoint gradients, with the surplus and imbalance terms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "ibp_device.h"
#include "ibp_devfun.h"
#include "ibp_kernels.h"
#include "ibp_lanes.h"

namespace ibp {

// outages per block row: 128 for the per-box sweep (enough blocks for one
// box), 512 for the box-tiled sweep, whose per-line partials (one float2 per
// row, box and line) then take half the traffic (4096 boxes: 14.16 -> 13.8 ms;
// 512 outages per row: 13.99 -> 13.73 ms for the whole backward; 1024 per row
// trades a slower sweep for a faster line pass, no net change;
// the chunk must be a compile-time constant for that: a runtime bound gave 14.07)
constexpr int kK5Chunk = 128;
constexpr int kK5ChunkTiled = 512;
constexpr int kK5Sub = 16;     // outages per butterfly reduction

// Sums v[0..31] over the 64 lanes of a wave; afterwards lanes 2i and 2i+1
// hold the total of v[i].
__device__ __forceinline__ float butterfly32(float (&v)[32]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = halve32(v[i], v[i + 16]);
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = halve16(v[i], v[i + 8]);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool up = lane & 8;
    const float send = up ? v[i] : v[i + 4];
    const float keep = up ? v[i + 4] : v[i];
    v[i] = keep + lane_xor<kDppXor8>(send);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const bool up = lane & 4;
    const float send = up ? v[i] : v[i + 2];
    const float keep = up ? v[i + 2] : v[i];
    v[i] = keep + __shfl_xor(send, 4, 64);
  }
  {
    const bool up = lane & 2;
    const float send = up ? v[0] : v[1];
    const float keep = up ? v[1] : v[0];
    v[0] = keep + lane_xor<kDppXor2>(send);
  }
  return v[0] + lane_xor<kDppXor1>(v[0]);
}

// One element of the outage sweep's VJP.  rlm = r_l - fmax_l and
// rlp = r_l + fmax_l per line.  Adds (dC, dR) to (gc, gr) and the
// outage-side contributions Lam dC, |Lam| dR to (pc, pr).  SIDES selects
// the penalty sides with a nonzero upstream weight: 3 both, 1 the lower
// side only (chi = 0: the gradient of f_hi), 2 the upper side only (clo = 0:
// the gradient of f_lo); a side whose weight is zero contributes exactly
// zero, so skipping it changes nothing but the sign of a zero.
template <int SIDES>
__device__ __forceinline__ void k5_elem(float lam, float lam0, float cc, float rc, float cl, float rlm, float rlp,
                                        float chi, float clo, float& gc, float& gr, float& pc, float& pr) {
  // The outaged line's own entry holds NaN: both activity tests fail and
  // dC = dR = 0 (the paper's mask M).  lam0 = finite_factor(lam) keeps the NaN
  // out of the outage-side products, which then add 0.
  const float C = fmaf(lam, cc, cl);
  const float a = fabsf(C);
  float hi = 0.0f, lo = 0.0f;
  if (SIDES & 2) {
    const float thi = a + fmaf(fabsf(lam), rc, rlm);  // |C| + R - fmax
    hi = thi > 0.0f ? chi : 0.0f;
  }
  if (SIDES & 1) {
    const float tlo = a - fmaf(fabsf(lam), rc, rlp);  // |C| - R - fmax
    lo = tlo > 0.0f ? clo : 0.0f;
  }
  const float s = SIDES == 3 ? hi + lo : (SIDES == 1 ? lo : hi);
  const float dR = SIDES == 3 ? hi - lo : (SIDES == 1 ? -lo : hi);
  // sign(C) (hi + lo) by flipping the sign bit when C is negative; C = 0
  // exactly only happens for a line whose flow interval is {0} here, where no
  // penalty is active and hi + lo = 0
  const float dC = __int_as_float(__float_as_int(s) ^ (__float_as_int(C) & (int)0x80000000));
  gc += dC;
  gr += dR;
  pc = fmaf(lam0, dC, pc);
  pr = fmaf(fabsf(lam0), dR, pr);
}

// Line data of the backward sweep for the four lines of float4 column `col`:
// centre, r - fmax and r + fmax (padding lines: 0, -FLT_MAX, +FLT_MAX).
__device__ __forceinline__ void line_radii(const DevNet& net, void* ws, const WsLayout& lay, int64_t b, int col,
                                           bool on, float4& c4, float4& rm4, float4& rp4) {
  c4 = make_float4(0.f, 0.f, 0.f, 0.f);
  rm4 = make_float4(-FLT_MAX, -FLT_MAX, -FLT_MAX, -FLT_MAX);
  rp4 = make_float4(FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX);
  if (!on) return;
  c4 = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lc) + b * net.Lp)[col];
  const float4 f4 = reinterpret_cast<const float4*>(net.fmax_c32)[col];
  const double* rf = ws_ptr<double>(ws, lay.lrf) + b * net.L;
  const int l0 = 4 * col;
  const float r0 = l0 < net.L ? (float)rf[l0] : 0.f, r1 = l0 + 1 < net.L ? (float)rf[l0 + 1] : 0.f;
  const float r2 = l0 + 2 < net.L ? (float)rf[l0 + 2] : 0.f, r3 = l0 + 3 < net.L ? (float)rf[l0 + 3] : 0.f;
  rm4 = make_float4(r0 - f4.x, r1 - f4.y, r2 - f4.z, r3 - f4.w);
  rp4 = make_float4(r0 + f4.x, r1 + f4.y, r2 + f4.z, r3 + f4.w);
}

__global__ __launch_bounds__(256) void k5_outage_vjp(DevNet net, void* ws, WsLayout lay, int64_t box0,
                                                     const double* __restrict__ g_lo,
                                                     const double* __restrict__ g_hi) {
  const int64_t b = box0 + blockIdx.z;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = blockIdx.x * 4 + w;
  const int col = tile * 64 + lane;
  const int Lp4 = net.Lp / 4;
  if (tile * 64 >= Lp4) return;  // whole wave beyond the lines (uniform)
  const bool on = col < Lp4;
  const int k0 = blockIdx.y * kK5Chunk;
  const int k1 = min(net.K, k0 + kK5Chunk);
  const float chi = (float)(-net.zeta_f * (g_lo ? g_lo[b] : 0.0));  // weight of an active P_hi
  const float clo = (float)(-net.zeta_f * (g_hi ? g_hi[b] : 0.0));  // weight of an active P_lo (dR gets -clo)
  // lines of this lane (padding lines: zero centre and radius, limit FLT_MAX)
  float4 c4 = make_float4(0.f, 0.f, 0.f, 0.f), rm4, rp4;
  line_radii(net, ws, lay, b, col, on, c4, rm4, rp4);
  const int4* cd = ws_ptr<int4>(ws, lay.ctg) + b * net.K;
  const float4* lam = reinterpret_cast<const float4*>(net.lodf) + col;
  float2* cpart = ws_ptr<float2>(ws, lay.cpart) + ((size_t)b * lay.k5_tiles + tile) * net.K;
  double gcl[4] = {0, 0, 0, 0}, grl[4] = {0, 0, 0, 0};
  for (int ks = k0; ks < k1; ks += kK5Sub) {
    float v[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = 0.0f;
    float gc[4] = {0, 0, 0, 0}, gr[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < kK5Sub; ++i) {
      const int k = ks + i;
      if (k < k1) {  // uniform
        const int4 d = cd[k];
        const float cc = __int_as_float(d.y), rc = __int_as_float(d.w);
        const float4 x = on ? lam[(size_t)k * Lp4] : make_float4(0.f, 0.f, 0.f, 0.f);
        float pc = 0.0f, pr = 0.0f;
        k5_elem<3>(x.x, finite_factor(x.x), cc, rc, c4.x, rm4.x, rp4.x, chi, clo, gc[0], gr[0], pc, pr);
        k5_elem<3>(x.y, finite_factor(x.y), cc, rc, c4.y, rm4.y, rp4.y, chi, clo, gc[1], gr[1], pc, pr);
        k5_elem<3>(x.z, finite_factor(x.z), cc, rc, c4.z, rm4.z, rp4.z, chi, clo, gc[2], gr[2], pc, pr);
        k5_elem<3>(x.w, finite_factor(x.w), cc, rc, c4.w, rm4.w, rp4.w, chi, clo, gc[3], gr[3], pc, pr);
        v[2 * i] = pc;
        v[2 * i + 1] = pr;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      gcl[j] += (double)gc[j];
      grl[j] += (double)gr[j];
    }
    const float tot = butterfly32(v);
    const int idx = lane >> 1;  // value index: outage ks + idx / 2, field idx % 2
    const int k = ks + (idx >> 1);
    if ((lane & 1) == 0 && k < k1) {
      float* dst = reinterpret_cast<float*>(cpart + k);
      dst[idx & 1] = tot;
    }
  }
  if (on) {
    float2* lp = ws_ptr<float2>(ws, lay.lpart) + ((size_t)b * lay.k5_by + blockIdx.y) * net.Lp + 4 * col;
#pragma unroll
    for (int j = 0; j < 4; ++j) lp[j] = make_float2((float)gcl[j], (float)grl[j]);
  }
}

// Many boxes: the outage sweep's VJP for 4 boxes x 256 lines per wave; the
// four waves of a block take four box tiles of the same line tile, so each
// outage-factor tile serves 16 boxes.  Per-outage sums of 4 outages x 4 boxes
// x 2 fields go through one 32-value butterfly.
constexpr int kBT5 = 4;

// One step of the box-tiled backward sweep: outages ks .. ks + 3 (FULL) or
// ks .. k1 - 1 for kBT5 boxes and the four lines of each lane; per-outage
// (centre, radius) partials through one 32-value butterfly, stored for box
// b0 + i at cp[(b0 + i) * box_stride + k].
template <int S, bool FULL>
__device__ __forceinline__ void k5b_step(const float4 (&x)[4], const float2 (&q)[kBT5][4], const float4 (&c4)[kBT5],
                                         const float4 (&rm4)[kBT5], const float4 (&rp4)[kBT5],
                                         const float (&chi)[kBT5], const float (&clo)[kBT5],
                                         float (&gc)[kBT5][4], float (&gr)[kBT5][4], int ks, int k1, int lane,
                                         int64_t b0, int64_t n_box, float2* cp, size_t box_stride) {
  const int nk = FULL ? 4 : min(4, k1 - ks);
  float v[32];
#pragma unroll
  for (int u = 0; u < 32; ++u) v[u] = 0.0f;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    if (FULL || kk < nk) {  // uniform
      const float l0x = finite_factor(x[kk].x), l0y = finite_factor(x[kk].y);
      const float l0z = finite_factor(x[kk].z), l0w = finite_factor(x[kk].w);
#pragma unroll
      for (int i = 0; i < kBT5; ++i) {
        const float cc = q[i][kk].x, rc = q[i][kk].y;
        float pc = 0.0f, pr = 0.0f;
        k5_elem<S>(x[kk].x, l0x, cc, rc, c4[i].x, rm4[i].x, rp4[i].x, chi[i], clo[i], gc[i][0], gr[i][0], pc, pr);
        k5_elem<S>(x[kk].y, l0y, cc, rc, c4[i].y, rm4[i].y, rp4[i].y, chi[i], clo[i], gc[i][1], gr[i][1], pc, pr);
        k5_elem<S>(x[kk].z, l0z, cc, rc, c4[i].z, rm4[i].z, rp4[i].z, chi[i], clo[i], gc[i][2], gr[i][2], pc, pr);
        k5_elem<S>(x[kk].w, l0w, cc, rc, c4[i].w, rm4[i].w, rp4[i].w, chi[i], clo[i], gc[i][3], gr[i][3], pc, pr);
        v[(kk * kBT5 + i) * 2] = pc;
        v[(kk * kBT5 + i) * 2 + 1] = pr;
      }
    }
    // The line accumulators are updated here, outage by outage: without the
    // (empty) pin the compiler defers every update of a branch-free step to
    // its end and holds all 64 elements' terms at once (256 registers).
#pragma unroll
    for (int i = 0; i < kBT5 && FULL; ++i)
      asm volatile("" : "+v"(gc[i][0]), "+v"(gc[i][1]), "+v"(gc[i][2]), "+v"(gc[i][3]), "+v"(gr[i][0]),
                   "+v"(gr[i][1]), "+v"(gr[i][2]), "+v"(gr[i][3]));
  }
  const float tot = butterfly32(v);
  const int idx = lane >> 1;  // (outage ks + idx / 8, box idx / 2 % 4, field idx % 2)
  const int k = ks + (idx >> 3);
  const int i = (idx >> 1) & 3;
  if ((lane & 1) == 0 && (FULL || k < k1) && b0 + i < n_box)
    reinterpret_cast<float*>(cp + (size_t)(b0 + i) * box_stride + k)[idx & 1] = tot;
}

// MODE 1 / 2: the caller asked for the gradient of f_hi / f_lo alone (the
// other weight pointer is null), so only that side's code is compiled into
// the kernel (fewer registers, more waves); MODE 3 picks the sides per wave.
template <int MODE>
__global__ __launch_bounds__(256) void k5b_outage_vjp(DevNet net, void* ws, WsLayout lay, int64_t n_box,
                                                      const double* __restrict__ g_lo,
                                                      const double* __restrict__ g_hi,
                                                      const float2* __restrict__ cb_all,
                                                      float2* __restrict__ cpart_all) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t b0 = ((int64_t)blockIdx.z * 4 + w) * kBT5;
  if (b0 >= n_box) return;
  const int tile = blockIdx.x;
  const int col = tile * 64 + lane;
  const int Lp4 = net.Lp / 4;
  const bool on = col < Lp4;
  const int k0 = blockIdx.y * kK5ChunkTiled;
  const int k1 = min(net.K, k0 + kK5ChunkTiled);
  int64_t bb[kBT5];
  float chi[kBT5], clo[kBT5];
  float4 c4[kBT5], rm4[kBT5], rp4[kBT5];
  const float2* cd[kBT5];
#pragma unroll
  for (int i = 0; i < kBT5; ++i) {
    bb[i] = min(b0 + i, n_box - 1);
    chi[i] = (float)(-net.zeta_f * (g_lo ? g_lo[bb[i]] : 0.0));
    clo[i] = (float)(-net.zeta_f * (g_hi ? g_hi[bb[i]] : 0.0));
    line_radii(net, ws, lay, bb[i], col, on, c4[i], rm4[i], rp4[i]);
    cd[i] = cb_all + bb[i] * net.K;
  }
  // lanes past the last column read the last one: their radii (line_radii)
  // keep every activity test false, so they add nothing
  const float4* lam = reinterpret_cast<const float4*>(net.lodf) + (on ? col : Lp4 - 1);
  float gc[kBT5][4], gr[kBT5][4];
#pragma unroll
  for (int i = 0; i < kBT5; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) gc[i][j] = gr[i][j] = 0.0f;
  // the wave's boxes share the side selection: upstream weights that are zero
  // for all of them (splitting asks for the gradient of f_hi alone) drop that
  // side's arithmetic
  bool no_hi = true, no_lo = true;
#pragma unroll
  for (int i = 0; i < kBT5; ++i) {
    no_hi = no_hi && chi[i] == 0.0f;
    no_lo = no_lo && clo[i] == 0.0f;
  }
  // Steps of four outages x kBT5 boxes x four lines per lane, each ending in
  // one butterfly over its 32 per-outage sums.  Full steps go in pairs over
  // two sets of factor rows, each set loaded one step before its use (rows
  // clamped to the block row, so full steps carry no bounds tests, and no
  // register copies between steps); the per-outage (centre, radius) pairs
  // come by scalar loads at the start of each step.  The last 1-3 outages of
  // the block row take the guarded step.
  auto sweep = [&](auto sides) {
    constexpr int S = decltype(sides)::value;
    float4 xn[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xn[u] = lam[(size_t)min(k0 + u, k1 - 1) * Lp4];
    int ks = k0;
    float4 xb[4];
    for (; ks + 8 <= k1; ks += 8) {
      float2 q[kBT5][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < kBT5; ++i) q[i][u] = cd[i][ks + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) xb[u] = lam[(size_t)min(ks + 4 + u, k1 - 1) * Lp4];
      __builtin_amdgcn_sched_barrier(0);
      k5b_step<S, true>(xn, q, c4, rm4, rp4, chi, clo, gc, gr, ks, k1, lane, b0, n_box,
                        cpart_all + (size_t)tile * net.K, (size_t)lay.k5_tiles * net.K);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < kBT5; ++i) q[i][u] = cd[i][ks + 4 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) xn[u] = lam[(size_t)min(ks + 8 + u, k1 - 1) * Lp4];
      __builtin_amdgcn_sched_barrier(0);
      k5b_step<S, true>(xb, q, c4, rm4, rp4, chi, clo, gc, gr, ks + 4, k1, lane, b0, n_box,
                        cpart_all + (size_t)tile * net.K, (size_t)lay.k5_tiles * net.K);
    }
    for (; ks + 4 <= k1; ks += 4) {
      float4 x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = xn[u];
      float2 q[kBT5][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < kBT5; ++i) q[i][u] = cd[i][ks + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) xn[u] = lam[(size_t)min(ks + 4 + u, k1 - 1) * Lp4];
      k5b_step<S, true>(x, q, c4, rm4, rp4, chi, clo, gc, gr, ks, k1, lane, b0, n_box,
                        cpart_all + (size_t)tile * net.K, (size_t)lay.k5_tiles * net.K);
    }
    if (ks < k1) {
      const int nk = k1 - ks;
      float2 q[kBT5][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < kBT5; ++i) q[i][u] = u < nk ? cd[i][ks + u] : make_float2(0.f, 0.f);
      k5b_step<S, false>(xn, q, c4, rm4, rp4, chi, clo, gc, gr, ks, k1, lane, b0, n_box,
                         cpart_all + (size_t)tile * net.K, (size_t)lay.k5_tiles * net.K);
    }
  };
  // Calls with both weights: the sides are picked per wave, and every step
  // keeps its per-outage branches, which bound the live temporaries (with
  // the branch-free steps above, or the step function, the two-sided code
  // takes 180-195 registers: two waves per SIMD for the whole kernel).
  auto sweep_guarded = [&](auto sides) {
    constexpr int S = decltype(sides)::value;
    float4 xn[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xn[u] = lam[(size_t)min(k0 + u, k1 - 1) * Lp4];
    for (int ks = k0; ks < k1; ks += 4) {
      const int nk = min(4, k1 - ks);
      float4 x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = xn[u];
      float2 q[kBT5][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < kBT5; ++i) q[i][u] = u < nk ? cd[i][ks + u] : make_float2(0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u) xn[u] = lam[(size_t)min(ks + 4 + u, k1 - 1) * Lp4];
      __builtin_amdgcn_sched_barrier(0);
      float v[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) v[u] = 0.0f;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        if (kk < nk) {  // uniform
#pragma unroll
          for (int i = 0; i < kBT5; ++i) {
            const float cc = q[i][kk].x, rc = q[i][kk].y;
            float pc = 0.0f, pr = 0.0f;
            k5_elem<S>(x[kk].x, finite_factor(x[kk].x), cc, rc, c4[i].x, rm4[i].x, rp4[i].x, chi[i], clo[i],
                       gc[i][0], gr[i][0], pc, pr);
            k5_elem<S>(x[kk].y, finite_factor(x[kk].y), cc, rc, c4[i].y, rm4[i].y, rp4[i].y, chi[i], clo[i],
                       gc[i][1], gr[i][1], pc, pr);
            k5_elem<S>(x[kk].z, finite_factor(x[kk].z), cc, rc, c4[i].z, rm4[i].z, rp4[i].z, chi[i], clo[i],
                       gc[i][2], gr[i][2], pc, pr);
            k5_elem<S>(x[kk].w, finite_factor(x[kk].w), cc, rc, c4[i].w, rm4[i].w, rp4[i].w, chi[i], clo[i],
                       gc[i][3], gr[i][3], pc, pr);
            v[(kk * kBT5 + i) * 2] = pc;
            v[(kk * kBT5 + i) * 2 + 1] = pr;
          }
        }
      }
      const float tot = butterfly32(v);
      const int idx = lane >> 1;  // (outage ks + idx / 8, box idx / 2 % 4, field idx % 2)
      const int k = ks + (idx >> 3);
      const int i = (idx >> 1) & 3;
      if ((lane & 1) == 0 && k < k1 && b0 + i < n_box) {
        float2* cp = cpart_all + ((size_t)(b0 + i) * lay.k5_tiles + tile) * net.K + k;
        reinterpret_cast<float*>(cp)[idx & 1] = tot;
      }
    }
  };
  if (MODE != 3)
    sweep(std::integral_constant<int, MODE>());
  else if (no_hi)
    sweep_guarded(std::integral_constant<int, 1>());
  else if (no_lo)
    sweep_guarded(std::integral_constant<int, 2>());
  else
    sweep_guarded(std::integral_constant<int, 3>());
  if (on) {
#pragma unroll
    for (int i = 0; i < kBT5; ++i) {
      if (b0 + i >= n_box) break;
      float2* lp = ws_ptr<float2>(ws, lay.lpart) + ((size_t)(b0 + i) * lay.k5_by + blockIdx.y) * net.Lp + 4 * col;
#pragma unroll
      for (int j = 0; j < 4; ++j) lp[j] = make_float2(gc[i][j], gr[i][j]);
    }
  }
}

// ---------------------------------------------------------------------------
// Screened sweep of the gradient of f_hi (box-tiled calls without g_lo).
//
// Only elements whose lower penalty max(|C| - R - fmax, 0) is active carry a
// gradient, and in sub-boxes they are few and sit on few lines (2000 buses,
// 4096 sub-boxes: 5% of the elements, on 11% of a box's lines).  The line
// screen of ibp_screen.hip marks, per tile of kScreenBoxes boxes, the lines
// that can hold one; K5p runs the dense sweep's exact test on those only.

// The screened sweep: a wave holds 64 Q outages (lanes) of one tile's boxes
// and walks the tile's candidate lines one at a time, the line's data in
// scalar registers and its factors one coalesced row segment (the next line's
// loads issued before the current line's arithmetic).  Per element the test
// (the dense sweep's, bit for bit) and the outage-side sums run on the vector
// ALUs; the line side needs two counts per box (active elements, and those
// among them with negative flow), which the test's lane masks give by scalar
// popcounts, added to the line's counter by one atomic per box and line.
template <int Q>
__global__ __launch_bounds__(256) void k5p_sweep(DevNet net, void* ws, WsLayout lay, int64_t n_box,
                                                 const double* __restrict__ g_hi, int n_chunk, int n_tg) {
  constexpr int S = kScreenBoxes;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // Work unit u = (chunk of 64 Q outages, group of 4 tiles: one per wave).
  // The blocks of one XCD (dispatch order: block id mod 8) take consecutive
  // units in chunk-major order, so each XCD streams one or two chunks and
  // their factor columns stay in its L2.
  const int U = n_chunk * n_tg;
  const int per = (U + 7) / 8;
  const int slot = blockIdx.x >> 3;
  const int u = (blockIdx.x & 7) * per + slot;
  if (slot >= per || u >= U) return;  // the whole block
  const int tile = (u % n_tg) * 4 + w;
  const bool on = tile < lay.k5s_tiles;
  const int kw = (u / n_tg) * 64 * Q;
  // the tile's candidate-line masks, staged in LDS: reading them there keeps
  // the walk free of vector-memory waits
  __shared__ uint64_t smk_all[4][kSparseMaxWords];
  uint64_t* smk = smk_all[w];
  const int words = net.Lp / 64;
  if (on) {
    const uint64_t* mask = ws_ptr<uint64_t>(ws, lay.smask) + (size_t)tile * words;
    for (int j = lane; j < words; j += 64) smk[j] = mask[j];
  }
  __syncthreads();
  if (!on) return;
  const int64_t b0 = (int64_t)tile * S;
  const float2* __restrict__ cb = ws_ptr<float2>(ws, lay.cb);
  float clo[S];
  int64_t bb[S];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    bb[i] = min(b0 + i, n_box - 1);
    clo[i] = (float)(-net.zeta_f * g_hi[bb[i]]);
  }
  float cc[Q][S], rc[Q][S], pc[Q][S], pr[Q][S];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = kw + 64 * q + lane;
    const int kq = min(k, net.K - 1);
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const float2 v = cb[bb[i] * net.K + kq];
      cc[q][i] = v.x;
      rc[q][i] = k < net.K ? v.y : INFINITY;  // lanes past the last outage: never active
      pc[q][i] = pr[q][i] = 0.0f;
    }
  }
  // line records through the constant address space: the kernel does not
  // write them, so their wave-uniform loads become scalar loads into SGPRs
  typedef __attribute__((address_space(4))) const float const_float;
  const_float* rec = (const_float*)(ws_ptr<float>(ws, lay.srec) + (size_t)tile * net.Lp * kScreenRecFloats);
  unsigned long long* cnt = ws_ptr<unsigned long long>(ws, lay.lcnt);
  // rows are padded to whole chunks (zero factors past the last outage, whose
  // tests fail: rc = inf)
  static_assert(64 * Q <= 256, "a chunk must fit the 256-outage row padding");
  const float* __restrict__ lamT = net.lodfT + kw + lane;
  // one candidate line: the exact test of the dense sweep on Q x S elements
  // per lane, outage-side sums in registers, line-side counts by popcount
  auto line_step = [&](int l, const float4& c4, const float4& r4, const float (&x)[Q]) {
    // each record value is read by Q elements' instructions: vector copies
    const float cl[S] = {vcopy(c4.x), vcopy(c4.y), vcopy(c4.z), vcopy(c4.w)};
    const float rl[S] = {vcopy(r4.x), vcopy(r4.y), vcopy(r4.z), vcopy(r4.w)};
    unsigned na[S], nn[S];
#pragma unroll
    for (int i = 0; i < S; ++i) na[i] = nn[i] = 0u;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const float C = fmaf(x[q], cc[q][i], cl[i]);
        const float T = fmaf(fabsf(x[q]), rc[q][i], rl[i]);
        // |C| - T > 0 exactly when |C| > T (denormals are kept); the NaN of
        // the outaged line's own factor fails it
        const bool act = fabsf(C) > T;
        const bool neg = C < 0.0f;
        const float mm = act ? x[q] : 0.0f;
        pc[q][i] += neg ? -mm : mm;
        pr[q][i] += fabsf(mm);
        const uint64_t ba = __builtin_amdgcn_ballot_w64(act);
        na[i] += (unsigned)__builtin_popcountll(ba);
        nn[i] += (unsigned)__builtin_popcountll(ba & __builtin_amdgcn_ballot_w64(neg));
      }
    }
    // lane i adds box i's counts
    int vlo = 0, vhi = 0;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      vlo = lane == i ? (int)na[i] : vlo;
      vhi = lane == i ? (int)nn[i] : vhi;
    }
    if (lane < S && b0 + lane < n_box && vlo != 0)
      atomicAdd(cnt + (b0 + lane) * net.Lp + l, ((unsigned long long)(unsigned)vhi << 32) | (unsigned)vlo);
  };
  // Walk the candidate lines (wave-uniform); each line's loads are issued
  // before the previous line's arithmetic.  Lane i holds mask word wb + i
  // (read out by readlane, so that finding the next line waits on no memory
  // access; reloaded from LDS every 64 words).
  int j = 0, wb = 0;
  uint64_t bits = 0;
  uint64_t mw = lane < words ? smk[lane] : 0ull;
  auto next = [&]() -> int {
    while (bits == 0) {
      if (j >= words) return -1;
      if (j - wb >= 64) {
        wb += 64;
        mw = wb + lane < words ? smk[wb + lane] : 0ull;
      }
      const int i = j - wb;
      bits = ((uint64_t)(unsigned)__builtin_amdgcn_readlane((int)(mw >> 32), i) << 32) |
             (unsigned)__builtin_amdgcn_readlane((int)(unsigned)mw, i);
      ++j;
    }
    const int l = (j - 1) * 64 + __builtin_ctzll(bits);
    bits &= bits - 1;
    return l;
  };
  int pl = -1;
  float4 pc4 = make_float4(0.f, 0.f, 0.f, 0.f), pr4 = pc4;
  float px[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) px[q] = 0.0f;
  for (int l = next(); l >= 0; l = next()) {
    const_float* rp = rec + kScreenRecFloats * (size_t)l;
    const float4 c4 = make_float4(rp[0], rp[1], rp[2], rp[3]), r4 = make_float4(rp[4], rp[5], rp[6], rp[7]);
    float x[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) x[q] = lamT[(size_t)l * net.Kp + 64 * q];
    if (pl >= 0) line_step(pl, pc4, pr4, px);
    pl = l;
    pc4 = c4;
    pr4 = r4;
#pragma unroll
    for (int q = 0; q < Q; ++q) px[q] = x[q];
  }
  if (pl >= 0) line_step(pl, pc4, pr4, px);
  float2* cp = ws_ptr<float2>(ws, lay.cpart);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = kw + 64 * q + lane;
#pragma unroll
    for (int i = 0; i < S; ++i)
      if (k < net.K && b0 + i < n_box)
        cp[(size_t)(b0 + i) * net.K + k] = make_float2(clo[i] * pc[q][i], -clo[i] * pr[q][i]);
  }
}

// Per line: base-case penalty gradient + outage-sweep partials (as the line
// itself and, if it is an outage line, as the outaged line).
// With `sparse` the outage sweep was the screened one: counts on the tile's
// candidate lines, per-outage sums as one [B][K] slot.
__global__ __launch_bounds__(256) void k5r_lines(DevNet net, void* ws, WsLayout lay, int64_t box0,
                                                 const double* __restrict__ g_lo,
                                                 const double* __restrict__ g_hi, int sparse) {
  const int64_t b = box0 + blockIdx.y;
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= net.Lp) return;
  float* gcf = ws_ptr<float>(ws, lay.gcf) + b * net.Lp;
  float* grf = ws_ptr<float>(ws, lay.grf) + b * net.Lp;
  if (l >= net.L) {
    gcf[l] = 0.0f;
    grf[l] = 0.0f;
    return;
  }
  const double zf = net.zeta_f, gl = g_lo ? g_lo[b] : 0.0, gh = g_hi ? g_hi[b] : 0.0;
  const double c = ws_ptr<double>(ws, lay.lcf)[b * net.L + l];
  const double r = ws_ptr<double>(ws, lay.lrf)[b * net.L + l];
  const double a = fabs(c), fb = net.fmax_b[l];
  const double hi = (a + r - fb > 0.0) ? -zf * gl : 0.0;
  const double lo = (a - r - fb > 0.0) ? -zf * gh : 0.0;
  const double s = c > 0.0 ? 1.0 : (c < 0.0 ? -1.0 : 0.0);
  double dc = s * (hi + lo), dr = hi - lo;
  if (sparse) {
    const int words = net.Lp / 64;
    const uint64_t m = ws_ptr<uint64_t>(ws, lay.smask)[(b / kScreenBoxes) * words + l / 64];
    if ((m >> (l & 63)) & 1ull) {
      // every active element adds sign(C) clo to the centre and -clo to the radius
      const unsigned long long c = ws_ptr<unsigned long long>(ws, lay.lcnt)[b * net.Lp + l];
      const double na = (double)(unsigned)c, nn = (double)(unsigned)(c >> 32);
      const double clo = -zf * gh;
      dc += clo * (na - 2.0 * nn);
      dr -= clo * na;
    }
    const int k = net.ctg_of_line[l];
    if (k >= 0) {
      const float2 q = ws_ptr<float2>(ws, lay.cpart)[(size_t)b * net.K + k];
      dc += q.x;
      dr += q.y;
    }
    gcf[l] = (float)dc;
    grf[l] = (float)dr;
    return;
  }
  const float2* lp = ws_ptr<float2>(ws, lay.lpart) + (size_t)b * lay.k5_by * net.Lp + l;
  for (int y = 0; y < lay.k5_by; ++y) {
    const float2 t = lp[(size_t)y * net.Lp];
    dc += t.x;
    dr += t.y;
  }
  const int k = net.ctg_of_line[l];
  if (k >= 0) {
    const float2* cp = ws_ptr<float2>(ws, lay.cpart) + (size_t)b * lay.k5_tiles * net.K + k;
    for (int t = 0; t < lay.k5_tiles; ++t) {
      const float2 q = cp[(size_t)t * net.K];
      dc += q.x;
      dr += q.y;
    }
  }
  gcf[l] = (float)dc;
  grf[l] = (float)dr;
}

// Per bus (two buses per wave): d c_inj = Phi^T d c_f, d r_inj = |Phi|^T d r_f.
__global__ __launch_bounds__(256) void k6_ptdf_t(DevNet net, void* ws, WsLayout lay, int64_t box0) {
  const int64_t b = box0 + blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int n0 = (blockIdx.x * 4 + w) * 2;
  if (n0 >= net.Np) return;
  const int Lp4 = net.Lp / 4;
  const float4* gc = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.gcf) + b * net.Lp);
  const float4* gr = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.grf) + b * net.Lp);
  const bool two = n0 + 1 < net.N;
  const float4* p0 = reinterpret_cast<const float4*>(net.phiT) + (size_t)min(n0, net.N - 1) * Lp4;
  const float4* p1 = reinterpret_cast<const float4*>(net.phiT) + (size_t)min(n0 + 1, net.N - 1) * Lp4;
  float a0 = 0, q0 = 0, a1 = 0, q1 = 0;
  if (n0 < net.N) {
    for (int j = lane; j < Lp4; j += 64) {
      const float4 c = gc[j], r = gr[j];
      const float4 x = ld_stream(p0 + j);
      a0 = fmaf(x.x, c.x, fmaf(x.y, c.y, fmaf(x.z, c.z, fmaf(x.w, c.w, a0))));
      q0 = fmaf(fabsf(x.x), r.x, fmaf(fabsf(x.y), r.y, fmaf(fabsf(x.z), r.z, fmaf(fabsf(x.w), r.w, q0))));
      if (two) {
        const float4 y = ld_stream(p1 + j);
        a1 = fmaf(y.x, c.x, fmaf(y.y, c.y, fmaf(y.z, c.z, fmaf(y.w, c.w, a1))));
        q1 = fmaf(fabsf(y.x), r.x, fmaf(fabsf(y.y), r.y, fmaf(fabsf(y.z), r.z, fmaf(fabsf(y.w), r.w, q1))));
      }
    }
  }
  const double s0 = wave_sum((double)a0), t0 = wave_sum((double)q0);
  const double s1 = wave_sum((double)a1), t1 = wave_sum((double)q1);
  if (lane == 0) {
    double* gci = ws_ptr<double>(ws, lay.gci) + b * net.Np;
    double* gri = ws_ptr<double>(ws, lay.gri) + b * net.Np;
    gci[n0] = n0 < net.N ? s0 : 0.0;
    gri[n0] = n0 < net.N ? t0 : 0.0;
    if (n0 + 1 < net.Np) {
      gci[n0 + 1] = two ? s1 : 0.0;
      gri[n0 + 1] = two ? t1 : 0.0;
    }
  }
}

// Many boxes: d c_inj[b, n] = sum_l dC[b, l] Phi[l, n] and d r_inj[b, n] =
// sum_l dR[b, l] |Phi[l, n]| as one tiled product over lines.  Tile 64 boxes
// x 64 buses, 32 lines per step staged in LDS; each thread owns a 4 x 4
// micro-tile of both products.  Each step's 32 products are summed in
// float32 and the step sums in float64, so the rounding error is that of
// 32-term float32 sums rather than of one float32 sum over every line.
constexpr int kGB = 64, kGN = 64, kGK = 32;

__global__ __launch_bounds__(256) void k6b_ptdf_t_tiled(DevNet net, void* ws, WsLayout lay, int64_t n_box) {
  __shared__ float Ac[kGK][kGB + 4];
  __shared__ float Ar[kGK][kGB + 4];
  __shared__ float Bp[kGK][kGN + 4];
  const int64_t b0 = (int64_t)blockIdx.y * kGB;
  const int n0 = blockIdx.x * kGN;
  const int t = threadIdx.x;
  const int tm = t / 16, tn = t % 16;  // micro-tile row (boxes) and column (buses)
  const float* gc = ws_ptr<float>(ws, lay.gcf);
  const float* gr = ws_ptr<float>(ws, lay.grf);
  double sum_c[4][4], sum_r[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) sum_c[i][j] = sum_r[i][j] = 0.0;
  // loader mapping: 64 rows x 32 lines = 512 float4 per operand -> 2 per thread
  for (int l0 = 0; l0 < net.Lp; l0 += kGK) {
    float acc_c[4][4], acc_r[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc_c[i][j] = acc_r[i][j] = 0.0f;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = t + q * 256;      // 0..511
      const int row = idx / 8;          // 0..63
      const int c4 = (idx % 8) * 4;     // line offset within the step
      const int64_t b = b0 + row;
      float4 vc = make_float4(0.f, 0.f, 0.f, 0.f), vr = vc, vp = vc;
      if (b < n_box) {
        vc = *reinterpret_cast<const float4*>(gc + b * net.Lp + l0 + c4);
        vr = *reinterpret_cast<const float4*>(gr + b * net.Lp + l0 + c4);
      }
      const int n = n0 + row;
      if (n < net.N) vp = *reinterpret_cast<const float4*>(net.phiT + (size_t)n * net.Lp + l0 + c4);
      Ac[c4 + 0][row] = vc.x; Ac[c4 + 1][row] = vc.y; Ac[c4 + 2][row] = vc.z; Ac[c4 + 3][row] = vc.w;
      Ar[c4 + 0][row] = vr.x; Ar[c4 + 1][row] = vr.y; Ar[c4 + 2][row] = vr.z; Ar[c4 + 3][row] = vr.w;
      Bp[c4 + 0][row] = vp.x; Bp[c4 + 1][row] = vp.y; Bp[c4 + 2][row] = vp.z; Bp[c4 + 3][row] = vp.w;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < kGK; ++k) {
      float ac[4], ar[4], bp[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ac[i] = Ac[k][tm * 4 + i];
        ar[i] = Ar[k][tm * 4 + i];
        bp[i] = Bp[k][tn * 4 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc_c[i][j] = fmaf(ac[i], bp[j], acc_c[i][j]);
          acc_r[i][j] = fmaf(ar[i], fabsf(bp[j]), acc_r[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        sum_c[i][j] += (double)acc_c[i][j];
        sum_r[i][j] += (double)acc_r[i][j];
      }
    __syncthreads();
  }
  double* gci = ws_ptr<double>(ws, lay.gci);
  double* gri = ws_ptr<double>(ws, lay.gri);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t b = b0 + tm * 4 + i;
    if (b >= n_box) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tn * 4 + j;
      if (n >= net.Np) continue;
      gci[b * net.Np + n] = n < net.N ? sum_c[i][j] : 0.0;
      gri[b * net.Np + n] = n < net.N ? sum_r[i][j] : 0.0;
    }
  }
}

// The same two products on the float32 matrix cores (v_mfma_f32_32x32x2f32):
// a wave owns 32 boxes x 32 buses of both, a block 2 x 2 waves.  Per step of 8
// lines each lane loads one float4 of its box row of dC and dR and of its bus
// row of the transposed PTDF (lines 4h .. 4h + 3 of the step for half-wave h),
// and the four components feed four MFMAs (k = h picks the line); |Phi| is
// the loaded value with its sign cleared.  Each 32-line chunk is summed in
// float32 on the matrix cores and the chunk sums in float64, as in the tiled
// vector kernel.  Blocks are dealt to the XCDs so that each XCD takes every
// eighth box tile with all of its bus tiles: a box tile's rows stay in that
// XCD's L2 while the transposed PTDF streams past.
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr int kMB = 64, kMN = 64;

__global__ __launch_bounds__(256) void k6m_ptdf_t_mfma(DevNet net, void* ws, WsLayout lay, int64_t n_box, int n_bt,
                                                      int n_nt) {
  const int id = blockIdx.x;
  const int slot = id >> 3;
  const int bt = (id & 7) + 8 * (slot / n_nt), nt = slot % n_nt;
  if (bt >= n_bt) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 31, h = lane >> 5;
  const int64_t box0 = (int64_t)bt * kMB + (w >> 1) * 32;
  const int bus = nt * kMN + (w & 1) * 32 + i;
  const int Lp = net.Lp;
  const size_t arow = (size_t)min(box0 + i, n_box - 1) * Lp + 4 * h;
  const float4* pc = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.gcf) + arow);
  const float4* pr = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.grf) + arow);
  const float4* pp = reinterpret_cast<const float4*>(net.phiT + (size_t)min(bus, net.N - 1) * Lp + 4 * h);
  double sc[16], sr[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) sc[e] = sr[e] = 0.0;
  for (int l0 = 0; l0 < Lp; l0 += 32) {
    float4 a[4], r[4], p[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = pc[(l0 + 8 * u) / 4];
      r[u] = pr[(l0 + 8 * u) / 4];
      p[u] = pp[(l0 + 8 * u) / 4];
    }
    // all twelve loads of the chunk in flight before its first MFMA (the
    // compiler would otherwise issue each step's loads after the previous
    // step's MFMAs and wait on them one step at a time)
    __builtin_amdgcn_sched_barrier(0);
    v16f ac = {}, ar = {};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ac = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u].x, p[u].x, ac, 0, 0, 0);
      ar = __builtin_amdgcn_mfma_f32_32x32x2f32(r[u].x, fabsf(p[u].x), ar, 0, 0, 0);
      ac = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u].y, p[u].y, ac, 0, 0, 0);
      ar = __builtin_amdgcn_mfma_f32_32x32x2f32(r[u].y, fabsf(p[u].y), ar, 0, 0, 0);
      ac = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u].z, p[u].z, ac, 0, 0, 0);
      ar = __builtin_amdgcn_mfma_f32_32x32x2f32(r[u].z, fabsf(p[u].z), ar, 0, 0, 0);
      ac = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u].w, p[u].w, ac, 0, 0, 0);
      ar = __builtin_amdgcn_mfma_f32_32x32x2f32(r[u].w, fabsf(p[u].w), ar, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      sc[e] += (double)ac[e];
      sr[e] += (double)ar[e];
    }
  }
  // accumulator e of lane (i, h) holds box row 8 (e / 4) + 4 h + e % 4, bus column i
  if (bus >= net.Np) return;
  double* gci = ws_ptr<double>(ws, lay.gci);
  double* gri = ws_ptr<double>(ws, lay.gri);
  const bool real = bus < net.N;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int64_t b = box0 + 8 * (e >> 2) + 4 * h + (e & 3);
    if (b < n_box) {
      gci[b * net.Np + bus] = real ? sc[e] : 0.0;
      gri[b * net.Np + bus] = real ? sr[e] : 0.0;
    }
  }
}

// Per input: endpoint gradients (injection, surplus and imbalance terms).
__global__ __launch_bounds__(256) void k7_endpoints(DevNet net, void* ws, WsLayout lay, int64_t box0,
                                                    const float* __restrict__ box_lo,
                                                    const float* __restrict__ box_hi,
                                                    const double* __restrict__ g_lo,
                                                    const double* __restrict__ g_hi,
                                                    double* __restrict__ d_lo, double* __restrict__ d_hi) {
  __shared__ double sh[4];
  const int64_t b = box0 + blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  // total injection interval and validity from the box-preparation partials
  const double* p1 = ws_ptr<double>(ws, lay.p1) + b * lay.n_p1 * kP1Fields;
  double cI = 0.0, rI = 0.0, bad = 0.0;
  for (int q = threadIdx.x; q < lay.n_p1; q += 256) {
    cI += p1[q * kP1Fields + kP1cI];
    rI += p1[q * kP1Fields + kP1rI];
    bad += p1[q * kP1Fields + kP1Bad];
  }
  cI = block_sum256(cI, sh);
  rI = block_sum256(rI, sh);
  bad = block_sum256(bad, sh);
  if (j >= net.X) return;
  const double gl = g_lo ? g_lo[b] : 0.0, gh = g_hi ? g_hi[b] : 0.0, zi = net.zeta_inj;
  const double aI = fabs(cI);
  const double hiI = (aI + rI > 0.0) ? -zi * gl : 0.0;
  const double loI = (aI - rI > 0.0) ? -zi * gh : 0.0;
  const double sI = cI > 0.0 ? 1.0 : (cI < 0.0 ? -1.0 : 0.0);
  const double dcI = sI * (hiI + loI), drI = hiI - loI;
  const double sj = j < net.G ? 1.0 : -1.0;
  const int n = net.dev_bus[j];
  const double wj = net.dev_w[j];
  double dc = sj * ws_ptr<double>(ws, lay.gci)[b * net.Np + n] + (gl + gh) * wj + sj * dcI;
  double dr = ws_ptr<double>(ws, lay.gri)[b * net.Np + n] + (gh - gl) * fabs(wj) + drI;
  if (net.seg_ptr) {
    const int s0 = net.seg_ptr[j], s1 = net.seg_ptr[j + 1];
    if (s1 > s0) {
      const double l = box_lo[b * net.X + j], h = box_hi[b * net.X + j];
      double lc, lr, hc, hr;
      curve_ibp_tangents(net.seg, s0, s1, 0.5 * (l + h), 0.5 * (h - l), lc, lr, hc, hr);
      // S_lo gets F_lo of a load and -F_hi of a generator; S_hi the other ends
      const double al = j < net.G ? -gh : gl, ah = j < net.G ? -gl : gh;
      dc += al * lc + ah * hc;
      dr += al * lr + ah * hr;
    }
  }
  const bool nanb = bad != 0.0;
  d_lo[b * net.X + j] = nanb ? NAN : 0.5 * (dc - dr);
  d_hi[b * net.X + j] = nanb ? NAN : 0.5 * (dc + dr);
}

void plan_backward(const DevNet& net, WsLayout& lay) {
  const int lp4 = net.Lp / 4;
  lay.k5_tiles = (lp4 + 63) / 64;
  lay.k5_chunk = lay.batched ? kK5ChunkTiled : kK5Chunk;
  lay.k5_by = std::max(1, (net.K + lay.k5_chunk - 1) / lay.k5_chunk);
}

hipError_t launch_backward_sweeps(const DevNet& net, int64_t n_box, void* ws, const WsLayout& lay,
                                  const float* box_lo, const float* box_hi, const double* g_lo, const double* g_hi, double* d_lo, double* d_hi,
                                  bool sparse, hipStream_t s, KernelTimer* tm) {
  sparse = sparse && !g_lo && g_hi && n_box >= kBatchMin && lay.batched && net.K > 0 && screen_fits(net, lay);
  if (sparse) {
    int t = tm->start(14, s);
    launch_line_screen(net, n_box, ws, lay, kScreenBackwardLower, s);
    tm->stop(t, s);
    t = tm->start(7, s);
    const int n_chunk = (net.K + 64 * kSparseQ - 1) / (64 * kSparseQ), n_tg = (lay.k5s_tiles + 3) / 4;
    const int per = (n_chunk * n_tg + 7) / 8;
    hipLaunchKernelGGL(k5p_sweep<kSparseQ>, dim3(8 * per), dim3(256), 0, s, net, ws, lay, n_box, g_hi, n_chunk,
                       n_tg);
    tm->stop(t, s);
  } else if (n_box >= kBatchMin && lay.batched && net.K > 0) {
    const int t = tm->start(7, s);
    const unsigned groups = (unsigned)(((n_box + kBT5 - 1) / kBT5 + 3) / 4);
    const dim3 grid(lay.k5_tiles, lay.k5_by, groups);
    const float2* cb_all = reinterpret_cast<const float2*>(static_cast<char*>(ws) + lay.cb);
    float2* cpart_all = reinterpret_cast<float2*>(static_cast<char*>(ws) + lay.cpart);
    if (!g_lo)
      hipLaunchKernelGGL(k5b_outage_vjp<1>, grid, dim3(256), 0, s, net, ws, lay, n_box, g_lo, g_hi, cb_all,
                         cpart_all);
    else if (!g_hi)
      hipLaunchKernelGGL(k5b_outage_vjp<2>, grid, dim3(256), 0, s, net, ws, lay, n_box, g_lo, g_hi, cb_all,
                         cpart_all);
    else
      hipLaunchKernelGGL(k5b_outage_vjp<3>, grid, dim3(256), 0, s, net, ws, lay, n_box, g_lo, g_hi, cb_all,
                         cpart_all);
    tm->stop(t, s);
  }
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    if (net.K > 0 && !(n_box >= kBatchMin && lay.batched)) {
      const int t = tm->start(7, s);
      hipLaunchKernelGGL(k5_outage_vjp, dim3((lay.k5_tiles + 3) / 4, lay.k5_by, nb), dim3(256), 0, s, net, ws,
                         lay, b0, g_lo, g_hi);
      tm->stop(t, s);
    }
    const int t = tm->start(13, s);
    hipLaunchKernelGGL(k5r_lines, dim3((net.Lp + 255) / 256, nb), dim3(256), 0, s, net, ws, lay, b0, g_lo, g_hi,
                       (int)sparse);
    tm->stop(t, s);
  }
  if (n_box >= kBatchMin) {
    const int t = tm->start(8, s);
    if (lay.k2_mfma) {
      const int n_bt = (int)((n_box + kMB - 1) / kMB), n_nt = (net.Np + kMN - 1) / kMN;
      hipLaunchKernelGGL(k6m_ptdf_t_mfma, dim3((unsigned)(8 * ((n_bt + 7) / 8) * n_nt)), dim3(256), 0, s, net, ws,
                         lay, n_box, n_bt, n_nt);
    } else {
      hipLaunchKernelGGL(k6b_ptdf_t_tiled, dim3((net.Np + kGN - 1) / kGN, (unsigned)((n_box + kGB - 1) / kGB)),
                         dim3(256), 0, s, net, ws, lay, n_box);
    }
    tm->stop(t, s);
  }
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    int t;
    if (n_box < kBatchMin) {
      t = tm->start(8, s);
      hipLaunchKernelGGL(k6_ptdf_t, dim3((net.Np + 7) / 8, nb), dim3(256), 0, s, net, ws, lay, b0);
      tm->stop(t, s);
    }
    t = tm->start(9, s);
    hipLaunchKernelGGL(k7_endpoints, dim3((net.X + 255) / 256, nb), dim3(256), 0, s, net, ws, lay, b0, box_lo,
                       box_hi, g_lo, g_hi, d_lo, d_hi);
    tm->stop(t, s);
  }
  return hipGetLastError();
}

}  // namespace ibp
