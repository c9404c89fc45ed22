// Linear-relaxation (CROWN-style) upper bound on max f over a box.
//
// The paper names convex relaxations (CROWN and its variants) as the tighter
// family beside IBP (Sec. I).  On this graph every penalty is a convex
// function of one affine pre-activation: phi(z) = max(|z| - t, 0) for a flow
// against its limit, |z| for the total imbalance.  For any s in {-1, 0, 1} the
// line s z - |s| t lies below phi for every z (a supporting line), so
//
//   f(x) <= S(x) - zeta_inj s_I z_I(x) - zeta_f sum_e (s_e z_e(x) - |s_e| t_e)
//
// holds at every x whatever the slopes are.  The right side is linear in x
// (plus the curve part), so its maximum over the box is
//   sum_j (G_j c_j + |G_j| r_j) + zeta_f sum_e |s_e| t_e  (+ curve interval),
// with G = w - zeta_inj s_I sign - zeta_f N^T Phi^T v and the line adjoint
//   v_l = s_l (base) + sum_k s_kl + [l = c(k)] sum_l' s_kl' Lam_l'k.
// The slope of an element is sign(C) when its padded interval lies beyond the
// limit (the K3 test t_lo > 0) and 0 otherwise: every line then attains IBP's
// lower penalty on the box, so the bound is never above IBP's f_hi in exact
// arithmetic.  The slope decision affects tightness only, never validity.
//
// Rigour: s in {-1, 0, 1} and float32 factors make the per-line sums exact
// small integers (int atomics, order-independent) and every s Lam product
// exact; per-outage sums add four products per lane in float32 and the rest
// in float64, and the transposed PTDF product runs in float64.  The
// coefficient error |G^ - G_exact| is bounded per input from
//   |Lam32 - Lam_exact| <= kappa0 |Lam32| + (2 eps_l + 2 |Lam| eps_c)/(1 - H_cc),
//   |Phi32 - Phi_exact| <= kappa0 |Phi32| + eps_l,
// the float64 accumulation bounds, and absolute sums carried beside each sum
// (vabs, ev); the box maximum adds E_j (|c_j| + r_j).
//
//   KC0  zero the per-line counters
//   KC1  outage sweep: slopes, per-line integer counts, per-outage float64 sums
//   KC2  per line: adjoint v, its absolute bound and error, limit totals
//   KC3  per bus: Phi^T v, |Phi|^T vabs, |Phi|^T ev (float64)
//   KC4  per input: coefficient, error bound, box maximum (and curve interval),
//        and the maximising vertex
//   KC5  per box: total, outward padding, min with IBP's f_hi
//
// Slopes come either from the box (an element has s = sign(C) when its padded
// interval lies beyond the limit) or from a reference point (s = sign(C) where
// the flow there exceeds the limit: the penalty's gradient at that point).
// The second family, taken at the box centre and then at points moving
// halfway towards each relaxation's maximising vertex, often reaches the LP
// optimum of the box; every pass gives a valid bound and the smallest is kept.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>

#include "ibp_devfun.h"
#include "ibp_kernels.h"
#include "ibp_lanes.h"

namespace ibp {

namespace {
constexpr int kKC = 16;   // outages per KC1 block
constexpr int kNB = 32;   // buses per KC3 block
}  // namespace

__global__ __launch_bounds__(256) void kc0_zero(int2* __restrict__ cnt, int64_t n) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i < n) cnt[i] = make_int2(0, 0);
}

// Slope of one element from the K3 quantities: C = fma(Lam, c_c, c_l),
// t_lo = |C| - fma(|Lam|, rho'_k, g_l) <= |C*| - R* - fmax.  NaN (the outaged
// line's own entry) compares false and gets slope 0.
__device__ __forceinline__ float crown_slope(float lam, float cc, float rk, float cl, float g) {
  const float C = fmaf(lam, cc, cl);
  const float tlo = fabsf(C) - fmaf(fabsf(lam), rk, g);
  return tlo > 0.0f ? copysignf(1.0f, C) : 0.0f;
}

// Slope from the flow at a reference point: C = fma(Lam, c_c(ref), c_l(ref)),
// s = sign(C) where |C| > fmax (the penalty's gradient there), else 0.
__device__ __forceinline__ float crown_slope_ref(float lam, float cc, float cl, float fmax) {
  const float C = fmaf(lam, cc, cl);
  return fabsf(C) > fmax ? copysignf(1.0f, C) : 0.0f;
}

// Sums v[0..23] (eight groups of three) over the 64 lanes of a wave by halving
// exchanges (12 + 6 + 3, then 3 x 3): afterwards every lane of the 8-lane group
// g = lane / 8 holds the totals of v[3g], v[3g + 1], v[3g + 2] in v[0..2].
__device__ __forceinline__ void halving_sum24(double (&v)[24]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 12; ++i) v[i] = halve32(v[i], v[i + 12]);
#pragma unroll
  for (int i = 0; i < 6; ++i) v[i] = halve16(v[i], v[i + 6]);
  {
    const bool up = lane & 8;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double send = up ? v[i] : v[i + 3];
      const double keep = up ? v[i + 3] : v[i];
      v[i] = keep + lane_xor<kDppXor8>(send);
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] += __shfl_xor(v[i], 4, 64);
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] += lane_xor<kDppXor2>(v[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] += lane_xor<kDppXor1>(v[i]);
}

// The same reduction for float32 values (the relaxation's per-outage sums:
// the KC2 error term covers their float32 rounding).
__device__ __forceinline__ void halving_sum24(float (&v)[24]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 12; ++i) v[i] = halve32(v[i], v[i + 12]);
#pragma unroll
  for (int i = 0; i < 6; ++i) v[i] = halve16(v[i], v[i + 6]);
  {
    const bool up = lane & 8;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float send = up ? v[i] : v[i + 3];
      const float keep = up ? v[i + 3] : v[i];
      v[i] = keep + lane_xor<kDppXor8>(send);
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] += __shfl_xor(v[i], 4, 64);
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] += lane_xor<kDppXor2>(v[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] += lane_xor<kDppXor1>(v[i]);
}

// Slopes of four lines x one outage; per-line counts in registers, the
// outage's three sums (s Lam, |s Lam|, count) into r[0..2].
// REF: c4 holds the line flows at the reference point and g4 the limits.
template <bool REF>
__device__ __forceinline__ void kc1_row(const float4& x, const int4& d, const float4& c4, const float4& g4,
                                        float (&cs)[4], float (&ca)[4], float* r) {
  const float cc = __int_as_float(d.y), rk = __int_as_float(d.z);
  float s[4];
  if (REF) {
    s[0] = crown_slope_ref(x.x, cc, c4.x, g4.x);
    s[1] = crown_slope_ref(x.y, cc, c4.y, g4.y);
    s[2] = crown_slope_ref(x.z, cc, c4.z, g4.z);
    s[3] = crown_slope_ref(x.w, cc, c4.w, g4.w);
  } else {
    s[0] = crown_slope(x.x, cc, rk, c4.x, g4.x);
    s[1] = crown_slope(x.y, cc, rk, c4.y, g4.y);
    s[2] = crown_slope(x.z, cc, rk, c4.z, g4.z);
    s[3] = crown_slope(x.w, cc, rk, c4.w, g4.w);
  }
  // s Lam is exact in float32; NaN entries carry s = 0 and a finite stand-in
  const float l[4] = {fminf(x.x, FLT_MAX), fminf(x.y, FLT_MAX), fminf(x.z, FLT_MAX), fminf(x.w, FLT_MAX)};
  // the four exact products are summed in float32, and so is the halving
  // reduction over the wave's 64 lanes: nine rounding levels, at most 9u of
  // the absolute sum (covered in KC2)
  float v = 0.0f, a = 0.0f, n = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    cs[i] += s[i];
    ca[i] += fabsf(s[i]);
    n += fabsf(s[i]);
    v += s[i] * l[i];
    a += fabsf(s[i] * l[i]);
  }
  r[0] = v;
  r[1] = a;
  r[2] = n;
}

// wsr: the reference points' forward workspace (REF), else unused.  Four
// waves per SIMD (111 registers, no spill) instead of the three the compiler
// picks unbounded: 8316 buses, one box, 85 -> 76 us.
template <bool REF>
__global__ __launch_bounds__(256, 4) void kc1_sweep(DevNet net, void* ws, const void* wsr, WsLayout lay,
                                                 int64_t box0) {
  __shared__ double shv[4][kKC][2];
  __shared__ float shn[4][kKC];
  const int64_t b = box0 + blockIdx.z;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int col = (blockIdx.x * 4 + w) * 64 + lane;  // float4 column: four lines per lane
  const int Lp4 = net.Lp / 4;
  const int k0 = blockIdx.y * kKC;
  const int k1 = min(net.K, k0 + kKC);
  const bool live = col < Lp4;
  float4 c4 = make_float4(0.f, 0.f, 0.f, 0.f), g4 = make_float4(FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX);
  void* wd = REF ? const_cast<void*>(wsr) : ws;  // where the slope decisions read from
  if (live && REF) {
    c4 = reinterpret_cast<const float4*>(ws_ptr<float>(wd, lay.lc) + b * net.Lp)[col];
    g4 = reinterpret_cast<const float4*>(net.fmax_c32)[col];
  } else if (live) {
    const double* bs = ws_ptr<double>(ws, lay.box) + b * kBoxSlots;
    const float vmax = __uint_as_float(*reinterpret_cast<const unsigned int*>(bs + kVmax));
    c4 = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lc) + b * net.Lp)[col];
    g4 = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lg) + b * net.Lp)[col];
    const float4 e4 = reinterpret_cast<const float4*>(net.line_eps)[col];
    g4 = make_float4(add_ru(g4.x, next_up_f32(e4.x * vmax)), add_ru(g4.y, next_up_f32(e4.y * vmax)),
                     add_ru(g4.z, next_up_f32(e4.z * vmax)), add_ru(g4.w, next_up_f32(e4.w * vmax)));
  }
  const int4* cd = ws_ptr<int4>(wd, lay.ctg) + b * net.K;
  const float4* lam = reinterpret_cast<const float4*>(net.lodf) + col;
  float cs[4] = {0.f, 0.f, 0.f, 0.f}, ca[4] = {0.f, 0.f, 0.f, 0.f};
  // groups of eight outages: eight rows in flight, then one halving reduction
  for (int kg = k0; kg < k1; kg += 8) {
    float r[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) r[i] = 0.0f;
    if (live) {
      float4 x[8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        x[i] = (kg + i < k1) ? ld_stream(lam + (size_t)(kg + i) * Lp4) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (kg + i < k1) kc1_row<REF>(x[i], cd[kg + i], c4, g4, cs, ca, r + 3 * i);
    }
    // a wave with no active element in the group skips the reduction
    bool act = false;
#pragma unroll
    for (int i = 0; i < 8; ++i) act |= r[3 * i + 2] != 0.0f;
    if (__any(act)) {
      halving_sum24(r);
    }
    // lane 8g holds outage kg + g (zeros when the wave skipped)
    if ((lane & 7) == 0 && kg + (lane >> 3) < k1) {
      const int q = kg - k0 + (lane >> 3);
      shv[w][q][0] = r[0];
      shv[w][q][1] = r[1];
      shn[w][q] = (float)r[2];
    }
  }
  __syncthreads();
  if (threadIdx.x < k1 - k0) {
    const int q = threadIdx.x;
    const double V = (shv[0][q][0] + shv[1][q][0]) + (shv[2][q][0] + shv[3][q][0]);
    const double A = (shv[0][q][1] + shv[1][q][1]) + (shv[2][q][1] + shv[3][q][1]);
    const double N = ((double)shn[0][q] + (double)shn[1][q]) + ((double)shn[2][q] + (double)shn[3][q]);
    ws_ptr<double4>(ws, lay.cv)[((size_t)b * lay.kc_bx + blockIdx.x) * net.K + k0 + q] =
        make_double4(V, A, N, 0.0);
  }
  if (live) {
    // per-line counts: integer atomics, so the totals do not depend on the order
    int2* cnt = ws_ptr<int2>(ws, lay.ccnt) + b * net.Lp + 4 * col;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (ca[i] != 0.0f) {
        atomicAdd(&cnt[i].x, (int)cs[i]);
        atomicAdd(&cnt[i].y, (int)ca[i]);
      }
  }
}

// Position of line l of box b in the adjoint array: box-major for the per-box
// and vector products, line-major (boxes contiguous) for the matrix-core
// product, whose lanes then load 16 consecutive boxes of one line.
__device__ __forceinline__ size_t lv_index(const WsLayout& lay, const DevNet& net, int64_t b, int l) {
  return lay.kc3_mfma ? (size_t)l * lay.kc3_bt + b : (size_t)b * net.Lp + l;
}

// Per line: v, vabs >= |v_exact|, ev >= |v^ - v_exact|; block partials of the
// limit total sum |s| t and of sum vabs.
__global__ __launch_bounds__(256) void kc2_lines(DevNet net, void* ws, const void* wsr, WsLayout lay,
                                                 int64_t box0) {
  __shared__ double sh[4];
  const int64_t b = box0 + blockIdx.y;
  const int l = blockIdx.x * 256 + threadIdx.x;
  double v = 0.0, va = 0.0, ev = 0.0, T = 0.0;
  if (l < net.L) {
    const double fb = net.fmax_b[l];
    double sb;
    if (wsr) {  // the base flow at the reference point
      const double cr = ws_ptr<double>(const_cast<void*>(wsr), lay.lcf)[b * net.L + l];
      sb = (fabs(cr) > fb) ? copysign(1.0, cr) : 0.0;
    } else {
      const double cf = ws_ptr<double>(ws, lay.lcf)[b * net.L + l];
      const double rf = ws_ptr<double>(ws, lay.lrf)[b * net.L + l];
      sb = (fabs(cf) - rf - fb > 0.0) ? copysign(1.0, cf) : 0.0;
    }
    const int2 n = ws_ptr<int2>(ws, lay.ccnt)[b * net.Lp + l];
    v = sb + (double)n.x;
    va = fabs(sb) + (double)n.y;
    T = fabs(sb) * fb + (double)n.y * net.fmax_c[l];
    const int k = net.ctg_of_line[l];
    if (k >= 0) {
      double V = 0.0, A = 0.0, N = 0.0;
      const double4* cv = ws_ptr<double4>(ws, lay.cv) + (size_t)b * lay.kc_bx * net.K + k;
      for (int t = 0; t < lay.kc_bx; ++t) {
        const double4 q = cv[(size_t)t * net.K];
        V += q.x;
        A += q.y;
        N += q.z;
      }
      // float32 sums of exact products within a wave (four per lane, then
      // six halving levels: <= 9u of their absolute sum), float64 sums over
      // waves and tiles; stored-factor errors
      const double gam = (net.Lp + lay.kc_bx + 16) * kU64 * 1.01;
      const double A1 = A * (1.0 + gam) * (1.0 + kKappa0) * (1.0 + 10.0 * kU32);
      ev = (kKappa0 + net.ctg_eps[k] + gam + 10.0 * kU32) * A1 + 2.0 * net.phi_err_max * net.ctg_inv[k] * N;
      v += V;
      va += A1 + ev;
    }
    // rounding of the two additions forming v
    ev = (ev + 2.0 * kU64 * va) * (1.0 + 4.0 * kU64);
    va = va * (1.0 + 4.0 * kU64) + ev;
  }
  if (l < net.Lp) ws_ptr<double4>(ws, lay.lv)[lv_index(lay, net, b, l)] = make_double4(v, va, ev, 0.0);
  T = block_sum256(T, sh);
  const double S = block_sum256(va, sh);
  if (threadIdx.x == 0) ws_ptr<double4>(ws, lay.ct)[b * lay.n_ct + blockIdx.x] = make_double4(T, S, 0.0, 0.0);
}

// Per bus n: y = sum_l Phi32[l, n] v_l, ya = sum_l |Phi32| vabs_l,
// ye = sum_l |Phi32| ev_l, over one 1024-line tile; kNB buses per block.
__global__ __launch_bounds__(256) void kc3_ptdf_t(DevNet net, void* ws, WsLayout lay, int64_t box0) {
  __shared__ double sh[4][kNB][3];
  const int64_t b = box0 + blockIdx.z;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int col = (blockIdx.x * 4 + w) * 64 + lane;
  const int Lp4 = net.Lp / 4;
  const bool live = col < Lp4;
  double v[4] = {0, 0, 0, 0}, va[4] = {0, 0, 0, 0}, ev[4] = {0, 0, 0, 0};
  if (live) {
    const double4* lv = ws_ptr<double4>(ws, lay.lv) + b * net.Lp + 4 * col;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double4 q = lv[i];
      v[i] = q.x;
      va[i] = q.y;
      ev[i] = q.z;
    }
  }
  const int n0 = blockIdx.y * kNB;
  const int n1 = min(net.N, n0 + kNB);
  const float4* ph = reinterpret_cast<const float4*>(net.phiT) + col;
  // groups of eight buses: eight rows in flight, then one halving reduction
  for (int ng = n0; ng < n1; ng += 8) {
    double r[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) r[i] = 0.0;
    if (live) {
      float4 x[8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        x[i] = (ng + i < n1) ? ld_stream(ph + (size_t)(ng + i) * Lp4) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double p[4] = {(double)x[i].x, (double)x[i].y, (double)x[i].z, (double)x[i].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          r[3 * i] = fma(p[q], v[q], r[3 * i]);
          r[3 * i + 1] = fma(fabs(p[q]), va[q], r[3 * i + 1]);
          r[3 * i + 2] = fma(fabs(p[q]), ev[q], r[3 * i + 2]);
        }
      }
    }
    halving_sum24(r);
    if ((lane & 7) == 0 && ng + (lane >> 3) < n1) {
      const int q = ng - n0 + (lane >> 3);
      sh[w][q][0] = r[0];
      sh[w][q][1] = r[1];
      sh[w][q][2] = r[2];
    }
  }
  __syncthreads();
  if (threadIdx.x < n1 - n0) {
    const int q = threadIdx.x;
    double o[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) o[f] = (sh[0][q][f] + sh[1][q][f]) + (sh[2][q][f] + sh[3][q][f]);
    ws_ptr<double4>(ws, lay.bpart)[((size_t)b * lay.kc3_bx + blockIdx.x) * net.Np + n0 + q] =
        make_double4(o[0], o[1], o[2], 0.0);
  }
}

// Chord of |z| over the total-injection interval [cI - rI - eI, cI + rI + eI]
// (float64, outward): slope a (sign of cI times alpha in [0, 1]) and an upper
// bound beta of the line's value at z = 0, so that |z| <= a z + beta on the
// interval.  With y = sign(cI) z the interval is [tl, th]; |y| at its two ends
// is th and |tl|, and alpha is the chord slope between them.
__device__ __forceinline__ void chord_imbalance(double cI, double rI, double eI, double& a, double& beta) {
  const double w = fabs(cI) + rI + eI;
  const double th = w * (1.0 + 4.0 * kU64);
  const double tl = (fabs(cI) - rI - eI) - 4.0 * kU64 * w;
  a = 0.0;
  beta = 0.0;
  if (th > 0.0) {
    const double ql = fabs(tl);
    const double al = fmin(fmax((th - ql) / (th - tl), 0.0), 1.0);
    const double bb = fmax(fma(-al, th, th), fma(-al, tl, ql));
    beta = bb + 4.0 * kU64 * (fabs(bb) + th + fabs(tl));
    a = copysign(al, cI);
  }
}

// Per input: coefficient G_j, its error bound E_j, and max over [lo_j, hi_j] of
// G_j x_j (plus the curve interval's upper end); block partials (sum, sum |.|).
// LOW: the chord relaxation's lower bound instead: min over [lo_j, hi_j] of
// G_j x_j (minus E_j |x_j|, plus the curve interval's lower end), the
// imbalance slope from its chord, whose intercept block 0 adds once per box;
// the vertex is the minimiser.
template <bool LOW>
__global__ __launch_bounds__(256) void kc4_inputs(DevNet net, void* ws, const void* wsr, WsLayout lay,
                                                  int64_t box0,
                                                  const float* __restrict__ box_lo,
                                                  const float* __restrict__ box_hi,
                                                  float* __restrict__ vertex) {
  __shared__ double sh[4];
  const int64_t b = box0 + blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  // imbalance slope: from the total injection interval, or at the reference point
  const double* p1 = ws_ptr<double>(wsr ? const_cast<void*>(wsr) : ws, lay.p1) + b * lay.n_p1 * kP1Fields;
  double cI = 0.0, rI = 0.0, aI = 0.0;
  for (int q = threadIdx.x; q < lay.n_p1; q += 256) {
    cI += p1[q * kP1Fields + kP1cI];
    rI += p1[q * kP1Fields + kP1rI];
    if (LOW) aI += p1[q * kP1Fields + kP1cIabs];
  }
  cI = block_sum256(cI, sh);
  rI = block_sum256(rI, sh);  // zero at a reference point
  double sI, bI = 0.0;
  if (LOW) {
    // float64 sums of n_p1 partials of n_p1 terms each: the same enclosure as K4's
    aI = block_sum256(aI, sh);
    const double eI = 2.0 * (lay.n_p1 + 16) * kU64 * 1.01 * (aI + rI);
    chord_imbalance(cI, rI, eI, sI, bI);
  } else {
    sI = (fabs(cI) - rI > 0.0) ? copysign(1.0, cI) : 0.0;
  }
  double SV = 0.0;
  for (int q = threadIdx.x; q < lay.n_ct; q += 256) SV += ws_ptr<double4>(ws, lay.ct)[b * lay.n_ct + q].y;
  SV = block_sum256(SV, sh) * (1.0 + (lay.n_ct + 16) * kU64 * 1.01);
  double h = 0.0, ha = 0.0;
  if (j < net.X) {
    const int n = net.dev_bus[j];
    double y = 0.0, ya = 0.0, ye = 0.0;
    const double4* bp = ws_ptr<double4>(ws, lay.bpart) + (size_t)b * lay.kc3_bx * net.Np + n;
    for (int t = 0; t < lay.kc3_bx; ++t) {
      const double4 q = bp[(size_t)t * net.Np];
      y += q.x;
      ya += q.y;
      ye += q.z;
    }
    // float64 products of float32 x float64 and sums over Lp lines + tiles
    const double gam = (net.Lp + lay.kc3_bx + 16) * kU64 * 1.01;
    ya *= (1.0 + gam);
    ye *= (1.0 + gam);
    const double sj = j < net.G ? 1.0 : -1.0;
    const double wj = net.dev_w[j], zi = net.zeta_inj, zf = net.zeta_f;
    const double G = wj - zi * sI * sj - zf * sj * y;
    // |y^ - (Phi_exact^T v_exact)_n| <= (kappa0 + gam) ya + (1 + kappa0) ye + 2 eps_max sum vabs
    const double E = zf * ((kKappa0 + gam) * ya + (1.0 + kKappa0) * ye + 2.0 * net.phi_err_max * SV) *
                         (1.0 + 8.0 * kU64) +
                     4.0 * kU64 * (fabs(wj) + zi + zf * fabs(y));
    const float l32 = box_lo[b * net.X + j], h32 = box_hi[b * net.X + j];
    if (vertex) vertex[b * net.X + j] = (G >= 0.0) != LOW ? h32 : l32;
    const double l = l32, hh = h32;
    const double c = 0.5 * (l + hh), r = 0.5 * (hh - l);
    const double m = fabs(c) + r;
    ha = fabs(G) * m + E * m;
    if (LOW) {
      h = G * c - fabs(G) * r - E * m;
      h -= 4.0 * kU64 * ha;
    } else {
      h = G * c + fabs(G) * r + E * m;
      h += 4.0 * kU64 * ha;
    }
    if (net.seg_ptr) {
      const int s0 = net.seg_ptr[j], s1 = net.seg_ptr[j + 1];
      if (s1 > s0) {
        double F_lo, F_hi, e;
        curve_ibp(net.seg, s0, s1, c, r, F_lo, F_hi, e);
        const double pad = e + kU64 * (fabs(F_lo) + fabs(F_hi));
        const double u = LOW ? (j < net.G ? -F_hi : F_lo) - pad : (j < net.G ? -F_lo : F_hi) + pad;
        h += u;
        ha += fabs(u);
      }
    }
  }
  if (LOW && blockIdx.x == 0 && threadIdx.x == 0) {
    // the imbalance line's intercept: -zeta_inj beta
    h -= net.zeta_inj * bI;
    ha += net.zeta_inj * fabs(bI);
  }
  h = block_sum256(h, sh);
  ha = block_sum256(ha, sh);
  if (threadIdx.x == 0) ws_ptr<double2>(ws, lay.cp)[b * lay.n_cp + blockIdx.x] = make_double2(h, ha);
}

// again: a later relaxation of the same call, kept only where it is smaller.
__global__ __launch_bounds__(256) void kc5_finalize(DevNet net, void* ws, WsLayout lay, int64_t box0,
                                                    double* __restrict__ f_hi, double* __restrict__ crown,
                                                    int again) {
  __shared__ double sh[4];
  const int64_t b = box0 + blockIdx.x;
  double H = 0.0, Ha = 0.0, T = 0.0;
  for (int q = threadIdx.x; q < lay.n_cp; q += 256) {
    const double2 t = ws_ptr<double2>(ws, lay.cp)[b * lay.n_cp + q];
    H += t.x;
    Ha += t.y;
  }
  for (int q = threadIdx.x; q < lay.n_ct; q += 256) T += ws_ptr<double4>(ws, lay.ct)[b * lay.n_ct + q].x;
  H = block_sum256(H, sh);
  Ha = block_sum256(Ha, sh);
  T = block_sum256(T, sh);
  if (threadIdx.x != 0) return;
  // sums of n_cp and n_ct partials, each a 256-term tree: float64 bound
  const double gam = (lay.n_cp + lay.n_ct + 300) * kU64 * 1.01;
  const double zT = net.zeta_f * T;
  const double ub = (H + zT) + gam * (Ha + fabs(H) + 2.0 * zT);
  const double prev = f_hi[b];
  const double out = (prev != prev || ub != ub) ? NAN : fmin(prev, ub);
  f_hi[b] = out;
  if (crown) crown[b] = (prev != prev) ? NAN : (again ? fmin(crown[b], ub) : ub);
}

// ---------------------------------------------------------------- many boxes
//
// Box-tiled forms of KC1 and KC3: every lane keeps four lines of four boxes,
// so each outage-factor or PTDF tile read from memory serves four boxes; the
// box tile is the fastest-varying block index, so blocks that read the same
// tile are dispatched together (dealt across the eight XCDs, so each tile is
// fetched into each XCD's L2 and shared there).  The partial
// arrays they write are those of the per-box kernels, so KC2, KC4 and KC5 are
// shared.
constexpr int kCB = 4;     // boxes per tile
constexpr int kKPB = 32;   // outages per KC1b block

template <bool REF>
__global__ __launch_bounds__(256) void kc1b_sweep(DevNet net, void* ws, const void* wsr, WsLayout lay,
                                                  int64_t n_box) {
  __shared__ double shv[4][kKPB][kCB][2];
  __shared__ float shn[4][kKPB][kCB];
  const int64_t bt = (int64_t)blockIdx.x * kCB;  // first box of the tile
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int col = (blockIdx.y * 4 + w) * 64 + lane;  // float4 column: four lines per lane
  const int Lp4 = net.Lp / 4;
  const int k0 = blockIdx.z * kKPB;
  const int k1 = min(net.K, k0 + kKPB);
  const bool live = col < Lp4;
  int64_t bb[kCB];
#pragma unroll
  for (int i = 0; i < kCB; ++i) bb[i] = min(bt + i, n_box - 1);
  float4 c4[kCB], g4[kCB];
  const int4* cd[kCB];
#pragma unroll
  for (int i = 0; i < kCB; ++i) {
    c4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    g4[i] = make_float4(FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX);
    cd[i] = ws_ptr<int4>(REF ? const_cast<void*>(wsr) : ws, lay.ctg) + bb[i] * net.K;
  }
  if (live && REF) {
    const float4 fc = reinterpret_cast<const float4*>(net.fmax_c32)[col];
#pragma unroll
    for (int i = 0; i < kCB; ++i) {
      c4[i] = reinterpret_cast<const float4*>(ws_ptr<float>(const_cast<void*>(wsr), lay.lc) + bb[i] * net.Lp)[col];
      g4[i] = fc;
    }
  } else if (live) {
    const float4 e4 = reinterpret_cast<const float4*>(net.line_eps)[col];
#pragma unroll
    for (int i = 0; i < kCB; ++i) {
      const double* bs = ws_ptr<double>(ws, lay.box) + bb[i] * kBoxSlots;
      const float vmax = __uint_as_float(*reinterpret_cast<const unsigned int*>(bs + kVmax));
      c4[i] = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lc) + bb[i] * net.Lp)[col];
      const float4 g = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lg) + bb[i] * net.Lp)[col];
      g4[i] = make_float4(add_ru(g.x, next_up_f32(e4.x * vmax)), add_ru(g.y, next_up_f32(e4.y * vmax)),
                          add_ru(g.z, next_up_f32(e4.z * vmax)), add_ru(g.w, next_up_f32(e4.w * vmax)));
    }
  }
  const float4* lam = reinterpret_cast<const float4*>(net.lodf) + col;
  float cs[kCB][4], ca[kCB][4];
#pragma unroll
  for (int i = 0; i < kCB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) cs[i][j] = ca[i][j] = 0.0f;
  // pairs of outages: 2 outages x 4 boxes x 3 sums in one halving reduction
  for (int kg = k0; kg < k1; kg += 2) {
    float r[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) r[i] = 0.0f;
    if (live) {
      float4 x[2];
#pragma unroll
      for (int o = 0; o < 2; ++o)
        x[o] = (kg + o < k1) ? ld_stream(lam + (size_t)(kg + o) * Lp4) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int o = 0; o < 2; ++o)
        if (kg + o < k1)
#pragma unroll
          for (int i = 0; i < kCB; ++i)
            kc1_row<REF>(x[o], cd[i][kg + o], c4[i], g4[i], cs[i], ca[i], r + 3 * (o * kCB + i));
    }
    bool act = false;
#pragma unroll
    for (int i = 0; i < 8; ++i) act |= r[3 * i + 2] != 0.0f;
    if (__any(act)) halving_sum24(r);
    // lane 8g holds outage kg + g / 4 of box g % 4
    if ((lane & 7) == 0) {
      const int g = lane >> 3, o = g / kCB, i = g % kCB;
      if (kg + o < k1) {
        shv[w][kg - k0 + o][i][0] = r[0];
        shv[w][kg - k0 + o][i][1] = r[1];
        shn[w][kg - k0 + o][i] = (float)r[2];
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < (k1 - k0) * kCB; t += 256) {
    const int q = t / kCB, i = t % kCB;
    if (bt + i >= n_box) continue;
    const double V = (shv[0][q][i][0] + shv[1][q][i][0]) + (shv[2][q][i][0] + shv[3][q][i][0]);
    const double A = (shv[0][q][i][1] + shv[1][q][i][1]) + (shv[2][q][i][1] + shv[3][q][i][1]);
    const double N = ((double)shn[0][q][i] + (double)shn[1][q][i]) + ((double)shn[2][q][i] + (double)shn[3][q][i]);
    ws_ptr<double4>(ws, lay.cv)[((size_t)(bt + i) * lay.kc_bx + blockIdx.y) * net.K + k0 + q] =
        make_double4(V, A, N, 0.0);
  }
  if (live) {
#pragma unroll
    for (int i = 0; i < kCB; ++i) {
      if (bt + i >= n_box) break;
      int2* cnt = ws_ptr<int2>(ws, lay.ccnt) + (bt + i) * net.Lp + 4 * col;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (ca[i][j] != 0.0f) {
          atomicAdd(&cnt[j].x, (int)cs[i][j]);
          atomicAdd(&cnt[j].y, (int)ca[i][j]);
        }
    }
  }
}

// Per bus n and four boxes: y = sum_l Phi32[l, n] v_l, ya, ye as in KC3, over
// one 1024-line tile; two buses per halving reduction, kNB buses per block.
__global__ __launch_bounds__(256) void kc3b_ptdf_t(DevNet net, void* ws, WsLayout lay, int64_t n_box) {
  __shared__ double sh[4][kNB][kCB][3];
  const int64_t bt = (int64_t)blockIdx.x * kCB;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int col = (blockIdx.y * 4 + w) * 64 + lane;
  const int Lp4 = net.Lp / 4;
  const bool live = col < Lp4;
  double v[kCB][4], va[kCB][4], ev[kCB][4];
#pragma unroll
  for (int i = 0; i < kCB; ++i) {
    const int64_t b = min(bt + i, n_box - 1);
    const double4* lv = ws_ptr<double4>(ws, lay.lv) + b * net.Lp + 4 * (live ? col : 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double4 q = live ? lv[j] : make_double4(0.0, 0.0, 0.0, 0.0);
      v[i][j] = q.x;
      va[i][j] = q.y;
      ev[i][j] = q.z;
    }
  }
  const int n0 = blockIdx.z * kNB;
  const int n1 = min(net.N, n0 + kNB);
  const float4* ph = reinterpret_cast<const float4*>(net.phiT) + col;
  for (int ng = n0; ng < n1; ng += 2) {
    double r[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) r[i] = 0.0;
    if (live) {
      float4 x[2];
#pragma unroll
      for (int o = 0; o < 2; ++o)
        x[o] = (ng + o < n1) ? ld_stream(ph + (size_t)(ng + o) * Lp4) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const double p[4] = {(double)x[o].x, (double)x[o].y, (double)x[o].z, (double)x[o].w};
#pragma unroll
        for (int i = 0; i < kCB; ++i) {
          double* q = r + 3 * (o * kCB + i);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            q[0] = fma(p[j], v[i][j], q[0]);
            q[1] = fma(fabs(p[j]), va[i][j], q[1]);
            q[2] = fma(fabs(p[j]), ev[i][j], q[2]);
          }
        }
      }
    }
    halving_sum24(r);
    if ((lane & 7) == 0) {
      const int g = lane >> 3, o = g / kCB, i = g % kCB;
      if (ng + o < n1) {
        sh[w][ng - n0 + o][i][0] = r[0];
        sh[w][ng - n0 + o][i][1] = r[1];
        sh[w][ng - n0 + o][i][2] = r[2];
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < (n1 - n0) * kCB; t += 256) {
    const int q = t / kCB, i = t % kCB;
    if (bt + i >= n_box) continue;
    double o[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) o[f] = (sh[0][q][i][f] + sh[1][q][i][f]) + (sh[2][q][i][f] + sh[3][q][i][f]);
    ws_ptr<double4>(ws, lay.bpart)[((size_t)(bt + i) * lay.kc3_bx + blockIdx.y) * net.Np + n0 + q] =
        make_double4(o[0], o[1], o[2], 0.0);
  }
}

// The same three products on the float64 matrix cores (v_mfma_f64_16x16x4f64)
// for the box-tiled path: D[bus][box] = sum over lines of A[bus][line] B[line][box]
// with A = Phi32^T (or |Phi32|^T) and B = v (or va, ev).  A wave owns 32
// buses x 32 boxes over one chunk of lines; per group of 16 lines each lane
// loads one float4 of the transposed PTDF per bus fragment (four lines of
// one bus: the A operands of four k-steps, line l0 + 4 k + s in step s) and
// one (v, va, ev) record per step and box fragment, and issues 48 MFMAs.  The
// four waves of a block take four 32-bus ranges of the same boxes.  Chunk z
// writes partial z of bpart (lay.kc3_bx chunks), summed by kc4_inputs.
// Operand layout as in the base-flow MFMA kernel: A[i][k] at lane i + 16 k,
// B[k][j] at lane j + 16 k, D[i][j] at lane j + 16 (i % 4), element i / 4.
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256, 2) void kc3m_ptdf_t(DevNet net, void* ws, WsLayout lay, int64_t n_box) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int n0 = (blockIdx.x * 4 + w) * 32;
  if (n0 >= net.N) return;  // whole wave past the last bus; no barrier follows
  const int64_t b0 = (int64_t)blockIdx.y * 32;
  const int i16 = lane & 15, k4 = lane >> 4;
  const int l_begin = blockIdx.z * lay.kc3_chunk;
  const int l_end = min(net.Lp, l_begin + lay.kc3_chunk);
  const float4* pa0 = reinterpret_cast<const float4*>(net.phiT + (size_t)min(n0 + i16, net.N - 1) * net.Lp + 4 * k4);
  const float4* pa1 =
      reinterpret_cast<const float4*>(net.phiT + (size_t)min(n0 + 16 + i16, net.N - 1) * net.Lp + 4 * k4);
  // line-major adjoint: lanes of one k4 read 16 consecutive boxes of a line
  // (boxes past n_box up to the 32-box tile are in the allocation; their
  // columns feed only outputs that are not written)
  const size_t bt = lay.kc3_bt;
  const double4* pb0 = ws_ptr<double4>(ws, lay.lv) + (size_t)(4 * k4) * bt + b0 + i16;
  const double4* pb1 = pb0 + 16;
  v4d y[2][2], ya[2][2], ye[2][2];
#pragma unroll
  for (int fi = 0; fi < 2; ++fi)
#pragma unroll
    for (int fj = 0; fj < 2; ++fj) y[fi][fj] = ya[fi][fj] = ye[fi][fj] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int l0 = l_begin; l0 < l_end; l0 += 16) {
    const float4 x0 = pa0[l0 / 4], x1 = pa1[l0 / 4];
    const float a0[4] = {x0.x, x0.y, x0.z, x0.w}, a1[4] = {x1.x, x1.y, x1.z, x1.w};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const double4 q0 = pb0[(size_t)(l0 + st) * bt], q1 = pb1[(size_t)(l0 + st) * bt];
      const double p0 = a0[st], p1 = a1[st];
      y[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(p0, q0.x, y[0][0], 0, 0, 0);
      y[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(p0, q1.x, y[0][1], 0, 0, 0);
      y[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(p1, q0.x, y[1][0], 0, 0, 0);
      y[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(p1, q1.x, y[1][1], 0, 0, 0);
      ya[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(p0), q0.y, ya[0][0], 0, 0, 0);
      ya[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(p0), q1.y, ya[0][1], 0, 0, 0);
      ya[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(p1), q0.y, ya[1][0], 0, 0, 0);
      ya[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(p1), q1.y, ya[1][1], 0, 0, 0);
      ye[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(p0), q0.z, ye[0][0], 0, 0, 0);
      ye[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(p0), q1.z, ye[0][1], 0, 0, 0);
      ye[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(p1), q0.z, ye[1][0], 0, 0, 0);
      ye[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(p1), q1.z, ye[1][1], 0, 0, 0);
    }
  }
  // element r of lane t: bus n0 + 16 fi + 4 r + t / 16, box b0 + 16 fj + t % 16
  double4* out = ws_ptr<double4>(ws, lay.bpart);
#pragma unroll
  for (int fj = 0; fj < 2; ++fj) {
    const int64_t b = b0 + 16 * fj + i16;
    if (b >= n_box) continue;
#pragma unroll
    for (int fi = 0; fi < 2; ++fi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = n0 + 16 * fi + 4 * r + k4;
        if (n < net.N)
          out[((size_t)b * lay.kc3_bx + blockIdx.z) * net.Np + n] =
              make_double4(y[fi][fj][r], ya[fi][fj][r], ye[fi][fj][r], 0.0);
      }
  }
}

// ---------------------------------------------------------------- lower bound
//
// Chord relaxation: every penalty phi(z) = max(|z| - t, 0) is convex, so on an
// interval that holds every value its pre-activation takes over the box it
// lies below the chord between the interval's ends.  With those lines
//
//   f(x) >= S(x) - zeta_inj (a_I z_I(x) + b_I) - zeta_f sum_e (a_e z_e(x) + b_e)
//
// at every x of the box; the right side is linear in x (plus the curve part),
// and its minimum over the box, taken with the same coefficient error bounds
// as the upper bound, is a certified lower bound on min f.
//
// Contingency elements (float32, per element): in y = sign(C) z - t the K3
// interval is [t_lo, t_hi] (exactly the floats K3 forms, which enclose the
// exact pre-activation range), and the penalty there is
// q(y) = max(|y + t| - t, 0).  An element with t_hi <= 0 has q = 0 on its whole
// interval and contributes nothing.  Otherwise the slope alpha (the chord
// slope, rounded to a multiple of 2^-24 in [0, 1]; any slope gives a valid
// line) and beta >= max(q(t_hi) - alpha t_hi, q(t_lo) - alpha t_lo) (rounded
// up) give q(y) <= alpha y + beta on [t_lo, t_hi] by convexity.  Each element's
// line is written around C' = c_l + Lam c_c (real arithmetic on the float32
// operands): a (z - C') + m with a = sign(C) alpha and m >= alpha (|C'| - t) +
// beta, so the constant of the relaxation is
//   sum_e b_e = sum_e m_e - sum_l c_l sum_k a_kl - sum_k c_c(k) sum_l a_kl Lam_kl,
// a sum of non-negative m (float32, relative error only) and two terms built
// from the per-line slope totals (exact integers in units of 2^-24) and the
// per-outage sums sum_l a Lam that the adjoint needs anyway.
constexpr int kCKB = 32;   // outages per block of the box-tiled chord sweep
constexpr int kCKB1 = 64;  // outages per block of the per-box chord sweep (half the per-line totals)
// the per-block line totals of the per-box sweep are int32 sums of at most
// kCKB1 slopes of at most 2^24 each
static_assert(((long long)kCKB1 << 24) < (1ll << 31), "per-block slope totals must fit in int32");
constexpr float kSlopeQ = 16777216.0f;  // 2^24

// One element: fixed-point slope magnitude qa and signed slope qs
// (a = qs / 2^24, |a| = alpha = qa / 2^24), and the value bound m (all zero
// when t_hi <= 0 or the entry is the outaged line's own, whose NaN fails the
// test).  Roundings (u = 2^-24, results in
// the normal range; FLT_MIN covers the rest):
//   - q0 = RN(-tl - 2 tq) is within u |q0| of the exact value, and
//     q0 (1 + 4u) + FLT_MIN, rounded, is above it;
//   - each of the two intercept candidates is within u of its magnitude, so
//     beta (1 + 4u), rounded, is above the exact maximum;
//   - y = alpha (|C| - tq) + beta carries the roundings of d = |C| - tq and
//     of the fma, and |C'| <= |C| (1 + u): the pad 8u (|C| + tq + |y|) and
//     FLT_MIN cover them with the final rounding.
__device__ __forceinline__ void chord_elem(float lam, float cc, float rk, float cl, float h, float g, float tq,
                                           float& qa, float& qs, float& m) {
  const float C = fmaf(lam, cc, cl);
  const float aC = fabsf(C);
  const float th = aC + fmaf(fabsf(lam), rk, h);
  const float tl = aC - fmaf(fabsf(lam), rk, g);
  const float q0 = fmaf(-2.0f, tq, -tl);
  const float ql = fmaxf(fmaxf(tl, fmaf(q0, 1.0f + 0x1p-22f, FLT_MIN)), 0.0f);
  // NaN (zero width) clamps to 0
  const float al = fminf(fmaxf((th - ql) * __builtin_amdgcn_rcpf(th - tl), 0.0f), 1.0f);
  const float qf = rintf(al * kSlopeQ);
  const float alq = qf * (1.0f / kSlopeQ);
  const float beta = fmaxf(fmaf(-alq, th, th), fmaf(-alq, tl, ql));
  const float bu = fmaf(fabsf(beta), 0x1p-22f, beta);
  const float y = fmaf(alq, aC - tq, bu);
  const float mm = fmaf(0x1p-21f, (aC + tq) + fabsf(y), y) + FLT_MIN;
  const bool act = th > 0.0f;
  qa = act ? qf : 0.0f;
  qs = copysignf(qa, C);
  m = act ? fmaxf(mm, 0.0f) : 0.0f;
}

// Four lines x one outage of one box: per-line fixed-point slope totals, and
// the outage's four sums (a Lam, |a Lam|, alpha, m) into r[0..3].
template <bool VCOPY>
__device__ __forceinline__ void chord_row(const float4& x, const int4& d, const float4& c4, const float4& h4,
                                          const float4& g4, const float4& t4, int (&cs)[4], int (&ca)[4],
                                          float* r) {
  // the outage's record (scalar loads) is read by three instructions per
  // line: vector copies where the registers allow (one box per lane)
  const float cc = VCOPY ? vcopy(__int_as_float(d.y)) : __int_as_float(d.y);
  const float rk = VCOPY ? vcopy(__int_as_float(d.z)) : __int_as_float(d.z);
  const float lam[4] = {x.x, x.y, x.z, x.w}, cl[4] = {c4.x, c4.y, c4.z, c4.w};
  const float hh[4] = {h4.x, h4.y, h4.z, h4.w}, gg[4] = {g4.x, g4.y, g4.z, g4.w};
  const float tt[4] = {t4.x, t4.y, t4.z, t4.w};
  float v = 0.0f, va = 0.0f, n = 0.0f, mm = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float qa, qs, m;
    chord_elem(lam[i], cc, rk, cl[i], hh[i], gg[i], tt[i], qa, qs, m);
    cs[i] += (int)qs;
    ca[i] += (int)qa;
    const float a = qs * (1.0f / kSlopeQ);
    // NaN entries carry a = 0 and a finite stand-in
    const float p = a * finite_factor(lam[i]);
    v += p;
    va += fabsf(p);
    n += fabsf(a);
    mm += m;
  }
  r[0] = v;
  r[1] = va;
  r[2] = n;
  r[3] = mm;
}

// Sums v[0..31] over the 64 lanes of a wave by halving exchanges (16 + 8 + 4 +
// 2 + 1, then one plain step): afterwards lanes 2g and 2g + 1 hold the total
// of v[g] in v[0].
__device__ __forceinline__ void halving_sum32(float (&v)[32]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = halve32(v[i], v[i + 16]);
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = halve16(v[i], v[i + 8]);
  {
    const bool up = lane & 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float send = up ? v[i] : v[i + 4];
      const float keep = up ? v[i + 4] : v[i];
      v[i] = keep + lane_xor<kDppXor8>(send);
    }
  }
  {
    const bool up = lane & 4;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float send = up ? v[i] : v[i + 2];
      const float keep = up ? v[i + 2] : v[i];
      v[i] = keep + __shfl_xor(send, 4, 64);
    }
  }
  {
    const bool up = lane & 2;
    const float send = up ? v[0] : v[1];
    const float keep = up ? v[1] : v[0];
    v[0] = keep + lane_xor<kDppXor2>(send);
  }
  v[0] += lane_xor<kDppXor1>(v[0]);
}

// Outage sweep of the chord relaxation: NB boxes per lane (1, or 2 or 4
// sharing every streamed outage-factor tile), four lines per lane, KB
// outages per block; 8 / NB outages x NB boxes x 4 sums per halving
// reduction.  Grid: (box tiles, line tiles, outage blocks).  MINB bounds the
// registers (one box: 6 waves per SIMD; two boxes: 5; four boxes: 3, the
// most that holds four boxes' line data without spilling).  Each element is
// a dependent chain of about 45 instructions with one reciprocal; the one-box
// sweep's time did not move with 3 to 6 waves per SIMD or 16 to 64 outages
// per block.
template <int NB, int MINB, int KB>
__global__ __launch_bounds__(256, MINB) void kc1c_chord(DevNet net, void* ws, WsLayout lay, int64_t n_box) {
  constexpr int OG = 8 / NB;
  __shared__ float sh[4][KB][NB][4];
  const int64_t bt = (int64_t)blockIdx.x * NB;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int col = (blockIdx.y * 4 + w) * 64 + lane;
  const int Lp4 = net.Lp / 4;
  const int k0 = blockIdx.z * KB;
  const int k1 = min(net.K, k0 + KB);
  const bool live = col < Lp4;
  int64_t bb[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) bb[i] = min(bt + i, n_box - 1);
  float4 c4[NB], h4[NB], g4[NB], t4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const int4* cd[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    c4[i] = h4[i] = g4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    cd[i] = ws_ptr<int4>(ws, lay.ctg) + bb[i] * net.K;
  }
  if (live) {
    const float4 e4 = reinterpret_cast<const float4*>(net.line_eps)[col];
    const float4 f4 = reinterpret_cast<const float4*>(net.fmax_c32)[col];
    // a float32 limit no larger than the float64 one
    constexpr float kDown = 1.0f - 0x1p-22f;
    t4 = make_float4(f4.x * kDown, f4.y * kDown, f4.z * kDown, f4.w * kDown);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const double* bs = ws_ptr<double>(ws, lay.box) + bb[i] * kBoxSlots;
      const float vmax = __uint_as_float(*reinterpret_cast<const unsigned int*>(bs + kVmax));
      const float ex = next_up_f32(e4.x * vmax), ey = next_up_f32(e4.y * vmax);
      const float ez = next_up_f32(e4.z * vmax), ew = next_up_f32(e4.w * vmax);
      c4[i] = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lc) + bb[i] * net.Lp)[col];
      const float4 h = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lh) + bb[i] * net.Lp)[col];
      const float4 g = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lg) + bb[i] * net.Lp)[col];
      h4[i] = make_float4(add_ru(h.x, ex), add_ru(h.y, ey), add_ru(h.z, ez), add_ru(h.w, ew));
      g4[i] = make_float4(add_ru(g.x, ex), add_ru(g.y, ey), add_ru(g.z, ez), add_ru(g.w, ew));
    }
  }
  const float4* lam = reinterpret_cast<const float4*>(net.lodf) + col;
  int cs[NB][4], ca[NB][4];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) cs[i][j] = ca[i][j] = 0;
  for (int kg = k0; kg < k1; kg += OG) {
    float r[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) r[i] = 0.0f;
    if (live) {
      float4 x[OG];
#pragma unroll
      for (int o = 0; o < OG; ++o)
        x[o] = (kg + o < k1) ? ld_stream(lam + (size_t)(kg + o) * Lp4) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int o = 0; o < OG; ++o)
        if (kg + o < k1)
#pragma unroll
          for (int i = 0; i < NB; ++i)
            chord_row<NB == 1>(x[o], cd[i][kg + o], c4[i], h4[i], g4[i], t4, cs[i], ca[i], r + 4 * (o * NB + i));
    }
    // a wave with no active element in the group skips the reduction
    bool act = false;
#pragma unroll
    for (int i = 0; i < 8; ++i) act |= (r[4 * i + 2] != 0.0f) | (r[4 * i + 3] != 0.0f);
    if (__any(act)) halving_sum32(r);
    // lane 2g holds sum g = 4 (o NB + i) + f (zeros when the wave skipped)
    if ((lane & 1) == 0) {
      const int g = lane >> 1, o = g / (4 * NB), i = (g >> 2) % NB;
      if (kg + o < k1) sh[w][kg - k0 + o][i][g & 3] = r[0];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < (k1 - k0) * NB; t += 256) {
    const int q = t / NB, i = t % NB;
    if (bt + i >= n_box) continue;
    double o[4];
#pragma unroll
    for (int f = 0; f < 4; ++f)
      o[f] = ((double)sh[0][q][i][f] + (double)sh[1][q][i][f]) + ((double)sh[2][q][i][f] + (double)sh[3][q][i][f]);
    ws_ptr<double4>(ws, lay.cv)[((size_t)(bt + i) * lay.kc_bx + blockIdx.y) * net.K + k0 + q] =
        make_double4(o[0], o[1], o[2], o[3]);
  }
  if (live && NB == 1 && lay.chp_z) {
    // one box: every block of outages targets the same lines, so atomics
    // would queue on the same addresses; each block stores its line totals
    // (at most KB 2^24 each) for the line kernel to add up
    int2* part = ws_ptr<int2>(ws, lay.chp) + ((size_t)bt * lay.chp_z + blockIdx.z) * net.Lp + 4 * col;
    reinterpret_cast<int4*>(part)[0] = make_int4(cs[0][0], ca[0][0], cs[0][1], ca[0][1]);
    reinterpret_cast<int4*>(part)[1] = make_int4(cs[0][2], ca[0][2], cs[0][3], ca[0][3]);
  } else if (live) {
    // per-line slope totals: 64-bit integer atomics, so the totals do not
    // depend on the order (at most K 2^24 per line)
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if (bt + i >= n_box) break;
      unsigned long long* cnt = ws_ptr<unsigned long long>(ws, lay.ccnt) + 2 * ((bt + i) * net.Lp + 4 * col);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (ca[i][j] != 0) {
          atomicAdd(&cnt[2 * j], (unsigned long long)(long long)cs[i][j]);
          atomicAdd(&cnt[2 * j + 1], (unsigned long long)(long long)ca[i][j]);
        }
    }
  }
}

// Per line of the chord relaxation: the base line's chord (float64), the
// adjoint v with vabs >= |v_exact| and ev >= |v^ - v_exact| as in KC2, and an
// upper bound T_l on the line's share of the relaxation's constant:
//   the base intercept, - c_l sum_k a_kl, and for the line's outage k
//   sum_l m_kl - c_c(k) sum_l a_kl Lam_kl (whose float32 rounding is bounded
//   by 12u sum |a Lam|: one product rounding, three in-lane additions, six
//   halving levels, with a spare u).
// Block partials (sum T_l, sum vabs, sum |terms of T_l|).
__global__ __launch_bounds__(256) void kc2c_lines(DevNet net, void* ws, WsLayout lay, int64_t box0) {
  __shared__ double sh[4];
  const int64_t b = box0 + blockIdx.y;
  const int l = blockIdx.x * 256 + threadIdx.x;
  double v = 0.0, va = 0.0, ev = 0.0, T = 0.0, Ta = 0.0;
  if (l < net.L) {
    const double fb = net.fmax_b[l];
    const double cf = ws_ptr<double>(ws, lay.lcf)[b * net.L + l];
    const double rf = ws_ptr<double>(ws, lay.lrf)[b * net.L + l];
    // base line: y = sign(cf) z - fb on [|cf| - rf - fb, |cf| + rf - fb] (outward)
    double ab = 0.0, tb = 0.0, tba = 0.0;
    {
      const double e = 4.0 * kU64 * (fabs(cf) + rf + fb);
      const double th = fabs(cf) + rf - fb + e;
      const double tl = fabs(cf) - rf - fb - e;
      if (th > 0.0) {
        const double q0 = -tl - 2.0 * fb;
        const double ql = fmax(fmax(tl, q0 + 4.0 * kU64 * (fabs(tl) + 2.0 * fb)), 0.0);
        const double al = fmin(fmax((th - ql) / (th - tl), 0.0), 1.0);
        double be = fmax(fma(-al, th, th), fma(-al, tl, ql));
        be += 4.0 * kU64 * (fabs(be) + th + fabs(tl) + ql);
        // the line alpha y + beta in z: a z + (beta - alpha fb)
        ab = copysign(al, cf);
        tb = be - al * fb;
        tba = fabs(be) + al * fb;
        tb += 2.0 * kU64 * tba;
      }
    }
    long long n0 = 0, n1 = 0;
    if (lay.chp_z) {
      // sixteen partials in flight per round (the grid is one thread per line)
      const int2* part = ws_ptr<int2>(ws, lay.chp) + (size_t)b * lay.chp_z * net.Lp + l;
      int z = 0;
      for (; z + 16 <= lay.chp_z; z += 16) {
        int2 q[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) q[i] = part[(size_t)(z + i) * net.Lp];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          n0 += q[i].x;
          n1 += q[i].y;
        }
      }
      for (; z < lay.chp_z; ++z) {
        const int2 q = part[(size_t)z * net.Lp];
        n0 += q.x;
        n1 += q.y;
      }
    } else {
      const long long* n = ws_ptr<long long>(ws, lay.ccnt) + 2 * (b * net.Lp + l);
      n0 = n[0];
      n1 = n[1];
    }
    const double nx = (double)n0 * (1.0 / 16777216.0), ny = (double)n1 * (1.0 / 16777216.0);
    const double cl = (double)ws_ptr<float>(ws, lay.lc)[b * net.Lp + l];
    v = ab + nx;
    va = fabs(ab) + ny;
    T = tb - cl * nx;
    Ta = tba + fabs(cl * nx);
    const int k = net.ctg_of_line[l];
    if (k >= 0) {
      double V = 0.0, A = 0.0, N = 0.0, M = 0.0;
      const double4* cv = ws_ptr<double4>(ws, lay.cv) + (size_t)b * lay.kc_bx * net.K + k;
      for (int t = 0; t < lay.kc_bx; ++t) {
        const double4 q = cv[(size_t)t * net.K];
        V += q.x;
        A += q.y;
        N += q.z;
        M += q.w;
      }
      const double gam = (net.Lp + lay.kc_bx + 16) * kU64 * 1.01;
      const double f32 = 1.0 + 12.0 * kU32;
      const double A1 = A * (1.0 + gam) * (1.0 + kKappa0) * f32;
      ev = (kKappa0 + net.ctg_eps[k] + gam + 12.0 * kU32) * A1 + 2.0 * net.phi_err_max * net.ctg_inv[k] * N * f32;
      v += V;
      va += A1 + ev;
      // this line is the outage's own: c_c(k) = c_l; V is within 12u A (float32
      // within a wave) plus gam A (float64 over waves and tiles) of its exact value
      const double M1 = M * (1.0 + gam) * f32;
      const double eV = fabs(cl) * (12.0 * kU32 + gam) * A1;
      T += M1 - cl * V + eV;
      Ta += M1 + fabs(cl * V) + eV;
    }
    ev = (ev + 2.0 * kU64 * va) * (1.0 + 4.0 * kU64);
    va = va * (1.0 + 4.0 * kU64) + ev;
    // products and the additions forming T
    T += 8.0 * kU64 * Ta;
    Ta *= (1.0 + 8.0 * kU64);
  }
  if (l < net.Lp) ws_ptr<double4>(ws, lay.lv)[lv_index(lay, net, b, l)] = make_double4(v, va, ev, 0.0);
  T = block_sum256(T, sh);
  const double S = block_sum256(va, sh);
  Ta = block_sum256(Ta, sh);
  if (threadIdx.x == 0) ws_ptr<double4>(ws, lay.ct)[b * lay.n_ct + blockIdx.x] = make_double4(T, S, Ta, 0.0);
}

// Per box: lower bound = sum of the input partials - zeta_f sum T_l, padded
// for the float64 sums; f_lo becomes the larger of IBP's and this bound.
__global__ __launch_bounds__(256) void kc5c_finalize(DevNet net, void* ws, WsLayout lay, int64_t box0,
                                                     double* __restrict__ f_lo, double* __restrict__ crown) {
  __shared__ double sh[4];
  const int64_t b = box0 + blockIdx.x;
  double H = 0.0, Ha = 0.0, T = 0.0, Ta = 0.0;
  for (int q = threadIdx.x; q < lay.n_cp; q += 256) {
    const double2 t = ws_ptr<double2>(ws, lay.cp)[b * lay.n_cp + q];
    H += t.x;
    Ha += t.y;
  }
  for (int q = threadIdx.x; q < lay.n_ct; q += 256) {
    const double4 t = ws_ptr<double4>(ws, lay.ct)[b * lay.n_ct + q];
    T += t.x;
    Ta += t.z;
  }
  H = block_sum256(H, sh);
  Ha = block_sum256(Ha, sh);
  T = block_sum256(T, sh);
  Ta = block_sum256(Ta, sh);
  if (threadIdx.x != 0) return;
  const double gam = (lay.n_cp + lay.n_ct + 300) * kU64 * 1.01;
  const double zT = net.zeta_f * T;
  const double lb = (H - zT) - gam * (Ha + fabs(H) + net.zeta_f * Ta + fabs(zT));
  const double prev = f_lo[b];
  f_lo[b] = (prev != prev || lb != lb) ? NAN : fmax(prev, lb);
  if (crown) crown[b] = (prev != prev) ? NAN : lb;
}

hipError_t launch_crown_lower(const DevNet& net, int64_t n_box, const float* lo, const float* hi, double* f_lo,
                              double* crown, float* vertex, void* ws, const WsLayout& lay, hipStream_t s,
                              KernelTimer* tm) {
  for (int64_t b0 = 0; b0 < n_box && !lay.chp_z; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(10, s);
    // two int64 totals per line: zeroed as pairs of int2
    const int64_t nz = 2 * (int64_t)nb * net.Lp;
    int2* cnt = reinterpret_cast<int2*>(static_cast<char*>(ws) + lay.ccnt) + 2 * b0 * net.Lp;
    hipLaunchKernelGGL(kc0_zero, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, cnt, nz);
    tm->stop(t, s);
  }
  if (net.K > 0) {
    const int t = tm->start(10, s);
    const unsigned kz = (unsigned)((net.K + kCKB - 1) / kCKB);
    if (n_box < kCB)
      hipLaunchKernelGGL((kc1c_chord<1, 5, kCKB1>), dim3((unsigned)n_box, lay.kc_bx, lay.chp_z), dim3(256), 0, s,
                         net, ws, lay, n_box);
    else if (lay.chord_nb == 1)
      hipLaunchKernelGGL((kc1c_chord<1, 5, kCKB>), dim3((unsigned)n_box, lay.kc_bx, kz), dim3(256), 0, s, net, ws,
                         lay, n_box);
    else if (lay.chord_nb == 2)
      hipLaunchKernelGGL((kc1c_chord<2, 5, kCKB>), dim3((unsigned)((n_box + 1) / 2), lay.kc_bx, kz), dim3(256), 0,
                         s, net, ws, lay, n_box);
    else
      hipLaunchKernelGGL((kc1c_chord<kCB, 1, kCKB>), dim3((unsigned)((n_box + kCB - 1) / kCB), lay.kc_bx, kz),
                         dim3(256), 0, s, net, ws, lay, n_box);
    tm->stop(t, s);
  }
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(11, s);
    hipLaunchKernelGGL(kc2c_lines, dim3(lay.n_ct, nb), dim3(256), 0, s, net, ws, lay, b0);
    if (n_box < kCB)
      hipLaunchKernelGGL(kc3_ptdf_t, dim3(lay.kc3_bx, lay.kc3_by, nb), dim3(256), 0, s, net, ws, lay, b0);
    tm->stop(t, s);
  }
  if (n_box >= kCB) {
    const int t = tm->start(11, s);
    if (lay.kc3_mfma)
      hipLaunchKernelGGL(kc3m_ptdf_t, dim3((net.N + 127) / 128, (unsigned)((n_box + 31) / 32), lay.kc3_bx),
                         dim3(256), 0, s, net, ws, lay, n_box);
    else
      hipLaunchKernelGGL(kc3b_ptdf_t, dim3((unsigned)((n_box + kCB - 1) / kCB), lay.kc3_bx, lay.kc3_by),
                         dim3(256), 0, s, net, ws, lay, n_box);
    tm->stop(t, s);
  }
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(12, s);
    hipLaunchKernelGGL(kc4_inputs<true>, dim3(lay.n_cp, nb), dim3(256), 0, s, net, ws, nullptr, lay, b0, lo, hi,
                       vertex);
    hipLaunchKernelGGL(kc5c_finalize, dim3(nb), dim3(256), 0, s, net, ws, lay, b0, f_lo, crown);
    tm->stop(t, s);
  }
  return hipGetLastError();
}

void plan_crown(const DevNet& net, int64_t n_box, WsLayout& lay, const Tune& t) {
  const int lp4 = net.Lp / 4;
  lay.kc_bx = (lp4 + 255) / 256;
  lay.kc_by = std::max(1, (net.K + kKC - 1) / kKC);
  lay.kc3_bx = (lp4 + 255) / 256;
  lay.kc3_by = (net.N + kNB - 1) / kNB;
  lay.kc3_mfma = 0;
  lay.kc3_chunk = net.Lp;
  if (t.k2b_mfma && n_box >= kCB) {
    // line chunks (multiples of 16) so that bus x box tiles x chunks fill the chip
    const int64_t blocks = (int64_t)((net.N + 127) / 128) * ((n_box + 31) / 32);
    int sc = (int)std::min<int64_t>(8, (2048 + blocks - 1) / blocks);
    sc = std::max(1, std::min(sc, net.Lp / 256));
    lay.kc3_mfma = 1;
    lay.kc3_bt = (int)((n_box + 31) / 32 * 32);
    lay.kc3_chunk = ((net.Lp + sc - 1) / sc + 15) & ~15;
    lay.kc3_bx = (net.Lp + lay.kc3_chunk - 1) / lay.kc3_chunk;
  }
  lay.n_cp = (net.X + 255) / 256;
  lay.n_ct = (net.L + 255) / 256;
  lay.chord_nb = t.chord_nb;
  // (with no outages there is no sweep: the zeroed totals serve)
  lay.chp_z = (n_box < kCB && net.K > 0) ? (net.K + kCKB1 - 1) / kCKB1 : 0;
}

// Reference points: the box centre first, then halfway towards the vertex that
// maximised the previous relaxation (float32; any point gives valid slopes).
__global__ __launch_bounds__(256) void kc_ref_update(int64_t n, const float* __restrict__ lo,
                                                     const float* __restrict__ hi, float* __restrict__ xref,
                                                     const float* __restrict__ vtx, int first) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= n) return;
  xref[i] = first ? 0.5f * lo[i] + 0.5f * hi[i] : 0.5f * xref[i] + 0.5f * vtx[i];
}

// One relaxation pass over every box; wsr != nullptr takes the slopes at the
// reference points whose forward data it holds.
static void relax_pass(const DevNet& net, int64_t n_box, const float* lo, const float* hi, double* f_hi,
                       double* crown, float* vertex, void* ws, const void* wsr, int again, const WsLayout& lay,
                       hipStream_t s, KernelTimer* tm) {
  const bool ref = wsr != nullptr;
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(10, s);
    const int64_t nz = (int64_t)nb * net.Lp;
    int2* cnt = reinterpret_cast<int2*>(static_cast<char*>(ws) + lay.ccnt) + b0 * net.Lp;
    hipLaunchKernelGGL(kc0_zero, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, cnt, nz);
    if (net.K > 0 && n_box < kCB) {
      if (ref)
        hipLaunchKernelGGL(kc1_sweep<true>, dim3(lay.kc_bx, lay.kc_by, nb), dim3(256), 0, s, net, ws, wsr, lay, b0);
      else
        hipLaunchKernelGGL(kc1_sweep<false>, dim3(lay.kc_bx, lay.kc_by, nb), dim3(256), 0, s, net, ws, wsr, lay,
                           b0);
    }
    tm->stop(t, s);
  }
  const unsigned tiles = (unsigned)((n_box + kCB - 1) / kCB);
  if (net.K > 0 && n_box >= kCB) {
    const int t = tm->start(10, s);
    const dim3 grid(tiles, lay.kc_bx, (net.K + kKPB - 1) / kKPB);
    if (ref)
      hipLaunchKernelGGL(kc1b_sweep<true>, grid, dim3(256), 0, s, net, ws, wsr, lay, n_box);
    else
      hipLaunchKernelGGL(kc1b_sweep<false>, grid, dim3(256), 0, s, net, ws, wsr, lay, n_box);
    tm->stop(t, s);
  }
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(11, s);
    hipLaunchKernelGGL(kc2_lines, dim3(lay.n_ct, nb), dim3(256), 0, s, net, ws, wsr, lay, b0);
    if (n_box < kCB)
      hipLaunchKernelGGL(kc3_ptdf_t, dim3(lay.kc3_bx, lay.kc3_by, nb), dim3(256), 0, s, net, ws, lay, b0);
    tm->stop(t, s);
  }
  if (n_box >= kCB) {
    const int t = tm->start(11, s);
    if (lay.kc3_mfma)
      hipLaunchKernelGGL(kc3m_ptdf_t, dim3((net.N + 127) / 128, (unsigned)((n_box + 31) / 32), lay.kc3_bx),
                         dim3(256), 0, s, net, ws, lay, n_box);
    else
      hipLaunchKernelGGL(kc3b_ptdf_t, dim3(tiles, lay.kc3_bx, lay.kc3_by), dim3(256), 0, s, net, ws, lay, n_box);
    tm->stop(t, s);
  }
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(12, s);
    hipLaunchKernelGGL(kc4_inputs<false>, dim3(lay.n_cp, nb), dim3(256), 0, s, net, ws, wsr, lay, b0, lo, hi, vertex);
    hipLaunchKernelGGL(kc5_finalize, dim3(nb), dim3(256), 0, s, net, ws, lay, b0, f_hi, crown, again);
    tm->stop(t, s);
  }
}

hipError_t launch_crown(const DevNet& net, int64_t n_box, const float* lo, const float* hi, int ref_iters,
                        double* f_hi, double* crown, float* vertex, void* ws, const WsLayout& lay, hipStream_t s,
                        KernelTimer* tm) {
  float* vtx = reinterpret_cast<float*>(static_cast<char*>(ws) + lay.vtx);
  float* xref = reinterpret_cast<float*>(static_cast<char*>(ws) + lay.xref);
  void* wsr = static_cast<char*>(ws) + lay.ref;
  relax_pass(net, n_box, lo, hi, f_hi, crown, ref_iters > 0 ? vtx : vertex, ws, nullptr, 0, lay, s, tm);
  const int64_t n = n_box * net.X;
  for (int it = 0; it < ref_iters; ++it) {
    hipLaunchKernelGGL(kc_ref_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, lo, hi, xref, vtx,
                       it == 0 ? 1 : 0);
    hipError_t e = launch_forward_prep(net, n_box, xref, xref, wsr, lay, s, tm);
    if (e != hipSuccess) return e;
    relax_pass(net, n_box, lo, hi, f_hi, crown, it + 1 == ref_iters ? vertex : vtx, ws, wsr, 1, lay, s, tm);
  }
  return hipGetLastError();
}

}  // namespace ibp
