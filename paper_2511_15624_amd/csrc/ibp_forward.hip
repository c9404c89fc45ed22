// Forward IBP kernels for gfx950 (MI355X): one box per grid slice.
//
//   K1  box -> per-bus injection centre/radius (Sec. II-A, p_inj = N_g p_g - N_d p_d),
//       surplus and imbalance intervals (Appendix eq. ibp_f; imbalance in the
//       closed form of E^T Phi - I = -e_slack 1^T).
//   K2  base flows c_f = Phi c, r_f = |Phi| r (Sec. III-C eq. IBP on Sec. II-A
//       eq. line flow ptdf), base overload penalties (Sec. III-A eq. slack-sfb),
//       and the per-line / per-outage constants K3 needs.
//   K3  every (outage, line) pair: post-outage flow interval (Sec. II-C eq. ctg
//       flow simplified, as line flow plus outage factor times the outaged
//       line's flow), overload penalties (eq. slack-Sc) and their sum
//       (eq. slack-sagg).  The outage-factor matrix is streamed once; the
//       K x L flow matrix is never stored.
//   K4  objective interval (eq. penalized-objective / ibp_f) per box.
//
// Float32 is used for the streamed data with outward padding folded into
// per-line and per-outage radii so that every bound encloses the exact
// interval of the float64 factors; all sums of penalties are float64.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "ibp_device.h"
#include "ibp_kernels.h"

namespace ibp {

// ---------------------------------------------------------------- helpers

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

template <typename T>
__device__ __forceinline__ T* ws_ptr(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

// ---------------------------------------------------------------- K1

__global__ __launch_bounds__(256) void k1_box_prep(DevNet net, const float* __restrict__ box_lo,
                                                   const float* __restrict__ box_hi, void* ws,
                                                   WsLayout lay, int64_t box0) {
  __shared__ double sh[4];
  const int64_t b = box0 + blockIdx.x;
  const int X = net.X, G = net.G;
  const float* lo = box_lo + b * X;
  const float* hi = box_hi + b * X;

  // surplus and total-injection sums over the inputs (float64; centre and
  // radius of float32 endpoints are exact in float64)
  double Sc = 0, Sr = 0, Sabs = 0, cI = 0, rI = 0, cIabs = 0, bad = 0;
  for (int j = threadIdx.x; j < X; j += 256) {
    const double l = lo[j], h = hi[j];
    if (!(l <= h) || !isfinite(l) || !isfinite(h)) bad = 1.0;
    const double c = 0.5 * (l + h), r = 0.5 * (h - l);
    const double w = net.dev_w[j];
    Sc += w * c;
    Sr += fabs(w) * r;
    Sabs += fabs(w * c) + fabs(w) * r;
    cI += (j < G) ? c : -c;
    rI += r;
    cIabs += fabs(c);
  }
  Sc = block_sum256(Sc, sh);
  Sr = block_sum256(Sr, sh);
  Sabs = block_sum256(Sabs, sh);
  cI = block_sum256(cI, sh);
  rI = block_sum256(rI, sh);
  cIabs = block_sum256(cIabs, sh);
  bad = block_sum256(bad, sh);

  // per-bus injection intervals, rounded outward to float32
  float* cinj = ws_ptr<float>(ws, lay.cinj) + b * net.Np;
  float* rpp = ws_ptr<float>(ws, lay.rpp) + b * net.Np;
  double Mc = 0, Mbox = 0, M2 = 0;
  for (int n = threadIdx.x; n < net.Np; n += 256) {
    if (n >= net.N) {
      cinj[n] = 0.0f;
      rpp[n] = 0.0f;
      continue;
    }
    double c = 0, r = 0, a = 0;
    int cnt = 0;
    for (int e = net.bus_ptr[n]; e < net.bus_ptr[n + 1]; ++e) {
      const int j = net.bus_dev[e];
      const double l = lo[j], h = hi[j];
      const double cj = 0.5 * (l + h), rj = 0.5 * (h - l);
      c += (j < G) ? cj : -cj;
      r += rj;
      a += fabs(cj);
      ++cnt;
    }
    // float64 summation error of c and r (cnt terms each)
    const double e64 = (cnt + 1) * kU64 * (a + r) * 1.01;
    const float c32 = (float)c;
    const float r32 = ru32((r + 2.0 * e64 + fabs(c - (double)c32)) * (1.0 + 4.0 * kU64));
    // radius inflated for the float32 rounding of the PTDF entries
    const float rp = ru32(((1.0 + kKappa0) * (double)r32 + kKappa0 * fabs((double)c32)) *
                          (1.0 + 4.0 * kU64));
    cinj[n] = c32;
    rpp[n] = rp;
    Mc += fabs((double)c32);
    Mbox += fabs((double)c32) + (double)r32;
    M2 += fabs((double)c32) + (double)rp;
  }
  Mc = block_sum256(Mc, sh);
  Mbox = block_sum256(Mbox, sh);
  M2 = block_sum256(M2, sh);

  // neutral padding lines for K3: zero centre, h = -FLT_MAX, g = +FLT_MAX
  float* lc = ws_ptr<float>(ws, lay.lc) + b * net.Lp;
  float* lh = ws_ptr<float>(ws, lay.lh) + b * net.Lp;
  float* lg = ws_ptr<float>(ws, lay.lg) + b * net.Lp;
  for (int l = net.L + threadIdx.x; l < net.Lp; l += 256) {
    lc[l] = 0.0f;
    lh[l] = -FLT_MAX;
    lg[l] = FLT_MAX;
  }

  if (threadIdx.x == 0) {
    double* bs = ws_ptr<double>(ws, lay.box) + b * kBoxSlots;
    // float64 reduction depth: X/256 serial terms plus the 8-level tree
    const double gam = (X / 256 + 12) * kU64 * 1.01;
    const double eS = gam * Sabs + 4.0 * kU64 * (fabs(Sc) + Sr);
    bs[kS_lo] = (Sc - Sr) - eS;
    bs[kS_hi] = (Sc + Sr) + eS;
    // 1^T s_inj interval: |sum p_inj| over the box (E^T Phi - I = -e_slack 1^T)
    const double eI = 2.0 * gam * (cIabs + rI);
    const double mag = (fabs(cI) + rI + eI) * (1.0 + 4.0 * kU64);
    const double mig = fabs(cI) - rI - eI;
    bs[kI_lo] = mig > 0.0 ? mig * (1.0 - 4.0 * kU64) : 0.0;
    bs[kI_hi] = mag;
    const double gN = (net.Np / 256 + 12) * kU64 * 1.01;
    bs[kMc] = Mc * (1.0 + gN);
    bs[kMbox] = Mbox * (1.0 + gN);
    // |c_f| + r_f <= sum |Phi| (|c| + r'') + pads <= M2 (1 + small) + phi_err_max Mbox
    bs[kM3] = (M2 * (1.0 + gN) * (1.0 + 1e-6) + 2.0 * net.phi_err_max * Mbox) * (1.0 + 1e-6);
    bs[kBad] = bad > 0.0 ? 1.0 : 0.0;
    bs[kVmax] = 0.0;  // K2 raises it with atomic max on the float bit pattern
  }
}

// ---------------------------------------------------------------- K2

// Per-line float64 epilogue: enclosing radius of the base flow, base penalties,
// and the per-line / per-outage constants of K3 (see the error model at K3).
__device__ __forceinline__ void k2_line_epilogue(const DevNet& net, int l, double cf, double rh,
                                                 double* bs, float* lc, float* lh, float* lg,
                                                 double* lcf, double* lrf, int4* ctg,
                                                 double& pb_hi, double& pb_lo) {
  const double Mc = bs[kMc], Mbox = bs[kMbox];
  const double gam = net.gamma64_n;
  // enclosing radius around the float64 centre cf: float64 accumulation of
  // |Phi32| r'' and Phi32 c32, and the float64 construction error of Phi
  const double rf = (rh * (1.0 + 2.0 * gam) + gam * Mc + net.phi_err[l] * Mbox) * (1.0 + 8.0 * kU64);
  const float cl = (float)cf;
  const double acl = fabs((double)cl);
  const double rl = rf + fabs(cf - (double)cl);
  lcf[l] = cf;
  lrf[l] = rf;

  // base overload penalty interval [max(|c|-r-fmax, 0), max(|c|+r-fmax, 0)]
  const double phib = net.fmax_b[l];
  const double a = fabs(cf);
  const double e = 4.0 * kU64 * (a + rf + phib);
  pb_hi += fmax(a + rf - phib + e, 0.0);
  pb_lo += fmax(a - rf - phib - e, 0.0);

  // K3 per-line constants
  const double phic = net.fmax_c[l];
  const double u1 = kU32 * (1.0 + kU32);
  const double dl = 2.0 * kU32 * (1.0 + kU32) * (1.0 + kU32);
  const double rho = rl + kU32 * acl;
  const double rhop = ((rho + dl * phic + u1 * acl) / (1.0 - dl)) * (1.0 + 16.0 * kU64) + 1e-36;
  lc[l] = cl;
  lh[l] = ru32(rhop - phic + 4.0 * kU64 * (rhop + phic));
  lg[l] = ru32((rhop + phic) * (1.0 + 4.0 * kU64));

  const int k = net.ctg_of_line[l];
  if (k >= 0) {
    const double Ek = net.ctg_eps[k] * (acl + rl);
    const double rk = (1.0 + kKappa0) * rl + (kKappa0 + kU32) * acl + Ek;
    const double rkp = ((rk + u1 * acl) / (1.0 - dl)) * (1.0 + 16.0 * kU64) + 1e-36;
    ctg[k] = make_int4(l, __float_as_int(cl), __float_as_int(ru32(rkp)), 0);
    const float v = ru32((acl + rl) * net.ctg_inv[k] * (1.0 + 4.0 * kU64));
    atomicMax(reinterpret_cast<unsigned int*>(bs + kVmax), __float_as_uint(v));
  }
}

template <int ROWS>
__global__ __launch_bounds__(256) void k2_base_flows(DevNet net, void* ws, WsLayout lay, int64_t box0) {
  const int64_t b = box0 + blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int gwave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * 4;
  const int n4 = net.Np / 4;
  const float4* cv = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.cinj) + b * net.Np);
  const float4* rv = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.rpp) + b * net.Np);
  double* bs = ws_ptr<double>(ws, lay.box) + b * kBoxSlots;
  float* lc = ws_ptr<float>(ws, lay.lc) + b * net.Lp;
  float* lh = ws_ptr<float>(ws, lay.lh) + b * net.Lp;
  float* lg = ws_ptr<float>(ws, lay.lg) + b * net.Lp;
  double* lcf = ws_ptr<double>(ws, lay.lcf) + b * net.L;
  double* lrf = ws_ptr<double>(ws, lay.lrf) + b * net.L;
  int4* ctg = ws_ptr<int4>(ws, lay.ctg) + b * net.K;

  double pb_hi = 0.0, pb_lo = 0.0;
  for (int r0 = gwave * ROWS; r0 < net.L; r0 += nwaves * ROWS) {
    double ac[ROWS], ar[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) ac[i] = ar[i] = 0.0;
    const float4* prow[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int row = min(r0 + i, net.L - 1);
      prow[i] = reinterpret_cast<const float4*>(net.phi + (size_t)row * net.Np);
    }
    for (int j = lane; j < n4; j += 64) {
      const float4 c4 = cv[j];
      const float4 r4 = rv[j];
      const double c0 = c4.x, c1 = c4.y, c2 = c4.z, c3 = c4.w;
      const double q0 = r4.x, q1 = r4.y, q2 = r4.z, q3 = r4.w;
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        const float4 p = prow[i][j];
        ac[i] = fma((double)p.x, c0, ac[i]);
        ac[i] = fma((double)p.y, c1, ac[i]);
        ac[i] = fma((double)p.z, c2, ac[i]);
        ac[i] = fma((double)p.w, c3, ac[i]);
        ar[i] = fma(fabs((double)p.x), q0, ar[i]);
        ar[i] = fma(fabs((double)p.y), q1, ar[i]);
        ar[i] = fma(fabs((double)p.z), q2, ar[i]);
        ar[i] = fma(fabs((double)p.w), q3, ar[i]);
      }
    }
    double cf = 0.0, rh = 0.0;
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const double s = wave_sum(ac[i]);
      const double t = wave_sum(ar[i]);
      if (lane == i) {
        cf = s;
        rh = t;
      }
    }
    if (lane < ROWS && r0 + lane < net.L)
      k2_line_epilogue(net, r0 + lane, cf, rh, bs, lc, lh, lg, lcf, lrf, ctg, pb_hi, pb_lo);
  }
  pb_hi = wave_sum(pb_hi);
  pb_lo = wave_sum(pb_lo);
  if (lane == 0) {
    double2* p2 = ws_ptr<double2>(ws, lay.p2) + b * lay.n_p2;
    p2[gwave] = make_double2(pb_hi, pb_lo);
  }
}

// ---------------------------------------------------------------- K3

// Error model (per element, float32 round-to-nearest, u = 2^-24):
//   C = fma(Lam, c_c, c_l),  A = fma(|Lam|, rho'_k, h_l),  B = fma(|Lam|, rho'_k, g_l)
//   t_hi = |C| + A,  t_lo = |C| - B
// with h_l >= rho'_l - fmax_l and g_l >= rho'_l + fmax_l.  With rho_l, rho_k
// the radii that enclose the exact interval around the computed C (line
// radii, the float32 storage error of Lam, the rounding of C) and
// delta = 2u (1 + u)^2,
//   rho'_l = (rho_l + delta fmax_l + u (1 + u) |c_l|) / (1 - delta),
//   rho'_k = (rho_k + u (1 + u) |c_c|) / (1 - delta)
// absorb the roundings of A, B, t_hi and t_lo, so t_hi >= |C*| + R* - fmax and
// t_lo <= |C*| - R* - fmax for the exact interval (C*, R*): max(t_hi, 0) and
// max(t_lo, 0) bound the exact penalties from above and below.  The float64
// construction error of the factors enters h_l and g_l once per tile
// (line_eps * Vmax).  The outaged line's own entry holds NaN, and
// max(NaN, 0) = 0 (IEEE maxNum), which removes it (the paper's mask M)
// without a branch.  Eight penalties are summed in float32 (three levels)
// before the float64 accumulation; K4 scales the totals by (1 +- 4u) for that.
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

template <int KC>
__global__ __launch_bounds__(256) void k3_contingency(DevNet net, void* ws, WsLayout lay, int64_t box0) {
  __shared__ double sh[8];
  const int64_t b = box0 + blockIdx.z;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int col = (blockIdx.x * 4 + w) * 64 + lane;  // float4 column
  const int Lp4 = net.Lp / 4;
  const int k0 = blockIdx.y * KC;
  const int k1 = min(net.K, k0 + KC);
  double acc_hi = 0.0, acc_lo = 0.0;
  if (col < Lp4) {
    const double* bs = ws_ptr<double>(ws, lay.box) + b * kBoxSlots;
    const float vmax = __uint_as_float(*reinterpret_cast<const unsigned int*>(bs + kVmax));
    const float4 c4 = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lc) + b * net.Lp)[col];
    float4 h4 = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lh) + b * net.Lp)[col];
    float4 g4 = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lg) + b * net.Lp)[col];
    const float4 e4 = reinterpret_cast<const float4*>(net.line_eps)[col];
    {
      const float ex = next_up_f32(e4.x * vmax), ey = next_up_f32(e4.y * vmax);
      const float ez = next_up_f32(e4.z * vmax), ew = next_up_f32(e4.w * vmax);
      h4 = make_float4(add_ru(h4.x, ex), add_ru(h4.y, ey), add_ru(h4.z, ez), add_ru(h4.w, ew));
      g4 = make_float4(add_ru(g4.x, ex), add_ru(g4.y, ey), add_ru(g4.z, ez), add_ru(g4.w, ew));
    }
    const int4* cd = ws_ptr<int4>(ws, lay.ctg) + b * net.K;
    const float4* lam = reinterpret_cast<const float4*>(net.lodf) + col;
    int k = k0;
    for (; k + 8 <= k1; k += 8) {
      float4 x[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = lam[(size_t)(k + i) * Lp4];
#pragma unroll
      for (int i = 0; i < 8; i += 2) k3_pair(x[i], cd[k + i], x[i + 1], cd[k + i + 1], c4, h4, g4, acc_hi, acc_lo);
    }
    for (; k + 2 <= k1; k += 2)
      k3_pair(lam[(size_t)k * Lp4], cd[k], lam[(size_t)(k + 1) * Lp4], cd[k + 1], c4, h4, g4, acc_hi, acc_lo);
    if (k < k1) {  // odd tail
      float a0, a1, a2, a3, b0, b1, b2, b3;
      const float4 x0 = lam[(size_t)k * Lp4];
      const int4 d0 = cd[k];
      const float cc0 = __int_as_float(d0.y), rk0 = __int_as_float(d0.z);
      k3_elem(x0.x, cc0, rk0, c4.x, h4.x, g4.x, a0, b0);
      k3_elem(x0.y, cc0, rk0, c4.y, h4.y, g4.y, a1, b1);
      k3_elem(x0.z, cc0, rk0, c4.z, h4.z, g4.z, a2, b2);
      k3_elem(x0.w, cc0, rk0, c4.w, h4.w, g4.w, a3, b3);
      acc_hi += (double)((a0 + a1) + (a2 + a3));
      acc_lo += (double)((b0 + b1) + (b2 + b3));
    }
  }
  acc_hi = wave_sum(acc_hi);
  acc_lo = wave_sum(acc_lo);
  if (lane == 0) {
    sh[w] = acc_hi;
    sh[4 + w] = acc_lo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double2* p3 = ws_ptr<double2>(ws, lay.p3) + b * lay.n_p3;
    p3[blockIdx.y * gridDim.x + blockIdx.x] =
        make_double2((sh[0] + sh[1]) + (sh[2] + sh[3]), (sh[4] + sh[5]) + (sh[6] + sh[7]));
  }
}

// ---------------------------------------------------------------- K4

__global__ __launch_bounds__(256) void k4_finalize(DevNet net, void* ws, WsLayout lay, int64_t box0,
                                                   double* __restrict__ f_lo,
                                                   double* __restrict__ f_hi,
                                                   double* __restrict__ terms) {
  __shared__ double sh[4];
  const int64_t b = box0 + blockIdx.x;
  const double2* p2 = ws_ptr<double2>(ws, lay.p2) + b * lay.n_p2;
  const double2* p3 = ws_ptr<double2>(ws, lay.p3) + b * lay.n_p3;
  double bh = 0, bl = 0, ch = 0, cl = 0;
  for (int i = threadIdx.x; i < lay.n_p2; i += 256) {
    bh += p2[i].x;
    bl += p2[i].y;
  }
  for (int i = threadIdx.x; i < lay.n_p3; i += 256) {
    ch += p3[i].x;
    cl += p3[i].y;
  }
  bh = block_sum256(bh, sh);
  bl = block_sum256(bl, sh);
  ch = block_sum256(ch, sh);
  cl = block_sum256(cl, sh);
  if (threadIdx.x != 0) return;
  const double* bs = ws_ptr<double>(ws, lay.box) + b * kBoxSlots;
  // float64 accumulation depth is far below L + K + 4096 additions per term
  const double gF = (double)(net.L + net.K + 4096) * kU64;
  const double Fb_hi = bh * (1.0 + gF), Fb_lo = bl * (1.0 - gF);
  const double Fc_hi = ch * (1.0 + 4.0 * kU32) * (1.0 + gF);
  const double Fc_lo = cl * (1.0 - 4.0 * kU32) * (1.0 - gF);
  const double zi = net.zeta_inj, zf = net.zeta_f;
  const double S_lo = bs[kS_lo], S_hi = bs[kS_hi], I_lo = bs[kI_lo], I_hi = bs[kI_hi];
  double hi = S_hi - zi * I_lo - zf * (Fb_lo + Fc_lo);
  hi += 8.0 * kU64 * (fabs(S_hi) + zi * I_lo + zf * (Fb_lo + Fc_lo));
  double lo = S_lo - zi * I_hi - zf * (Fb_hi + Fc_hi);
  lo -= 8.0 * kU64 * (fabs(S_lo) + zi * I_hi + zf * (Fb_hi + Fc_hi));
  if (bs[kBad] != 0.0) {
    lo = hi = NAN;
  }
  f_lo[b] = lo;
  f_hi[b] = hi;
  if (terms) {
    double* t = terms + b * 8;
    const bool bad = bs[kBad] != 0.0;
    t[0] = bad ? NAN : S_lo;
    t[1] = bad ? NAN : S_hi;
    t[2] = bad ? NAN : I_lo;
    t[3] = bad ? NAN : I_hi;
    t[4] = bad ? NAN : Fb_lo;
    t[5] = bad ? NAN : Fb_hi;
    t[6] = bad ? NAN : Fc_lo;
    t[7] = bad ? NAN : Fc_hi;
  }
}

// ---------------------------------------------------------------- launchers

constexpr int kK2Rows = 4;
constexpr int kK3Kc = 32;

void plan_single(const DevNet& net, int64_t n_box, WsLayout& lay, int num_cus) {
  // K2: grid-stride over groups of kK2Rows rows, a few waves per SIMD
  const int groups = (net.L + kK2Rows - 1) / kK2Rows;
  const int want_waves = num_cus * 4 * 4;
  lay.k2_blocks = std::max(1, std::min((groups + 3) / 4, want_waves / 4));
  lay.n_p2 = lay.k2_blocks * 4;
  // K3: 4 waves x 256 lines per block, kK3Kc outages per block
  const int lp4 = net.Lp / 4;
  lay.k3_bx = (lp4 + 255) / 256;
  lay.k3_by = std::max(1, (net.K + kK3Kc - 1) / kK3Kc);
  lay.n_p3 = lay.k3_bx * lay.k3_by;
  (void)n_box;
}

hipError_t launch_forward_single(const DevNet& net, int64_t n_box, const float* lo, const float* hi,
                                 double* f_lo, double* f_hi, double* terms, void* ws,
                                 const WsLayout& lay, hipStream_t s, KernelTimer* tm) {
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    int t = tm->start(0, s);
    hipLaunchKernelGGL(k1_box_prep, dim3(nb), dim3(256), 0, s, net, lo, hi, ws, lay, b0);
    tm->stop(t, s);
    t = tm->start(1, s);
    hipLaunchKernelGGL(k2_base_flows<kK2Rows>, dim3(lay.k2_blocks, nb), dim3(256), 0, s, net, ws, lay, b0);
    tm->stop(t, s);
    if (net.K > 0) {
      t = tm->start(2, s);
      hipLaunchKernelGGL(k3_contingency<kK3Kc>, dim3(lay.k3_bx, lay.k3_by, nb), dim3(256), 0, s, net, ws,
                         lay, b0);
      tm->stop(t, s);
    }
    t = tm->start(3, s);
    hipLaunchKernelGGL(k4_finalize, dim3(nb), dim3(256), 0, s, net, ws, lay, b0, f_lo, f_hi, terms);
    tm->stop(t, s);
  }
  return hipGetLastError();
}

}  // namespace ibp
