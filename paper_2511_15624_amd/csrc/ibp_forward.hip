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
#include "ibp_devfun.h"
#include "ibp_kernels.h"

namespace ibp {

// ---------------------------------------------------------------- K1

// Injection interval of bus n, p_inj = N_g p_g - N_d p_d, in float64:
// out = (c, r''), where r'' covers the summation error of c and r and the
// float32 storage error of the PTDF entries it will multiply; mc = |c|,
// mbox = |c| + r'.  The centre stays in float64 (the base-flow sweeps multiply
// it in float64), so no float32 rounding of it enters the radius.  The
// endpoints of the bus's first four devices are loaded together; further
// devices (rare) follow in a loop.  Terms are added in device order.
__device__ __forceinline__ void bus_injection(const DevNet& net, const float* __restrict__ lo,
                                              const float* __restrict__ hi, int n, double2& out, double& mc,
                                              double& mbox) {
  const int4 d4 = net.bus_dev4[n];
  const int e0 = net.bus_ptr[n], e1 = net.bus_ptr[n + 1];
  const int js[4] = {d4.x, d4.y, d4.z, d4.w};
  float l4[4], h4[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = max(js[q], 0);
    l4[q] = lo[j];
    h4[q] = hi[j];
  }
  double c = 0, r = 0, a = 0;
  int cnt = 0;
  auto add = [&](int j, double l, double h) {
    const double cj = 0.5 * (l + h), rj = 0.5 * (h - l);
    c += (j < net.G) ? cj : -cj;
    r += rj;
    a += fabs(cj);
    ++cnt;
  };
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (js[q] >= 0) add(js[q], l4[q], h4[q]);
  for (int e = e0 + 4; e < e1; ++e) {
    const int j = net.bus_dev[e];
    add(j, lo[j], hi[j]);
  }
  // float64 summation error of c and r (cnt terms each): the computed centre
  // is off by at most e64, so the radius grows by 2 e64 (and by 4 u64 for the
  // roundings of these additions)
  const double e64 = (cnt + 1) * kU64 * (a + r) * 1.01;
  const double r1 = (r + 2.0 * e64) * (1.0 + 4.0 * kU64);
  // radius inflated for the float32 rounding of the PTDF entries
  const double rp = ((1.0 + kKappa0) * r1 + kKappa0 * fabs(c)) * (1.0 + 4.0 * kU64);
  out = make_double2(c, rp);
  mc = fabs(c);
  mbox = fabs(c) + r1;
}

// Per-input terms of the box-preparation sums: surplus (linear part and
// curves), total injection, validity.  Centre and radius of float32 endpoints
// are exact in float64.
__device__ __forceinline__ void input_terms(const DevNet& net, int i, double l, double h, double w,
                                            double (&v)[kP1Fields]) {
  if (!(l <= h) || !isfinite(l) || !isfinite(h)) v[kP1Bad] += 1.0;
  const double c = 0.5 * (l + h), r = 0.5 * (h - l);
  v[kP1Sc] += w * c;
  v[kP1Sr] += fabs(w) * r;
  v[kP1Sabs] += fabs(w * c) + fabs(w) * r;
  v[kP1cI] += (i < net.G) ? c : -c;
  v[kP1rI] += r;
  v[kP1cIabs] += fabs(c);
  if (net.seg_ptr) {
    // curve term: loads add [F_lo, F_hi], generators subtract it
    const int s0 = net.seg_ptr[i], s1 = net.seg_ptr[i + 1];
    if (s1 > s0) {
      double F_lo, F_hi, e;
      curve_ibp(net.seg, s0, s1, c, r, F_lo, F_hi, e);
      const double sc = (i < net.G ? -0.5 : 0.5) * (F_lo + F_hi);
      const double sr = 0.5 * (F_hi - F_lo) + e + 1.01 * kU64 * (fabs(F_lo) + fabs(F_hi));
      v[kP1Sc] += sc;
      v[kP1Sr] += sr;
      v[kP1Sabs] += fabs(sc) + sr;
    }
  }
}

// Neutral padding lines for K3 (zero centre, h = -FLT_MAX, g = +FLT_MAX) and
// the box's Vmax slot cleared; run by one block per box.
__device__ __forceinline__ void box_slots_init(const DevNet& net, void* ws, const WsLayout& lay, int64_t b) {
  float* lc = ws_ptr<float>(ws, lay.lc) + b * net.Lp;
  float* lh = ws_ptr<float>(ws, lay.lh) + b * net.Lp;
  float* lg = ws_ptr<float>(ws, lay.lg) + b * net.Lp;
  for (int l = net.L + (int)threadIdx.x; l < net.Lp; l += blockDim.x) {
    lc[l] = 0.0f;
    lh[l] = -FLT_MAX;
    lg[l] = FLT_MAX;
  }
  if (threadIdx.x == 0) ws_ptr<double>(ws, lay.box)[b * kBoxSlots + kVmax] = 0.0;
}

// One wave per 64 buses / 64 inputs of a box (the box-tiled path): injection
// intervals to the workspace and partial float64 sums for the surplus, the
// total injection and the padding constants.
__global__ __launch_bounds__(64) void k1_box_prep(DevNet net, const float* __restrict__ box_lo,
                                                  const float* __restrict__ box_hi, void* ws,
                                                  WsLayout lay, int64_t box0) {
  const int64_t b = box0 + blockIdx.y;
  const int i = blockIdx.x * 64 + threadIdx.x;
  const float* lo = box_lo + b * net.X;
  const float* hi = box_hi + b * net.X;
  double v[kP1Fields];
#pragma unroll
  for (int f = 0; f < kP1Fields; ++f) v[f] = 0.0;
  // this lane's input, loaded before the bus's dependent loads start
  const int ix = min(i, net.X - 1);
  const double li = lo[ix], hi_i = hi[ix], wi = net.dev_w[ix];
  double2 cr = make_double2(0.0, 0.0);
  if (i < net.N) bus_injection(net, lo, hi, i, cr, v[kP1Mc], v[kP1Mbox]);
  if (i < net.X) input_terms(net, i, li, hi_i, wi, v);
  if (i < net.Np) ws_ptr<double2>(ws, lay.inj)[b * net.Np + i] = cr;
#pragma unroll
  for (int f = 0; f < kP1Fields; ++f) v[f] = wave_sum(v[f]);
  if (threadIdx.x < kP1Fields) {
    double* rec = ws_ptr<double>(ws, lay.p1) + (b * lay.n_p1 + blockIdx.x) * kP1Fields;
    double val = 0.0;
#pragma unroll
    for (int f = 0; f < kP1Fields; ++f)
      if (threadIdx.x == f) val = v[f];
    rec[threadIdx.x] = val;
  }
  if (blockIdx.x == 0) box_slots_init(net, ws, lay, b);
}

// ---------------------------------------------------------------- K2

// Per-line data of the epilogue, loaded together before any of it is used.
struct LineConst {
  double phi_err, fmax_b, fmax_c;
  double2 ctg;  // (ctg_eps, ctg_inv) of the line's outage
  int k;        // outage index or -1
};

__device__ __forceinline__ LineConst load_line_const(const DevNet& net, int l) {
  return LineConst{net.phi_err[l], net.fmax_b[l], net.fmax_c[l], net.line_ctg[l], net.ctg_of_line[l]};
}

// Per-line float64 epilogue: enclosing radius of the base flow, base penalties,
// and the per-line / per-outage constants of K3 (see the error model at K3).
// Returns the float bits of (|c_c| + r_c) / (1 - H_cc) rounded up if the line
// is an outage line (0 otherwise), for the caller's max reduction.
__device__ __forceinline__ unsigned line_epilogue(const DevNet& net, int l, const LineConst& q, double cf,
                                                  double rh, double Mc, double Mbox, float* lc, float* lh,
                                                  float* lg, double* lcf, double* lrf, int4* ctg, float2* cb,
                                                  double& pb_hi, double& pb_lo) {
  const double gam = net.gamma64_n;
  // enclosing radius around the float64 centre cf: float64 accumulation of
  // |Phi32| r'' and Phi32 c, and the float64 construction error of Phi
  const double rf = (rh * (1.0 + 2.0 * gam) + gam * Mc + q.phi_err * Mbox) * (1.0 + 8.0 * kU64);
  const float cl = (float)cf;
  const double acl = fabs((double)cl);
  const double rl = rf + fabs(cf - (double)cl);
  lcf[l] = cf;
  lrf[l] = rf;

  // base overload penalty interval [max(|c|-r-fmax, 0), max(|c|+r-fmax, 0)]
  const double phib = q.fmax_b;
  const double a = fabs(cf);
  const double e = 4.0 * kU64 * (a + rf + phib);
  pb_hi += fmax(a + rf - phib + e, 0.0);
  pb_lo += fmax(a - rf - phib - e, 0.0);

  // K3 per-line constants
  const double phic = q.fmax_c;
  constexpr double u1 = kU32 * (1.0 + kU32);
  constexpr double dl = 2.0 * kU32 * (1.0 + kU32) * (1.0 + kU32);
  constexpr double inv1md = 1.0 / (1.0 - dl);  // the 16 u64 factor covers its rounding
  const double rho = rl + kU32 * acl;
  const double rhop = ((rho + dl * phic + u1 * acl) * inv1md) * (1.0 + 16.0 * kU64) + 1e-36;
  lc[l] = cl;
  lh[l] = ru32(rhop - phic + 4.0 * kU64 * (rhop + phic));
  lg[l] = ru32((rhop + phic) * (1.0 + 4.0 * kU64));

  if (q.k >= 0) {
    const double Ek = q.ctg.x * (acl + rl);
    const double rk = (1.0 + kKappa0) * rl + (kKappa0 + kU32) * acl + Ek;
    const double rkp = ((rk + u1 * acl) * inv1md) * (1.0 + 16.0 * kU64) + 1e-36;
    // fourth field: the unpadded radius, read by the backward sweep
    ctg[q.k] = make_int4(l, __float_as_int(cl), __float_as_int(ru32(rkp)), __float_as_int((float)rf));
    // the box-tiled backward sweep reads (centre, unpadded radius) of four
    // outages as two 16-byte scalar loads
    if (cb) cb[q.k] = make_float2(cl, (float)rf);
    const float v = ru32((acl + rl) * q.ctg.y * (1.0 + 4.0 * kU64));
    return __float_as_uint(v);
  }
  return 0u;
}

constexpr int kK2eThreads = 256;
constexpr int kK2eBy = 16;  // base-flow partials per line loaded in one round

// One line per lane, kK2eThreads lines per block: combine the K2 partials of
// every bus chunk and run the line epilogue; one base-penalty partial per wave
// (64 lines) and one max-reduction atomic per block.  Every load that does
// not depend on another is issued before the first use (the line index is
// clamped; partials that do not exist are skipped by wave-uniform or lane
// masks, not loaded twice), so the kernel waits on memory about twice
// instead of once per dependent step.
__global__ __launch_bounds__(kK2eThreads) void k2e_lines(DevNet net, void* ws, WsLayout lay, int64_t box0) {
  const int64_t b = box0 + blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int l = blockIdx.x * kK2eThreads + threadIdx.x;
  const int lq = min(l, net.L - 1);
  const double* p1 = ws_ptr<double>(ws, lay.p1) + b * lay.n_p1 * kP1Fields;
  const double2* part = ws_ptr<double2>(ws, lay.part2) + (size_t)b * lay.k2_by * net.Lp + lq;
  const int nby = lay.k2_by;

  // every wave sums all box-preparation partials of Mc and Mbox itself
  double mc = 0.0, mb = 0.0;
  double2 t[kK2eBy];
  LineConst q;
  {
    double xm[4], xb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = lane + 64 * u;
      xm[u] = xb[u] = 0.0;
      if (j < lay.n_p1) {
        xm[u] = p1[j * kP1Fields + kP1Mc];
        xb[u] = p1[j * kP1Fields + kP1Mbox];
      }
    }
#pragma unroll
    for (int y = 0; y < kK2eBy; ++y)
      if (y < nby) t[y] = part[(size_t)y * net.Lp];
    q = load_line_const(net, lq);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      mc += xm[u];
      mb += xb[u];
    }
  }
  for (int j = lane + 256; j < lay.n_p1; j += 64) {
    mc += p1[j * kP1Fields + kP1Mc];
    mb += p1[j * kP1Fields + kP1Mbox];
  }
  double cf[4] = {0, 0, 0, 0}, rh[4] = {0, 0, 0, 0};
#pragma unroll
  for (int y = 0; y < kK2eBy; ++y)
    if (y < nby) {
      cf[y & 3] += t[y].x;
      rh[y & 3] += t[y].y;
    }
  for (int y = kK2eBy; y < nby; ++y) {
    const double2 u = part[(size_t)y * net.Lp];
    cf[y & 3] += u.x;
    rh[y & 3] += u.y;
  }
  const double g = (lay.n_p1 + 16) * kU64 * 1.01;
  mc = wave_sum(mc) * (1.0 + g);
  mb = wave_sum(mb) * (1.0 + g);
  double pb_hi = 0.0, pb_lo = 0.0;
  unsigned vm = 0u;
  if (l < net.L)
    vm = line_epilogue(net, l, q, (cf[0] + cf[1]) + (cf[2] + cf[3]), (rh[0] + rh[1]) + (rh[2] + rh[3]), mc, mb,
                       ws_ptr<float>(ws, lay.lc) + b * net.Lp, ws_ptr<float>(ws, lay.lh) + b * net.Lp,
                       ws_ptr<float>(ws, lay.lg) + b * net.Lp, ws_ptr<double>(ws, lay.lcf) + b * net.L,
                       ws_ptr<double>(ws, lay.lrf) + b * net.L, ws_ptr<int4>(ws, lay.ctg) + b * net.K,
                       lay.cb ? ws_ptr<float2>(ws, lay.cb) + b * net.K : nullptr, pb_hi, pb_lo);
  // max over the wave (non-negative floats order like their bit patterns)
  vm = wave_max_u32(vm);
  pb_hi = wave_sum(pb_hi);
  pb_lo = wave_sum(pb_lo);
  // one atomic per block: same-address atomics from every wave queue up
  const int wi = blockIdx.x * (kK2eThreads / 64) + w;
  __shared__ unsigned svm[kK2eThreads / 64];
  if (lane == 0) svm[w] = vm;
  if (lane == 0 && wi < lay.n_p2) ws_ptr<double2>(ws, lay.p2)[b * lay.n_p2 + wi] = make_double2(pb_hi, pb_lo);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned m = 0u;
#pragma unroll
    for (int q = 0; q < kK2eThreads / 64; ++q) m = max(m, svm[q]);
    if (m != 0u)
      atomicMax(reinterpret_cast<unsigned int*>(ws_ptr<double>(ws, lay.box) + b * kBoxSlots + kVmax), m);
  }
}

// Base flows c_f = Phi c and rho = |Phi| r'' in float64, streaming the
// transposed PTDF: each lane owns four lines, each wave a chunk of NC buses
// whose (c, r'') it reads as wave-uniform scalars.  The four waves of a block
// share the line tile; their sums are combined in LDS and written as one
// partial per block row (bus chunk).
template <int NC>
__global__ __launch_bounds__(256) void k2_base_flows(DevNet net, void* ws, WsLayout lay, int64_t box0,
                                                     const double2* __restrict__ inj_all) {
  __shared__ double sh[3][64][8];
  const int64_t b = box0 + blockIdx.z;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int col = blockIdx.x * 64 + lane;  // float4 column
  const int Lp4 = net.Lp / 4;
  const int n0 = (blockIdx.y * 4 + w) * NC;
  const int n1 = min(net.N, n0 + NC);
  double ac0 = 0, ac1 = 0, ac2 = 0, ac3 = 0, ar0 = 0, ar1 = 0, ar2 = 0, ar3 = 0;
  if (col < Lp4) {
    const double2* __restrict__ inj = inj_all + b * net.Np;
    const float4* ph = reinterpret_cast<const float4*>(net.phiT) + col;
    int n = n0;
    for (; n + 8 <= n1; n += 8) {
      float4 x[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = ld_stream(ph + (size_t)(n + i) * Lp4);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double2 cr = inj[n + i];
        ac0 = fma((double)x[i].x, cr.x, ac0);
        ac1 = fma((double)x[i].y, cr.x, ac1);
        ac2 = fma((double)x[i].z, cr.x, ac2);
        ac3 = fma((double)x[i].w, cr.x, ac3);
        ar0 = fma(fabs((double)x[i].x), cr.y, ar0);
        ar1 = fma(fabs((double)x[i].y), cr.y, ar1);
        ar2 = fma(fabs((double)x[i].z), cr.y, ar2);
        ar3 = fma(fabs((double)x[i].w), cr.y, ar3);
      }
    }
    for (; n < n1; ++n) {
      const float4 x = ld_stream(ph + (size_t)n * Lp4);
      const double2 cr = inj[n];
      ac0 = fma((double)x.x, cr.x, ac0);
      ac1 = fma((double)x.y, cr.x, ac1);
      ac2 = fma((double)x.z, cr.x, ac2);
      ac3 = fma((double)x.w, cr.x, ac3);
      ar0 = fma(fabs((double)x.x), cr.y, ar0);
      ar1 = fma(fabs((double)x.y), cr.y, ar1);
      ar2 = fma(fabs((double)x.z), cr.y, ar2);
      ar3 = fma(fabs((double)x.w), cr.y, ar3);
    }
  }
  if (w > 0) {
    double* d = sh[w - 1][lane];
    d[0] = ac0; d[1] = ac1; d[2] = ac2; d[3] = ac3;
    d[4] = ar0; d[5] = ar1; d[6] = ar2; d[7] = ar3;
  }
  __syncthreads();
  if (w == 0 && col < Lp4) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double* d = sh[q][lane];
      ac0 += d[0]; ac1 += d[1]; ac2 += d[2]; ac3 += d[3];
      ar0 += d[4]; ar1 += d[5]; ar2 += d[6]; ar3 += d[7];
    }
    double2* out = ws_ptr<double2>(ws, lay.part2) + ((size_t)b * lay.k2_by + blockIdx.y) * net.Lp + 4 * col;
    out[0] = make_double2(ac0, ar0);
    out[1] = make_double2(ac1, ar1);
    out[2] = make_double2(ac2, ar2);
    out[3] = make_double2(ac3, ar3);
  }
}

// ---------------------------------------------------------------- K4

__device__ __forceinline__ void objective_interval(const DevNet& net, const WsLayout& lay, int64_t b,
                                                   const double (&x)[12], double* __restrict__ f_lo,
                                                   double* __restrict__ f_hi, double* __restrict__ terms);

// Objective interval of one box from all partial sums, run by one block of T
// threads after every partial is visible.  The first T partials of each kind
// are loaded in one group (clamped indices, masked adds); loops take the rest.
template <int T>
__device__ void finalize_box(const DevNet& net, void* ws, const WsLayout& lay, int64_t b,
                             double* __restrict__ f_lo, double* __restrict__ f_hi,
                             double* __restrict__ terms) {
  const double* p1 = ws_ptr<double>(ws, lay.p1) + b * lay.n_p1 * kP1Fields;
  const double2* p2 = ws_ptr<double2>(ws, lay.p2) + b * lay.n_p2;
  const double2* p3 = ws_ptr<double2>(ws, lay.p3) + b * lay.n_p3;
  constexpr int kQ3 = 32;  // outage-sweep partials per thread in the first group
  const int tid = threadIdx.x;
  double v[kP1Fields];
  double bh = 0, bl = 0;
  double ch[4] = {0, 0, 0, 0}, cl[4] = {0, 0, 0, 0};
  {
    const int j1 = min(tid, lay.n_p1 - 1);
    double x1[kP1Fields];
#pragma unroll
    for (int f = kP1Sc; f < kP1Fields; ++f) x1[f] = p1[j1 * kP1Fields + f];
    const double2 x2 = p2[min(tid, lay.n_p2 - 1)];
    double2 x3[kQ3];
    const int n3 = lay.n_p3;
#pragma unroll
    for (int q = 0; q < kQ3; ++q) x3[q] = p3[max(0, min(tid + q * T, n3 - 1))];
#pragma unroll
    for (int f = 0; f < kP1Fields; ++f) v[f] = (f >= kP1Sc && tid < lay.n_p1) ? x1[f] : 0.0;
    if (tid < lay.n_p2) {
      bh = x2.x;
      bl = x2.y;
    }
#pragma unroll
    for (int q = 0; q < kQ3; ++q)
      if (tid + q * T < n3) {
        ch[q & 3] += x3[q].x;
        cl[q & 3] += x3[q].y;
      }
  }
  for (int j = tid + T; j < lay.n_p1; j += T)
#pragma unroll
    for (int f = kP1Sc; f < kP1Fields; ++f) v[f] += p1[j * kP1Fields + f];
  for (int i = tid + T; i < lay.n_p2; i += T) {
    const double2 x = p2[i];
    bh += x.x;
    bl += x.y;
  }
  for (int i = tid + kQ3 * T; i < lay.n_p3; i += T) {
    const double2 x = p3[i];
    ch[0] += x.x;
    cl[0] += x.y;
  }
  // one combined block reduction of the 12 running sums
  constexpr int W = T / 64;
  __shared__ double red[W][12];
  double x[12];
#pragma unroll
  for (int f = 0; f < 8; ++f) x[f] = v[kP1Sc + f];
  x[8] = bh;
  x[9] = bl;
  x[10] = (ch[0] + ch[1]) + (ch[2] + ch[3]);
  x[11] = (cl[0] + cl[1]) + (cl[2] + cl[3]);
#pragma unroll
  for (int f = 0; f < 12; ++f) x[f] = wave_sum(x[f]);
  if ((tid & 63) == 0)
#pragma unroll
    for (int f = 0; f < 12; ++f) red[tid >> 6][f] = x[f];
  __syncthreads();
  __shared__ double tot[12];
  if (tid < 12) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < W; ++q) t += red[q][tid];
    tot[tid] = t;
  }
  __syncthreads();
  if (tid != 0) return;
#pragma unroll
  for (int f = 0; f < 12; ++f) x[f] = tot[f];
  objective_interval(net, lay, b, x, f_lo, f_hi, terms);
}

// Objective interval of box b from its summed terms: x[0..7] the box-
// preparation fields from kP1Sc on (surplus centre, radius and magnitude,
// total injection centre, radius and magnitude, invalid count), x[8], x[9]
// the base penalties (hi, lo), x[10], x[11] the outage penalties (hi, lo).
__device__ __forceinline__ void objective_interval(const DevNet& net, const WsLayout& lay, int64_t b,
                                                   const double (&x)[12], double* __restrict__ f_lo,
                                                   double* __restrict__ f_hi, double* __restrict__ terms) {
  double v[kP1Fields];
#pragma unroll
  for (int f = 0; f < 8; ++f) v[kP1Sc + f] = x[f];
  const double bh = x[8];
  const double bl = x[9];
  // one-sided calls: the side not computed is bounded trivially (upper bound
  // of the outage penalties +inf, lower bound 0)
  const double chs = lay.sides == 1 ? INFINITY : x[10];
  const double cls = lay.sides == 2 ? 0.0 : x[11];

  // surplus and imbalance intervals; float64 reduction depth <= n_p1 + 16
  const double gam = (lay.n_p1 + 16) * kU64 * 1.01;
  const double Sc = v[kP1Sc], Sr = v[kP1Sr];
  const double eS = gam * v[kP1Sabs] + 4.0 * kU64 * (fabs(Sc) + Sr);
  const double S_lo = (Sc - Sr) - eS, S_hi = (Sc + Sr) + eS;
  // 1^T s_inj = |sum p_inj| since E^T Phi - I = -e_slack 1^T
  const double cI = v[kP1cI], rI = v[kP1rI];
  const double eI = 2.0 * gam * (v[kP1cIabs] + rI);
  const double I_hi = (fabs(cI) + rI + eI) * (1.0 + 4.0 * kU64);
  const double mig = fabs(cI) - rI - eI;
  const double I_lo = mig > 0.0 ? mig * (1.0 - 4.0 * kU64) : 0.0;

  // float64 accumulation depth is far below L + K + 4096 additions per term
  const double gF = (double)(net.L + net.K + 4096) * kU64;
  const double Fb_hi = bh * (1.0 + gF), Fb_lo = bl * (1.0 - gF);
  const double Fc_hi = chs * (1.0 + 4.0 * kU32) * (1.0 + gF);
  const double Fc_lo = cls * (1.0 - 4.0 * kU32) * (1.0 - gF);
  const double zi = net.zeta_inj, zf = net.zeta_f;
  double hi = S_hi - zi * I_lo - zf * (Fb_lo + Fc_lo);
  hi += 8.0 * kU64 * (fabs(S_hi) + zi * I_lo + zf * (Fb_lo + Fc_lo));
  double lo = S_lo - zi * I_hi - zf * (Fb_hi + Fc_hi);
  lo -= 8.0 * kU64 * (fabs(S_lo) + zi * I_hi + zf * (Fb_hi + Fc_hi));
  const bool bad = v[kP1Bad] != 0.0;
  if (bad) lo = hi = NAN;
  f_lo[b] = lo;
  f_hi[b] = hi;
  if (terms) {
    double* t = terms + b * 8;
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

// One block of T threads per box.
template <int T>
__global__ __launch_bounds__(T) void k4_finalize(DevNet net, void* ws, WsLayout lay, int64_t box0,
                                                 double* __restrict__ f_lo, double* __restrict__ f_hi,
                                                 double* __restrict__ terms) {
  finalize_box<T>(net, ws, lay, box0 + blockIdx.x, f_lo, f_hi, terms);
}

static void launch_k4(const DevNet& net, void* ws, const WsLayout& lay, int64_t b0, int nb, double* f_lo,
                      double* f_hi, double* terms, hipStream_t s) {
  hipLaunchKernelGGL(k4_finalize<256>, dim3(nb), dim3(256), 0, s, net, ws, lay, b0, f_lo, f_hi, terms);
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
// The outage sweep of one block: four waves x 256 lines (float4 column `col`
// of each lane) x outages [k0, k1) of box b, with the construction-error
// padding of the box's vmax; returns the block's penalty sums (hi, lo) in
// thread 0.
template <int KC>
__device__ __forceinline__ double2 k3_block(const DevNet& net, void* ws, const WsLayout& lay, int64_t b, int col,
                                            int k0, int k1, float vmax) {
  __shared__ double sh[8];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int Lp4 = net.Lp / 4;
  double acc_hi = 0.0, acc_lo = 0.0;
  if (col < Lp4) {
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
      for (int i = 0; i < 8; ++i) x[i] = ld_stream(lam + (size_t)(k + i) * Lp4);
#pragma unroll
      for (int i = 0; i < 8; i += 2) k3_pair(x[i], cd[k + i], x[i + 1], cd[k + i + 1], c4, h4, g4, acc_hi, acc_lo);
    }
    for (; k + 2 <= k1; k += 2)
      k3_pair(ld_stream(lam + (size_t)k * Lp4), cd[k], ld_stream(lam + (size_t)(k + 1) * Lp4), cd[k + 1], c4, h4,
              g4, acc_hi, acc_lo);
    if (k < k1) {  // odd tail
      float a0, a1, a2, a3, b0, b1, b2, b3;
      const float4 x0 = ld_stream(lam + (size_t)k * Lp4);
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
  return make_double2((sh[0] + sh[1]) + (sh[2] + sh[3]), (sh[4] + sh[5]) + (sh[6] + sh[7]));
}

template <int KC>
__global__ __launch_bounds__(256) void k3_contingency(DevNet net, void* ws, WsLayout lay, int64_t box0) {
  const int64_t b = box0 + blockIdx.z;
  const int col = (blockIdx.x * 4 + (int)(threadIdx.x >> 6)) * 64 + (int)(threadIdx.x & 63);  // float4 column
  const double* bs = ws_ptr<double>(ws, lay.box) + b * kBoxSlots;
  const float vmax = __uint_as_float(*reinterpret_cast<const unsigned int*>(bs + kVmax));
  const int k0 = blockIdx.y * KC;
  const double2 t = k3_block<KC>(net, ws, lay, b, col, k0, min(net.K, k0 + KC), vmax);
  if (threadIdx.x == 0) ws_ptr<double2>(ws, lay.p3)[b * lay.n_p3 + blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// ---------------------------------------------------------------- small networks

// One block per box for the smallest networks (at most kMicroBuses buses,
// kMicroLines lines and kMicroElems outage elements).  A dispatch costs about
// 2.4 us on this part, so the five dependent launches of the general path
// dominate such calls (18.4 us at 14 buses); here the whole call is one
// launch and one block, its phases separated by block barriers, every
// intermediate in LDS (the workspace receives the per-line data and the
// box-preparation record too, for the relaxation and backward kernels that
// read them).  The arithmetic is that of the multi-kernel path (the same
// device functions; the outage elements in pairs of outages, k3_pair, so the
// float32 penalty sums have the same depth), so the padding is unchanged.
// Every load that does not depend on another is issued before the first use.
// SWEEP = false stops after the line epilogue (the backward's preparation).
constexpr int kMicroBuses = 256;
constexpr int kMicroLines = 1024;
constexpr int kMicroElems = 65536;

template <bool SWEEP>
__global__ __launch_bounds__(256) void km_box(DevNet net, const float* __restrict__ box_lo,
                                              const float* __restrict__ box_hi, void* ws, WsLayout lay, int64_t box0,
                                              double* __restrict__ f_lo, double* __restrict__ f_hi,
                                              double* __restrict__ terms) {
  __shared__ double2 inj[kMicroBuses];
  __shared__ float s_lc[kMicroLines], s_lh[kMicroLines], s_lg[kMicroLines];
  __shared__ int4 s_ctg[kMicroElems / 64];
  __shared__ double red[4][kP1Fields + 4];
  __shared__ unsigned redm[4];
  const int64_t b = box0 + blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const float* lo = box_lo + b * net.X;
  const float* hi = box_hi + b * net.X;
  // line constants of this thread's first line, loaded with the box
  const int l0 = min(tid, net.L - 1);
  const LineConst q0 = load_line_const(net, l0);
  double v[kP1Fields];
#pragma unroll
  for (int f = 0; f < kP1Fields; ++f) v[f] = 0.0;
  if (tid < net.N) {
    double2 cr;
    bus_injection(net, lo, hi, tid, cr, v[kP1Mc], v[kP1Mbox]);
    inj[tid] = cr;
  }
  for (int i = tid; i < net.X; i += 256) input_terms(net, i, lo[i], hi[i], net.dev_w[i], v);
  box_slots_init(net, ws, lay, b);
  for (int l = net.L + tid; l < net.Lp; l += 256) {
    s_lc[l] = 0.0f;
    s_lh[l] = -FLT_MAX;
    s_lg[l] = FLT_MAX;
  }
#pragma unroll
  for (int f = 0; f < kP1Fields; ++f) v[f] = wave_sum(v[f]);
  if (lane == 0)
#pragma unroll
    for (int f = 0; f < kP1Fields; ++f) red[w][f] = v[f];
  __syncthreads();
#pragma unroll
  for (int f = 0; f < kP1Fields; ++f) v[f] = (red[0][f] + red[1][f]) + (red[2][f] + red[3][f]);
  if (tid < kP1Fields) ws_ptr<double>(ws, lay.p1)[b * kP1Fields + tid] = v[tid];
  const double g = (net.N + 64) * kU64 * 1.01;
  const double mc = v[kP1Mc] * (1.0 + g), mb = v[kP1Mbox] * (1.0 + g);

  // base flows (sixteen PTDF loads in flight per step) and the line epilogue
  double pb_hi = 0.0, pb_lo = 0.0;
  unsigned vm = 0u;
  for (int l = tid; l < net.L; l += 256) {
    double cf = 0.0, rh = 0.0;
    for (int n0 = 0; n0 < net.N; n0 += 16) {
      float x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = n0 + u < net.N ? net.phiT[(size_t)(n0 + u) * net.Lp + l] : 0.0f;
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (n0 + u < net.N) {
          const double2 cr = inj[n0 + u];
          cf = fma((double)x[u], cr.x, cf);
          rh = fma(fabs((double)x[u]), cr.y, rh);
        }
    }
    const LineConst q = l == l0 ? q0 : load_line_const(net, l);
    vm = max(vm, line_epilogue(net, l, q, cf, rh, mc, mb, s_lc, s_lh, s_lg, ws_ptr<double>(ws, lay.lcf) + b * net.L,
                               ws_ptr<double>(ws, lay.lrf) + b * net.L, s_ctg,
                               lay.cb ? ws_ptr<float2>(ws, lay.cb) + b * net.K : nullptr, pb_hi, pb_lo));
  }
  vm = wave_max_u32(vm);
  pb_hi = wave_sum(pb_hi);
  pb_lo = wave_sum(pb_lo);
  if (lane == 0) {
    red[w][kP1Fields] = pb_hi;
    red[w][kP1Fields + 1] = pb_lo;
    redm[w] = vm;
  }
  __syncthreads();
  const unsigned vmb = max(max(redm[0], redm[1]), max(redm[2], redm[3]));
  const float vmax = __uint_as_float(vmb);
  // the per-line and per-outage data for the kernels that run after this one
  float* wlc = ws_ptr<float>(ws, lay.lc) + b * net.Lp;
  float* wlh = ws_ptr<float>(ws, lay.lh) + b * net.Lp;
  float* wlg = ws_ptr<float>(ws, lay.lg) + b * net.Lp;
  for (int l = tid; l < net.L; l += 256) {
    wlc[l] = s_lc[l];
    wlh[l] = s_lh[l];
    wlg[l] = s_lg[l];
  }
  int4* wctg = ws_ptr<int4>(ws, lay.ctg) + b * net.K;
  for (int k = tid; k < net.K; k += 256) wctg[k] = s_ctg[k];
  if (tid == 0) *reinterpret_cast<unsigned*>(ws_ptr<double>(ws, lay.box) + b * kBoxSlots + kVmax) = vmb;
  if (!SWEEP) return;

  // outage sweep: items (column of four lines, pair of outages), columns fastest
  const int Lp4 = net.Lp / 4;
  const int np = net.K / 2;
  double acc_hi = 0.0, acc_lo = 0.0;
  const float4* lam = reinterpret_cast<const float4*>(net.lodf);
  auto column = [&](int col, float4& c4, float4& h4, float4& g4) {
    const float4 e4 = reinterpret_cast<const float4*>(net.line_eps)[col];
    c4 = make_float4(s_lc[4 * col], s_lc[4 * col + 1], s_lc[4 * col + 2], s_lc[4 * col + 3]);
    h4 = make_float4(add_ru(s_lh[4 * col], next_up_f32(e4.x * vmax)), add_ru(s_lh[4 * col + 1], next_up_f32(e4.y * vmax)),
                     add_ru(s_lh[4 * col + 2], next_up_f32(e4.z * vmax)), add_ru(s_lh[4 * col + 3], next_up_f32(e4.w * vmax)));
    g4 = make_float4(add_ru(s_lg[4 * col], next_up_f32(e4.x * vmax)), add_ru(s_lg[4 * col + 1], next_up_f32(e4.y * vmax)),
                     add_ru(s_lg[4 * col + 2], next_up_f32(e4.z * vmax)), add_ru(s_lg[4 * col + 3], next_up_f32(e4.w * vmax)));
  };
  for (int it = tid; it < np * Lp4; it += 256) {
    const int col = it % Lp4, k = 2 * (it / Lp4);
    const float4 x0 = lam[(size_t)k * Lp4 + col], x1 = lam[(size_t)(k + 1) * Lp4 + col];
    float4 c4, h4, g4;
    column(col, c4, h4, g4);
    k3_pair(x0, s_ctg[k], x1, s_ctg[k + 1], c4, h4, g4, acc_hi, acc_lo);
  }
  if (net.K & 1) {  // the last outage of an odd count, alone
    const int k = net.K - 1;
    for (int col = tid; col < Lp4; col += 256) {
      const float4 x0 = lam[(size_t)k * Lp4 + col];
      float4 c4, h4, g4;
      column(col, c4, h4, g4);
      const float cc0 = __int_as_float(s_ctg[k].y), rk0 = __int_as_float(s_ctg[k].z);
      float a0, a1, a2, a3, q0a, q1, q2, q3;
      k3_elem(x0.x, cc0, rk0, c4.x, h4.x, g4.x, a0, q0a);
      k3_elem(x0.y, cc0, rk0, c4.y, h4.y, g4.y, a1, q1);
      k3_elem(x0.z, cc0, rk0, c4.z, h4.z, g4.z, a2, q2);
      k3_elem(x0.w, cc0, rk0, c4.w, h4.w, g4.w, a3, q3);
      acc_hi += (double)((a0 + a1) + (a2 + a3));
      acc_lo += (double)((q0a + q1) + (q2 + q3));
    }
  }
  acc_hi = wave_sum(acc_hi);
  acc_lo = wave_sum(acc_lo);
  if (lane == 0) {
    red[w][kP1Fields + 2] = acc_hi;
    red[w][kP1Fields + 3] = acc_lo;
  }
  __syncthreads();
  if (tid != 0) return;
  double x[12];
#pragma unroll
  for (int f = 0; f < 8; ++f) x[f] = v[kP1Sc + f];
#pragma unroll
  for (int f = 0; f < 4; ++f)
    x[8 + f] = (red[0][kP1Fields + f] + red[1][kP1Fields + f]) + (red[2][kP1Fields + f] + red[3][kP1Fields + f]);
  objective_interval(net, lay, b, x, f_lo, f_hi, terms);
}

// ---------------------------------------------------------------- K4

// ---------------------------------------------------------------- launchers

bool tune_valid(const Tune& t) {
  const bool nc = t.k2_nc == 32 || t.k2_nc == 64 || t.k2_nc == 128 || t.k2_nc == 256 || t.k2_nc == 512;
  const bool kc = t.k3_kc == 16 || t.k3_kc == 32 || t.k3_kc == 64 || t.k3_kc == 128;
  return nc && kc;
}

bool tune_batched_valid(const Tune& t) {
  return (t.k3_bt == 2 || t.k3_bt == 4 || t.k3_bt == 8) && t.k3_rows >= 0 && t.k3_rows <= 4096 &&
         t.k3_xcd >= -1 && t.k3_xcd <= 1 && (t.k2b_mfma == 0 || t.k2b_mfma == 1) && t.k2_by >= 0 && t.k2_by <= 8;
}

void plan_single(const DevNet& net, int64_t n_box, WsLayout& lay, const Tune& t) {
  (void)n_box;
  const int lp4 = net.Lp / 4;
  lay.k2_nc = t.k2_nc;
  lay.k3_kc = t.k3_kc;
  // the smallest networks: one launch, one block per box (km_box)
  lay.small = net.N <= kMicroBuses && net.L <= kMicroLines && (int64_t)net.K * net.Lp <= kMicroElems;
  lay.n_p1 = lay.small ? 1 : (std::max(net.Np, net.X) + 63) / 64;
  lay.k2_bx = (lp4 + 63) / 64;
  lay.k2_by = std::max(1, (net.N + 4 * t.k2_nc - 1) / (4 * t.k2_nc));
  lay.n_p2 = (net.L + 63) / 64;  // one base-penalty partial per epilogue wave
  // K3: 4 waves x 256 lines per block, k3_kc outages per block
  lay.k3_bx = (lp4 + 255) / 256;
  lay.k3_by = std::max(1, (net.K + t.k3_kc - 1) / t.k3_kc);
  lay.n_p3 = net.K > 0 ? lay.k3_bx * lay.k3_by : 0;
  if (lay.small) lay.n_p2 = lay.n_p3 = 1;
}

template <int NC>
static void launch_k2(const DevNet& net, void* ws, const WsLayout& lay, int64_t b0, int nb, hipStream_t s,
                      KernelTimer* tm) {
  tm->launch(1, k2_base_flows<NC>, dim3(lay.k2_bx, lay.k2_by, nb), dim3(256), s, net, ws, lay, b0,
             reinterpret_cast<const double2*>(static_cast<char*>(ws) + lay.inj));
}

template <int KC>
static void launch_k3(const DevNet& net, void* ws, const WsLayout& lay, int64_t b0, int nb, hipStream_t s,
                      KernelTimer* tm) {
  tm->launch(2, k3_contingency<KC>, dim3(lay.k3_bx, lay.k3_by, nb), dim3(256), s, net, ws, lay, b0);
}

hipError_t launch_forward_single(const DevNet& net, int64_t n_box, const float* lo, const float* hi,
                                 double* f_lo, double* f_hi, double* terms, void* ws,
                                 const WsLayout& lay, hipStream_t s, KernelTimer* tm) {
  if (lay.small) {
    for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
      const int nb = (int)std::min<int64_t>(65535, n_box - b0);
      tm->launch(2, km_box<true>, dim3(nb), dim3(256), s, net, lo, hi, ws, lay, b0, f_lo, f_hi, terms);
    }
    return hipGetLastError();
  }
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    tm->launch(0, k1_box_prep, dim3(lay.n_p1, nb), dim3(64), s, net, lo, hi, ws, lay, b0);
    switch (lay.k2_nc) {
      case 32: launch_k2<32>(net, ws, lay, b0, nb, s, tm); break;
      case 64: launch_k2<64>(net, ws, lay, b0, nb, s, tm); break;
      case 256: launch_k2<256>(net, ws, lay, b0, nb, s, tm); break;
      case 512: launch_k2<512>(net, ws, lay, b0, nb, s, tm); break;
      default: launch_k2<128>(net, ws, lay, b0, nb, s, tm); break;
    }
    tm->launch(4, k2e_lines, dim3((net.L + kK2eThreads - 1) / kK2eThreads, nb), dim3(kK2eThreads), s, net, ws,
               lay, b0);
    if (net.K > 0) {
      switch (lay.k3_kc) {
        case 32: launch_k3<32>(net, ws, lay, b0, nb, s, tm); break;
        case 64: launch_k3<64>(net, ws, lay, b0, nb, s, tm); break;
        case 128: launch_k3<128>(net, ws, lay, b0, nb, s, tm); break;
        default: launch_k3<16>(net, ws, lay, b0, nb, s, tm); break;
      }
    }
    tm->launch(3, k4_finalize<256>, dim3(nb), dim3(256), s, net, ws, lay, b0, f_lo, f_hi, terms);
  }
  return hipGetLastError();
}

hipError_t launch_forward_prep(const DevNet& net, int64_t n_box, const float* lo, const float* hi, void* ws,
                               const WsLayout& lay, hipStream_t s, KernelTimer* tm) {
  if (lay.small) {
    for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
      const int nb = (int)std::min<int64_t>(65535, n_box - b0);
      const int t = tm->start(0, s);
      hipLaunchKernelGGL(km_box<false>, dim3(nb), dim3(256), 0, s, net, lo, hi, ws, lay, b0, nullptr, nullptr,
                         nullptr);
      tm->stop(t, s);
    }
    return hipGetLastError();
  }
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(0, s);
    hipLaunchKernelGGL(k1_box_prep, dim3(lay.n_p1, nb), dim3(64), 0, s, net, lo, hi, ws, lay, b0);
    tm->stop(t, s);
  }
  if (lay.batched) {
    const hipError_t e = launch_batched_sweeps(net, n_box, ws, lay, s, tm, 0);
    if (e != hipSuccess) return e;
  } else {
    for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
      const int nb = (int)std::min<int64_t>(65535, n_box - b0);
      switch (lay.k2_nc) {
        case 32: launch_k2<32>(net, ws, lay, b0, nb, s, tm); break;
        case 64: launch_k2<64>(net, ws, lay, b0, nb, s, tm); break;
        case 256: launch_k2<256>(net, ws, lay, b0, nb, s, tm); break;
        case 512: launch_k2<512>(net, ws, lay, b0, nb, s, tm); break;
        default: launch_k2<128>(net, ws, lay, b0, nb, s, tm); break;
      }
    }
  }
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(4, s);
    hipLaunchKernelGGL(k2e_lines, dim3((net.L + kK2eThreads - 1) / kK2eThreads, nb), dim3(kK2eThreads), 0, s,
                       net, ws, lay, b0);
    tm->stop(t, s);
  }
  return hipGetLastError();
}

hipError_t launch_forward(const DevNet& net, int64_t n_box, const float* lo, const float* hi, double* f_lo,
                          double* f_hi, double* terms, void* ws, const WsLayout& lay, hipStream_t s,
                          KernelTimer* tm) {
  if (!lay.batched) return launch_forward_single(net, n_box, lo, hi, f_lo, f_hi, terms, ws, lay, s, tm);
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(0, s);
    hipLaunchKernelGGL(k1_box_prep, dim3(lay.n_p1, nb), dim3(64), 0, s, net, lo, hi, ws, lay, b0);
    tm->stop(t, s);
  }
  launch_batched_sweeps(net, n_box, ws, lay, s, tm, 0);
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(4, s);
    hipLaunchKernelGGL(k2e_lines, dim3((net.L + kK2eThreads - 1) / kK2eThreads, nb), dim3(kK2eThreads), 0, s,
                       net, ws, lay, b0);
    tm->stop(t, s);
  }
  launch_batched_sweeps(net, n_box, ws, lay, s, tm, 1);
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    const int t = tm->start(3, s);
    launch_k4(net, ws, lay, b0, nb, f_lo, f_hi, terms, s);
    tm->stop(t, s);
  }
  return hipGetLastError();
}

}  // namespace ibp
