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

#include "ibp_device.h"
#include "ibp_devfun.h"
#include "ibp_kernels.h"

namespace ibp {

constexpr int kK5Chunk = 128;  // outages per block row
constexpr int kK5Sub = 16;     // outages per butterfly reduction

__device__ __forceinline__ float sgnf(float x) { return x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f); }

// Sums v[0..31] over the 64 lanes of a wave; afterwards lanes 2i and 2i+1
// hold the total of v[i].
__device__ __forceinline__ float butterfly32(float (&v)[32]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const bool up = lane & 32;
    const float send = up ? v[i] : v[i + 16];
    const float keep = up ? v[i + 16] : v[i];
    v[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const bool up = lane & 16;
    const float send = up ? v[i] : v[i + 8];
    const float keep = up ? v[i + 8] : v[i];
    v[i] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool up = lane & 8;
    const float send = up ? v[i] : v[i + 4];
    const float keep = up ? v[i + 4] : v[i];
    v[i] = keep + __shfl_xor(send, 8, 64);
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
    v[0] = keep + __shfl_xor(send, 2, 64);
  }
  return v[0] + __shfl_xor(v[0], 1, 64);
}

// One element of the outage sweep's VJP.  Returns (dC, dR) and adds the
// outage-side contributions Lam dC, |Lam| dR to (pc, pr).
__device__ __forceinline__ void k5_elem(float lam, float cc, float rc, float cl, float rl, float fm, float chi,
                                        float clo, float& gc, float& gr, float& pc, float& pr) {
  // The outaged line's own entry holds NaN: C and R are NaN, both activity
  // tests fail and dC = dR = 0 (the paper's mask M); lam0 keeps the NaN out of
  // the outage-side products.
  const float C = fmaf(lam, cc, cl);
  const float R = fmaf(fabsf(lam), rc, rl);
  const float a = fabsf(C);
  const float hi = (a + R - fm > 0.0f) ? chi : 0.0f;
  const float lo = (a - R - fm > 0.0f) ? clo : 0.0f;
  const float dC = sgnf(C) * (hi + lo);
  const float dR = hi - lo;
  const float lam0 = (lam == lam) ? lam : 0.0f;
  gc += dC;
  gr += dR;
  pc = fmaf(lam0, dC, pc);
  pr = fmaf(fabsf(lam0), dR, pr);
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
  const float chi = (float)(-net.zeta_f * g_lo[b]);  // weight of an active P_hi
  const float clo = (float)(-net.zeta_f * g_hi[b]);  // weight of an active P_lo (dR gets -clo)
  // lines of this lane (padding lines: zero centre and radius, limit FLT_MAX)
  float4 c4 = make_float4(0.f, 0.f, 0.f, 0.f), r4 = c4, f4 = make_float4(FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX);
  if (on) {
    c4 = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lc) + b * net.Lp)[col];
    const double* rf = ws_ptr<double>(ws, lay.lrf) + b * net.L;
    const int l0 = 4 * col;
    r4 = make_float4(l0 < net.L ? (float)rf[l0] : 0.f, l0 + 1 < net.L ? (float)rf[l0 + 1] : 0.f,
                     l0 + 2 < net.L ? (float)rf[l0 + 2] : 0.f, l0 + 3 < net.L ? (float)rf[l0 + 3] : 0.f);
    f4 = reinterpret_cast<const float4*>(net.fmax_c32)[col];
  }
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
        k5_elem(x.x, cc, rc, c4.x, r4.x, f4.x, chi, clo, gc[0], gr[0], pc, pr);
        k5_elem(x.y, cc, rc, c4.y, r4.y, f4.y, chi, clo, gc[1], gr[1], pc, pr);
        k5_elem(x.z, cc, rc, c4.z, r4.z, f4.z, chi, clo, gc[2], gr[2], pc, pr);
        k5_elem(x.w, cc, rc, c4.w, r4.w, f4.w, chi, clo, gc[3], gr[3], pc, pr);
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

// Per line: base-case penalty gradient + outage-sweep partials (as the line
// itself and, if it is an outage line, as the outaged line).
__global__ __launch_bounds__(256) void k5r_lines(DevNet net, void* ws, WsLayout lay, int64_t box0,
                                                 const double* __restrict__ g_lo,
                                                 const double* __restrict__ g_hi) {
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
  const double zf = net.zeta_f, gl = g_lo[b], gh = g_hi[b];
  const double c = ws_ptr<double>(ws, lay.lcf)[b * net.L + l];
  const double r = ws_ptr<double>(ws, lay.lrf)[b * net.L + l];
  const double a = fabs(c), fb = net.fmax_b[l];
  const double hi = (a + r - fb > 0.0) ? -zf * gl : 0.0;
  const double lo = (a - r - fb > 0.0) ? -zf * gh : 0.0;
  const double s = c > 0.0 ? 1.0 : (c < 0.0 ? -1.0 : 0.0);
  double dc = s * (hi + lo), dr = hi - lo;
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

// Per input: endpoint gradients (injection, surplus and imbalance terms).
__global__ __launch_bounds__(256) void k7_endpoints(DevNet net, void* ws, WsLayout lay, int64_t box0,
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
  const double gl = g_lo[b], gh = g_hi[b], zi = net.zeta_inj;
  const double aI = fabs(cI);
  const double hiI = (aI + rI > 0.0) ? -zi * gl : 0.0;
  const double loI = (aI - rI > 0.0) ? -zi * gh : 0.0;
  const double sI = cI > 0.0 ? 1.0 : (cI < 0.0 ? -1.0 : 0.0);
  const double dcI = sI * (hiI + loI), drI = hiI - loI;
  const double sj = j < net.G ? 1.0 : -1.0;
  const int n = net.dev_bus[j];
  const double wj = net.dev_w[j];
  const double dc = sj * ws_ptr<double>(ws, lay.gci)[b * net.Np + n] + (gl + gh) * wj + sj * dcI;
  const double dr = ws_ptr<double>(ws, lay.gri)[b * net.Np + n] + (gh - gl) * fabs(wj) + drI;
  const bool nanb = bad != 0.0;
  d_lo[b * net.X + j] = nanb ? NAN : 0.5 * (dc - dr);
  d_hi[b * net.X + j] = nanb ? NAN : 0.5 * (dc + dr);
}

void plan_backward(const DevNet& net, WsLayout& lay) {
  const int lp4 = net.Lp / 4;
  lay.k5_tiles = (lp4 + 63) / 64;
  lay.k5_by = std::max(1, (net.K + kK5Chunk - 1) / kK5Chunk);
}

hipError_t launch_backward_sweeps(const DevNet& net, int64_t n_box, void* ws, const WsLayout& lay,
                                  const double* g_lo, const double* g_hi, double* d_lo, double* d_hi,
                                  hipStream_t s, KernelTimer* tm) {
  for (int64_t b0 = 0; b0 < n_box; b0 += 65535) {
    const int nb = (int)std::min<int64_t>(65535, n_box - b0);
    int t = tm->start(7, s);
    if (net.K > 0)
      hipLaunchKernelGGL(k5_outage_vjp, dim3((lay.k5_tiles + 3) / 4, lay.k5_by, nb), dim3(256), 0, s, net, ws,
                         lay, b0, g_lo, g_hi);
    hipLaunchKernelGGL(k5r_lines, dim3((net.Lp + 255) / 256, nb), dim3(256), 0, s, net, ws, lay, b0, g_lo, g_hi);
    tm->stop(t, s);
    t = tm->start(8, s);
    hipLaunchKernelGGL(k6_ptdf_t, dim3((net.Np + 7) / 8, nb), dim3(256), 0, s, net, ws, lay, b0);
    tm->stop(t, s);
    t = tm->start(9, s);
    hipLaunchKernelGGL(k7_endpoints, dim3((net.X + 255) / 256, nb), dim3(256), 0, s, net, ws, lay, b0, g_lo, g_hi,
                       d_lo, d_hi);
    tm->stop(t, s);
  }
  return hipGetLastError();
}

}  // namespace ibp
