// Line screen of the one-sided sweeps, and the screened forward sweep.
//
// A one-sided quantity sums (or differentiates) one penalty side over every
// outage x line element: the lower penalties max(|C| - R - fmax, 0) for f_hi,
// the upper ones max(|C| + R - fmax, 0) for f_lo (Sec. III-A eqs. (slack-Sc),
// (slack-sagg); Sec. III-C eq. (IBP)).  Post-outage flows are
// C = c_l + Lam c_c and R = r_l + |Lam| r_c (Sec. II-C, eq. ctg flow
// simplified), so with w_k = |c_c| - r_c (lower) or |c_c| + r_c (upper) for
// the outaged line of outage k, every element of line l obeys
//   |C| - R - fmax <= (|c_l| - (r_l + fmax)) + |Lam_lk| max(w_k, 0),
//   |C| + R - fmax <= (|c_l| + (r_l - fmax)) + |Lam_lk| w_k.
// A line on which the right-hand side stays below zero for every outage and
// every box of a tile holds no active element there, and contributes nothing.
// In sub-boxes few lines can (2000 buses, 4096 sub-boxes: 19% of the
// (4-box tile, line) pairs for the lower penalties; at the boxes' centre
// points 39% for the upper ones).
//
// K5w takes per tile and outage the largest max(w_k, 0) over the tile's
// boxes; K5s, per tile and line, the largest |Lam_lk| W_k over the outages
// (one multiply and one max per factor and tile, 16 or 4 tiles per block
// sharing each factor load) and marks the line where base + that > -margin.
// margin is 32 float32 unit roundoffs of the largest magnitude either test adds
// (the screen's own bound and the sweep's test take 12 between them), so no
// line with an active element goes unmarked.  The radii and limits are those
// of the sweep the screen serves: the backward's unpadded ones, or the
// forward's padded r' and fmax -/+ r' (which only make its penalties
// smaller on the lower side; on the upper side they enter the bound).  Marked
// lines get their tile record (the four boxes' centres and radius terms),
// which the sweeps read by scalar loads.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "ibp_device.h"
#include "ibp_devfun.h"
#include "ibp_kernels.h"
#include "ibp_lanes.h"

namespace ibp {

constexpr int kScreenChunk = 128;  // outages per LDS chunk of the screen

// Tiles per screen block: 16 share every factor load when that still gives
// about two blocks per CU (4096 boxes at 2000 buses: 0.69 ms; 32 tiles gave
// too few blocks, 1.30 ms), otherwise 4 (1024 boxes: 16 tiles left the chip
// under-filled with 208 blocks).
inline int screen_tiles(const DevNet& net, const WsLayout& lay) {
  const int64_t line_blocks = (net.Lp + 255) / 256;
  return ((int64_t)lay.k5s_tiles + 15) / 16 * line_blocks >= 512 ? 16 : 4;
}

// The per-outage (centre, radius) the sweep of `mode` uses: the backward's
// (centre, unpadded radius) pairs, or the forward's (centre, padded r').
template <int MODE>
__device__ __forceinline__ float2 outage_cr(const DevNet& net, void* ws, const WsLayout& lay, int64_t b, int k) {
  if (MODE == kScreenBackwardLower) return ws_ptr<float2>(ws, lay.cb)[b * net.K + k];
  const int4 d = ws_ptr<int4>(ws, lay.ctg)[b * net.K + k];
  return make_float2(__int_as_float(d.y), __int_as_float(d.z));
}

// The per-line radius term of the sweep's test for box b: r + fmax
// (backward), or the forward sweep's padded g = r' + fmax and
// h = r' - fmax, each raised by the line's construction error times the box's
// largest outage magnitude exactly as that sweep forms them.
template <int MODE>
__device__ __forceinline__ float line_term(const DevNet& net, void* ws, const WsLayout& lay, int64_t b, int l,
                                           float fc) {
  if (MODE == kScreenBackwardLower) return (float)ws_ptr<double>(ws, lay.lrf)[b * net.L + l] + fc;
  const double* bs = ws_ptr<double>(ws, lay.box) + b * kBoxSlots;
  const float vmax = __uint_as_float(*reinterpret_cast<const unsigned int*>(bs + kVmax));
  const float ex = next_up_f32(net.line_eps[l] * vmax);
  const float v = ws_ptr<float>(ws, MODE == kScreenForwardLower ? lay.lg : lay.lh)[b * net.Lp + l];
  return add_ru(v, ex);
}

// The forward sweep's padded g of box b and line l (the lower penalties' term
// of a two-sided sweep), formed as K3b forms it.
__device__ __forceinline__ float line_g(const DevNet& net, void* ws, const WsLayout& lay, int64_t b, int l) {
  const double* bs = ws_ptr<double>(ws, lay.box) + b * kBoxSlots;
  const float vmax = __uint_as_float(*reinterpret_cast<const unsigned int*>(bs + kVmax));
  return add_ru(ws_ptr<float>(ws, lay.lg)[b * net.Lp + l], next_up_f32(net.line_eps[l] * vmax));
}

// K5w: per tile and outage W (zero past the last outage); per tile and block
// of 256 outages the largest |c_c| + r_c, for the margin.
template <int MODE>
__global__ __launch_bounds__(256) void k5w_tile_max(DevNet net, void* ws, WsLayout lay, int64_t n_box) {
  constexpr int S = kScreenBoxes;
  __shared__ unsigned zs[4];
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int64_t t = blockIdx.y;
  float wv = 0.0f, z = 0.0f;
  if (k < net.K) {
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const int64_t b = t * S + i;
      if (b < n_box) {
        const float2 v = outage_cr<MODE>(net, ws, lay, b, k);
        wv = fmaxf(wv, MODE >= kScreenForwardUpper ? fabsf(v.x) + v.y : fabsf(v.x) - v.y);
        z = fmaxf(z, fabsf(v.x) + v.y);
      }
    }
  }
  if (k < net.Kp) ws_ptr<float>(ws, lay.sw)[t * net.Kp + k] = wv;
  // non-negative floats order like their bit patterns
  const unsigned zb = wave_max_u32(__float_as_uint(z));
  if ((threadIdx.x & 63) == 0) zs[threadIdx.x >> 6] = zb;
  __syncthreads();
  if (threadIdx.x == 0)
    ws_ptr<float>(ws, lay.sz)[t * lay.k5w_bx + blockIdx.x] =
        __uint_as_float(max(max(zs[0], zs[1]), max(zs[2], zs[3])));
}

// K5s: one line per lane, G tiles per block, the tiles' W staged
// in LDS kScreenChunk outages at a time.
template <int MODE, int G>
__global__ __launch_bounds__(256) void k5s_screen(DevNet net, void* ws, WsLayout lay, int64_t n_box) {
  constexpr int S = kScreenBoxes;
  static_assert(S == 4, "a tile's line record holds four boxes");
  static_assert(G % 4 == 0, "tiles are read from LDS as float4");
  __shared__ __align__(16) float wsh[kScreenChunk][G];
  __shared__ float zsh[G];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l = blockIdx.x * 256 + tid;
  const bool lon = l < net.L;
  const int lq = min(l, net.Lp - 1);
  const int64_t tile0 = (int64_t)blockIdx.y * G;
  const int ntile = (int)min<int64_t>(G, lay.k5s_tiles - tile0);
  const float* W = ws_ptr<float>(ws, lay.sw) + tile0 * net.Kp;
  if (tid < G) {
    float z = 0.0f;
    if (tid < ntile)
      for (int j = 0; j < lay.k5w_bx; ++j) z = fmaxf(z, ws_ptr<float>(ws, lay.sz)[(tile0 + tid) * lay.k5w_bx + j]);
    zsh[tid] = z;
  }
  float m[G];
#pragma unroll
  for (int g = 0; g < G; ++g) m[g] = 0.0f;
  const float* lam = net.lodf + lq;
  for (int k0 = 0; k0 < net.K; k0 += kScreenChunk) {
    const int nk = min(kScreenChunk, net.K - k0);
    __syncthreads();
    for (int idx = tid; idx < kScreenChunk * G; idx += 256) {
      const int kk = idx % kScreenChunk, g = idx / kScreenChunk;
      wsh[kk][g] = (g < ntile && kk < nk) ? W[(size_t)g * net.Kp + k0 + kk] : 0.0f;
    }
    __syncthreads();
    // |Lam| W: the outaged line's own factor is NaN, and fmaxf keeps m there;
    // rows past the chunk's end read its last row against W = 0
    for (int kk = 0; kk < nk; kk += 4) {
      float a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = fabsf(lam[(size_t)(k0 + min(kk + u, nk - 1)) * net.Lp]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int g4 = 0; g4 < G / 4; ++g4) {
          const float4 wv = *reinterpret_cast<const float4*>(&wsh[kk + u][4 * g4]);
          m[4 * g4 + 0] = fmaxf(m[4 * g4 + 0], a[u] * wv.x);
          m[4 * g4 + 1] = fmaxf(m[4 * g4 + 1], a[u] * wv.y);
          m[4 * g4 + 2] = fmaxf(m[4 * g4 + 2], a[u] * wv.z);
          m[4 * g4 + 3] = fmaxf(m[4 * g4 + 3], a[u] * wv.w);
        }
      }
    }
  }
  const float fc = lon ? net.fmax_c32[l] : 0.0f;
  const float amax = lon ? net.lam_max[l] : 0.0f;
  const float* lc = ws_ptr<float>(ws, lay.lc);
  const int words = net.Lp / 64;
  const int word = blockIdx.x * 4 + w;
  // a box past the end gets a record that never tests active
  constexpr float kOff = MODE >= kScreenForwardUpper ? -INFINITY : INFINITY;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (g >= ntile) break;  // uniform
    const int64_t t = tile0 + g;
    float cv[S], rv[S], gv[S];
    float base = -FLT_MAX, sc = 0.0f;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const int64_t b = t * S + i;
      cv[i] = 0.0f;
      rv[i] = kOff;
      gv[i] = INFINITY;
      if (lon && b < n_box) {
        cv[i] = lc[b * net.Lp + l];
        rv[i] = line_term<MODE>(net, ws, lay, b, l, fc);
        base = fmaxf(base, MODE >= kScreenForwardUpper ? fabsf(cv[i]) + rv[i] : fabsf(cv[i]) - rv[i]);
        sc = fmaxf(sc, fabsf(cv[i]) + fabsf(rv[i]));
      }
    }
    const float margin = 0x1p-19f * (sc + amax * zsh[g]);
    const bool flag = lon && base + m[g] > -margin;
    const uint64_t bits = __builtin_amdgcn_ballot_w64(flag);
    if (lane == 0 && word < words) ws_ptr<uint64_t>(ws, lay.smask)[t * words + word] = bits;
    if (flag) {
      float4* rec = reinterpret_cast<float4*>(ws_ptr<float>(ws, lay.srec) + ((size_t)t * net.Lp + l) * kScreenRecFloats);
      rec[0] = make_float4(cv[0], cv[1], cv[2], cv[3]);
      rec[1] = make_float4(rv[0], rv[1], rv[2], rv[3]);
      if (MODE == kScreenForwardBoth) {
#pragma unroll
        for (int i = 0; i < S; ++i)
          if (lon && t * S + i < n_box) gv[i] = line_g(net, ws, lay, t * S + i, l);
        rec[2] = make_float4(gv[0], gv[1], gv[2], gv[3]);
      }
      if (MODE == kScreenBackwardLower) {
#pragma unroll
        for (int i = 0; i < S; ++i)
          if (t * S + i < n_box) ws_ptr<uint64_t>(ws, lay.lcnt)[(t * S + i) * net.Lp + l] = 0ull;
      }
    }
  }
}

template <int MODE>
static void launch_screen_mode(const DevNet& net, int64_t n_box, void* ws, const WsLayout& lay, hipStream_t s) {
  hipLaunchKernelGGL(k5w_tile_max<MODE>, dim3(lay.k5w_bx, lay.k5s_tiles), dim3(256), 0, s, net, ws, lay, n_box);
  const unsigned gx = (net.Lp + 255) / 256;
  if (screen_tiles(net, lay) == 16)
    hipLaunchKernelGGL((k5s_screen<MODE, 16>), dim3(gx, (lay.k5s_tiles + 15) / 16), dim3(256), 0, s, net, ws, lay,
                       n_box);
  else
    hipLaunchKernelGGL((k5s_screen<MODE, 4>), dim3(gx, (lay.k5s_tiles + 3) / 4), dim3(256), 0, s, net, ws, lay,
                       n_box);
}

void launch_line_screen(const DevNet& net, int64_t n_box, void* ws, const WsLayout& lay, int mode, hipStream_t s) {
  if (mode == kScreenBackwardLower)
    launch_screen_mode<kScreenBackwardLower>(net, n_box, ws, lay, s);
  else if (mode == kScreenForwardLower)
    launch_screen_mode<kScreenForwardLower>(net, n_box, ws, lay, s);
  else if (mode == kScreenForwardUpper)
    launch_screen_mode<kScreenForwardUpper>(net, n_box, ws, lay, s);
  else
    launch_screen_mode<kScreenForwardBoth>(net, n_box, ws, lay, s);
}

// K3p: the one-sided forward sweep over the marked lines.  A wave holds 64 Q
// outages (lanes) of one tile's boxes and walks the tile's marked lines (the
// same walk as the backward's K5p); each element is k3_elem's, bit for bit
// (the same float32 operations on the same values), and each line's Q
// elements per box are summed in float32 (depth 2, within the depth-3 sums
// the padding of the outage-penalty total allows) and added in float64.
// Per (box, chunk of 64 Q outages) one float64 partial, in the slot the
// finalize sums; slots past the last chunk are cleared.
template <int SIDES, int Q>
__global__ __launch_bounds__(256) void k3p_sweep(DevNet net, void* ws, WsLayout lay, int64_t n_box, int n_chunk,
                                                 int n_tg) {
  constexpr int S = kScreenBoxes;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // unit u = (chunk, group of 4 tiles: one per wave), chunk-major, and the
  // blocks of one XCD (block id mod 8) on consecutive units
  const int U = n_chunk * n_tg;
  const int per = (U + 7) / 8;
  const int slot = blockIdx.x >> 3;
  const int u = (blockIdx.x & 7) * per + slot;
  if (slot >= per || u >= U) return;  // the whole block
  const int tile = (u % n_tg) * 4 + w;
  const bool on = tile < lay.k5s_tiles;
  const int chunk = u / n_tg;
  const int kw = chunk * 64 * Q;
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
  int64_t bb[S];
#pragma unroll
  for (int i = 0; i < S; ++i) bb[i] = min(b0 + i, n_box - 1);
  // per-lane outage data; lanes past the last outage get r' = inf (their
  // factors are the zero padding, and 0 x inf = NaN fails every test)
  float cc[Q][S], rk[Q][S];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = kw + 64 * q + lane;
    const int kq = min(k, net.K - 1);
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const int4 d = ws_ptr<int4>(ws, lay.ctg)[bb[i] * net.K + kq];
      cc[q][i] = __int_as_float(d.y);
      rk[q][i] = k < net.K ? __int_as_float(d.z) : INFINITY;
    }
  }
  double acc[S], acc2[S];  // SIDES 3: acc the upper penalties, acc2 the lower
#pragma unroll
  for (int i = 0; i < S; ++i) acc[i] = acc2[i] = 0.0;
  typedef __attribute__((address_space(4))) const float const_float;
  const_float* rec = (const_float*)(ws_ptr<float>(ws, lay.srec) + (size_t)tile * net.Lp * kScreenRecFloats);
  static_assert(64 * Q <= 256, "a chunk must fit the 256-outage row padding");
  const float* __restrict__ lamT = net.lodfT + kw + lane;
  // records: SIDES 1 (centres, g), SIDES 2 (centres, h), SIDES 3 (centres,
  // h, g)
  auto line_step = [&](const float4& c4, const float4& r4, const float4& g4, const float (&x)[Q]) {
    // each record value is read by Q elements' instructions: vector copies
    const float cl[S] = {vcopy(c4.x), vcopy(c4.y), vcopy(c4.z), vcopy(c4.w)};
    const float rl[S] = {vcopy(r4.x), vcopy(r4.y), vcopy(r4.z), vcopy(r4.w)};
    const float gl[S] = {SIDES == 3 ? vcopy(g4.x) : 0.0f, SIDES == 3 ? vcopy(g4.y) : 0.0f,
                         SIDES == 3 ? vcopy(g4.z) : 0.0f, SIDES == 3 ? vcopy(g4.w) : 0.0f};
#pragma unroll
    for (int i = 0; i < S; ++i) {
      float p[Q], p2[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        float a, b;
        k3_elem<SIDES>(x[q], cc[q][i], rk[q][i], cl[i], rl[i], SIDES == 3 ? gl[i] : rl[i], a, b);
        p[q] = SIDES == 1 ? b : a;
        p2[q] = b;
      }
      static_assert(Q == 4, "the float32 sum is written for four outages");
      acc[i] += (double)((p[0] + p[1]) + (p[2] + p[3]));
      if (SIDES == 3) acc2[i] += (double)((p2[0] + p2[1]) + (p2[2] + p2[3]));
    }
  };
  // marked-line walk (wave-uniform): lane i holds mask word wb + i, read out
  // by readlane; each line's loads issued before the previous line's sums
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
  bool pending = false;
  float4 pc4 = make_float4(0.f, 0.f, 0.f, 0.f), pr4 = pc4, pg4 = pc4;
  float px[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) px[q] = 0.0f;
  for (int l = next(); l >= 0; l = next()) {
    const_float* rp = rec + kScreenRecFloats * (size_t)l;
    const float4 c4 = make_float4(rp[0], rp[1], rp[2], rp[3]), r4 = make_float4(rp[4], rp[5], rp[6], rp[7]);
    const float4 g4 = SIDES == 3 ? make_float4(rp[8], rp[9], rp[10], rp[11]) : r4;
    float x[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) x[q] = lamT[(size_t)l * net.Kp + 64 * q];
    if (pending) line_step(pc4, pr4, pg4, px);
    pending = true;
    pc4 = c4;
    pr4 = r4;
    pg4 = g4;
#pragma unroll
    for (int q = 0; q < Q; ++q) px[q] = x[q];
  }
  if (pending) line_step(pc4, pr4, pg4, px);
  double2* p3 = ws_ptr<double2>(ws, lay.p3);
#pragma unroll
  for (int i = 0; i < S; ++i) {
    const double t = wave_sum(acc[i]);
    const double t2 = SIDES == 3 ? wave_sum(acc2[i]) : 0.0;
    if (lane == 0 && b0 + i < n_box) {
      p3[(b0 + i) * lay.n_p3 + chunk] = SIDES == 1 ? make_double2(0.0, t) : make_double2(t, t2);
      if (chunk == 0)
        for (int c = n_chunk; c < lay.n_p3; ++c) p3[(b0 + i) * lay.n_p3 + c] = make_double2(0.0, 0.0);
    }
  }
}

void launch_screened_forward_sweep(const DevNet& net, int64_t n_box, void* ws, const WsLayout& lay, int sides,
                                   hipStream_t s) {
  const int n_chunk = (net.K + 64 * kSparseQ - 1) / (64 * kSparseQ), n_tg = (lay.k5s_tiles + 3) / 4;
  const int per = (n_chunk * n_tg + 7) / 8;
  if (sides == 1)
    hipLaunchKernelGGL((k3p_sweep<1, kSparseQ>), dim3(8 * per), dim3(256), 0, s, net, ws, lay, n_box, n_chunk, n_tg);
  else if (sides == 2)
    hipLaunchKernelGGL((k3p_sweep<2, kSparseQ>), dim3(8 * per), dim3(256), 0, s, net, ws, lay, n_box, n_chunk, n_tg);
  else
    hipLaunchKernelGGL((k3p_sweep<3, kSparseQ>), dim3(8 * per), dim3(256), 0, s, net, ws, lay, n_box, n_chunk, n_tg);
}

}  // namespace ibp
