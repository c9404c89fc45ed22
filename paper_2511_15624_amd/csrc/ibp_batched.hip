// Box-tiled forward kernels for many boxes at once (sub-boxes and periods).
//
// Every box still gets the IBP of Sec. III-C through the graph of the
// Appendix; what changes is the data reuse.  A wave owns 256 lines and a tile
// of kBT boxes, and the four waves of a block take four box tiles of the same
// line tile, so each PTDF / outage-factor tile read from memory serves
// 4 x kBT boxes.  Grids are laid out so that blocks sharing a tile get the same
// linear id modulo 8: dispatch places consecutive ids on the 8 XCDs in turn,
// so those blocks run on one XCD and hit its L2.
//
// The arithmetic per element and the error model are those of the single-box
// kernels (float64 base-flow accumulation; float32 outage sweep with radii
// padded per line and per outage).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "ibp_device.h"
#include "ibp_devfun.h"
#include "ibp_kernels.h"

namespace ibp {

constexpr int kBT = 4;  // boxes per wave tile of the vector base-flow sweep (and the outage sweep's default)

// Base flows for kBT boxes x 256 lines per wave, over every bus.
__global__ __launch_bounds__(256) void k2b_base_flows(DevNet net, void* ws, WsLayout lay, int64_t n_box,
                                                      const double2* __restrict__ inj_all) {
  const int Lp4 = net.Lp / 4;
  if ((int)blockIdx.x * 64 >= Lp4) return;  // padding block of the grid
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t b0 = ((int64_t)blockIdx.y * 4 + w) * kBT;
  if (b0 >= n_box) return;
  const int col = blockIdx.x * 64 + lane;
  int64_t bb[kBT];
#pragma unroll
  for (int i = 0; i < kBT; ++i) bb[i] = min(b0 + i, n_box - 1);
  double ac[kBT][4], ar[kBT][4];
#pragma unroll
  for (int i = 0; i < kBT; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) ac[i][j] = ar[i][j] = 0.0;
  if (col < Lp4) {
    const float4* ph = reinterpret_cast<const float4*>(net.phiT) + col;
    int n = 0;
    for (; n + 8 <= net.N; n += 8) {
      float4 x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = ph[(size_t)(n + u) * Lp4];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double p0 = x[u].x, p1 = x[u].y, p2 = x[u].z, p3 = x[u].w;
#pragma unroll
        for (int i = 0; i < kBT; ++i) {
          const double2 cr = inj_all[bb[i] * net.Np + n + u];
          ac[i][0] = fma(p0, cr.x, ac[i][0]);
          ac[i][1] = fma(p1, cr.x, ac[i][1]);
          ac[i][2] = fma(p2, cr.x, ac[i][2]);
          ac[i][3] = fma(p3, cr.x, ac[i][3]);
          ar[i][0] = fma(fabs(p0), cr.y, ar[i][0]);
          ar[i][1] = fma(fabs(p1), cr.y, ar[i][1]);
          ar[i][2] = fma(fabs(p2), cr.y, ar[i][2]);
          ar[i][3] = fma(fabs(p3), cr.y, ar[i][3]);
        }
      }
    }
    for (; n < net.N; ++n) {
      const float4 x = ph[(size_t)n * Lp4];
      const double p0 = x.x, p1 = x.y, p2 = x.z, p3 = x.w;
#pragma unroll
      for (int i = 0; i < kBT; ++i) {
        const double2 cr = inj_all[bb[i] * net.Np + n];
        ac[i][0] = fma(p0, cr.x, ac[i][0]);
        ac[i][1] = fma(p1, cr.x, ac[i][1]);
        ac[i][2] = fma(p2, cr.x, ac[i][2]);
        ac[i][3] = fma(p3, cr.x, ac[i][3]);
        ar[i][0] = fma(fabs(p0), cr.y, ar[i][0]);
        ar[i][1] = fma(fabs(p1), cr.y, ar[i][1]);
        ar[i][2] = fma(fabs(p2), cr.y, ar[i][2]);
        ar[i][3] = fma(fabs(p3), cr.y, ar[i][3]);
      }
    }
#pragma unroll
    for (int i = 0; i < kBT; ++i) {
      if (b0 + i >= n_box) break;
      double2* out = ws_ptr<double2>(ws, lay.part2) + (size_t)(b0 + i) * net.Lp + 4 * col;
      out[0] = make_double2(ac[i][0], ar[i][0]);
      out[1] = make_double2(ac[i][1], ar[i][1]);
      out[2] = make_double2(ac[i][2], ar[i][2]);
      out[3] = make_double2(ac[i][3], ar[i][3]);
    }
  }
}

// Base flows on the float64 matrix cores (v_mfma_f64_16x16x4f64): the two
// products C_c = Phi C and C_r = |Phi| R over 32 boxes at once are dense
// GEMMs (lines x buses times buses x boxes).  One wave owns 64 lines x 32
// boxes: per step of four buses each lane loads one float4 of the transposed
// PTDF (four consecutive lines of one bus) and the (c, r) pairs of two boxes
// at that bus, and issues 16 MFMAs (four line fragments x two box fragments x
// centre and radius).  Line fragment m holds the lines l0 + 4 i + m
// (i = 0..15), so the float4's components are the lane's A operands of the
// four fragments.  The four waves of a block take the four 64-line tiles of
// the same 32 boxes, so a box's injections are read once per block from L2.
// Operand layout (lane t): A[i][k] = lane i + 16 k, B[k][j] = lane j + 16 k,
// D[i][j] = lane j + 16 (i % 4), element i / 4.  Products of a float32 factor
// and a float64 injection are accumulated in float64 (any order is covered by
// the same accumulation bound as the vector kernels).
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256, 2) void k2b_base_flows_mfma(DevNet net, void* ws, WsLayout lay, int64_t n_box,
                                                              const double2* __restrict__ inj_all) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int l0 = (blockIdx.x * 4 + w) * 64;
  if (l0 >= net.Lp) return;  // whole wave beyond the padded lines; no barrier follows
  const int64_t b0 = (int64_t)blockIdx.y * 32;
  const int i16 = lane & 15, k4 = lane >> 4;
  const int Lp4 = net.Lp / 4;
  // bus chunk blockIdx.z of k2_by (chunk starts are multiples of four, so no
  // step reaches into the next chunk; the last chunk ends at N)
  const int nb0 = blockIdx.z * lay.k2_chunk;
  const int nb1 = min(net.N, nb0 + lay.k2_chunk);
  if (nb0 >= nb1) return;
  const float4* pa = reinterpret_cast<const float4*>(net.phiT + l0 + 4 * i16);
  const double2* pb0 = inj_all + min(b0 + i16, n_box - 1) * net.Np + k4;
  const double2* pb1 = inj_all + min(b0 + 16 + i16, n_box - 1) * net.Np + k4;
  v4d ac[4][2], ar[4][2];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int j = 0; j < 2; ++j) ac[m][j] = ar[m][j] = v4d{0.0, 0.0, 0.0, 0.0};
  const int N = net.N;
  // rows past the last bus are clamped to it; their injections are zero.  The
  // next step's operands are loaded before this step's MFMAs (the scheduling
  // barrier keeps the compiler from sinking the loads to their use; the last
  // step reloads its own operands).
  const int n_last = nb0 + ((nb1 - nb0 - 1) & ~3);
  float4 xn = pa[(size_t)min(nb0 + k4, N - 1) * Lp4];
  double2 c0n = pb0[nb0], c1n = pb1[nb0];
  for (int n = nb0; n < nb1; n += 4) {
    const float4 x = xn;
    const double2 c0 = c0n, c1 = c1n;
    const int nn = min(n + 4, n_last);
    xn = pa[(size_t)min(nn + k4, N - 1) * Lp4];
    c0n = pb0[nn];
    c1n = pb1[nn];
    __builtin_amdgcn_sched_barrier(0);
    const double a[4] = {(double)x.x, (double)x.y, (double)x.z, (double)x.w};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      ac[m][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], c0.x, ac[m][0], 0, 0, 0);
      ac[m][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], c1.x, ac[m][1], 0, 0, 0);
      ar[m][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(a[m]), c0.y, ar[m][0], 0, 0, 0);
      ar[m][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(a[m]), c1.y, ar[m][1], 0, 0, 0);
    }
  }
  // element r of lane t is row i = 4 r + t / 16 of each fragment: for box
  // b0 + 16 j + (t % 16), fragment m gives line l0 + 4 i + m, so the lane
  // holds four runs of four consecutive lines, l0 + 16 r + 4 (t / 16) + m
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int64_t b = b0 + 16 * j + i16;
    if (b < n_box) {
      double2* out = ws_ptr<double2>(ws, lay.part2) + ((size_t)b * lay.k2_by + blockIdx.z) * net.Lp + l0 + 4 * k4;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int m = 0; m < 4; ++m) out[16 * r + m] = make_double2(ac[m][j][r], ar[m][j][r]);
    }
  }
}

// Outage sweep for kBT boxes x 256 lines per wave over one block row of outages.
// SIDES as in k3_elem: one-sided calls compute only the penalty bound they need.
//
// Block order: blocks are dealt to the eight XCDs in turn, each XCD with its
// own L2.  When the outage factors exceed the last-level cache (lay.k3_xcd),
// the linear block index is remapped so that each XCD takes a contiguous
// range of (line tile, outage block) tiles with all their box tiles: the
// blocks resident on one XCD then stream the same factor rows, fetched into
// its L2 once (8316 buses, 256 boxes: 5.05 -> 4.61 ms).  With the factors in
// the last-level cache the plain order is faster (2000 buses: 27.3 against
// 28.4 ms).  The order changes no sum.
template <int SIDES, int kBT>
__global__ __launch_bounds__(256) void k3b_contingency(DevNet net, void* ws, WsLayout lay, int64_t n_box) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  if (lay.k3_xcd) {
    const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z, nb = gx * gy * gz;
    const unsigned bid = bx + gx * (by + gy * bz);
    // XCD j = bid % 8 takes positions [start_j, start_j + count_j) of the
    // tile-major order (count_j = nb / 8, plus one for the first nb % 8)
    const unsigned j = bid & 7u, li = bid >> 3, q = nb >> 3, r = nb & 7u;
    const unsigned p = (j < r ? j * (q + 1u) : r * (q + 1u) + (j - r) * q) + li;
    bz = p % gz;
    const unsigned d = p / gz;
    bx = d % gx;
    by = d / gx;
  }
  const int64_t b0 = ((int64_t)bz * 4 + w) * kBT;
  if (b0 >= n_box) return;
  const int col = bx * 64 + lane;
  const int Lp4 = net.Lp / 4;
  const int k0 = by * lay.k3_kper;
  const int k1 = min(net.K, k0 + lay.k3_kper);
  int64_t bb[kBT];
#pragma unroll
  for (int i = 0; i < kBT; ++i) bb[i] = min(b0 + i, n_box - 1);
  double acc_hi[kBT], acc_lo[kBT];
#pragma unroll
  for (int i = 0; i < kBT; ++i) acc_hi[i] = acc_lo[i] = 0.0;
  if (col < Lp4) {
    float4 c4[kBT], h4[kBT], g4[kBT];
    const int4* cd[kBT];
    const float4 e4 = reinterpret_cast<const float4*>(net.line_eps)[col];
#pragma unroll
    for (int i = 0; i < kBT; ++i) {
      const double* bs = ws_ptr<double>(ws, lay.box) + bb[i] * kBoxSlots;
      const float vmax = __uint_as_float(*reinterpret_cast<const unsigned int*>(bs + kVmax));
      c4[i] = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lc) + bb[i] * net.Lp)[col];
      const float4 h = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lh) + bb[i] * net.Lp)[col];
      const float4 g = reinterpret_cast<const float4*>(ws_ptr<float>(ws, lay.lg) + bb[i] * net.Lp)[col];
      const float ex = next_up_f32(e4.x * vmax), ey = next_up_f32(e4.y * vmax);
      const float ez = next_up_f32(e4.z * vmax), ew = next_up_f32(e4.w * vmax);
      h4[i] = make_float4(add_ru(h.x, ex), add_ru(h.y, ey), add_ru(h.z, ez), add_ru(h.w, ew));
      g4[i] = make_float4(add_ru(g.x, ex), add_ru(g.y, ey), add_ru(g.z, ez), add_ru(g.w, ew));
      cd[i] = ws_ptr<int4>(ws, lay.ctg) + bb[i] * net.K;
    }
    const float4* lam = reinterpret_cast<const float4*>(net.lodf) + col;
    int k = k0;
    const int n4 = (k1 - k0) / 4;
    if (n4 > 0) {
      // per-outage (centre, padded radius) of the next four outages are
      // loaded (scalar loads) before this step's arithmetic, so the step
      // waits on scalar memory once instead of once per box (the last step
      // reloads its own outages)
      const int k_last = k0 + 4 * (n4 - 1);
      int2 qn[kBT][4];
#pragma unroll
      for (int i = 0; i < kBT; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int4 d = cd[i][k0 + u];
          qn[i][u] = make_int2(d.y, d.z);
        }
      for (; k <= k_last; k += 4) {
        int2 q[kBT][4];
#pragma unroll
        for (int i = 0; i < kBT; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) q[i][u] = qn[i][u];
        const int kn = min(k + 4, k_last);
        float4 x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = lam[(size_t)(k + u) * Lp4];
#pragma unroll
        for (int i = 0; i < kBT; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int4 d = cd[i][kn + u];
            qn[i][u] = make_int2(d.y, d.z);
          }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < kBT; ++i) {
          k3_pair<SIDES>(x[0], make_int4(0, q[i][0].x, q[i][0].y, 0), x[1], make_int4(0, q[i][1].x, q[i][1].y, 0),
                         c4[i], h4[i], g4[i], acc_hi[i], acc_lo[i]);
          k3_pair<SIDES>(x[2], make_int4(0, q[i][2].x, q[i][2].y, 0), x[3], make_int4(0, q[i][3].x, q[i][3].y, 0),
                         c4[i], h4[i], g4[i], acc_hi[i], acc_lo[i]);
        }
      }
    }
    for (; k < k1; ++k) {
      const float4 x0 = lam[(size_t)k * Lp4];
#pragma unroll
      for (int i = 0; i < kBT; ++i) {
        const int4 d0 = cd[i][k];
        const float cc0 = __int_as_float(d0.y), rk0 = __int_as_float(d0.z);
        float a0, a1, a2, a3, q0, q1, q2, q3;
        k3_elem<SIDES>(x0.x, cc0, rk0, c4[i].x, h4[i].x, g4[i].x, a0, q0);
        k3_elem<SIDES>(x0.y, cc0, rk0, c4[i].y, h4[i].y, g4[i].y, a1, q1);
        k3_elem<SIDES>(x0.z, cc0, rk0, c4[i].z, h4[i].z, g4[i].z, a2, q2);
        k3_elem<SIDES>(x0.w, cc0, rk0, c4[i].w, h4[i].w, g4[i].w, a3, q3);
        if (SIDES & 2) acc_hi[i] += (double)((a0 + a1) + (a2 + a3));
        if (SIDES & 1) acc_lo[i] += (double)((q0 + q1) + (q2 + q3));
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kBT; ++i) {
    const double hs = wave_sum(acc_hi[i]);
    const double ls = wave_sum(acc_lo[i]);
    if (lane == 0 && b0 + i < n_box) {
      double2* p3 = ws_ptr<double2>(ws, lay.p3) + (b0 + i) * lay.n_p3;
      p3[by * gridDim.x + bx] = make_double2(hs, ls);
    }
  }
}

// Outage rows of the box-tiled sweep chosen by rule: enough waves in flight,
// at least 32 outages per row, and k3_bx * rows a multiple of 8 when that is
// near (blocks that share an outage tile then share an XCD).
int batched_rows_rule(const DevNet& net, int k3_bx, int64_t groups) {
  int rows = 1;
  const int max_rows = std::max(1, net.K / 32);
  while (rows < max_rows && (int64_t)k3_bx * rows * groups * 4 < 16384) rows *= 2;
  rows = std::min(rows, max_rows);
  for (int r = rows; r <= std::min(max_rows, rows * 2); ++r)
    if ((k3_bx * r) % 8 == 0) {
      rows = r;
      break;
    }
  return rows;
}

void plan_batched(const DevNet& net, int64_t n_box, WsLayout& lay, const Tune& t) {
  const int lp4 = net.Lp / 4;
  lay.batched = 1;
  lay.n_p1 = (std::max(net.Np, net.X) + 63) / 64;
  lay.k2_bx = (lp4 + 63) / 64;
  lay.k2_gx = (lay.k2_bx + 7) / 8 * 8;  // blocks of one line tile share an XCD
  // outage factors larger than the last-level cache: XCD-aware sweep order
  lay.k3_xcd = (int64_t)net.K * net.Lp * 4 > (128ll << 20) ? 1 : 0;
  lay.k2_by = 1;
  lay.k2_chunk = net.N;
  if (t.k2b_mfma) {
    // split the buses when the line x box tiles alone give few blocks; each
    // chunk writes its own partial sums, which the line epilogue adds
    const int64_t blocks = (int64_t)((net.Lp / 64 + 3) / 4) * ((n_box + 31) / 32);
    int by = (int)std::min<int64_t>(8, (2048 + blocks - 1) / blocks);
    by = std::max(1, std::min(by, net.N / 256));
    if (t.k2_by > 0) by = std::min(t.k2_by, std::max(1, net.N / 4));
    lay.k2_chunk = ((net.N + by - 1) / by + 3) & ~3;
    lay.k2_by = (net.N + lay.k2_chunk - 1) / lay.k2_chunk;
  }
  lay.n_p2 = (net.L + 63) / 64;
  lay.k3_bt = t.k3_bt;
  const int64_t nbt = (n_box + lay.k3_bt - 1) / lay.k3_bt;
  const int64_t groups = (nbt + 3) / 4;
  lay.k3_bx = (lp4 + 63) / 64;
  int rows = batched_rows_rule(net, lay.k3_bx, groups);
  if (t.k3_rows > 0) rows = std::min(t.k3_rows, std::max(1, net.K));
  if (t.k3_xcd >= 0) lay.k3_xcd = t.k3_xcd;
  lay.k3_by = rows;
  lay.k3_kper = net.K > 0 ? (net.K + rows - 1) / rows : 0;
  lay.n_p3 = net.K > 0 ? lay.k3_bx * rows : 0;
  lay.k2_nc = 0;
  lay.k3_kc = lay.k3_kper;
  lay.k2_mfma = t.k2b_mfma;
}

hipError_t launch_batched_sweeps(const DevNet& net, int64_t n_box, void* ws, const WsLayout& lay, hipStream_t s,
                                 KernelTimer* tm, int phase) {
  const int64_t nbt = (n_box + kBT - 1) / kBT;
  const unsigned groups = (unsigned)((nbt + 3) / 4);
  const int64_t nbt3 = (n_box + lay.k3_bt - 1) / lay.k3_bt;
  const unsigned groups3 = (unsigned)((nbt3 + 3) / 4);
  if (phase == 0) {
    const int t = tm->start(5, s);
    const double2* inj = reinterpret_cast<const double2*>(static_cast<char*>(ws) + lay.inj);
    if (lay.k2_mfma)
      hipLaunchKernelGGL(k2b_base_flows_mfma,
                         dim3((net.Lp / 64 + 3) / 4, (unsigned)((n_box + 31) / 32), (unsigned)lay.k2_by), dim3(256),
                         0, s, net, ws, lay, n_box, inj);
    else
      hipLaunchKernelGGL(k2b_base_flows, dim3(lay.k2_gx, groups), dim3(256), 0, s, net, ws, lay, n_box, inj);
    tm->stop(t, s);
  } else if (net.K > 0 && lay.fscreen) {
    // the line screen, then the sweep over the marked lines only
    int t = tm->start(15, s);
    launch_line_screen(net, n_box, ws, lay,
                       lay.sides == 1 ? kScreenForwardLower : lay.sides == 2 ? kScreenForwardUpper : kScreenForwardBoth,
                       s);
    tm->stop(t, s);
    t = tm->start(6, s);
    launch_screened_forward_sweep(net, n_box, ws, lay, lay.sides, s);
    tm->stop(t, s);
  } else if (net.K > 0) {
    const int t = tm->start(6, s);
    const dim3 grid(lay.k3_bx, lay.k3_by, groups3);
    auto go = [&](auto bt) {
      constexpr int BT = decltype(bt)::value;
      if (lay.sides == 1)
        hipLaunchKernelGGL((k3b_contingency<1, BT>), grid, dim3(256), 0, s, net, ws, lay, n_box);
      else if (lay.sides == 2)
        hipLaunchKernelGGL((k3b_contingency<2, BT>), grid, dim3(256), 0, s, net, ws, lay, n_box);
      else
        hipLaunchKernelGGL((k3b_contingency<3, BT>), grid, dim3(256), 0, s, net, ws, lay, n_box);
    };
    if (lay.k3_bt == 2)
      go(std::integral_constant<int, 2>());
    else if (lay.k3_bt == 8)
      go(std::integral_constant<int, 8>());
    else
      go(std::integral_constant<int, 4>());
    tm->stop(t, s);
  }
  return hipGetLastError();
}

}  // namespace ibp
