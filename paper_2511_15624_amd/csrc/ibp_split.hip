// Gradient-ranked bisection of input boxes (branching on the input domain).
//
// The paper bounds max f over a box with IBP and names branch and bound as the
// way to tighten such bounds (Sec. I, Sec. V).  Here every root box keeps a
// list of leaf boxes that partition it; one round, per root:
//   1. select the leaf with the largest upper bound f_hi,
//   2. split it at the midpoint of the coordinate j maximising
//      (d f_hi / d hi_j - d f_hi / d lo_j) * r_j  (= d f_hi / d r_j * r_j),
//   3. the caller bounds the two children and their centre points; the root's
//      upper bound is the largest leaf f_hi and its lower bound on max f the
//      largest certified value f_lo at a centre point.
// Leaves of root r live in slots r*S .. r*S + S-1; slots >= n_used are empty.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "ibp_kernels.h"

namespace ibp {

// One wave per root: leaf with the largest f_hi among the used slots (ties to
// the lowest slot; a NaN leaf only wins when every leaf is NaN, then slot 0).
// The lanes then copy it to sel_lo/sel_hi (row r), coalesced.
__global__ __launch_bounds__(64) void split_select(int64_t R, int S, int n_used, int X,
                                                   const float* __restrict__ leaf_lo,
                                                   const float* __restrict__ leaf_hi,
                                                   const double* __restrict__ leaf_fhi, int64_t* __restrict__ sel,
                                                   float* __restrict__ sel_lo, float* __restrict__ sel_hi) {
  const int64_t r = blockIdx.x;
  const int lane = threadIdx.x;
  double bv = -INFINITY;
  int bq = -1;
  for (int q = lane; q < n_used; q += 64) {
    const double v = leaf_fhi[r * S + q];
    if (v == v && (bq < 0 || v > bv)) {
      bv = v;
      bq = q;
    }
  }
  for (int m = 32; m >= 1; m >>= 1) {
    const double ov = __shfl_xor(bv, m, 64);
    const int oq = __shfl_xor(bq, m, 64);
    if (oq >= 0 && (bq < 0 || ov > bv || (ov == bv && oq < bq))) {
      bv = ov;
      bq = oq;
    }
  }
  const int64_t best = r * S + (bq < 0 ? 0 : bq);
  if (lane == 0) sel[r] = best;
  for (int j = lane; j < X; j += 64) {
    sel_lo[r * X + j] = leaf_lo[best * X + j];
    sel_hi[r * X + j] = leaf_hi[best * X + j];
  }
}

// One wave per root: split coordinate from the gradient, children written to
// slot sel[r] (first half) and slot r*S + n_used (second half); also the two
// children's centre points as zero-width boxes (rows 2r, 2r+1 of cen_*),
// and the children themselves (rows 2r, 2r+1 of kid_*).
__global__ __launch_bounds__(64) void split_bisect(int64_t R, int S, int n_used, int X,
                                                   float* __restrict__ leaf_lo, float* __restrict__ leaf_hi,
                                                   const int64_t* __restrict__ sel,
                                                   const float* __restrict__ sel_lo,
                                                   const float* __restrict__ sel_hi,
                                                   const double* __restrict__ g_lo,
                                                   const double* __restrict__ g_hi,
                                                   float* __restrict__ kid_lo, float* __restrict__ kid_hi,
                                                   float* __restrict__ cen) {
  const int64_t r = blockIdx.x;
  const int lane = threadIdx.x;
  const float* lo = sel_lo + r * X;
  const float* hi = sel_hi + r * X;
  double best = -1.0;
  int bj = -1;
  for (int j = lane; j < X; j += 64) {
    const double w = 0.5 * ((double)hi[j] - (double)lo[j]);
    if (!(w > 0.0)) continue;
    const float mid = 0.5f * lo[j] + 0.5f * hi[j];
    if (!(mid > lo[j] && mid < hi[j])) continue;  // no float32 strictly inside
    const double score = (g_hi[r * X + j] - g_lo[r * X + j]) * w;
    if (score > best || bj < 0) {
      best = score;
      bj = j;
    }
  }
  // wave argmax (ties to the lowest index)
  for (int m = 32; m >= 1; m >>= 1) {
    const double ob = __shfl_xor(best, m, 64);
    const int oj = __shfl_xor(bj, m, 64);
    if (oj >= 0 && (bj < 0 || ob > best || (ob == best && oj < bj))) {
      best = ob;
      bj = oj;
    }
  }
  const int64_t s0 = sel[r];
  const int64_t s1 = r * S + n_used;
  float mid = 0.0f;
  if (bj >= 0) mid = 0.5f * lo[bj] + 0.5f * hi[bj];
  for (int j = lane; j < X; j += 64) {
    const float l = lo[j], h = hi[j];
    // first child [l, mid] on coordinate bj, second [mid, h]; a leaf that
    // cannot be split keeps itself and gets an identical twin
    const float h0 = (j == bj) ? mid : h;
    const float l1 = (j == bj) ? mid : l;
    leaf_lo[s0 * X + j] = l;
    leaf_hi[s0 * X + j] = h0;
    leaf_lo[s1 * X + j] = l1;
    leaf_hi[s1 * X + j] = h;
    kid_lo[(2 * r) * X + j] = l;
    kid_hi[(2 * r) * X + j] = h0;
    kid_lo[(2 * r + 1) * X + j] = l1;
    kid_hi[(2 * r + 1) * X + j] = h;
    cen[(2 * r) * X + j] = 0.5f * l + 0.5f * h0;
    cen[(2 * r + 1) * X + j] = 0.5f * l1 + 0.5f * h;
  }
}

// One thread per root: scatter the children's f_hi, refresh the root's upper
// bound (the smaller of its previous value and the largest leaf f_hi) and
// lower bound (largest certified centre value).
__global__ void split_update(int64_t R, int S, int n_used_after, const int64_t* __restrict__ sel,
                             const double* __restrict__ kid_fhi, const double* __restrict__ cen_flo,
                             double* __restrict__ leaf_fhi, double* __restrict__ root_ub,
                             double* __restrict__ root_lb) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= R) return;
  leaf_fhi[sel[r]] = kid_fhi[2 * r];
  leaf_fhi[r * S + n_used_after - 1] = kid_fhi[2 * r + 1];
  double ub = -INFINITY;
  for (int q = 0; q < n_used_after; ++q) ub = fmax(ub, leaf_fhi[r * S + q]);
  root_ub[r] = fmin(root_ub[r], ub);  // both bound max f over the root; keep the smaller
  root_lb[r] = fmax(root_lb[r], fmax(cen_flo[2 * r], cen_flo[2 * r + 1]));
}

hipError_t launch_split_select(int64_t R, int S, int n_used, int X, const float* leaf_lo, const float* leaf_hi,
                               const double* leaf_fhi, int64_t* sel, float* sel_lo, float* sel_hi, hipStream_t s) {
  hipLaunchKernelGGL(split_select, dim3((unsigned)R), dim3(64), 0, s, R, S, n_used, X, leaf_lo, leaf_hi, leaf_fhi,
                     sel, sel_lo, sel_hi);
  return hipGetLastError();
}

hipError_t launch_split_bisect(int64_t R, int S, int n_used, int X, float* leaf_lo, float* leaf_hi,
                               const int64_t* sel, const float* sel_lo, const float* sel_hi, const double* g_lo,
                               const double* g_hi, float* kid_lo, float* kid_hi, float* cen, hipStream_t s) {
  hipLaunchKernelGGL(split_bisect, dim3((unsigned)R), dim3(64), 0, s, R, S, n_used, X, leaf_lo, leaf_hi, sel,
                     sel_lo, sel_hi, g_lo, g_hi, kid_lo, kid_hi, cen);
  return hipGetLastError();
}

hipError_t launch_split_update(int64_t R, int S, int n_used_after, const int64_t* sel, const double* kid_fhi,
                               const double* cen_flo, double* leaf_fhi, double* root_ub, double* root_lb,
                               hipStream_t s) {
  hipLaunchKernelGGL(split_update, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, R, S, n_used_after, sel,
                     kid_fhi, cen_flo, leaf_fhi, root_ub, root_lb);
  return hipGetLastError();
}

}  // namespace ibp
