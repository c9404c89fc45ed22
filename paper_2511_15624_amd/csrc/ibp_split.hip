// Branch and bound over input boxes (branching on the input domain).
//
// The paper bounds max f over a box with IBP, names branch and bound as the
// way to tighten such bounds (Sec. I, Sec. V), and screens instances for
// max f < 0 (welfare-negative or infeasible, Sec. III-D eq. (inf-or-wn)).
// Every root box keeps a list of leaf boxes that partition it; one round, for
// the roots in an active list:
//   1. select the leaf with the largest upper bound f_hi,
//   2. split it at the midpoint of the coordinate j maximising
//      (d f_hi / d hi_j - d f_hi / d lo_j) * r_j  (= d f_hi / d r_j * r_j),
//   3. the caller bounds the two children and a set of points inside them
//      (zero-width boxes, so f_lo there is a certified value of f at a point);
//      the root's upper bound becomes min(previous, largest leaf f_hi), its
//      lower bound on max f the largest certified point value, and the point
//      that attains it is kept,
//   4. screening marks roots whose sign of max f is certified (upper bound
//      < 0: welfare-negative; lower bound >= 0: not) or whose gap is closed,
//      and compacts the list of roots still open.
// Leaves of root r live in slots r*S .. r*S + S-1; slots >= n_leaf[r] are
// empty.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "ibp_kernels.h"

namespace ibp {

__device__ __forceinline__ int64_t root_of(const int64_t* roots, int64_t i) { return roots ? roots[i] : i; }

// One wave per active root: leaf with the largest f_hi among the used slots
// (ties to the lowest slot; a NaN leaf only wins when every leaf is NaN, then
// slot 0).  The lanes copy it to sel_lo/sel_hi (row i), coalesced.
__global__ __launch_bounds__(64) void split_select(int64_t n, const int64_t* __restrict__ roots, int S,
                                                   const int* __restrict__ n_leaf, int X,
                                                   const float* __restrict__ leaf_lo,
                                                   const float* __restrict__ leaf_hi,
                                                   const double* __restrict__ leaf_fhi, int64_t* __restrict__ sel,
                                                   float* __restrict__ sel_lo, float* __restrict__ sel_hi) {
  const int64_t i = blockIdx.x;
  const int64_t r = root_of(roots, i);
  const int lane = threadIdx.x;
  const int used = min(S, max(1, n_leaf[r]));
  double bv = -INFINITY;
  int bq = -1;
  for (int q = lane; q < used; q += 64) {
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
  if (lane == 0) sel[i] = best;
  for (int j = lane; j < X; j += 64) {
    sel_lo[i * X + j] = leaf_lo[best * X + j];
    sel_hi[i * X + j] = leaf_hi[best * X + j];
  }
}

// One wave per active root: split coordinate from the gradient, children
// written to slot sel[i] (first half) and slot r*S + n_leaf[r] (second half,
// only while n_leaf[r] < S); also the children themselves (rows 2i, 2i+1 of
// kid_*) and their centre points (rows 2i, 2i+1 of cen).
__global__ __launch_bounds__(64) void split_bisect(int64_t n, const int64_t* __restrict__ roots, int S,
                                                   const int* __restrict__ n_leaf, int X,
                                                   float* __restrict__ leaf_lo, float* __restrict__ leaf_hi,
                                                   const int64_t* __restrict__ sel,
                                                   const float* __restrict__ sel_lo,
                                                   const float* __restrict__ sel_hi,
                                                   const double* __restrict__ g_lo,
                                                   const double* __restrict__ g_hi,
                                                   float* __restrict__ kid_lo, float* __restrict__ kid_hi,
                                                   float* __restrict__ cen) {
  const int64_t i = blockIdx.x;
  const int64_t r = root_of(roots, i);
  const int lane = threadIdx.x;
  const float* lo = sel_lo + i * X;
  const float* hi = sel_hi + i * X;
  double best = -1.0;
  int bj = -1;
  for (int j = lane; j < X; j += 64) {
    const double w = 0.5 * ((double)hi[j] - (double)lo[j]);
    if (!(w > 0.0)) continue;
    const float mid = 0.5f * lo[j] + 0.5f * hi[j];
    if (!(mid > lo[j] && mid < hi[j])) continue;  // no float32 strictly inside
    const double score = (g_hi[i * X + j] - g_lo[i * X + j]) * w;
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
  const int nl = n_leaf[r];
  const bool room = nl >= 1 && nl < S;
  const int64_t s0 = sel[i];
  const int64_t s1 = r * S + nl;
  float mid = 0.0f;
  if (bj >= 0 && room) mid = 0.5f * lo[bj] + 0.5f * hi[bj];
  const int cut = room ? bj : -1;  // a full root gets two copies of its leaf
  for (int j = lane; j < X; j += 64) {
    const float l = lo[j], h = hi[j];
    // first child [l, mid] on coordinate cut, second [mid, h]; a leaf that
    // cannot be split keeps itself and gets an identical twin
    const float h0 = (j == cut) ? mid : h;
    const float l1 = (j == cut) ? mid : l;
    if (room) {
      leaf_lo[s0 * X + j] = l;
      leaf_hi[s0 * X + j] = h0;
      leaf_lo[s1 * X + j] = l1;
      leaf_hi[s1 * X + j] = h;
    }
    kid_lo[(2 * i) * X + j] = l;
    kid_hi[(2 * i) * X + j] = h0;
    kid_lo[(2 * i + 1) * X + j] = l1;
    kid_hi[(2 * i + 1) * X + j] = h;
    cen[(2 * i) * X + j] = 0.5f * l + 0.5f * h0;
    cen[(2 * i + 1) * X + j] = 0.5f * l1 + 0.5f * h;
  }
}

// One wave per active root: scatter the children's f_hi, refresh the root's
// upper bound (the smaller of its previous value and the largest leaf f_hi)
// and lower bound (largest certified point value; the point is copied to
// root_x when it improves), and count the new leaf.
__global__ __launch_bounds__(64) void split_update(int64_t n, const int64_t* __restrict__ roots, int S,
                                                   int* __restrict__ n_leaf, const int64_t* __restrict__ sel,
                                                   const double* __restrict__ kid_fhi, int pts,
                                                   const double* __restrict__ point_flo,
                                                   const float* __restrict__ points, int X,
                                                   double* __restrict__ leaf_fhi, double* __restrict__ root_ub,
                                                   double* __restrict__ root_lb, float* __restrict__ root_x) {
  const int64_t i = blockIdx.x;
  const int64_t r = root_of(roots, i);
  const int lane = threadIdx.x;
  const int nl = n_leaf[r];
  const bool room = nl >= 1 && nl < S;
  const int after = room ? nl + 1 : nl;
  double ub = -INFINITY;
  for (int q = lane; q < after; q += 64) {
    double v;
    if (room && r * S + q == sel[i])
      v = kid_fhi[2 * i];
    else if (room && q == nl)
      v = kid_fhi[2 * i + 1];
    else
      v = leaf_fhi[r * S + q];
    ub = fmax(ub, v);
  }
  for (int m = 32; m >= 1; m >>= 1) ub = fmax(ub, __shfl_xor(ub, m, 64));
  // best certified point (ties to the lowest index)
  double bv = -INFINITY;
  int bp = -1;
  for (int p = lane; p < pts; p += 64) {
    const double v = point_flo[i * pts + p];
    if (v == v && (bp < 0 || v > bv)) {
      bv = v;
      bp = p;
    }
  }
  for (int m = 32; m >= 1; m >>= 1) {
    const double ov = __shfl_xor(bv, m, 64);
    const int op = __shfl_xor(bp, m, 64);
    if (op >= 0 && (bp < 0 || ov > bv || (ov == bv && op < bp))) {
      bv = ov;
      bp = op;
    }
  }
  const double lb_prev = root_lb[r];
  const bool better = bp >= 0 && (bv > lb_prev || !(lb_prev == lb_prev));
  if (better && root_x)
    for (int j = lane; j < X; j += 64) root_x[r * X + j] = points[((int64_t)i * pts + bp) * X + j];
  if (lane == 0) {
    if (room) {
      leaf_fhi[sel[i]] = kid_fhi[2 * i];
      leaf_fhi[r * S + nl] = kid_fhi[2 * i + 1];
      n_leaf[r] = nl + 1;
    }
    root_ub[r] = fmin(root_ub[r], ub);  // both bound max f over the root; keep the smaller
    if (better) root_lb[r] = bv;
  }
}

// Status of every root and the compacted list of open roots (one block; a
// block-wide scan keeps the list in ascending order).
//   1: upper bound < 0 (max f < 0 certified: welfare-negative or infeasible)
//   2: lower bound >= 0 (a point with f >= 0 is certified)
//   3: gap closed: ub - lb <= rel_tol * max(1, |ub|)
//   4: a bound is NaN (invalid box)
//   0: open
__global__ __launch_bounds__(1024) void split_screen(int64_t R, const double* __restrict__ root_ub,
                                                     const double* __restrict__ root_lb, double rel_tol,
                                                     int* __restrict__ status, int64_t* __restrict__ open_roots,
                                                     int64_t* __restrict__ n_open) {
  __shared__ int wsum[16];
  __shared__ int64_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t c0 = 0; c0 < R; c0 += 1024) {
    const int64_t r = c0 + threadIdx.x;
    int st = -1;
    if (r < R) {
      const double ub = root_ub[r], lb = root_lb[r];
      if (!(ub == ub) || !(lb == lb))
        st = 4;
      else if (ub < 0.0)
        st = 1;
      else if (lb >= 0.0)
        st = 2;
      else if (ub - lb <= rel_tol * fmax(1.0, fabs(ub)))
        st = 3;
      else
        st = 0;
      status[r] = st;
    }
    const int open = st == 0 ? 1 : 0;
    // inclusive scan within the wave, then across the 16 waves
    int x = open;
    for (int m = 1; m < 64; m <<= 1) {
      const int y = __shfl_up(x, m, 64);
      if (lane >= m) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int off = 0;
    for (int q = 0; q < w; ++q) off += wsum[q];
    int total = 0;
    for (int q = 0; q < 16; ++q) total += wsum[q];
    if (open) open_roots[base + off + x - 1] = r;
    __syncthreads();
    if (threadIdx.x == 0) base += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_open = base;
}

hipError_t launch_split_select(int64_t n, const int64_t* roots, int S, const int* n_leaf, int X,
                               const float* leaf_lo, const float* leaf_hi, const double* leaf_fhi, int64_t* sel,
                               float* sel_lo, float* sel_hi, hipStream_t s) {
  hipLaunchKernelGGL(split_select, dim3((unsigned)n), dim3(64), 0, s, n, roots, S, n_leaf, X, leaf_lo, leaf_hi,
                     leaf_fhi, sel, sel_lo, sel_hi);
  return hipGetLastError();
}

hipError_t launch_split_bisect(int64_t n, const int64_t* roots, int S, const int* n_leaf, int X, float* leaf_lo,
                               float* leaf_hi, const int64_t* sel, const float* sel_lo, const float* sel_hi,
                               const double* g_lo, const double* g_hi, float* kid_lo, float* kid_hi, float* cen,
                               hipStream_t s) {
  hipLaunchKernelGGL(split_bisect, dim3((unsigned)n), dim3(64), 0, s, n, roots, S, n_leaf, X, leaf_lo, leaf_hi,
                     sel, sel_lo, sel_hi, g_lo, g_hi, kid_lo, kid_hi, cen);
  return hipGetLastError();
}

hipError_t launch_split_update(int64_t n, const int64_t* roots, int S, int* n_leaf, const int64_t* sel,
                               const double* kid_fhi, int pts, const double* point_flo, const float* points, int X,
                               double* leaf_fhi, double* root_ub, double* root_lb, float* root_x, hipStream_t s) {
  hipLaunchKernelGGL(split_update, dim3((unsigned)n), dim3(64), 0, s, n, roots, S, n_leaf, sel, kid_fhi, pts,
                     point_flo, points, X, leaf_fhi, root_ub, root_lb, root_x);
  return hipGetLastError();
}

hipError_t launch_split_screen(int64_t R, const double* root_ub, const double* root_lb, double rel_tol, int* status,
                               int64_t* open_roots, int64_t* n_open, hipStream_t s) {
  hipLaunchKernelGGL(split_screen, dim3(1), dim3(1024), 0, s, R, root_ub, root_lb, rel_tol, status, open_roots,
                     n_open);
  return hipGetLastError();
}

}  // namespace ibp
