// Launchers of the HIP kernels (defined in the .hip sources).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>

#include <vector>

#include "ibp_device.h"

namespace ibp {

// Optional per-kernel event timing (see ibp_set_kernel_timing).
struct KernelTimer {
  bool enabled = false;
  struct Rec {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  // Records an event before a launch; returns the index to close with stop().
  int start(int id, hipStream_t s) {
    if (!enabled) return -1;
    Rec r{id, nullptr, nullptr};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void stop(int idx, hipStream_t s) {
    if (idx >= 0) (void)hipEventRecord(recs[idx].b, s);
  }
  // Launches `kernel`; while timing is enabled the start and end are recorded
  // by the dispatch itself (no event packets queued around it, so the
  // duration is the kernel's own).
  template <typename K, typename... A>
  void launch(int id, K kernel, dim3 grid, dim3 block, hipStream_t s, A... args) {
    Rec r{id, nullptr, nullptr};
    if (enabled && (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess)) r.a = r.b = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, r.a, r.b, 0, args...);
    if (r.a && r.b) recs.push_back(r);
  }
};

// Tile parameters of the streaming kernels (chosen by the autotuner or the
// IBP_TILE environment variable, e.g. "k2nc=64,k3kc=32,k2b=0,ckb=4").
struct Tune {
  int k2_nc = 128;  // buses per wave in the base-flow sweep: 32, 64, 128, 256 or 512
  int k3_kc = 16;   // outages per block in the outage sweep: 16, 32, 64 or 128
  int k2b_mfma = 1; // box-tiled base flows on the float64 matrix cores (0: vector FMA)
  int chord_nb = 1; // boxes per lane in the box-tiled chord-relaxation sweep: 1, 2 or 4
  // box-tiled forward (the autotuner's batched candidates)
  int k3_bt = 4;    // boxes per wave in the box-tiled outage sweep: 2, 4 or 8
  int k3_rows = 0;  // outage rows of that sweep (0: the rule of batched_rows_rule)
  int k3_xcd = -1;  // its XCD-aware block order: 0 off, 1 on, -1 by cache size
  int k2_by = 0;    // bus chunks of the matrix-core base flows (0: by rule)
  int k5_sparse = 1; // box-tiled gradient of f_hi: screened sweep over candidate lines (0: dense sweep)
  int k3_sparse = 1; // box-tiled one-sided forward: screened sweep over candidate lines (0: dense sweep)
  int k3_scr = 0;    // box-tiled calls bounding f_lo screen the upper penalties (as IBP_F_SCREEN_UPPER)
};

// Line screen of the one-sided sweeps (see ibp_screen.hip): boxes per tile
// (the tile shares its marked lines and every factor load), outages per lane
// of the screened sweeps, and the mask words per tile they stage in LDS.
constexpr int kScreenBoxes = 4;
constexpr int kSparseQ = 4;
constexpr int kSparseMaxWords = 512;  // networks up to 32768 lines
// What a screen bounds: the lower penalties with the backward's unpadded
// radii (gradient of f_hi), or the forward's padded lower / upper penalties
// (one-sided bound f_hi / f_lo).
// kScreenForwardBoth: the upper-penalty screen of a two-sided forward (a line
// with no active upper penalty has no active lower one either), recording
// both sides' terms.
enum ScreenMode : int {
  kScreenBackwardLower = 0,
  kScreenForwardLower = 1,
  kScreenForwardUpper = 2,
  kScreenForwardBoth = 3
};
// Floats per (tile, line) record: the four boxes' centres and two radius terms.
constexpr int kScreenRecFloats = 12;
// The screen's regions are laid out and the network fits the sweeps' LDS masks.
inline bool screen_fits(const DevNet& net, const WsLayout& lay) {
  return lay.k5s_tiles > 0 && net.Lp / 64 <= kSparseMaxWords;
}
// Marks, per tile of kScreenBoxes boxes, the lines that can hold an active
// penalty of the mode's kind (masks, line records; for the backward also
// zeroed line counters).
void launch_line_screen(const DevNet& net, int64_t n_box, void* ws, const WsLayout& lay, int mode, hipStream_t s);
// The box-tiled forward sweep over the marked lines (sides 1: lower
// penalties, 2: upper, 3: both), after launch_line_screen with the matching
// mode; writes the outage-penalty partials that the finalize reads.
void launch_screened_forward_sweep(const DevNet& net, int64_t n_box, void* ws, const WsLayout& lay, int sides,
                                   hipStream_t s);
bool tune_valid(const Tune& t);
bool tune_batched_valid(const Tune& t);
int batched_rows_rule(const DevNet& net, int k3_bx, int64_t groups);

// Grid shapes and partial-sum counts of the single-box-per-slice forward path.
void plan_single(const DevNet& net, int64_t n_box, WsLayout& lay, const Tune& t);

// Box-tiled plan (n_box >= kBatchMin and no IBP_F_PLAIN).
void plan_batched(const DevNet& net, int64_t n_box, WsLayout& lay, const Tune& t);
constexpr int64_t kBatchMin = 4;

// Batched base-flow sweep (phase 0) or outage sweep (phase 1).
hipError_t launch_batched_sweeps(const DevNet& net, int64_t n_box, void* ws, const WsLayout& lay, hipStream_t s,
                                 KernelTimer* tm, int phase);

// Forward bounds for n_box boxes with the plan in `lay` (single or batched).
hipError_t launch_forward(const DevNet& net, int64_t n_box, const float* lo, const float* hi, double* f_lo,
                          double* f_hi, double* terms, void* ws, const WsLayout& lay, hipStream_t s,
                          KernelTimer* tm);

// Forward preparation only (K1, base flows, line epilogue): everything the
// backward kernels read.
hipError_t launch_forward_prep(const DevNet& net, int64_t n_box, const float* lo, const float* hi, void* ws,
                               const WsLayout& lay, hipStream_t s, KernelTimer* tm);

// Backward grid shapes, and the backward kernels after launch_forward_prep.
// `sparse`: the gradient of f_hi alone (no g_lo) takes the screened sweep.
void plan_backward(const DevNet& net, WsLayout& lay);
hipError_t launch_backward_sweeps(const DevNet& net, int64_t n_box, void* ws, const WsLayout& lay,
                                  const float* box_lo, const float* box_hi, const double* g_lo,
                                  const double* g_hi, double* d_lo, double* d_hi, bool sparse, hipStream_t s,
                                  KernelTimer* tm);

// Linear-relaxation upper bound after a forward pass (see ibp_crown.hip).
void plan_crown(const DevNet& net, int64_t n_box, WsLayout& lay, const Tune& t);
hipError_t launch_crown(const DevNet& net, int64_t n_box, const float* lo, const float* hi, int ref_iters,
                        double* f_hi, double* crown, float* vertex, void* ws, const WsLayout& lay, hipStream_t s,
                        KernelTimer* tm);
// Chord-relaxation lower bound after a forward call on the same workspace:
// f_lo[b] = max(f_lo[b], bound); crown (optional) the bound alone; vertex
// (optional) the minimiser of the linear part.
hipError_t launch_crown_lower(const DevNet& net, int64_t n_box, const float* lo, const float* hi, double* f_lo,
                              double* crown, float* vertex, void* ws, const WsLayout& lay, hipStream_t s,
                              KernelTimer* tm);

// Branch-and-bound rounds over input boxes (see ibp_split.hip).
hipError_t launch_split_select(int64_t n, const int64_t* roots, int S, const int* n_leaf, int X,
                               const float* leaf_lo, const float* leaf_hi, const double* leaf_fhi, int64_t* sel,
                               float* sel_lo, float* sel_hi, hipStream_t s);
hipError_t launch_split_bisect(int64_t n, const int64_t* roots, int S, const int* n_leaf, int X, float* leaf_lo,
                               float* leaf_hi, const int64_t* sel, const float* sel_lo, const float* sel_hi,
                               const double* g_lo, const double* g_hi, float* kid_lo, float* kid_hi, float* cen,
                               hipStream_t s);
hipError_t launch_split_update(int64_t n, const int64_t* roots, int S, int* n_leaf, const int64_t* sel,
                               const double* kid_fhi, int pts, const double* point_flo, const float* points, int X,
                               double* leaf_fhi, double* root_ub, double* root_lb, float* root_x, hipStream_t s);
hipError_t launch_split_screen(int64_t R, const double* root_ub, const double* root_lb, double rel_tol, int* status,
                               int64_t* open_roots, int64_t* n_open, hipStream_t s);

// Streaming-read probe (see ibp_probe.hip): 2048 per-block partial sums.
hipError_t launch_read_probe(const float4* src, int64_t n, float* partial, hipStream_t s);
hipError_t launch_alu_probe(float* out, int64_t iters, int scalar, hipStream_t s);

// K1..K4 for n_box boxes, each box handled by its own grid slice.
hipError_t launch_forward_single(const DevNet& net, int64_t n_box, const float* lo, const float* hi,
                                 double* f_lo, double* f_hi, double* terms, void* ws,
                                 const WsLayout& lay, hipStream_t s, KernelTimer* tm);

}  // namespace ibp
