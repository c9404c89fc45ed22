// Device-side data of a built network and the per-call workspace layout.
// Shared by the kernels and the host launcher code of libibp.
#pragma once

#include <cstddef>
#include <cstdint>

namespace ibp {

// float32 unit roundoff and float64 unit roundoff
constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24
constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53
// relative error of storing a float64 factor as float32 (round to nearest),
// measured against the stored value: |x - fl(x)| <= u |fl(x)| / (1 - u)
constexpr double kKappa0 = kU32 * (1.0 + 1.0 / 1048576.0);

// Per-box scalar slots in the workspace (float64).
enum BoxSlot : int {
  kVmax = 0,  // float bits (low 32 bits): max over outages of (|c_c| + r_c) / (1 - H_cc)
  kBoxSlots = 2
};

// Fields of the per-block partial record written by the box-preparation kernel.
enum P1Field : int {
  kP1Mc = 0,   // sum |c_n|
  kP1Mbox,     // sum (|c_n| + r'_n)
  kP1Sc,       // sum w_j c_j        (surplus centre)
  kP1Sr,       // sum |w_j| r_j      (surplus radius)
  kP1Sabs,     // sum |w_j c_j| + |w_j| r_j
  kP1cI,       // sum gens c - sum loads c   (total injection centre)
  kP1rI,       // sum r                      (total injection radius)
  kP1cIabs,    // sum |c|
  kP1Bad,      // number of invalid inputs
  kP1Fields = 10
};

// Network data on the device (everything the kernels read), passed by value.
struct DevNet {
  int N, L, K, G, D, X;
  int Np, Lp;  // padded row strides of the PTDF (buses) and outage factors (lines)
  int Kp;      // padded row stride of the line-major outage factors (outages, a multiple of 256; zero padding)
  const float* phiT;        // [N x Lp] float32 PTDF transposed (row n = column n of Phi), zero padding
  const float* lodf;        // [K x Lp] float32 outage factors, NaN at (k, c(k)), zero padding
  const float* lodfT;       // [L x Kp] the same factors line-major (row l: every outage's factor on line l)
  const float* lam_max;     // [Lp] max over outages of |factor| on the line, rounded up (0 on padding lines)
  const double* fmax_b;     // [L]
  const double* fmax_c;     // [L]
  const double* phi_err;    // [L] absolute float64 PTDF error bound of the row
  const int* ctg_of_line;   // [L] contingency index or -1
  const int* ctg_line;      // [K]
  const double* ctg_eps;    // [K] 2 phi_err[c] / (1 - H_cc)
  const double* ctg_inv;    // [K] 1 / (1 - H_cc)
  const double2* line_ctg;  // [L] (ctg_eps, ctg_inv) of the outage of line l, (0, 0) if it has none
  const float* line_eps;    // [Lp] 2 phi_err[l], rounded up (0 on padding lines)
  const float* fmax_c32;    // [Lp] post-outage limit as float32 (FLT_MAX on padding lines)
  const int* dev_bus;       // [X] bus of each input (generators, then loads)
  const int* bus_ptr;       // [N + 1] CSR over buses of the devices on each bus
  const int* bus_dev;       // [X] device indices (0..G-1 generators, G..X-1 loads)
  const int4* bus_dev4;     // [N] the first four entries of bus_dev for each bus, -1 where it has fewer
  const double* dev_w;      // [X] -cost for generators, +value for loads
  const int* seg_ptr;       // [X + 1] curve segments of each input, or nullptr (linear costs only)
  const double4* seg;       // [S] (slope a, shift b, cap U, |U| if finite else 0)
  double zeta_inj, zeta_f;
  double phi_err_max;
  double gamma64_n;         // float64 accumulation bound for one PTDF row
};

// Workspace carve-up for n_box boxes.  Offsets in bytes from the base pointer.
struct WsLayout {
  size_t inj = 0;                  // double2 [B][Np]: (c32, r'') of the injections, as float64
  size_t p1 = 0;                   // double [B][n_p1][kP1Fields]: box-preparation partial sums
  size_t part2 = 0;                // double2 [B][n_by][Lp]: base-flow partial sums (centre, radius)
  size_t box = 0;                  // double [B][kBoxSlots]
  size_t lc = 0, lh = 0, lg = 0;   // float [B][Lp]: line centre, h = rho'-fmax, g = rho'+fmax
  size_t lcf = 0, lrf = 0;         // double [B][L]: base-flow centre and enclosing radius
  size_t ctg = 0;                  // int4 [B][K]: (line, centre bits, rho' bits, unpadded radius bits)
  size_t p2 = 0;                   // double2 [B][n_p2]: base-penalty partial sums (hi, lo)
  size_t p3 = 0;                   // double2 [B][n_p3]: contingency partial sums (hi, lo)
  size_t lpart = 0;                // float2 [B][k5_by][Lp]: backward per-line partials (d centre, d radius)
  size_t cpart = 0;                // float2 [B][k5_tiles][K]: backward per-outage partials
  size_t gcf = 0, grf = 0;         // float [B][Lp]: backward line gradients (centre, radius)
  size_t gci = 0, gri = 0;         // double [B][Np]: backward injection gradients
  size_t cb = 0;                   // float2 [B][K]: backward per-outage (centre, unpadded radius); 0: absent
  size_t total = 0;
  int n_p1 = 0, n_p2 = 0, n_p3 = 0;
  int k2_bx = 0, k2_by = 0;        // K2 grid per box (line tiles x bus chunks)
  int k3_bx = 0, k3_by = 0;        // K3 grid per box (line tiles x outage chunks)
  int k2_nc = 0, k3_kc = 0;        // tile parameters used
  int batched = 0;                 // 1: box-tiled kernels (boxes share every streamed tile)
  int small = 0;                   // 1: smallest networks, one launch and one block per box (km_box)
  int sides = 3;                   // penalty sides of the outage sweep: 3 both, 1 lower (f_hi), 2 upper (f_lo)
  int k2_gx = 0;                   // batched base flows: grid x (line tiles padded to a multiple of 8)
  int k2_mfma = 0;                 // batched base flows on the float64 matrix cores
  int k2_chunk = 0;                // batched base flows: buses per chunk (k2_by chunks, a multiple of 4)
  int k3_kper = 0;                 // batched outage sweep: outages per block row
  int k3_bt = 4;                   // batched outage sweep: boxes per wave
  int k5_by = 0, k5_tiles = 0;     // backward outage sweep: outage chunks, line tiles
  int k5_chunk = 0;                // outages per backward chunk
  // screened backward sweep of the gradient of f_hi (box-tiled calls): the
  // lines that may hold an active lower-penalty element, per tile of boxes
  int k5s_tiles = 0;               // tiles of kScreenBoxes boxes (0: not laid out)
  int fscreen = 0;                 // one-sided box-tiled forward calls take the screened sweep
  size_t smask = 0;                // uint64 [tiles][Lp / 64]: candidate-line bit masks
  size_t srec = 0;                 // float [tiles][Lp][12]: the tile's boxes' centres and radius terms
  size_t lcnt = 0;                 // uint64 [B][Lp]: active-element counts (negative-flow count << 32 | count)
  size_t sw = 0;                   // float [tiles][Kp]: per tile and outage, max over its boxes of max(|c_c| - r_c, 0)
  size_t sz = 0;                   // float [tiles][k5w_bx]: per tile and 256 outages, max |c_c| + r_c
  int k5w_bx = 0;                  // blocks of 256 outages (Kp / 256 rounded up)
  // linear-relaxation bound (present with the CROWN flag)
  size_t ccnt = 0;                 // int2 [B][Lp]: per-line (sum s, sum |s|) over outages
  size_t cv = 0;                   // double4 [B][kc_bx][K]: per-outage (sum s Lam, sum |s Lam|, count)
  size_t lv = 0;                   // double4 [B][Lp]: per-line (v, vabs, ev); [Lp][kc3_bt] with kc3_mfma
  int kc3_bt = 0;                  // box stride of the line-major adjoint (n_box rounded up to 32)
  size_t bpart = 0;                // double4 [B][kc3_bx][Np]: per-bus (y, ya, ye) partials
  size_t cp = 0;                   // double2 [B][n_cp]: per-input partial sums
  size_t ct = 0;                   // double2 [B][n_ct]: per-line partial sums (limit total, sum vabs)
  int kc_bx = 0, kc_by = 0, kc3_bx = 0, kc3_by = 0, n_cp = 0, n_ct = 0;
  int chord_nb = 1;                // boxes per lane of the box-tiled chord sweep
  int k3_xcd = 0;                  // box-tiled outage sweep in XCD-aware block order
  size_t chp = 0;                  // int2 [B][chp_z][Lp]: per-box chord sweep, per-block line totals
  int chp_z = 0;                   // outage blocks of the per-box chord sweep (0: box-tiled, atomics)
  int kc3_mfma = 0, kc3_chunk = 0; // box-tiled transposed PTDF on the matrix cores: lines per chunk (kc3_bx chunks)
  // reference points of the relaxation (present with the reference flag)
  size_t fwd_total = 0;            // bytes of the forward arrays above (inj .. p3)
  size_t ref = 0;                  // a second forward region, for the reference points
  size_t xref = 0, vtx = 0;        // float [B][X]: reference points, maximising vertices
};

}  // namespace ibp
