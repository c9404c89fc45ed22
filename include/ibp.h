/*
 * ibp.h -- C ABI of libibp: certified interval bounds on the soft-constrained
 * SC-DCOPF market surplus by interval bound propagation (IBP), on MI355X.
 *
 * Paper: "Fast and Certified Bounding of Security-Constrained DCOPF via
 * Interval Bound Propagation" (Tekeler, Chevalier, Zhong, Zhang).
 *
 * For each input box  p_g in [pg_lo, pg_hi],  p_d in [pd_lo, pd_hi]
 * (Appendix, eq. (f-ibp)) the library returns  [f_lo, f_hi]  with
 *
 *     f_lo <= min_box f_ibp  and  f_hi >= max_box f_ibp,
 *
 * where f_ibp is the explicit graph of the Appendix, eq. (ibp_f):
 *   surplus  sum_j value_j p_d,j - sum_i cost_i p_g,i  (linear costs), plus
 *            optional piecewise-linear curves sum_j F*_j(p_d,j) - sum_i F*_i(p_g,i)
 *            in the ReLU form of Sec. III-B (see ibp_network_desc),
 *   minus zeta_inj * 1^T |(E^T Phi - I) p_inj|        (Sec. III-A, eq. slack-sinj),
 *   minus zeta_f * 1^T max(|Phi p_inj| - fmax_b, 0)    (eq. slack-sfb),
 *   minus zeta_f * sum over N-1 outages and lines of
 *         max(|post-outage flow| - fmax_c, 0)          (eqs. slack-Sc, slack-sagg),
 * with p_inj = N_g p_g - N_d p_d (Sec. II-A), the PTDF Phi of eq. (line flow
 * ptdf) and post-outage flows from the rank-1 outage update of Sec. II-C,
 * eq. (ctg flow simplified).  The bounds are those of IBP (Sec. III-C, eq. IBP)
 * through that graph, computed in float32 with outward padding so that they
 * enclose the exact-arithmetic IBP bounds.
 *
 * Conventions for every call:
 *   - Sizes are element counts.  Indices are 0-based int32.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *     memory on the device the network was built for.
 *   - The library never takes ownership of caller memory.
 *   - Errors that the host can detect are returned synchronously and nothing is
 *     launched; ibp_last_error() then gives a message (thread-local, valid until
 *     the next call on the same thread).
 *   - Compute calls are asynchronous on the given stream (a hipStream_t passed as
 *     void*; NULL means the default stream).
 */
#ifndef IBP_H_
#define IBP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ibp_status {
  IBP_OK = 0,
  IBP_E_INVALID_ARG = 1,     /* NULL pointer, size or index out of range, non-positive b/fmax/zeta */
  IBP_E_DISCONNECTED = 2,    /* base network not connected (reduced admittance singular) */
  IBP_E_ISLANDING_CTG = 3,   /* an explicitly listed outage disconnects the network */
  IBP_E_ILL_CONDITIONED = 4, /* 1 - H_cc < 1e-6 for some outage (rank-1 update near singular) */
  IBP_E_OUT_OF_MEMORY = 5,   /* host or device allocation failed */
  IBP_E_DEVICE = 6,          /* a HIP runtime call failed */
  IBP_E_WORKSPACE = 7,       /* workspace NULL or smaller than ibp_workspace_bytes() */
  IBP_E_HOST_ONLY = 8        /* compute call on a handle built with IBP_DEVICE_HOST_ONLY */
} ibp_status;

/* Network description (all host memory; copied by ibp_build_network).
 * Sec. II-A: buses, lines with susceptance b (Y_D = diag(b)), slack bus whose
 * row/column is removed from the reduced matrices; Sec. II-B/C: base-case and
 * post-outage flow limits; Sec. II-D: penalty weights zeta_inj, zeta_f. */
typedef struct ibp_network_desc {
  int32_t n_bus;            /* N >= 2 */
  int32_t n_line;           /* L >= 1 */
  int32_t slack_bus;        /* in [0, N) */
  const int32_t* line_from; /* [L] in [0, N), from != to */
  const int32_t* line_to;   /* [L] */
  const double* line_b;     /* [L] susceptance > 0 */
  const double* fmax_base;  /* [L] base-case limit > 0 */
  const double* fmax_ctg;   /* [L] post-outage limit > 0 */
  int32_t n_gen;            /* G >= 0 */
  const int32_t* gen_bus;   /* [G] */
  const double* gen_cost;   /* [G] linear cost, $/p.u.-h (any sign) */
  int32_t n_load;           /* D >= 0, G + D >= 1 */
  const int32_t* load_bus;  /* [D] */
  const double* load_value; /* [D] linear value, $/p.u.-h (any sign) */
  double zeta_inj;          /* >= 0 */
  double zeta_f;            /* >= 0 */
  int32_t n_ctg;            /* K; ignored when ctg_line is NULL */
  const int32_t* ctg_line;  /* [K] distinct non-islanding lines, or NULL for
                               every non-islanding line in ascending order */
  /* Optional piecewise-linear cost (generators) and value (loads) curves of
   * Sec. III-B, eqs. (single ReLU) and (combined ReLUs).  Input j (generators
   * first, then loads) owns segments seg_ptr[j] .. seg_ptr[j+1]-1; its curve is
   *   F*_0(x) = 0,  F*_i(x) = min(F*_{i-1}(x) + a_i max(x - b_i, 0), U_i),
   * with slope a_i = seg_a[i], shift b_i = seg_b[i], cap U_i = seg_U[i].  The
   * surplus adds F* of every load and subtracts F* of every generator, on top
   * of the linear terms (set gen_cost / load_value to 0 for curves only).
   * seg_ptr == NULL: linear costs only (the other three are then ignored). */
  const int32_t* seg_ptr;   /* [G + D + 1], seg_ptr[0] = 0, non-decreasing */
  const double* seg_a;      /* [seg_ptr[G + D]] finite */
  const double* seg_b;      /* [seg_ptr[G + D]] finite */
  const double* seg_U;      /* [seg_ptr[G + D]] finite or +infinity */
} ibp_network_desc;

typedef struct ibp_network ibp_network;

typedef struct ibp_network_info {
  int32_t n_bus, n_line, n_ctg, n_gen, n_load, n_input; /* n_input = G + D */
  int32_t device;             /* HIP device ordinal, or IBP_DEVICE_HOST_ONLY */
  double min_one_minus_hcc;   /* smallest 1 - H_cc over the outages */
  double phi_abs_err;         /* a-posteriori bound on |Phi64 - Phi_exact| (max over entries) */
  size_t device_bytes;        /* device memory held by the handle */
  double build_seconds;       /* wall time of the float64 construction */
} ibp_network_info;

#define IBP_DEVICE_HOST_ONLY (-1)

/* ibp_build_network -- float64 construction of PTDF (Sec. II-A, eq. line flow
 * ptdf) and of the outage factors (Sec. II-C, rank-1 update and eq. ctg flow
 * simplified), rounding to float32 and upload to `device`.
 * device = IBP_DEVICE_HOST_ONLY builds on the host only (no HIP call at all);
 * such a handle supports query/export/free but no compute call.
 * Synchronous.  On success *out owns host and device memory until
 * ibp_free_network.  Errors: INVALID_ARG, DISCONNECTED, ISLANDING_CTG,
 * ILL_CONDITIONED, OUT_OF_MEMORY, DEVICE. */
ibp_status ibp_build_network(const ibp_network_desc* desc, int device, ibp_network** out);

/* Fills *info (host).  Errors: INVALID_ARG on NULL. */
ibp_status ibp_network_query(const ibp_network* net, ibp_network_info* info);

/* Copies the K outaged line indices (host int32[K]). */
ibp_status ibp_network_ctg_lines(const ibp_network* net, int32_t* out);

/* Copies the float64 factors the float32 device copies were rounded from:
 * ptdf (host, L x N row-major, slack column zero) and lodf (host, K x L
 * row-major: row k is the outage-distribution column of outage k, entry
 * (k, c(k)) holds the raw value H_cc / (1 - H_cc) and is never used).
 * Either pointer may be NULL. */
ibp_status ibp_network_export(const ibp_network* net, double* ptdf, double* lodf);

/* Releases everything held by the handle.  NULL is allowed. */
void ibp_free_network(ibp_network* net);

/* Flags for the compute calls. */
#define IBP_F_NONE 0u
#define IBP_F_PLAIN 1u    /* per-box single-box kernels even for n_box > 1 (reference form for batching) */
#define IBP_F_BACKWARD 4u /* workspace query only: size for ibp_bound_backward (includes the forward's) */
#define IBP_F_CROWN 8u    /* workspace query only: size for ibp_crown_bound_boxes (includes the forward's) */
#define IBP_F_CROWN_REF 16u /* workspace query only: ibp_crown_bound_boxes with ref_iters > 0 */
/* One-sided calls of ibp_bound_boxes / ibp_crown_bound_boxes (and of
 * ibp_bound_backward, see there), for callers that use one bound only (branch
 * and bound bounds children from above and evaluates points from below).  The box-tiled outage sweep then computes only
 * the penalty side that bound needs (about half its arithmetic).  The other
 * output stays a valid bound: with IBP_F_UPPER_ONLY f_lo is -INFINITY (terms:
 * Fc_hi = +INFINITY); with IBP_F_LOWER_ONLY the outage penalties' lower bound
 * is taken as 0, so f_hi is larger than the two-sided call's (terms: Fc_lo = 0).
 * The requested bound is the two-sided call's: bit for bit on the per-box
 * path (fewer than 4 boxes, or IBP_F_PLAIN); on the box-tiled path the sweep
 * runs only on the lines that a screen (per tile of 4 boxes, a bound over all
 * outages at once) finds able to hold an active penalty of that side, which
 * changes the float32 summation order of the outage penalties (1e-6 relative
 * at most; the bound is certified either way; IBP_TILE=k3s=0 at
 * ibp_build_network keeps the dense sweep).  IBP_F_UPPER_ONLY calls always
 * take the screen (the lower penalties of f_hi are active on few lines:
 * 2000 buses, 8192 sub-boxes, 12.2 -> 7.8 ms).  Calls that bound f_lo (two-
 * sided, or IBP_F_LOWER_ONLY) take it only with IBP_F_SCREEN_UPPER: the
 * screen then bounds the upper penalties (a line with none active has no
 * active lower penalty either) and the sweep sums both sides, or the upper
 * side alone, over the marked lines.  That pays where few lines carry an
 * active upper penalty (the centre points of sub-boxes: 12.3 -> 9.3 ms at
 * 8192 points; 18 x 1024 period sub-boxes, two-sided: 37.1 -> 30.1 ms) and
 * costs more than it saves on wide sub-boxes (1024 of them, lower bound
 * alone: 2.1 against 1.6 ms).  At most one of the two side flags;
 * IBP_F_SCREEN_UPPER not with IBP_F_UPPER_ONLY. */
#define IBP_F_UPPER_ONLY 32u
#define IBP_F_LOWER_ONLY 64u
#define IBP_F_SCREEN_UPPER 512u
/* Forward then backward on the same boxes (the differentiation form: the
 * bound, then its gradient, as torch.autograd runs them).  IBP_F_KEEP_PREP
 * (ibp_bound_boxes): lay the workspace out as for ibp_bound_backward (it must
 * hold ibp_workspace_bytes(net, n_box, flags | IBP_F_BACKWARD), which the
 * query with IBP_F_KEEP_PREP also returns) and leave the forward
 * intermediates (injections, base flows, line and outage constants) in it.
 * IBP_F_REUSE_PREP (ibp_bound_backward): take those intermediates instead of
 * recomputing them (the backward's box preparation, base flows and line
 * epilogue: about 2 of its 12 ms at 2000 buses x 4096 boxes).  The library
 * keeps, per handle and workspace, what the last call on that workspace left
 * there: an ibp_bound_boxes call with IBP_F_KEEP_PREP, or any
 * ibp_bound_backward, leaves the intermediates of its boxes (box pointers,
 * n_box, IBP_F_PLAIN and the handle's tiles recorded); any other compute call
 * on the workspace, a tile change, or a call split into chunks (more than
 * 16 x 65535 boxes) leaves none.  IBP_F_REUSE_PREP is refused with
 * INVALID_ARG unless the record matches the call; the box values themselves
 * must not change in between (not checked). */
#define IBP_F_KEEP_PREP 128u
#define IBP_F_REUSE_PREP 256u

/* Bytes of device workspace a compute call needs for n_box boxes (0 on error). */
size_t ibp_workspace_bytes(const ibp_network* net, int64_t n_box, uint32_t flags);

/* ibp_bound_boxes -- IBP bounds of f_ibp over n_box boxes (Appendix, eqs.
 * (ibp_f), (f-ibp); Sec. III-C, eq. IBP).
 *   box_lo, box_hi : device float32 [n_box x X], row-major, X = G + D inputs,
 *                    generators first, then loads.  The float32 values are the box.
 *   f_lo, f_hi     : device float64 [n_box], written.
 *   terms          : device float64 [n_box x 8] or NULL; per box the intervals
 *                    S_lo, S_hi (surplus), I_lo, I_hi (1^T s_inj), Fb_lo, Fb_hi
 *                    (1^T s_fb), Fc_lo, Fc_hi (s_agg), each already padded.
 *   ws, ws_bytes   : device workspace of at least ibp_workspace_bytes(net, n_box, flags).
 * flags: 0, IBP_F_PLAIN, IBP_F_UPPER_ONLY or IBP_F_LOWER_ONLY (or PLAIN with one
 * of the other two; 0 and IBP_F_LOWER_ONLY optionally with IBP_F_SCREEN_UPPER),
 * each optionally with IBP_F_KEEP_PREP.
 * A box with a non-finite endpoint or lo > hi gets NaN outputs; other boxes are
 * unaffected.  Concurrent calls on one handle are safe with distinct workspaces.
 * Errors: INVALID_ARG, WORKSPACE, HOST_ONLY, DEVICE. */
ibp_status ibp_bound_boxes(const ibp_network* net, int64_t n_box,
                           const float* box_lo, const float* box_hi,
                           double* f_lo, double* f_hi, double* terms,
                           void* ws, size_t ws_bytes, void* stream, uint32_t flags);

/* ibp_bound_boxes_noalloc -- ibp_bound_boxes for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same results, bit
 * for bit, but the workspace is a library-owned device array of
 * IBP_NOALLOC_SCRATCH_BYTES per GPU (reserved when the library's code is
 * loaded on a device and held until the process ends; its address is taken at
 * ibp_build_network, or at the first call on a device).  The call allocates
 * nothing and queues no memset: every slot the kernels accumulate into is
 * cleared by the first kernel of the call itself.
 *   box_lo, box_hi, f_lo, f_hi, terms, flags: as for ibp_bound_boxes.
 * Every call on one GPU shares that GPU's array and leaves its contents behind:
 * calls that overlap in time on one GPU (on different streams, from different
 * threads, or with different networks) race on it and must be serialised by the
 * caller, for example by issuing them on one stream.
 * Errors: INVALID_ARG, HOST_ONLY, DEVICE, and WORKSPACE when the call needs more
 * than IBP_NOALLOC_SCRATCH_BYTES (ibp_workspace_bytes(net, n_box, flags) says
 * how much; 32 MiB holds one box of an 8316-bus, 14000-line, 8000-outage
 * network about fifteen times over). */
#define IBP_NOALLOC_SCRATCH_BYTES (32u << 20)
ibp_status ibp_bound_boxes_noalloc(const ibp_network* net, int64_t n_box,
                                   const float* box_lo, const float* box_hi,
                                   double* f_lo, double* f_hi, double* terms,
                                   void* stream, uint32_t flags);

/* ibp_bound_backward -- vector-Jacobian product of the (unpadded) IBP map:
 *   g_box_lo[b, j] = d(g_f_lo[b] f_lo[b] + g_f_hi[b] f_hi[b]) / d box_lo[b, j],
 *   g_box_hi likewise (device float64 [n_box x X], overwritten).
 * Subgradient convention: sign(0) = 0 and max(z, 0) is active iff z > 0.
 * g_f_lo, g_f_hi: device float64 [n_box].  The workspace must hold
 * ibp_workspace_bytes(net, n_box, flags | IBP_F_BACKWARD); the call recomputes
 * the forward intermediates in it (unless IBP_F_REUSE_PREP) and leaves them
 * there.  A box with invalid endpoints gets NaN
 * gradients.  flags: 0 or IBP_F_PLAIN, optionally with IBP_F_UPPER_ONLY (the
 * VJP of f_hi alone: g_f_lo is not read and may be NULL) or IBP_F_LOWER_ONLY
 * (of f_lo alone: g_f_hi not read); the one-sided sweeps carry only that
 * side's arithmetic; and optionally IBP_F_REUSE_PREP (see above).  Errors as
 * the forward call. */
ibp_status ibp_bound_backward(const ibp_network* net, int64_t n_box,
                              const float* box_lo, const float* box_hi,
                              const double* g_f_lo, const double* g_f_hi,
                              double* g_box_lo, double* g_box_hi,
                              void* ws, size_t ws_bytes, void* stream, uint32_t flags);

/* ibp_backward_screen_lines -- what the screened outage sweep of the last
 * backward call did (the gradient of f_hi alone, Appendix eq. (ibp_f) through
 * the lower penalties of Sec. III-A eq. (slack-Sc)).  Calls of ibp_bound_backward
 * with IBP_F_UPPER_ONLY on 4 or more boxes (not IBP_F_PLAIN) first mark, per
 * tile of 4 boxes, the lines on which some outage can make the lower penalty
 * active (a bound over the tile, with a rounding margin), then run the outage
 * sweep on those lines only; the gradient is that of the dense sweep up to
 * float32 summation order (IBP_TILE=k5s=0 at ibp_build_network keeps the
 * dense sweep).  After such a call on workspace `ws` with n_box boxes (at most
 * 16 x 65535; a call split into chunks is not covered), this returns the
 * number of marked (tile, line) pairs (*n_marked) and of all pairs (*n_pairs =
 * tiles x lines).  Reads the workspace on `stream` and waits for it.  After
 * any other call on `ws` the numbers are meaningless.
 * Errors: INVALID_ARG (NULL, or sizes with no screened sweep), WORKSPACE,
 * HOST_ONLY, DEVICE. */
ibp_status ibp_backward_screen_lines(const ibp_network* net, int64_t n_box, const void* ws, size_t ws_bytes,
                                     void* stream, int64_t* n_marked, int64_t* n_pairs);

/* ibp_crown_bound_boxes -- IBP bounds tightened by a linear relaxation of the
 * penalties (the CROWN family of convex relaxations the paper cites beside
 * IBP, Sec. I).  Every penalty max(|z| - t, 0) and the imbalance |z| is
 * convex, so a supporting line s z - |s| t (s in {-1, 0, 1}) lies below it
 * everywhere; with these lines the objective is bounded above by a linear
 * function of the inputs (plus the interval of any piecewise-linear curves)
 * whose exact maximum over the box is computed with outward rounding.  The
 * first relaxation takes the slope of an element as the sign of its flow when
 * IBP's interval for it lies beyond the limit, else 0 (never looser than IBP).
 * With ref_iters > 0, ref_iters further relaxations take the slopes from the
 * flows at reference points (sign where the flow exceeds the limit there, else
 * 0): first the box centre, then each point moved halfway (float32) towards
 * the vertex that maximised the previous relaxation.  Every relaxation is a
 * valid bound; the smallest is kept.
 *   f_lo, f_hi : device float64 [n_box]: IBP's f_lo, and min(IBP f_hi,
 *                relaxation bound) -- both still certified.
 *   ref_iters  : 0 .. 64 reference-point relaxations after the first.
 *   crown_hi   : device float64 [n_box] or NULL: the smallest relaxation bound
 *                alone.
 *   vertex     : device float32 [n_box x X] or NULL: the box vertex that
 *                maximises the last relaxation's linear part (hi_j where its
 *                coefficient is >= 0, else lo_j), a candidate point for
 *                lower bounds on max f.
 *   ws, ws_bytes: at least ibp_workspace_bytes(net, n_box, flags | IBP_F_CROWN)
 *                (| IBP_F_CROWN_REF when ref_iters > 0).
 * flags: 0, IBP_F_PLAIN, IBP_F_UPPER_ONLY (forward kernels as in
 * ibp_bound_boxes; with UPPER_ONLY f_lo is -INFINITY).  Invalid boxes get NaN.
 * Errors: INVALID_ARG, WORKSPACE, HOST_ONLY, DEVICE. */
ibp_status ibp_crown_bound_boxes(const ibp_network* net, int64_t n_box,
                                 const float* box_lo, const float* box_hi, int32_t ref_iters,
                                 double* f_lo, double* f_hi, double* crown_hi, float* vertex,
                                 void* ws, size_t ws_bytes, void* stream, uint32_t flags);

/* ibp_crown_lower_boxes -- IBP bounds with f_lo tightened by a linear
 * relaxation of the penalties (the CROWN family of convex relaxations the
 * paper cites beside IBP, Sec. I), the counterpart of ibp_crown_bound_boxes
 * for the lower bound.  Every penalty max(|z| - t, 0) and the imbalance |z| is
 * convex, so on the IBP interval of its pre-activation it lies below its chord;
 * with these lines the objective is bounded below by a linear function of the
 * inputs (plus the interval of any piecewise-linear curves) whose exact
 * minimum over the box is computed with outward rounding.  Chord slopes are
 * rounded to multiples of 2^-24 (any slope gives a valid line; the intercept
 * is formed for the rounded slope).  In exact arithmetic the relaxation is
 * never below IBP's f_lo; the call keeps the larger of the two.
 *   f_lo, f_hi : device float64 [n_box]: max(IBP f_lo, relaxation bound), and
 *                IBP's f_hi -- both certified.
 *   crown_lo   : device float64 [n_box] or NULL: the relaxation bound alone.
 *   vertex     : device float32 [n_box x X] or NULL: the box vertex that
 *                minimises the relaxation's linear part (lo_j where its
 *                coefficient is >= 0, else hi_j), a candidate point for upper
 *                bounds on min f.
 *   ws, ws_bytes: at least ibp_workspace_bytes(net, n_box, flags | IBP_F_CROWN).
 * flags: 0, IBP_F_PLAIN, IBP_F_LOWER_ONLY (forward kernels as in
 * ibp_bound_boxes; with LOWER_ONLY f_hi is the one-sided call's).  Invalid
 * boxes get NaN.
 * Errors: INVALID_ARG, WORKSPACE, HOST_ONLY, DEVICE. */
ibp_status ibp_crown_lower_boxes(const ibp_network* net, int64_t n_box,
                                 const float* box_lo, const float* box_hi,
                                 double* f_lo, double* f_hi, double* crown_lo, float* vertex,
                                 void* ws, size_t ws_bytes, void* stream, uint32_t flags);

/* Kernel timing for benchmarks and profiling.  While enabled, every compute
 * call on `net` records a HIP event pair for each kernel it queues, on the
 * call's stream (for the single-box forward kernels the events are recorded by
 * the dispatch itself, so they time the kernel alone; elsewhere they are queued
 * around it).  ibp_kernel_times() waits for those events and returns, per
 * kernel id, the summed milliseconds and the number of launches since the last
 * read (then clears them).  Kernel ids: 0 box preparation, 1 base flows,
 * 2 outage sweep, 3 finalize, 4 line epilogue, 5 batched base flows,
 * 6 batched outage sweep, 7 backward outage sweep, 8 backward transposed PTDF,
 * 9 backward endpoints, 10 relaxation outage sweep, 11 relaxation line adjoint
 * and transposed PTDF, 12 relaxation inputs and finalize, 13 backward
 * per-line (base-case) terms, 14 backward line screen (the gradient of f_hi
 * alone in box-tiled calls, before its outage sweep), 15 forward line screen
 * (one-sided box-tiled calls, before their outage sweep, id 6).
 * Not thread-safe with concurrent compute calls on the same handle. */
#define IBP_N_KERNEL_IDS 16
ibp_status ibp_set_kernel_timing(ibp_network* net, int enable);
ibp_status ibp_kernel_times(ibp_network* net, int32_t n_ids, double* total_ms, int64_t* count);

/* Tile parameters of the two streaming kernels: k2_nc buses per wave in the
 * base-flow sweep (32, 64, 128, 256, 512) and k3_kc outages per block in the outage
 * sweep (16, 32, 64, 128).  They change the workspace size; results do not
 * depend on them beyond float64 summation order.  ibp_autotune() times every
 * pair on the caller's boxes (forward calls on `stream`, synchronizing) and
 * keeps the fastest; `chosen` (host int32[2], nullable) receives it.  The
 * workspace must hold ibp_workspace_bytes(net, n_box, IBP_F_AUTOTUNE).
 * Neither call may run concurrently with compute calls on the same handle.
 * The environment variable IBP_TILE, read by ibp_build_network, sets the same
 * parameters ("k2nc=64,k3kc=32"); "k2b=0" in it makes calls of 4 or more
 * boxes compute their base flows with vector float64 FMA instead of the
 * float64 matrix cores (the default; both sum the same products); "ckb=2"
 * or "ckb=4" makes the box-tiled chord-relaxation sweep of
 * ibp_crown_lower_boxes keep two or four boxes per lane instead of one (same
 * results). */
#define IBP_F_AUTOTUNE 2u /* workspace query only: size for every tile pair */
ibp_status ibp_set_tile(ibp_network* net, int32_t k2_nc, int32_t k3_kc);
ibp_status ibp_autotune(ibp_network* net, int64_t n_box, const float* box_lo, const float* box_hi,
                        void* ws, size_t ws_bytes, void* stream, int32_t* chosen);

/* Tile parameters of the box-tiled path (calls of 4 or more boxes; time
 * indices and sub-boxes batched into one launch, Sec. IV-A): boxes per wave of
 * the outage sweep (k3_bt: 2, 4 or 8), its outage rows (k3_rows: 0 for the
 * built-in rule, else 1..4096), its XCD-aware block order (k3_xcd: 0 off, 1 on,
 * -1 on when the outage factors exceed 128 MiB), the base-flow engine (k2_mfma:
 * 1 float64 matrix cores, 0 vector FMA) and its bus chunks (k2_by: 0 for the
 * rule, else 1..8).  Results do not depend on them beyond float64 summation
 * order.  ibp_autotune_batched() times the candidates around the current
 * parameters on the caller's n_box >= 4 boxes (forward kernels on `stream`,
 * synchronizing; the base flows first, then the outage sweep with the chosen
 * base flows, then the same sweep over the lines the upper-penalty screen
 * marks, kept in the screen-upper setting below if faster) and keeps the
 * fastest; `chosen` (host int32[5], nullable) receives (k3_bt, k3_rows,
 * k3_xcd, k2_mfma, k2_by).  The workspace must hold
 * ibp_workspace_bytes(net, n_box, IBP_F_AUTOTUNE).  ibp_get_tile() copies the
 * current parameters (host int32[7]: k2_nc, k3_kc, k3_bt, k3_rows, k3_xcd,
 * k2_mfma, k2_by).  None of the three may run concurrently with compute calls
 * on the same handle.  Errors: INVALID_ARG, WORKSPACE, HOST_ONLY, DEVICE. */
ibp_status ibp_set_tile_batched(ibp_network* net, int32_t k3_bt, int32_t k3_rows, int32_t k3_xcd,
                                int32_t k2_mfma, int32_t k2_by);
ibp_status ibp_get_tile(const ibp_network* net, int32_t* out);
ibp_status ibp_autotune_batched(ibp_network* net, int64_t n_box, const float* box_lo, const float* box_hi,
                                void* ws, size_t ws_bytes, void* stream, int32_t* chosen);

/* Screen-upper setting of the box-tiled path: with `on` = 1 every box-tiled
 * call that bounds f_lo (two-sided or IBP_F_LOWER_ONLY) behaves as if it
 * carried IBP_F_SCREEN_UPPER (bounds within the 1e-6 relative reordering that
 * flag states, still certified; the workspace those calls need
 * grows by the screen's regions, so query ibp_workspace_bytes after changing
 * it).  Default 0; ibp_autotune_batched() sets it; IBP_TILE "scru=1" sets it
 * at network build.  ibp_get_screen_upper() reads it into *on (host int32).
 * Not concurrently with compute calls on the same handle.  Errors:
 * INVALID_ARG. */
ibp_status ibp_set_screen_upper(ibp_network* net, int32_t on);
ibp_status ibp_get_screen_upper(const ibp_network* net, int32_t* on);

/* Branch and bound over input boxes (the paper names branch and bound over
 * the inputs as the way to tighten IBP bounds, Sec. I and Sec. V, and screens
 * instances for max f < 0, Sec. III-D eq. (inf-or-wn)).
 * Every root owns `slots` leaf slots: leaf q of root r is row r*slots + q of
 * leaf_lo/leaf_hi (device float32 [n_root*slots x n_input]) with its upper
 * bound in leaf_fhi (device float64 [n_root*slots]); n_leaf (device int32
 * [n_root]) counts the used slots, which partition the root.  A round works on
 * n_act active roots: roots (device int64 [n_act], ascending, or NULL for
 * roots 0..n_act-1).  Rows "i" below are dense over the active list.
 *   ibp_split_select: per active root, the leaf with the largest f_hi; its
 *     row index goes to sel (device int64 [n_act]) and a copy to
 *     sel_lo/sel_hi (device float32 [n_act x n_input]).
 *   (the caller runs ibp_bound_backward on sel_lo/sel_hi with g_f_lo = 0,
 *    g_f_hi = 1 to get g_lo/g_hi)
 *   ibp_split_bisect: splits the selected leaf at the float32 midpoint of the
 *     coordinate j maximising (g_hi_j - g_lo_j) * (hi_j - lo_j)/2; the halves
 *     replace slot sel and fill slot n_leaf[r] when n_leaf[r] < slots (a root
 *     with no free slot is left unchanged), and are written to kid_lo/kid_hi
 *     (device [2*n_act x n_input], rows 2i, 2i+1) with their centre points in
 *     centers (same shape).  A leaf with no float32 strictly inside any
 *     coordinate is duplicated.
 *   (the caller bounds the children and evaluates points_per_root points per
 *    root as zero-width boxes: points device float32
 *    [n_act x points_per_root x n_input], their f_lo in point_flo)
 *   ibp_split_update: writes the children's f_hi into leaf_fhi, increments
 *     n_leaf, sets root_ub[r] = min(root_ub[r], max leaf f_hi) and
 *     root_lb[r] = max(root_lb[r], best point value) (device float64
 *     [n_root]); when the point improves root_lb and root_x is not NULL, the
 *     point is copied to row r of root_x (device float32 [n_root x n_input]).
 *   ibp_split_screen: status[r] (device int32 [n_root]) = 1 if root_ub < 0
 *     (max f < 0 certified: welfare-negative or infeasible), 2 if
 *     root_lb >= 0 (a point with f >= 0 certified), 3 if
 *     root_ub - root_lb <= rel_tol * max(1, |root_ub|), 4 if a bound is NaN,
 *     else 0 (open); the open roots are written to open_roots (device int64
 *     [n_root], ascending) and their count to *n_open (device int64).
 * All asynchronous on `stream`; host-checkable errors: INVALID_ARG. */
ibp_status ibp_split_select(int64_t n_act, const int64_t* roots, int32_t slots, const int32_t* n_leaf,
                            int32_t n_input, const float* leaf_lo, const float* leaf_hi,
                            const double* leaf_fhi, int64_t* sel, float* sel_lo, float* sel_hi,
                            void* stream);
ibp_status ibp_split_bisect(int64_t n_act, const int64_t* roots, int32_t slots, const int32_t* n_leaf,
                            int32_t n_input, float* leaf_lo, float* leaf_hi, const int64_t* sel,
                            const float* sel_lo, const float* sel_hi,
                            const double* g_lo, const double* g_hi,
                            float* kid_lo, float* kid_hi, float* centers, void* stream);
ibp_status ibp_split_update(int64_t n_act, const int64_t* roots, int32_t slots, int32_t* n_leaf,
                            const int64_t* sel, const double* kid_fhi, int32_t points_per_root,
                            const double* point_flo, const float* points, int32_t n_input,
                            double* leaf_fhi, double* root_ub, double* root_lb, float* root_x,
                            void* stream);
ibp_status ibp_split_screen(int64_t n_root, const double* root_ub, const double* root_lb, double rel_tol,
                            int32_t* status, int64_t* open_roots, int64_t* n_open, void* stream);

/* ibp_read_probe -- streams n_float4 float4 values from device memory `src`
 * (16-byte aligned) with the load pattern of the library's HBM-bound sweeps
 * (nontemporal float4 loads, eight in flight per lane; 2048 blocks x 256
 * threads, each block a contiguous range) and writes 2048 per-block float32
 * sums to `partial` (device, caller owned).  For calibration: the caller times
 * it on `stream` to measure the read rate those sweeps can reach.  Asynchronous.  Errors: INVALID_ARG (NULL or
 * misaligned pointer, n_float4 < 1), DEVICE. */
#define IBP_READ_PROBE_PARTIALS 2048
ibp_status ibp_read_probe(const void* src, int64_t n_float4, float* partial, void* stream);

/* ibp_alu_probe -- float32 FMA issue-rate probe: 2048 blocks x 256 threads,
 * each lane running eight independent chains a <- 0.5 a + 1 (fused
 * multiply-add) for `iters` steps (1 .. 2^24), then writing the sum of its
 * chains to out[lane] (device float32[IBP_ALU_PROBE_LANES], caller owned;
 * 16.0 exactly once iters >= 64).  scalar_operand = 0 keeps every operand in a
 * vector register; 1 reads the multiplier from a scalar register.  For
 * calibration: the caller times it on `stream`; 2^22 x 8 x iters lane FMAs over
 * the time is the vector-ALU rate the ALU-bound sweeps are priced against.
 * Asynchronous.  Errors: INVALID_ARG, DEVICE. */
#define IBP_ALU_PROBE_LANES 524288
ibp_status ibp_alu_probe(float* out, int64_t iters, int32_t scalar_operand, void* stream);

/* Last error message of the calling thread ("" if none). */
const char* ibp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IBP_H_ */
