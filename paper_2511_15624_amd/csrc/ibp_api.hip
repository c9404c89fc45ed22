// C ABI of libibp (declared in include/ibp.h): handle lifetime, float32
// packing and upload of the float64 factors, workspace sizing, argument
// checks and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ibp_device.h"
#include "ibp_internal.h"
#include "ibp_kernels.h"

// The forward intermediates a workspace holds after a call that leaves them
// (ibp_bound_boxes with IBP_F_KEEP_PREP, or any ibp_bound_backward), for
// ibp_bound_backward with IBP_F_REUSE_PREP.
struct PrepTag {
  const void* ws;
  int64_t n_box;
  const float* lo;
  const float* hi;
  bool plain;
  uint64_t tiles;  // tile generation of the handle when they were made
};

struct ibp_network {
  ibp::HostNet h;
  int device = IBP_DEVICE_HOST_ONLY;
  int num_cus = 256;
  ibp::DevNet dn{};
  std::vector<void*> allocs;
  size_t device_bytes = 0;
  ibp::KernelTimer timer;
  ibp::Tune tune;
  uint64_t tile_gen = 0;  // bumped whenever the tiles (and so the workspace layout) change
  mutable std::mutex prep_mu;
  mutable std::vector<PrepTag> prep;  // at most one record per workspace
};

// Library-owned workspace of ibp_bound_boxes_noalloc: one copy per GPU the
// library runs on, held until the process ends.  In host code the name is a
// host-side stand-in, not a device address: kernels get the per-device address
// taken by hipGetSymbolAddress (g_scratch below), never the name itself.
static __device__ __align__(256) unsigned char scratch[IBP_NOALLOC_SCRATCH_BYTES];

namespace {

// Last error message of this thread: a fixed buffer, so that reporting an
// allocation failure allocates nothing.
constexpr size_t kErrBytes = 512;
thread_local char g_err[kErrBytes];

void set_err(const char* msg) {
  std::strncpy(g_err, msg, kErrBytes - 1);
  g_err[kErrBytes - 1] = 0;
}

// Device address of `scratch` on each device, taken once per device with that
// device current (at network construction, or at the first no-allocation call).
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxScratchDevices] = {};

ibp_status fail(ibp_status s, const char* msg) {
  set_err(msg);
  return s;
}
ibp_status fail(ibp_status s, const std::string& msg) { return fail(s, msg.c_str()); }

// Every entry point runs its body under this guard: no C++ exception crosses
// the C boundary.  Host allocation failures (std::bad_alloc, and the
// length errors of impossible sizes) become IBP_E_OUT_OF_MEMORY; anything
// else thrown is reported the same way with its message.  Whatever the body
// had allocated is owned by RAII objects or the handle and freed by then.
template <typename F>
ibp_status guarded(F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(IBP_E_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(IBP_E_OUT_OF_MEMORY, e.what());
  } catch (...) {
    return fail(IBP_E_OUT_OF_MEMORY, "host resource exhausted");
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Timing events and scratch output of an autotuning call, released on every
// exit (hipFree waits for the queued work that may still use the buffer).
struct TuneScratch {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void* buf = nullptr;
  bool init(size_t bytes) {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return false;
    return bytes == 0 || hipMalloc(&buf, bytes) == hipSuccess;
  }
  ~TuneScratch() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (buf) (void)hipFree(buf);
  }
};

// Records of kept forward intermediates (see PrepTag): every compute call on
// a workspace first forgets that workspace's record; the calls that leave the
// intermediates behind then record them.
void prep_forget(const ibp_network* net, const void* ws) {
  std::lock_guard<std::mutex> lock(net->prep_mu);
  auto& v = net->prep;
  v.erase(std::remove_if(v.begin(), v.end(), [&](const PrepTag& t) { return t.ws == ws; }), v.end());
}

void prep_record(const ibp_network* net, const PrepTag& tag) {
  std::lock_guard<std::mutex> lock(net->prep_mu);
  auto& v = net->prep;
  v.erase(std::remove_if(v.begin(), v.end(), [&](const PrepTag& t) { return t.ws == tag.ws; }), v.end());
  v.push_back(tag);
}

bool prep_matches(const ibp_network* net, const PrepTag& tag) {
  std::lock_guard<std::mutex> lock(net->prep_mu);
  for (const PrepTag& t : net->prep)
    if (t.ws == tag.ws)
      return t.n_box == tag.n_box && t.lo == tag.lo && t.hi == tag.hi && t.plain == tag.plain &&
             t.tiles == tag.tiles;
  return false;
}

// Address of this device's `scratch` copy; the device must be current.
ibp_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxScratchDevices)
    return fail(IBP_E_DEVICE, "no-allocation scratch: device ordinal beyond " + std::to_string(kMaxScratchDevices));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(IBP_E_DEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                    hipGetErrorString(e));
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return IBP_OK;
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <typename T>
ibp_status upload(ibp_network* net, const T* src, size_t count, const T** dst) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
  if (hipMalloc(&p, bytes) != hipSuccess)
    return fail(IBP_E_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  net->allocs.push_back(p);
  net->device_bytes += bytes;
  if (count && hipMemcpy(p, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(IBP_E_DEVICE, "hipMemcpy to device failed");
  *dst = static_cast<const T*>(p);
  return IBP_OK;
}

void clear_timer(ibp_network* net) {
  for (auto& r : net->timer.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  net->timer.recs.clear();
}

void release_device(ibp_network* net) {
  if (net->device >= 0) {
    DeviceGuard g(net->device);
    clear_timer(net);
    for (void* p : net->allocs) (void)hipFree(p);
  }
  net->allocs.clear();
  net->device_bytes = 0;
}

ibp_status to_device(ibp_network* net, int device) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
    return fail(IBP_E_DEVICE, "no HIP device available");
  if (device < 0 || device >= count)
    return fail(IBP_E_INVALID_ARG, "device ordinal out of range");
  DeviceGuard g(device);
  if (!g.ok) return fail(IBP_E_DEVICE, "hipSetDevice failed");
  net->device = device;
  {
    void* sp = nullptr;
    const ibp_status ss = scratch_address(device, &sp);
    if (ss != IBP_OK) return ss;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    net->num_cus = cus;

  const ibp::HostNet& h = net->h;
  ibp::DevNet& d = net->dn;
  d.N = h.N;
  d.L = h.L;
  d.K = h.K;
  d.G = h.G;
  d.D = h.D;
  d.X = h.G + h.D;
  d.Np = round_up(h.N, 64);
  d.Lp = round_up(h.L, 64);
  d.zeta_inj = h.zeta_inj;
  d.zeta_f = h.zeta_f;
  d.phi_err_max = h.phi_err_max;
  // float64 sums of N products of a float32 PTDF entry and a float64
  // injection: each step rounds the product (when not fused) and the sum
  d.gamma64_n = (double)(2 * h.N + 64) * ibp::kU64 * 1.01;

  ibp_status st;
  {
    // transposed PTDF, bus-major: row n holds the flows on every line for a unit
    // injection at bus n (column n of Phi); padding lines are zero
    std::vector<float> phiT((size_t)h.N * d.Lp, 0.0f);
    ibp::parallel_for(h.N, 64, [&](int64_t a, int64_t b) {
      for (int64_t n = a; n < b; ++n) {
        float* row = phiT.data() + (size_t)n * d.Lp;
        for (int l = 0; l < h.L; ++l) row[l] = (float)h.phi[(size_t)l * h.N + n];
      }
    });
    if ((st = upload(net, phiT.data(), phiT.size(), &d.phiT)) != IBP_OK) return st;
  }
  {
    std::vector<float> lodf32((size_t)std::max(1, h.K) * d.Lp, 0.0f);
    for (int k = 0; k < h.K; ++k) {
      float* row = lodf32.data() + (size_t)k * d.Lp;
      const double* src = h.lodf.data() + (size_t)k * h.L;
      for (int l = 0; l < h.L; ++l) row[l] = (float)src[l];
      row[h.ctg_line[k]] = std::numeric_limits<float>::quiet_NaN();  // outaged line's own entry
    }
    if ((st = upload(net, lodf32.data(), (size_t)h.K * d.Lp, &d.lodf)) != IBP_OK) return st;
    // line-major copy (the screened backward sweep keeps one line per wave and
    // the outages on the lanes) and the largest |factor| of each line
    std::vector<float>().swap(lodf32);
    d.Kp = round_up(std::max(1, h.K), 256);  // whole 256-outage chunks of the screened sweep
    std::vector<float> lt((size_t)std::max(1, h.L) * d.Kp, 0.0f);
    std::vector<float> amax(d.Lp, 0.0f);
    const int n_lb = (h.L + 63) / 64;
    ibp::parallel_for(n_lb, 1, [&](int64_t a, int64_t b) {
      for (int64_t lb = a; lb < b; ++lb) {
        // 64 lines at a time: each outage row is read as one contiguous run
        const int l0 = (int)lb * 64, l1 = std::min(h.L, l0 + 64);
        float am[64] = {};
        for (int k = 0; k < h.K; ++k) {
          const double* src = h.lodf.data() + (size_t)k * h.L;
          const int c = h.ctg_line[k];
          for (int l = l0; l < l1; ++l) {
            const float v = (float)src[l];
            lt[(size_t)l * d.Kp + k] = v;
            if (l != c) am[l - l0] = std::max(am[l - l0], std::fabs(v));
          }
        }
        for (int l = l0; l < l1; ++l)
          amax[l] = am[l - l0] == 0.0f ? 0.0f : std::nextafter(am[l - l0], std::numeric_limits<float>::infinity());
      }
    });
    for (int k = 0; k < h.K; ++k) lt[(size_t)h.ctg_line[k] * d.Kp + k] = std::numeric_limits<float>::quiet_NaN();
    if ((st = upload(net, lt.data(), lt.size(), &d.lodfT)) != IBP_OK) return st;
    if ((st = upload(net, amax.data(), amax.size(), &d.lam_max)) != IBP_OK) return st;
  }
  if ((st = upload(net, h.fmax_base.data(), h.L, &d.fmax_b)) != IBP_OK) return st;
  if ((st = upload(net, h.fmax_ctg.data(), h.L, &d.fmax_c)) != IBP_OK) return st;
  if ((st = upload(net, h.phi_err.data(), h.L, &d.phi_err)) != IBP_OK) return st;
  if ((st = upload(net, h.ctg_of_line.data(), h.L, &d.ctg_of_line)) != IBP_OK) return st;
  if ((st = upload(net, h.ctg_line.data(), h.K, &d.ctg_line)) != IBP_OK) return st;
  {
    // outage-factor error from the PTDF error (rank-1 update of Sec. II-C):
    // |dLam[l,k]| <= (2 eps_l + 2 |Lam| eps_c) / (1 - H_cc); the eps_c part goes into
    // the outage radius, the eps_l part is applied per tile with the box's
    // max_k (|c_c| + r_c) / (1 - H_cc)
    std::vector<double> eps(h.K), inv(h.K);
    for (int k = 0; k < h.K; ++k) {
      eps[k] = 2.0 * h.phi_err[h.ctg_line[k]] / h.one_m_hcc[k] * (1.0 + 1e-12);
      inv[k] = 1.0 / h.one_m_hcc[k] * (1.0 + 1e-12);
    }
    if ((st = upload(net, eps.data(), eps.size(), &d.ctg_eps)) != IBP_OK) return st;
    if ((st = upload(net, inv.data(), inv.size(), &d.ctg_inv)) != IBP_OK) return st;
    // the same constants indexed by line, so that a per-line kernel loads them
    // together with its other line data
    std::vector<double2> lk(std::max(1, h.L), make_double2(0.0, 0.0));
    for (int k = 0; k < h.K; ++k) lk[h.ctg_line[k]] = make_double2(eps[k], inv[k]);
    if ((st = upload(net, lk.data(), lk.size(), &d.line_ctg)) != IBP_OK) return st;
    std::vector<float> le(d.Lp, 0.0f);
    for (int l = 0; l < h.L; ++l) {
      // 2 eps_l plus the float32 subnormal spacing of a stored factor, rounded up
      const double v = (2.0 * h.phi_err[l] + std::ldexp(1.0, -149)) * (1.0 + 1.0 / 1024.0);
      float f = (float)v;
      if ((double)f < v) f = std::nextafter(f, std::numeric_limits<float>::infinity());
      le[l] = f;
    }
    if ((st = upload(net, le.data(), le.size(), &d.line_eps)) != IBP_OK) return st;
  }
  {
    std::vector<float> fc(d.Lp, std::numeric_limits<float>::max());
    for (int l = 0; l < h.L; ++l) fc[l] = (float)h.fmax_ctg[l];
    if ((st = upload(net, fc.data(), fc.size(), &d.fmax_c32)) != IBP_OK) return st;
    std::vector<int> db(h.G + h.D);
    for (int g = 0; g < h.G; ++g) db[g] = h.gen_bus[g];
    for (int j = 0; j < h.D; ++j) db[h.G + j] = h.load_bus[j];
    if ((st = upload(net, db.data(), db.size(), &d.dev_bus)) != IBP_OK) return st;
  }
  {
    const int X = h.G + h.D;
    std::vector<int> ptr(h.N + 1, 0), dev(X);
    std::vector<double> w(X);
    for (int g = 0; g < h.G; ++g) ptr[h.gen_bus[g] + 1]++;
    for (int j = 0; j < h.D; ++j) ptr[h.load_bus[j] + 1]++;
    for (int n = 0; n < h.N; ++n) ptr[n + 1] += ptr[n];
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int g = 0; g < h.G; ++g) dev[fill[h.gen_bus[g]]++] = g;
    for (int j = 0; j < h.D; ++j) dev[fill[h.load_bus[j]]++] = h.G + j;
    for (int g = 0; g < h.G; ++g) w[g] = -h.gen_cost[g];
    for (int j = 0; j < h.D; ++j) w[h.G + j] = h.load_value[j];
    if ((st = upload(net, ptr.data(), ptr.size(), &d.bus_ptr)) != IBP_OK) return st;
    if ((st = upload(net, dev.data(), dev.size(), &d.bus_dev)) != IBP_OK) return st;
    std::vector<int4> dev4(h.N, make_int4(-1, -1, -1, -1));
    for (int n = 0; n < h.N; ++n) {
      int* q = &dev4[n].x;
      for (int e = ptr[n]; e < std::min(ptr[n + 1], ptr[n] + 4); ++e) q[e - ptr[n]] = dev[e];
    }
    if ((st = upload(net, dev4.data(), dev4.size(), &d.bus_dev4)) != IBP_OK) return st;
    if ((st = upload(net, w.data(), w.size(), &d.dev_w)) != IBP_OK) return st;
  }
  d.seg_ptr = nullptr;
  d.seg = nullptr;
  if (!h.seg_ptr.empty()) {
    const size_t S = h.seg_a.size();
    std::vector<double4> seg(S);
    for (size_t i = 0; i < S; ++i) {
      const double U = h.seg_U[i];
      seg[i] = make_double4(h.seg_a[i], h.seg_b[i], U, std::isfinite(U) ? std::fabs(U) : 0.0);
    }
    if ((st = upload(net, h.seg_ptr.data(), h.seg_ptr.size(), &d.seg_ptr)) != IBP_OK) return st;
    if ((st = upload(net, seg.data(), seg.size(), &d.seg)) != IBP_OK) return st;
  }
  if (hipDeviceSynchronize() != hipSuccess) return fail(IBP_E_DEVICE, "device synchronize failed");
  // default tiles: the longest bus chunk that still gives the base-flow sweep
  // about 3.5 waves per CU (longer streams per wave beat more waves: at 8316
  // buses 512 buses per wave, 3.7 waves per CU, stream faster than 256 at
  // 7.1), and short outage chunks (many waves in flight)
  {
    const int lt = (d.Lp / 4 + 63) / 64;
    int nc = 32;
    for (int c : {512, 256, 128, 64}) {
      if ((int64_t)lt * ((h.N + c - 1) / c) * 2 >= 7LL * net->num_cus) {
        nc = c;
        break;
      }
    }
    net->tune.k2_nc = nc;
    net->tune.k3_kc = 16;
  }
  if (const char* e = std::getenv("IBP_TILE")) {
    ibp::Tune t = net->tune;
    int v = 0;
    if (const char* p = std::strstr(e, "k2nc=")) t.k2_nc = (v = std::atoi(p + 5)) ? v : t.k2_nc;
    if (const char* p = std::strstr(e, "k3kc=")) t.k3_kc = (v = std::atoi(p + 5)) ? v : t.k3_kc;
    if (const char* p = std::strstr(e, "k2b=")) t.k2b_mfma = std::atoi(p + 4) != 0;
    if (const char* p = std::strstr(e, "ckb=")) t.chord_nb = std::atoi(p + 4);
    if (const char* p = std::strstr(e, "bt=")) t.k3_bt = std::atoi(p + 3);
    if (const char* p = std::strstr(e, "rows=")) t.k3_rows = std::atoi(p + 5);
    if (const char* p = std::strstr(e, "xcd=")) t.k3_xcd = std::atoi(p + 4);
    if (const char* p = std::strstr(e, "k2by=")) t.k2_by = std::atoi(p + 5);
    if (const char* p = std::strstr(e, "k5s=")) t.k5_sparse = std::atoi(p + 4) != 0;
    if (const char* p = std::strstr(e, "k3s=")) t.k3_sparse = std::atoi(p + 4) != 0;
    if (const char* p = std::strstr(e, "scru=")) t.k3_scr = std::atoi(p + 5) != 0;
    if (ibp::tune_valid(t) && ibp::tune_batched_valid(t) && (t.chord_nb == 1 || t.chord_nb == 2 || t.chord_nb == 4)) net->tune = t;
  }
  return IBP_OK;
}

ibp::WsLayout layout_for(const ibp_network* net, int64_t n_box, const ibp::Tune& tune, bool batched);

// Box-tiled candidates of the autotuner around the current tiles `t`: the
// outage sweep's boxes per wave, outage rows (half, the rule's and twice) and
// block order, and the base flows' engine and bus chunks.
std::vector<ibp::Tune> sweep_candidates(const ibp_network* net, int64_t n_box, const ibp::Tune& t) {
  const ibp::DevNet& d = net->dn;
  std::vector<ibp::Tune> out;
  for (int bt : {2, 4, 8}) {
    const int64_t groups = ((n_box + bt - 1) / bt + 3) / 4;
    const int r = ibp::batched_rows_rule(d, (d.Lp / 4 + 63) / 64, groups);
    std::vector<int> rows{r};
    if (r / 2 >= 1) rows.push_back(r / 2);
    if (2 * r <= std::max(1, d.K / 16)) rows.push_back(2 * r);
    for (int rw : rows)
      for (int x : {0, 1}) {
        ibp::Tune c = t;
        c.k3_bt = bt;
        c.k3_rows = rw;
        c.k3_xcd = x;
        out.push_back(c);
      }
  }
  return out;
}

std::vector<ibp::Tune> flow_candidates(const ibp_network* net, const ibp::Tune& t) {
  std::vector<ibp::Tune> out;
  for (int by : {1, 2, 4, 8}) {
    if (by > 1 && by > net->dn.N / 256) break;
    ibp::Tune c = t;
    c.k2b_mfma = 1;
    c.k2_by = by;
    out.push_back(c);
  }
  ibp::Tune v = t;
  v.k2b_mfma = 0;
  v.k2_by = 0;
  out.push_back(v);
  return out;
}

// Appends the line screen's regions (masks, line records, tile maxima) to a
// box-tiled layout; fscreen says whether the screened forward sweep fits it
// (one outage-penalty partial per chunk of 64 kSparseQ outages in the
// finalize's slots).
void add_screen(const ibp::DevNet& d, const ibp::Tune& tune, int64_t n_box, ibp::WsLayout& lay) {
  const size_t B = (size_t)std::max<int64_t>(1, n_box);
  size_t off = lay.total;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  lay.k5s_tiles = (int)((B + ibp::kScreenBoxes - 1) / ibp::kScreenBoxes);
  const size_t tiles = (size_t)lay.k5s_tiles;
  lay.smask = take(tiles * (d.Lp / 64) * sizeof(uint64_t));
  lay.srec = take(tiles * d.Lp * ibp::kScreenRecFloats * sizeof(float));
  lay.k5w_bx = (d.Kp + 255) / 256;
  lay.sw = take(tiles * d.Kp * sizeof(float));
  lay.sz = take(tiles * lay.k5w_bx * sizeof(float));
  lay.total = off;
  const int n_chunk = (d.K + 64 * ibp::kSparseQ - 1) / (64 * ibp::kSparseQ);
  lay.fscreen = tune.k3_sparse && ibp::screen_fits(d, lay) && n_chunk <= lay.n_p3;
}

ibp::WsLayout layout(const ibp_network* net, int64_t n_box, uint32_t flags) {
  if (flags & IBP_F_AUTOTUNE) {
    // the largest layout over every tile pair (smallest tiles give most
    // partials), and from kBatchMin boxes on over every box-tiled candidate
    ibp::Tune t = net->tune;
    t.k2_nc = 32;
    t.k3_kc = 16;
    ibp::WsLayout big = layout_for(net, n_box, t, false);
    if (n_box >= ibp::kBatchMin) {
      for (const ibp::Tune& f : flow_candidates(net, net->tune))
        for (const ibp::Tune& c : sweep_candidates(net, n_box, f)) {
          ibp::WsLayout l = layout_for(net, n_box, c, true);
          // and the upper-penalty screen, timed on the chosen tiles
          if (net->dn.K > 0) add_screen(net->dn, c, n_box, l);
          if (l.total > big.total) big = l;
        }
    }
    return big;
  }
  const bool batched = n_box >= ibp::kBatchMin && !(flags & IBP_F_PLAIN);
  ibp::WsLayout lay = layout_for(net, n_box, net->tune, batched);
  if (flags & (IBP_F_BACKWARD | IBP_F_KEEP_PREP)) {
    const ibp::DevNet& d = net->dn;
    const size_t B = (size_t)std::max<int64_t>(1, n_box);
    ibp::plan_backward(d, lay);
    size_t off = lay.total;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off = align256(off + bytes);
      return o;
    };
    lay.lpart = take(B * lay.k5_by * d.Lp * 2 * sizeof(float));
    lay.cpart = take(B * lay.k5_tiles * std::max(1, d.K) * 2 * sizeof(float));
    lay.gcf = take(B * d.Lp * sizeof(float));
    lay.grf = take(B * d.Lp * sizeof(float));
    lay.gci = take(B * d.Np * sizeof(double));
    lay.gri = take(B * d.Np * sizeof(double));
    if (lay.batched && d.K > 0) {
      lay.cb = take(B * d.K * 2 * sizeof(float));
      lay.lcnt = take(B * d.Lp * sizeof(uint64_t));
    }
    lay.total = off;
  }
  // the line screen of the one-sided sweeps (the backward's gradient of f_hi,
  // the forward's one-sided bounds) and of screened calls bounding f_lo
  const bool one_sided = (flags & (IBP_F_UPPER_ONLY | IBP_F_LOWER_ONLY)) != 0;
  const bool scr_upper = (flags & IBP_F_SCREEN_UPPER) || (net->tune.k3_scr && !(flags & IBP_F_UPPER_ONLY));
  if (lay.batched && net->dn.K > 0 && (one_sided || scr_upper || (flags & (IBP_F_BACKWARD | IBP_F_KEEP_PREP)))) {
    add_screen(net->dn, net->tune, n_box, lay);
    const bool side_ok = (flags & IBP_F_UPPER_ONLY) || scr_upper;
    lay.fscreen = side_ok && lay.fscreen;
  } else {
    lay.fscreen = 0;
  }
  if (flags & (IBP_F_CROWN | IBP_F_CROWN_REF)) {
    const ibp::DevNet& d = net->dn;
    const size_t B = (size_t)std::max<int64_t>(1, n_box);
    ibp::plan_crown(d, n_box, lay, net->tune);
    size_t off = lay.total;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off = align256(off + bytes);
      return o;
    };
    lay.ccnt = take(B * d.Lp * 2 * sizeof(long long));  // int2 counts, or int64 slope totals
    lay.cv = take(B * lay.kc_bx * std::max(1, d.K) * 4 * sizeof(double));
    lay.lv = take(std::max<size_t>(B, (size_t)lay.kc3_bt) * d.Lp * 4 * sizeof(double));
    lay.bpart = take(B * lay.kc3_bx * d.Np * 4 * sizeof(double));
    lay.cp = take(B * lay.n_cp * 2 * sizeof(double));
    lay.ct = take(B * lay.n_ct * 4 * sizeof(double));
    if (lay.chp_z) lay.chp = take(B * lay.chp_z * d.Lp * 2 * sizeof(int));
    if (flags & IBP_F_CROWN_REF) {
      lay.ref = take(lay.fwd_total);
      lay.xref = take(B * d.X * sizeof(float));
      lay.vtx = take(B * d.X * sizeof(float));
    }
    lay.total = off;
  }
  return lay;
}

ibp::WsLayout layout_for(const ibp_network* net, int64_t n_box, const ibp::Tune& tune, bool batched = false) {
  const ibp::DevNet& d = net->dn;
  ibp::WsLayout lay;
  if (batched)
    ibp::plan_batched(d, n_box, lay, tune);
  else
    ibp::plan_single(d, n_box, lay, tune);
  const size_t B = (size_t)std::max<int64_t>(1, n_box);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  lay.inj = take(B * d.Np * 2 * sizeof(double));
  lay.p1 = take(B * lay.n_p1 * ibp::kP1Fields * sizeof(double));
  lay.part2 = take(B * lay.k2_by * d.Lp * 2 * sizeof(double));
  lay.box = take(B * ibp::kBoxSlots * sizeof(double));
  lay.lc = take(B * d.Lp * sizeof(float));
  lay.lh = take(B * d.Lp * sizeof(float));
  lay.lg = take(B * d.Lp * sizeof(float));
  lay.lcf = take(B * d.L * sizeof(double));
  lay.lrf = take(B * d.L * sizeof(double));
  lay.ctg = take(B * std::max(1, d.K) * 4 * sizeof(int));
  lay.p2 = take(B * std::max(1, lay.n_p2) * 2 * sizeof(double));
  lay.p3 = take(B * std::max(1, lay.n_p3) * 2 * sizeof(double));
  lay.total = off;
  lay.fwd_total = off;
  return lay;
}

ibp_status check_compute_args(const ibp_network* net, int64_t n_box, const void* lo, const void* hi,
                              const void* a, const void* b, void* ws, size_t ws_bytes,
                              uint32_t flags, ibp::WsLayout& lay) {
  if (!net) return fail(IBP_E_INVALID_ARG, "network handle is NULL");
  if (net->device < 0) return fail(IBP_E_HOST_ONLY, "network was built host-only");
  if (n_box < 0) return fail(IBP_E_INVALID_ARG, "n_box < 0");
  if (flags & ~uint32_t(IBP_F_PLAIN | IBP_F_BACKWARD | IBP_F_CROWN | IBP_F_CROWN_REF | IBP_F_UPPER_ONLY |
                        IBP_F_LOWER_ONLY | IBP_F_KEEP_PREP | IBP_F_REUSE_PREP | IBP_F_SCREEN_UPPER))
    return fail(IBP_E_INVALID_ARG, "unknown flag bits");
  if ((flags & IBP_F_SCREEN_UPPER) && (flags & IBP_F_UPPER_ONLY))
    return fail(IBP_E_INVALID_ARG, "IBP_F_SCREEN_UPPER is for calls that bound f_lo");
  if ((flags & IBP_F_UPPER_ONLY) && (flags & IBP_F_LOWER_ONLY))
    return fail(IBP_E_INVALID_ARG, "IBP_F_UPPER_ONLY and IBP_F_LOWER_ONLY exclude each other");
  if (n_box == 0) return IBP_OK;
  if (!lo || !hi || !a || !b) return fail(IBP_E_INVALID_ARG, "a required device pointer is NULL");
  lay = layout(net, n_box, flags);
  lay.sides = (flags & IBP_F_UPPER_ONLY) ? 1 : (flags & IBP_F_LOWER_ONLY) ? 2 : 3;
  if (!ws || ws_bytes < lay.total)
    return fail(IBP_E_WORKSPACE, "workspace needs " + std::to_string(lay.total) + " bytes, got " +
                                     std::to_string(ws_bytes));
  return IBP_OK;
}

// Box-tiled calls of more boxes than one launch sequence can take (the outage
// sweeps put 16 boxes per block along the third grid dimension, at most 65535)
// run as consecutive chunks on the same stream and workspace.
constexpr int64_t kTiledChunk = 16 * 65535;

// Calls f(first box, box count, layout) per chunk; the layout of every chunk
// fits in the workspace the whole call was checked against.
template <typename F>
ibp_status for_chunks(const ibp_network* net, int64_t n_box, uint32_t flags, const ibp::WsLayout& lay,
                      size_t ws_bytes, F f) {
  if (!lay.batched || n_box <= kTiledChunk) return f(0, n_box, lay);
  for (int64_t b = 0; b < n_box; b += kTiledChunk) {
    const int64_t nc = std::min(kTiledChunk, n_box - b);
    ibp::WsLayout lc = layout(net, nc, flags);
    lc.sides = lay.sides;
    if (lc.total > ws_bytes) return fail(IBP_E_WORKSPACE, "workspace too small for a chunk of the call");
    const ibp_status st = f(b, nc, lc);
    if (st != IBP_OK) return st;
  }
  return IBP_OK;
}

}  // namespace

extern "C" {

ibp_status ibp_build_network(const ibp_network_desc* desc, int device, ibp_network** out) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (!out) return fail(IBP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (device < IBP_DEVICE_HOST_ONLY) return fail(IBP_E_INVALID_ARG, "device ordinal out of range");
    // the handle is owned here until construction succeeds: a failure or an
    // exception at any step frees it and every device allocation it holds
    struct Owner {
      ibp_network* p;
      ~Owner() {
        if (p) {
          release_device(p);
          delete p;
        }
      }
    } own{new (std::nothrow) ibp_network()};
    if (!own.p) return fail(IBP_E_OUT_OF_MEMORY, "host allocation failed");
    ibp_network* net = own.p;
    std::string err;
    ibp_status st;
    try {
      st = ibp::build_host(desc, net->h, err);
    } catch (const std::bad_alloc&) {
      st = IBP_E_OUT_OF_MEMORY;
      err = "host allocation failed during construction";
    }
    if (st != IBP_OK) return fail(st, err);
    if (device >= 0) {
      try {
        st = to_device(net, device);
      } catch (const std::bad_alloc&) {
        st = fail(IBP_E_OUT_OF_MEMORY, "host allocation failed while packing float32 factors");
      }
      if (st != IBP_OK) return st;  // the message is set; Owner frees the handle
    }
    own.p = nullptr;
    *out = net;
    return IBP_OK;
  });
}

ibp_status ibp_network_query(const ibp_network* net, ibp_network_info* info) {
  return guarded([&]() -> ibp_status {
    if (!net || !info) return fail(IBP_E_INVALID_ARG, "NULL argument");
    info->n_bus = net->h.N;
    info->n_line = net->h.L;
    info->n_ctg = net->h.K;
    info->n_gen = net->h.G;
    info->n_load = net->h.D;
    info->n_input = net->h.G + net->h.D;
    info->device = net->device;
    info->min_one_minus_hcc = net->h.min_one_m_hcc;
    info->phi_abs_err = net->h.phi_err_max;
    info->device_bytes = net->device_bytes;
    info->build_seconds = net->h.build_seconds;
    return IBP_OK;
  });
}

ibp_status ibp_network_ctg_lines(const ibp_network* net, int32_t* out) {
  return guarded([&]() -> ibp_status {
    if (!net || (!out && net->h.K > 0)) return fail(IBP_E_INVALID_ARG, "NULL argument");
    if (net->h.K) std::memcpy(out, net->h.ctg_line.data(), sizeof(int32_t) * net->h.K);
    return IBP_OK;
  });
}

ibp_status ibp_network_export(const ibp_network* net, double* ptdf, double* lodf) {
  return guarded([&]() -> ibp_status {
    if (!net) return fail(IBP_E_INVALID_ARG, "network handle is NULL");
    // (no copy at all from an empty matrix: K = 0 leaves the outage factors empty)
    if (ptdf && !net->h.phi.empty()) std::memcpy(ptdf, net->h.phi.data(), sizeof(double) * net->h.phi.size());
    if (lodf && !net->h.lodf.empty()) std::memcpy(lodf, net->h.lodf.data(), sizeof(double) * net->h.lodf.size());
    return IBP_OK;
  });
}

void ibp_free_network(ibp_network* net) {
  if (!net) return;
  release_device(net);
  delete net;
}

size_t ibp_workspace_bytes(const ibp_network* net, int64_t n_box, uint32_t flags) {
  if (!net || net->device < 0 || n_box < 0) return 0;
  try {
    return layout(net, n_box, flags).total;
  } catch (...) {
    set_err("host allocation failed");
    return 0;
  }
}

ibp_status ibp_bound_boxes(const ibp_network* net, int64_t n_box, const float* box_lo,
                           const float* box_hi, double* f_lo, double* f_hi, double* terms, void* ws,
                           size_t ws_bytes, void* stream, uint32_t flags) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    ibp::WsLayout lay;
    if (flags & IBP_F_REUSE_PREP) return fail(IBP_E_INVALID_ARG, "IBP_F_REUSE_PREP is a backward flag");
    ibp_status st = check_compute_args(net, n_box, box_lo, box_hi, f_lo, f_hi, ws, ws_bytes, flags, lay);
    if (st != IBP_OK || n_box == 0) return st;
    DeviceGuard g(net->device);
    if (!g.ok) return fail(IBP_E_DEVICE, "hipSetDevice failed");
    prep_forget(net, ws);
    const int64_t X = net->dn.X;
    st = for_chunks(net, n_box, flags, lay, ws_bytes, [&](int64_t b, int64_t nc, const ibp::WsLayout& lc) {
      hipError_t e = ibp::launch_forward(net->dn, nc, box_lo + b * X, box_hi + b * X, f_lo + b, f_hi + b,
                                         terms ? terms + 8 * b : nullptr, ws, lc, static_cast<hipStream_t>(stream),
                                         const_cast<ibp::KernelTimer*>(&net->timer));
      if (e != hipSuccess) return fail(IBP_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
      return IBP_OK;
    });
    // one pass over all boxes (a call split into chunks keeps only its last chunk's)
    if (st == IBP_OK && (flags & IBP_F_KEEP_PREP) && (!lay.batched || n_box <= kTiledChunk))
      prep_record(net, PrepTag{ws, n_box, box_lo, box_hi, (flags & IBP_F_PLAIN) != 0, net->tile_gen});
    return st;
  });
}

ibp_status ibp_bound_boxes_noalloc(const ibp_network* net, int64_t n_box, const float* box_lo,
                                   const float* box_hi, double* f_lo, double* f_hi, double* terms, void* stream,
                                   uint32_t flags) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (!net) return fail(IBP_E_INVALID_ARG, "network handle is NULL");
    if (net->device < 0) return fail(IBP_E_HOST_ONLY, "network was built host-only");
    if (flags & ~uint32_t(IBP_F_PLAIN | IBP_F_UPPER_ONLY | IBP_F_LOWER_ONLY | IBP_F_SCREEN_UPPER))
      return fail(IBP_E_INVALID_ARG,
                  "flags: only IBP_F_PLAIN, IBP_F_UPPER_ONLY, IBP_F_LOWER_ONLY and IBP_F_SCREEN_UPPER are accepted");
    if ((flags & IBP_F_SCREEN_UPPER) && (flags & IBP_F_UPPER_ONLY))
      return fail(IBP_E_INVALID_ARG, "IBP_F_SCREEN_UPPER is for calls that bound f_lo");
    if (n_box < 0) return fail(IBP_E_INVALID_ARG, "n_box < 0");
    if (n_box == 0) return IBP_OK;
    const size_t need = layout(net, n_box, flags).total;
    if (need > IBP_NOALLOC_SCRATCH_BYTES)
      return fail(IBP_E_WORKSPACE, std::to_string(n_box) + " boxes need " + std::to_string(need) +
                                       " bytes of workspace, more than the " +
                                       std::to_string((size_t)IBP_NOALLOC_SCRATCH_BYTES) +
                                       " bytes of the library's scratch: use ibp_bound_boxes with a workspace, "
                                       "or fewer boxes per call");
    DeviceGuard g(net->device);
    if (!g.ok) return fail(IBP_E_DEVICE, "hipSetDevice failed");
    void* ws = nullptr;
    ibp_status st = scratch_address(net->device, &ws);
    if (st != IBP_OK) return st;
    ibp::WsLayout lay;
    st = check_compute_args(net, n_box, box_lo, box_hi, f_lo, f_hi, ws, IBP_NOALLOC_SCRATCH_BYTES, flags, lay);
    if (st != IBP_OK) return st;
    // no kernel timing here: its events would be created per call
    ibp::KernelTimer off;
    const int64_t X = net->dn.X;
    return for_chunks(net, n_box, flags, lay, IBP_NOALLOC_SCRATCH_BYTES,
                      [&](int64_t b, int64_t nc, const ibp::WsLayout& lc) {
                        hipError_t e = ibp::launch_forward(net->dn, nc, box_lo + b * X, box_hi + b * X, f_lo + b,
                                                           f_hi + b, terms ? terms + 8 * b : nullptr, ws, lc,
                                                           static_cast<hipStream_t>(stream), &off);
                        if (e != hipSuccess)
                          return fail(IBP_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
                        return IBP_OK;
                      });
  });
}

ibp_status ibp_bound_backward(const ibp_network* net, int64_t n_box, const float* box_lo,
                              const float* box_hi, const double* g_f_lo, const double* g_f_hi,
                              double* g_box_lo, double* g_box_hi, void* ws, size_t ws_bytes,
                              void* stream, uint32_t flags) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    ibp::WsLayout lay;
    // one-sided: the weight of the other bound is not read (taken as zero)
    const bool up = flags & IBP_F_UPPER_ONLY, low = flags & IBP_F_LOWER_ONLY;
    ibp_status st = check_compute_args(net, n_box, box_lo, box_hi, up ? g_f_hi : g_f_lo, low ? g_f_lo : g_f_hi, ws,
                                       ws_bytes, flags | IBP_F_BACKWARD, lay);
    if (st != IBP_OK || n_box == 0) return st;
    if (!g_box_lo || !g_box_hi) return fail(IBP_E_INVALID_ARG, "a required device pointer is NULL");
    if (up) g_f_lo = nullptr;
    if (low) g_f_hi = nullptr;
    if (flags & IBP_F_KEEP_PREP) return fail(IBP_E_INVALID_ARG, "IBP_F_KEEP_PREP is a forward flag");
    const PrepTag tag{ws, n_box, box_lo, box_hi, (flags & IBP_F_PLAIN) != 0, net->tile_gen};
    const bool reuse = (flags & IBP_F_REUSE_PREP) != 0;
    if (reuse && !prep_matches(net, tag))
      return fail(IBP_E_INVALID_ARG,
                  "IBP_F_REUSE_PREP: the workspace does not hold the forward intermediates of these boxes (an "
                  "ibp_bound_boxes call with IBP_F_KEEP_PREP on the same boxes, flags, tiles and workspace)");
    DeviceGuard g(net->device);
    if (!g.ok) return fail(IBP_E_DEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    ibp::KernelTimer* tm = const_cast<ibp::KernelTimer*>(&net->timer);
    const int64_t X = net->dn.X;
    if (!reuse) prep_forget(net, ws);
    st = for_chunks(net, n_box, flags | IBP_F_BACKWARD, lay, ws_bytes,
                    [&](int64_t b, int64_t nc, const ibp::WsLayout& lc) {
                      const float *lo = box_lo + b * X, *hi = box_hi + b * X;
                      hipError_t e = reuse ? hipSuccess : ibp::launch_forward_prep(net->dn, nc, lo, hi, ws, lc, s, tm);
                      if (e == hipSuccess)
                        e = ibp::launch_backward_sweeps(net->dn, nc, ws, lc, lo, hi, g_f_lo ? g_f_lo + b : nullptr,
                                                        g_f_hi ? g_f_hi + b : nullptr, g_box_lo + b * X,
                                                        g_box_hi + b * X, net->tune.k5_sparse != 0, s, tm);
                      if (e != hipSuccess)
                        return fail(IBP_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
                      return IBP_OK;
                    });
    // the backward leaves the forward intermediates of its boxes in the workspace
    if (st == IBP_OK && !reuse && (!lay.batched || n_box <= kTiledChunk)) prep_record(net, tag);
    return st;
  });
}

ibp_status ibp_backward_screen_lines(const ibp_network* net, int64_t n_box, const void* ws, size_t ws_bytes,
                                     void* stream, int64_t* n_marked, int64_t* n_pairs) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (!net || !ws || !n_marked || !n_pairs) return fail(IBP_E_INVALID_ARG, "NULL argument");
    if (net->device < 0) return fail(IBP_E_HOST_ONLY, "the network was built without a device");
    if (n_box < ibp::kBatchMin || n_box > kTiledChunk || net->dn.K == 0)
      return fail(IBP_E_INVALID_ARG, "no screened sweep for this number of boxes or network");
    const ibp::WsLayout lay = layout(net, n_box, IBP_F_BACKWARD);
    if (!lay.batched || lay.k5s_tiles == 0) return fail(IBP_E_INVALID_ARG, "no screened sweep for these sizes");
    if (ws_bytes < lay.total) return fail(IBP_E_WORKSPACE, "workspace smaller than the backward call's");
    DeviceGuard g(net->device);
    if (!g.ok) return fail(IBP_E_DEVICE, "hipSetDevice failed");
    const size_t words = (size_t)net->dn.Lp / 64, n = (size_t)lay.k5s_tiles * words;
    std::vector<uint64_t> m(n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(m.data(), static_cast<const char*>(ws) + lay.smask, n * sizeof(uint64_t),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(IBP_E_DEVICE, "copy of the screen's line masks failed");
    int64_t c = 0;
    for (uint64_t v : m) c += __builtin_popcountll(v);
    *n_marked = c;
    *n_pairs = (int64_t)lay.k5s_tiles * net->dn.L;
    return IBP_OK;
  });
}

ibp_status ibp_crown_bound_boxes(const ibp_network* net, int64_t n_box, const float* box_lo,
                                 const float* box_hi, int32_t ref_iters, double* f_lo, double* f_hi,
                                 double* crown_hi, float* vertex, void* ws, size_t ws_bytes, void* stream,
                                 uint32_t flags) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (flags & ~uint32_t(IBP_F_PLAIN | IBP_F_UPPER_ONLY))
      return fail(IBP_E_INVALID_ARG, "flags: only IBP_F_PLAIN and IBP_F_UPPER_ONLY are accepted");
    if (ref_iters < 0 || ref_iters > 64) return fail(IBP_E_INVALID_ARG, "ref_iters must be in [0, 64]");
    ibp::WsLayout lay;
    const uint32_t need = flags | IBP_F_CROWN | (ref_iters > 0 ? IBP_F_CROWN_REF : 0u);
    ibp_status st = check_compute_args(net, n_box, box_lo, box_hi, f_lo, f_hi, ws, ws_bytes, need, lay);
    if (st != IBP_OK || n_box == 0) return st;
    DeviceGuard g(net->device);
    if (!g.ok) return fail(IBP_E_DEVICE, "hipSetDevice failed");
    prep_forget(net, ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    ibp::KernelTimer* tm = const_cast<ibp::KernelTimer*>(&net->timer);
    const int64_t X = net->dn.X;
    return for_chunks(net, n_box, need, lay, ws_bytes, [&](int64_t b, int64_t nc, const ibp::WsLayout& lc) {
      const float *lo = box_lo + b * X, *hi = box_hi + b * X;
      hipError_t e = ibp::launch_forward(net->dn, nc, lo, hi, f_lo + b, f_hi + b, nullptr, ws, lc, s, tm);
      if (e == hipSuccess)
        e = ibp::launch_crown(net->dn, nc, lo, hi, ref_iters, f_hi + b, crown_hi ? crown_hi + b : nullptr,
                              vertex ? vertex + b * X : nullptr, ws, lc, s, tm);
      if (e != hipSuccess) return fail(IBP_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
      return IBP_OK;
    });
  });
}

ibp_status ibp_crown_lower_boxes(const ibp_network* net, int64_t n_box, const float* box_lo,
                                 const float* box_hi, double* f_lo, double* f_hi, double* crown_lo, float* vertex,
                                 void* ws, size_t ws_bytes, void* stream, uint32_t flags) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (flags & ~uint32_t(IBP_F_PLAIN | IBP_F_LOWER_ONLY))
      return fail(IBP_E_INVALID_ARG, "flags: only IBP_F_PLAIN and IBP_F_LOWER_ONLY are accepted");
    ibp::WsLayout lay;
    const uint32_t need = flags | IBP_F_CROWN;
    ibp_status st = check_compute_args(net, n_box, box_lo, box_hi, f_lo, f_hi, ws, ws_bytes, need, lay);
    if (st != IBP_OK) return st;
    if (n_box == 0) return IBP_OK;
    DeviceGuard g(net->device);
    if (!g.ok) return fail(IBP_E_DEVICE, "hipSetDevice failed");
    prep_forget(net, ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    ibp::KernelTimer* tm = const_cast<ibp::KernelTimer*>(&net->timer);
    const int64_t X = net->dn.X;
    return for_chunks(net, n_box, need, lay, ws_bytes, [&](int64_t b, int64_t nc, const ibp::WsLayout& lc) {
      const float *lo = box_lo + b * X, *hi = box_hi + b * X;
      hipError_t e = ibp::launch_forward(net->dn, nc, lo, hi, f_lo + b, f_hi + b, nullptr, ws, lc, s, tm);
      if (e == hipSuccess)
        e = ibp::launch_crown_lower(net->dn, nc, lo, hi, f_lo + b, crown_lo ? crown_lo + b : nullptr,
                                    vertex ? vertex + b * X : nullptr, ws, lc, s, tm);
      if (e != hipSuccess) return fail(IBP_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
      return IBP_OK;
    });
  });
}

ibp_status ibp_set_kernel_timing(ibp_network* net, int enable) {
  return guarded([&]() -> ibp_status {
    if (!net) return fail(IBP_E_INVALID_ARG, "network handle is NULL");
    if (net->device < 0) return fail(IBP_E_HOST_ONLY, "network was built host-only");
    net->timer.enabled = enable != 0;
    return IBP_OK;
  });
}

ibp_status ibp_kernel_times(ibp_network* net, int32_t n_ids, double* total_ms, int64_t* count) {
  return guarded([&]() -> ibp_status {
    if (!net || !total_ms || !count || n_ids < 0) return fail(IBP_E_INVALID_ARG, "NULL argument");
    if (net->device < 0) return fail(IBP_E_HOST_ONLY, "network was built host-only");
    DeviceGuard g(net->device);
    for (int i = 0; i < n_ids; ++i) {
      total_ms[i] = 0.0;
      count[i] = 0;
    }
    ibp_status st = IBP_OK;
    for (auto& r : net->timer.recs) {
      float ms = 0.0f;
      if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
        st = fail(IBP_E_DEVICE, "reading kernel timing events failed");
        continue;
      }
      if (r.id >= 0 && r.id < n_ids) {
        total_ms[r.id] += ms;
        count[r.id] += 1;
      }
    }
    clear_timer(net);
    return st;
  });
}

ibp_status ibp_set_tile(ibp_network* net, int32_t k2_nc, int32_t k3_kc) {
  return guarded([&]() -> ibp_status {
    if (!net) return fail(IBP_E_INVALID_ARG, "network handle is NULL");
    ibp::Tune t = net->tune;
    t.k2_nc = k2_nc;
    t.k3_kc = k3_kc;
    if (!ibp::tune_valid(t)) return fail(IBP_E_INVALID_ARG, "unsupported tile parameters");
    net->tune = t;
    ++net->tile_gen;
    return IBP_OK;
  });
}

ibp_status ibp_autotune(ibp_network* net, int64_t n_box, const float* box_lo, const float* box_hi,
                        void* ws, size_t ws_bytes, void* stream, int32_t* chosen) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (!net) return fail(IBP_E_INVALID_ARG, "network handle is NULL");
    if (net->device < 0) return fail(IBP_E_HOST_ONLY, "network was built host-only");
    if (n_box <= 0 || !box_lo || !box_hi) return fail(IBP_E_INVALID_ARG, "need at least one device box");
    const ibp::WsLayout big = layout(net, n_box, IBP_F_AUTOTUNE);
    if (!ws || ws_bytes < big.total)
      return fail(IBP_E_WORKSPACE, "autotune workspace needs " + std::to_string(big.total) + " bytes");
    DeviceGuard g(net->device);
    if (!g.ok) return fail(IBP_E_DEVICE, "hipSetDevice failed");
    prep_forget(net, ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // events and scratch outputs for the timing runs
    TuneScratch sc;
    if (!sc.init(sizeof(double) * 2 * n_box)) return fail(IBP_E_OUT_OF_MEMORY, "autotune events or output buffer");
    double* f = static_cast<double*>(sc.buf);
    const hipEvent_t e0 = sc.e0, e1 = sc.e1;
    const int ncs[] = {32, 64, 128, 256, 512};
    const int kcs[] = {16, 32, 64, 128};
    float best = 1e30f;
    ibp::Tune best_t = net->tune;
    ibp::KernelTimer off;
    ibp_status st = IBP_OK;
    for (int nc : ncs) {
      for (int kc : kcs) {
        ibp::Tune t = net->tune;
        t.k2_nc = nc;
        t.k3_kc = kc;
        const ibp::WsLayout lay = layout_for(net, n_box, t, false);
        float ms = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {  // first round warms up
          (void)hipEventRecord(e0, s);
          for (int it = 0; it < 3; ++it)
            if (ibp::launch_forward_single(net->dn, n_box, box_lo, box_hi, f, f + n_box, nullptr, ws, lay, s,
                                           &off) != hipSuccess)
              st = fail(IBP_E_DEVICE, "autotune launch failed");
          (void)hipEventRecord(e1, s);
          if (hipEventSynchronize(e1) != hipSuccess) st = fail(IBP_E_DEVICE, "autotune synchronize failed");
          (void)hipEventElapsedTime(&ms, e0, e1);
        }
        if (st == IBP_OK && ms < best) {
          best = ms;
          best_t = t;
        }
      }
    }
    if (st != IBP_OK) return st;
    net->tune = best_t;
    ++net->tile_gen;
    if (chosen) {
      chosen[0] = best_t.k2_nc;
      chosen[1] = best_t.k3_kc;
    }
    return IBP_OK;
  });
}

ibp_status ibp_set_tile_batched(ibp_network* net, int32_t k3_bt, int32_t k3_rows, int32_t k3_xcd, int32_t k2_mfma,
                                int32_t k2_by) {
  return guarded([&]() -> ibp_status {
    if (!net) return fail(IBP_E_INVALID_ARG, "network handle is NULL");
    ibp::Tune t = net->tune;
    t.k3_bt = k3_bt;
    t.k3_rows = k3_rows;
    t.k3_xcd = k3_xcd;
    t.k2b_mfma = k2_mfma;
    t.k2_by = k2_by;
    if (!ibp::tune_batched_valid(t)) return fail(IBP_E_INVALID_ARG, "unsupported box-tiled tile parameters");
    net->tune = t;
    ++net->tile_gen;
    return IBP_OK;
  });
}

ibp_status ibp_set_screen_upper(ibp_network* net, int32_t on) {
  return guarded([&]() -> ibp_status {
    if (!net) return fail(IBP_E_INVALID_ARG, "network handle is NULL");
    if (on != 0 && on != 1) return fail(IBP_E_INVALID_ARG, "on must be 0 or 1");
    net->tune.k3_scr = on;
    ++net->tile_gen;
    return IBP_OK;
  });
}

ibp_status ibp_get_screen_upper(const ibp_network* net, int32_t* on) {
  return guarded([&]() -> ibp_status {
    if (!net || !on) return fail(IBP_E_INVALID_ARG, "NULL argument");
    *on = net->tune.k3_scr;
    return IBP_OK;
  });
}

ibp_status ibp_get_tile(const ibp_network* net, int32_t* out) {
  return guarded([&]() -> ibp_status {
    if (!net || !out) return fail(IBP_E_INVALID_ARG, "NULL argument");
    const ibp::Tune& t = net->tune;
    const int32_t v[7] = {t.k2_nc, t.k3_kc, t.k3_bt, t.k3_rows, t.k3_xcd, t.k2b_mfma, t.k2_by};
    std::memcpy(out, v, sizeof(v));
    return IBP_OK;
  });
}

ibp_status ibp_autotune_batched(ibp_network* net, int64_t n_box, const float* box_lo, const float* box_hi,
                                void* ws, size_t ws_bytes, void* stream, int32_t* chosen) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (!net) return fail(IBP_E_INVALID_ARG, "network handle is NULL");
    if (net->device < 0) return fail(IBP_E_HOST_ONLY, "network was built host-only");
    if (n_box < ibp::kBatchMin || !box_lo || !box_hi)
      return fail(IBP_E_INVALID_ARG, "the box-tiled autotuner needs at least 4 device boxes");
    if (n_box > 16 * 65535) return fail(IBP_E_INVALID_ARG, "too many boxes for one tuning launch");
    const ibp::WsLayout big = layout(net, n_box, IBP_F_AUTOTUNE);
    if (!ws || ws_bytes < big.total)
      return fail(IBP_E_WORKSPACE, "autotune workspace needs " + std::to_string(big.total) + " bytes");
    DeviceGuard g(net->device);
    if (!g.ok) return fail(IBP_E_DEVICE, "hipSetDevice failed");
    prep_forget(net, ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    TuneScratch sc;
    if (!sc.init(0)) return fail(IBP_E_DEVICE, "autotune events");
    const hipEvent_t e0 = sc.e0, e1 = sc.e1;
    ibp::KernelTimer off;
    ibp_status st = IBP_OK;
    auto time_it = [&](auto launch) {
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {  // the first run warms up
        float ms = 0.0f;
        (void)hipEventRecord(e0, s);
        if (launch() != hipSuccess) st = fail(IBP_E_DEVICE, "autotune launch failed");
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) st = fail(IBP_E_DEVICE, "autotune synchronize failed");
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) best = std::min(best, ms);
      }
      return best;
    };
    // base flows: box preparation once, then every engine / chunking (each
    // writes only its own partials)
    ibp::Tune best_t = net->tune;
    {
      float best = 1e30f;
      for (const ibp::Tune& c : flow_candidates(net, net->tune)) {
        ibp::WsLayout lay = layout_for(net, n_box, c, true);
        if (ibp::launch_forward_prep(net->dn, n_box, box_lo, box_hi, ws, lay, s, &off) != hipSuccess)
          st = fail(IBP_E_DEVICE, "autotune preparation failed");
        const float ms = time_it([&] { return ibp::launch_batched_sweeps(net->dn, n_box, ws, lay, s, &off, 0); });
        if (st == IBP_OK && ms < best) {
          best = ms;
          best_t.k2b_mfma = c.k2b_mfma;
          best_t.k2_by = c.k2_by;
        }
      }
    }
    // outage sweep: the chosen base flows prepared once, then every candidate
    // (the line data sit before the per-call partials, at the same offsets)
    if (st == IBP_OK && net->dn.K > 0) {
      ibp::WsLayout prep = layout_for(net, n_box, best_t, true);
      if (ibp::launch_forward_prep(net->dn, n_box, box_lo, box_hi, ws, prep, s, &off) != hipSuccess)
        st = fail(IBP_E_DEVICE, "autotune preparation failed");
      float best = 1e30f;
      ibp::Tune pick = best_t;
      for (const ibp::Tune& c : sweep_candidates(net, n_box, best_t)) {
        ibp::WsLayout lay = layout_for(net, n_box, c, true);
        const float ms = time_it([&] { return ibp::launch_batched_sweeps(net->dn, n_box, ws, lay, s, &off, 1); });
        if (st == IBP_OK && ms < best) {
          best = ms;
          pick = c;
        }
      }
      best_t = pick;
      // the two-sided sweep over the lines the upper-penalty screen marks,
      // against the dense one just picked (it pays where few lines carry an
      // active upper penalty: narrow boxes)
      ibp::Tune ts = best_t;
      ts.k3_sparse = 1;
      ibp::WsLayout lay = layout_for(net, n_box, ts, true);
      add_screen(net->dn, ts, n_box, lay);
      best_t.k3_scr = 0;
      if (lay.fscreen) {
        lay.sides = 3;
        const float ms = time_it([&] { return ibp::launch_batched_sweeps(net->dn, n_box, ws, lay, s, &off, 1); });
        if (st == IBP_OK && ms < best) best_t.k3_scr = 1;
      }
    }
    if (st != IBP_OK) return st;
    net->tune = best_t;
    ++net->tile_gen;
    if (chosen) {
      chosen[0] = best_t.k3_bt;
      chosen[1] = best_t.k3_rows;
      chosen[2] = best_t.k3_xcd;
      chosen[3] = best_t.k2b_mfma;
      chosen[4] = best_t.k2_by;
    }
    return IBP_OK;
  });
}

ibp_status ibp_split_select(int64_t n_act, const int64_t* roots, int32_t slots, const int32_t* n_leaf,
                            int32_t n_input, const float* leaf_lo, const float* leaf_hi, const double* leaf_fhi,
                            int64_t* sel, float* sel_lo, float* sel_hi, void* stream) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (n_act < 0 || slots < 1 || n_input < 1) return fail(IBP_E_INVALID_ARG, "bad split sizes");
    if (n_act == 0) return IBP_OK;
    if (n_act > 0x7fffffff) return fail(IBP_E_INVALID_ARG, "too many roots");
    if (!n_leaf || !leaf_lo || !leaf_hi || !leaf_fhi || !sel || !sel_lo || !sel_hi)
      return fail(IBP_E_INVALID_ARG, "a required device pointer is NULL");
    hipError_t e = ibp::launch_split_select(n_act, roots, slots, n_leaf, n_input, leaf_lo, leaf_hi, leaf_fhi, sel,
                                            sel_lo, sel_hi, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IBP_OK : fail(IBP_E_DEVICE, hipGetErrorString(e));
  });
}

ibp_status ibp_split_bisect(int64_t n_act, const int64_t* roots, int32_t slots, const int32_t* n_leaf,
                            int32_t n_input, float* leaf_lo, float* leaf_hi, const int64_t* sel,
                            const float* sel_lo, const float* sel_hi, const double* g_lo, const double* g_hi,
                            float* kid_lo, float* kid_hi, float* centers, void* stream) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (n_act < 0 || slots < 2 || n_input < 1) return fail(IBP_E_INVALID_ARG, "bad split sizes (need slots >= 2)");
    if (n_act == 0) return IBP_OK;
    if (n_act > 0x7fffffff) return fail(IBP_E_INVALID_ARG, "too many roots");
    if (!n_leaf || !leaf_lo || !leaf_hi || !sel || !sel_lo || !sel_hi || !g_lo || !g_hi || !kid_lo || !kid_hi ||
        !centers)
      return fail(IBP_E_INVALID_ARG, "a required device pointer is NULL");
    hipError_t e = ibp::launch_split_bisect(n_act, roots, slots, n_leaf, n_input, leaf_lo, leaf_hi, sel, sel_lo,
                                            sel_hi, g_lo, g_hi, kid_lo, kid_hi, centers,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IBP_OK : fail(IBP_E_DEVICE, hipGetErrorString(e));
  });
}

ibp_status ibp_split_update(int64_t n_act, const int64_t* roots, int32_t slots, int32_t* n_leaf,
                            const int64_t* sel, const double* kid_fhi, int32_t points_per_root,
                            const double* point_flo, const float* points, int32_t n_input, double* leaf_fhi,
                            double* root_ub, double* root_lb, float* root_x, void* stream) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (n_act < 0 || slots < 2 || points_per_root < 0 || n_input < 1)
      return fail(IBP_E_INVALID_ARG, "bad split sizes");
    if (n_act == 0) return IBP_OK;
    if (n_act > 0x7fffffff) return fail(IBP_E_INVALID_ARG, "too many roots");
    if (!n_leaf || !sel || !kid_fhi || !leaf_fhi || !root_ub || !root_lb ||
        (points_per_root > 0 && !point_flo) || (root_x && points_per_root > 0 && !points))
      return fail(IBP_E_INVALID_ARG, "a required device pointer is NULL");
    hipError_t e = ibp::launch_split_update(n_act, roots, slots, n_leaf, sel, kid_fhi, points_per_root, point_flo,
                                            points, n_input, leaf_fhi, root_ub, root_lb, root_x,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IBP_OK : fail(IBP_E_DEVICE, hipGetErrorString(e));
  });
}

ibp_status ibp_split_screen(int64_t n_root, const double* root_ub, const double* root_lb, double rel_tol,
                            int32_t* status, int64_t* open_roots, int64_t* n_open, void* stream) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (n_root < 0 || !(rel_tol >= 0.0)) return fail(IBP_E_INVALID_ARG, "bad screening arguments");
    if (!root_ub || !root_lb || !status || !open_roots || !n_open)
      return fail(IBP_E_INVALID_ARG, "a required device pointer is NULL");
    hipError_t e = ibp::launch_split_screen(n_root, root_ub, root_lb, rel_tol, status, open_roots, n_open,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IBP_OK : fail(IBP_E_DEVICE, hipGetErrorString(e));
  });
}

ibp_status ibp_read_probe(const void* src, int64_t n_float4, float* partial, void* stream) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (!src || !partial || n_float4 < 1) return fail(IBP_E_INVALID_ARG, "read probe needs a buffer and a size");
    if (reinterpret_cast<uintptr_t>(src) % 16 != 0) return fail(IBP_E_INVALID_ARG, "read probe source not 16-byte aligned");
    hipError_t e = ibp::launch_read_probe(static_cast<const float4*>(src), n_float4, partial,
                                          static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IBP_OK : fail(IBP_E_DEVICE, hipGetErrorString(e));
  });
}

ibp_status ibp_alu_probe(float* out, int64_t iters, int32_t scalar_operand, void* stream) {
  return guarded([&]() -> ibp_status {
    g_err[0] = 0;
    if (!out || iters < 1 || iters > (int64_t(1) << 24) || (scalar_operand != 0 && scalar_operand != 1))
      return fail(IBP_E_INVALID_ARG, "ALU probe needs an output, 1 <= iters <= 2^24 and an operand mode of 0 or 1");
    hipError_t e = ibp::launch_alu_probe(out, iters, scalar_operand, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IBP_OK : fail(IBP_E_DEVICE, hipGetErrorString(e));
  });
}

const char* ibp_last_error(void) { return g_err; }

}  // extern "C"
