// Float64 host construction of the network factors (the one-off setup step).
//
//  * Reduced admittance Y_Br = E_r^T Y_D E_r (Sec. II-A), dense, slack removed.
//  * Its inverse through a blocked Cholesky factor: Y_Br = C C^T, W = C^{-1},
//    Y_Br^{-1} = W^T W.
//  * PTDF rows  Phi[l, :] = b_l (Y_Br^{-1}[from_l, :] - Y_Br^{-1}[to_l, :]),
//    i.e. Phi_r = Y_D E_r Y_Br^{-1} of eq. (line flow ptdf), slack column zero.
//  * Outage factors from the rank-1 update of Sec. II-C: with
//    H[l, m] = Phi[l, from_m] - Phi[l, to_m], the post-outage flow of line l
//    after losing line c is f_l + H[l, c] / (1 - H[c, c]) * f_c, which is the
//    paper's eq. (ctg flow simplified) written per line (the factor
//    H[l, c] / (1 - H[c, c]) equals -B[k, l] / b_c with the paper's B).
//  * An a-posteriori bound on the PTDF error from the residual
//    R = Phi_r Y_Br - Y_D E_r:  |Phi_r - Phi_exact| <= |R| |Y_Br^{-1}|.
//
// Everything here is plain C++ (no HIP); the work is split over host threads.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <limits>
#include <cstring>
#include <exception>
#include <functional>
#include <mutex>
#include <queue>
#include <utility>
#include <thread>
#include <cstdlib>

#include "ibp_internal.h"

namespace ibp {

void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& body) {
  if (n <= 0) return;
  unsigned hw = std::thread::hardware_concurrency();
  if (const char* e = std::getenv("IBP_HOST_THREADS")) hw = (unsigned)std::max(1, atoi(e));
  int64_t chunks = (n + grain - 1) / grain;
  int64_t nt = std::min<int64_t>(std::max(1u, hw), chunks);
  if (nt <= 1) {
    body(0, n);
    return;
  }
  // Workers take chunks until none is left.  A worker that throws stops the
  // others from taking more and its exception is rethrown here after every
  // thread has joined; a thread that cannot be started (resource limits)
  // leaves its share to the others and to the calling thread, which always
  // works too.  No exception leaves a joinable thread behind.
  std::atomic<int64_t> next{0};
  std::exception_ptr err;
  std::mutex err_mu;
  auto work = [&]() {
    try {
      for (;;) {
        int64_t c = next.fetch_add(1);
        if (c >= chunks) break;
        int64_t a = c * grain, b = std::min(n, a + grain);
        body(a, b);
      }
    } catch (...) {
      next.store(chunks);
      std::lock_guard<std::mutex> lock(err_mu);
      if (!err) err = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  try {
    th.reserve(nt - 1);
    for (int64_t t = 0; t + 1 < nt; ++t) th.emplace_back(work);
  } catch (...) {
    // fewer threads than asked for: the ones started and this one finish
  }
  work();
  for (auto& t : th) t.join();
  if (err) std::rethrow_exception(err);
}

std::vector<uint8_t> find_bridges(int N, const std::vector<int32_t>& from,
                                  const std::vector<int32_t>& to) {
  const int L = (int)from.size();
  std::vector<int> head(N + 1, 0), adj_to(2 * L), adj_line(2 * L);
  for (int l = 0; l < L; ++l) {
    head[from[l] + 1]++;
    head[to[l] + 1]++;
  }
  for (int n = 0; n < N; ++n) head[n + 1] += head[n];
  std::vector<int> fill(head.begin(), head.end() - 1);
  for (int l = 0; l < L; ++l) {
    adj_to[fill[from[l]]] = to[l];
    adj_line[fill[from[l]]++] = l;
    adj_to[fill[to[l]]] = from[l];
    adj_line[fill[to[l]]++] = l;
  }
  std::vector<int> disc(N, -1), low(N, 0), it(N, 0), via(N, -1);
  std::vector<uint8_t> bridge(L, 0);
  std::vector<int> stack;
  int t = 0;
  for (int root = 0; root < N; ++root) {
    if (disc[root] >= 0) continue;
    disc[root] = low[root] = t++;
    it[root] = head[root];
    stack.push_back(root);
    while (!stack.empty()) {
      int v = stack.back();
      if (it[v] < head[v + 1]) {
        int e = it[v]++;
        int w = adj_to[e], l = adj_line[e];
        if (l == via[v]) continue;
        if (disc[w] < 0) {
          disc[w] = low[w] = t++;
          via[w] = l;
          it[w] = head[w];
          stack.push_back(w);
        } else {
          low[v] = std::min(low[v], disc[w]);
        }
      } else {
        stack.pop_back();
        if (!stack.empty()) {
          int p = stack.back();
          low[p] = std::min(low[p], low[v]);
          if (low[v] > disc[p]) bridge[via[v]] = 1;
        }
      }
    }
  }
  return bridge;
}

namespace {

// C[i, j] -= sum_{p in [p0, p1)} A[i, p] * B[j, p] for a 4 x 4 block of rows;
// A and B rows are contiguous in p (row-major, leading dimension ld).
typedef double v4d __attribute__((vector_size(32)));

inline double hsum(v4d v) { return (v[0] + v[1]) + (v[2] + v[3]); }

inline v4d load4(const double* p) {
  v4d v;
  std::memcpy(&v, p, sizeof(v));
  return v;
}

// out[a][b] = sum_{p in [p0, p1)} A[ia[a]*ld + p] * B[jb[b]*ld + p]
template <int MA, int MB>
inline void dot_block(const double* A, const double* B, int64_t ld, const int64_t* ia,
                      const int64_t* jb, int64_t p0, int64_t p1, double out[MA][MB]) {
  v4d acc[MA][MB];
  for (int a = 0; a < MA; ++a)
    for (int b = 0; b < MB; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  int64_t p = p0;
  for (; p + 4 <= p1; p += 4) {
    v4d x[MA], y[MB];
    for (int a = 0; a < MA; ++a) x[a] = load4(A + ia[a] * ld + p);
    for (int b = 0; b < MB; ++b) y[b] = load4(B + jb[b] * ld + p);
    for (int a = 0; a < MA; ++a)
      for (int b = 0; b < MB; ++b) acc[a][b] += x[a] * y[b];
  }
  for (int a = 0; a < MA; ++a)
    for (int b = 0; b < MB; ++b) {
      double s = hsum(acc[a][b]);
      for (int64_t q = p; q < p1; ++q) s += A[ia[a] * ld + q] * B[jb[b] * ld + q];
      out[a][b] = s;
    }
}

// Lower Cholesky in place (row-major n x n, lower triangle used).  Returns
// false if a pivot is not positive.
bool cholesky_lower(double* A, int64_t n) {
  const int64_t NB = 96;
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    const int64_t k1 = std::min(n, k0 + NB);
    // 1. unblocked factor of the diagonal block
    for (int64_t j = k0; j < k1; ++j) {
      double d = A[j * n + j];
      for (int64_t p = k0; p < j; ++p) d -= A[j * n + p] * A[j * n + p];
      if (!(d > 0.0)) return false;
      d = std::sqrt(d);
      A[j * n + j] = d;
      for (int64_t i = j + 1; i < k1; ++i) {
        double s = A[i * n + j];
        for (int64_t p = k0; p < j; ++p) s -= A[i * n + p] * A[j * n + p];
        A[i * n + j] = s / d;
      }
    }
    // 2. panel rows below: A[i, k0:k1] <- A[i, k0:k1] C_kk^{-T}
    parallel_for(n - k1, 64, [&](int64_t a, int64_t b) {
      for (int64_t i = k1 + a; i < k1 + b; ++i) {
        double* ri = A + i * n;
        for (int64_t j = k0; j < k1; ++j) {
          double s = ri[j];
          const double* rj = A + j * n;
          for (int64_t p = k0; p < j; ++p) s -= ri[p] * rj[p];
          ri[j] = s / rj[j];
        }
      }
    });
    // 3. trailing update of the lower triangle: A[i, j] -= A[i, k0:k1] . A[j, k0:k1]
    const int64_t m = n - k1;
    const int64_t T = 4;
    const int64_t nbk = (m + T - 1) / T;
    parallel_for(nbk, 4, [&](int64_t a, int64_t b) {
      for (int64_t bi = a; bi < b; ++bi) {
        const int64_t i0 = k1 + bi * T;
        int64_t ia[4];
        for (int t = 0; t < 4; ++t) ia[t] = std::min(i0 + t, n - 1);
        for (int64_t j0 = k1; j0 <= std::min(i0 + T - 1, n - 1); j0 += T) {
          int64_t jb[4];
          for (int t = 0; t < 4; ++t) jb[t] = std::min(j0 + t, n - 1);
          double out[4][4];
          dot_block<4, 4>(A, A, n, ia, jb, k0, k1, out);
          for (int x = 0; x < 4; ++x) {
            const int64_t i = i0 + x;
            if (i >= n) break;
            for (int y = 0; y < 4; ++y) {
              const int64_t j = j0 + y;
              if (j >= n || j > i) break;
              A[i * n + j] -= out[x][y];
            }
          }
        }
      }
    });
  }
  return true;
}

// Given the lower Cholesky factor C (row-major, lower part of A), returns the
// full symmetric inverse of C C^T in `inv` (row-major n x n).
void spd_inverse_from_cholesky(const double* C, int64_t n, std::vector<double>& inv) {
  // Wt = (C^{-1})^T stored row-major, i.e. row j of Wt is column j of W = C^{-1};
  // Wt is upper triangular: Wt[j, p] = W[p, j] for p >= j.
  // Column j of W solves C w = e_j: w_p = 0 for p < j, w_j = 1 / C_jj,
  // w_p = -(sum_{q=j}^{p-1} C[p, q] w_q) / C_pp.  Blocked by groups of columns,
  // each group handled by one thread with dot products over contiguous rows.
  std::vector<double> Wt((size_t)n * n, 0.0);
  const int64_t GB = 16;  // columns of W per task
  const int64_t TP = 4;   // rows of C per tile
  const int64_t ng = (n + GB - 1) / GB;
  parallel_for(ng, 1, [&](int64_t a, int64_t b) {
    for (int64_t g = a; g < b; ++g) {
      const int64_t j0 = g * GB, j1 = std::min(n, j0 + GB);
      for (int64_t p0 = j0; p0 < n; p0 += TP) {
        const int64_t p1 = std::min(n, p0 + TP);
        double out[TP][GB];
        for (int64_t x = 0; x < TP; ++x)
          for (int64_t y = 0; y < GB; ++y) out[x][y] = 0.0;
        if (p0 > j0) {
          int64_t ia[TP];
          for (int64_t t = 0; t < TP; ++t) ia[t] = std::min(p0 + t, n - 1);
          for (int64_t y0 = 0; y0 < GB; y0 += 2) {
            int64_t jb[2] = {std::min(j0 + y0, n - 1), std::min(j0 + y0 + 1, n - 1)};
            double o[TP][2];
            dot_block<TP, 2>(C, Wt.data(), n, ia, jb, j0, p0, o);
            for (int64_t x = 0; x < TP; ++x) {
              out[x][y0] = o[x][0];
              out[x][y0 + 1] = o[x][1];
            }
          }
        }
        // finish the rows of this tile in order (they depend on each other)
        for (int64_t p = p0; p < p1; ++p) {
          const double* cp = C + p * n;
          const double inv_d = 1.0 / cp[p];
          for (int64_t j = j0; j < j1; ++j) {
            double* w = Wt.data() + j * n;
            if (p < j) continue;
            if (p == j) {
              w[p] = inv_d;
              continue;
            }
            double s = out[p - p0][j - j0];
            for (int64_t q = std::max(p0, j); q < p; ++q) s += cp[q] * w[q];
            w[p] = -s * inv_d;
          }
        }
      }
    }
  });
  // inv[i, j] = sum_{p >= max(i, j)} Wt[i, p] Wt[j, p]
  inv.assign((size_t)n * n, 0.0);
  const int64_t T = 4;
  const int64_t nb = (n + T - 1) / T;
  parallel_for(nb, 2, [&](int64_t a, int64_t b) {
    for (int64_t bi = a; bi < b; ++bi) {
      const int64_t i0 = bi * T;
      int64_t ia[4];
      for (int t = 0; t < 4; ++t) ia[t] = std::min(i0 + t, n - 1);
      for (int64_t j0 = 0; j0 <= std::min(i0 + T - 1, n - 1); j0 += T) {
        int64_t jb[4];
        for (int t = 0; t < 4; ++t) jb[t] = std::min(j0 + t, n - 1);
        // entries beyond each row's own start are zero in Wt, so summing from
        // max(i0, j0) is exact for every pair in the block
        double out[4][4];
        dot_block<4, 4>(Wt.data(), Wt.data(), n, ia, jb, std::max(i0, j0), n, out);
        for (int x = 0; x < 4; ++x) {
          const int64_t i = i0 + x;
          if (i >= n) break;
          for (int y = 0; y < 4; ++y) {
            const int64_t j = j0 + y;
            if (j >= n || j > i) break;
            inv[i * n + j] = out[x][y];
            inv[j * n + i] = out[x][y];
          }
        }
      }
    }
  });
}


}  // namespace

// Largest over buses of the least path resistance sum_j 1/b_j from the slack,
// rounded up: every 1/b_j and every partial sum carries at most one float64
// rounding, so (1 + 2 u)^(N + 1) >= 1 + 2.1 (N + 1) u covers them all.
static double max_path_resistance(const HostNet& net) {
  const int N = net.N, L = net.L;
  std::vector<int> head(N + 1, 0), adj(2 * L);
  for (int l = 0; l < L; ++l) {
    head[net.line_from[l] + 1]++;
    head[net.line_to[l] + 1]++;
  }
  for (int b = 0; b < N; ++b) head[b + 1] += head[b];
  std::vector<int> fill(head.begin(), head.end() - 1);
  for (int l = 0; l < L; ++l) {
    adj[fill[net.line_from[l]]++] = l;
    adj[fill[net.line_to[l]]++] = l;
  }
  std::vector<double> dist(N, std::numeric_limits<double>::infinity());
  std::vector<uint8_t> done(N, 0);
  using Item = std::pair<double, int>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  dist[net.slack] = 0.0;
  heap.push({0.0, net.slack});
  while (!heap.empty()) {
    const auto [d, v] = heap.top();
    heap.pop();
    if (done[v]) continue;
    done[v] = 1;
    for (int e = head[v]; e < head[v + 1]; ++e) {
      const int l = adj[e];
      const int w = net.line_from[l] == v ? net.line_to[l] : net.line_from[l];
      const double nd = d + 1.0 / net.line_b[l];
      if (nd < dist[w]) {
        dist[w] = nd;
        heap.push({nd, w});
      }
    }
  }
  double m = 0.0;
  for (int b = 0; b < N; ++b) m = std::max(m, dist[b]);
  return m * (1.0 + 2.1 * (N + 1) * std::ldexp(1.0, -53));
}

ibp_status build_host(const ibp_network_desc* d, HostNet& net, std::string& err) {
  auto t0 = std::chrono::steady_clock::now();
  if (!d) {
    err = "desc is NULL";
    return IBP_E_INVALID_ARG;
  }
  const int N = d->n_bus, L = d->n_line, G = d->n_gen, D = d->n_load;
  if (N < 2 || L < 1 || G < 0 || D < 0 || G + D < 1) {
    err = "need n_bus >= 2, n_line >= 1, n_gen + n_load >= 1";
    return IBP_E_INVALID_ARG;
  }
  if (d->slack_bus < 0 || d->slack_bus >= N) {
    err = "slack_bus out of range";
    return IBP_E_INVALID_ARG;
  }
  if (!d->line_from || !d->line_to || !d->line_b || !d->fmax_base || !d->fmax_ctg ||
      (G > 0 && (!d->gen_bus || !d->gen_cost)) || (D > 0 && (!d->load_bus || !d->load_value))) {
    err = "a required array pointer is NULL";
    return IBP_E_INVALID_ARG;
  }
  if (!(d->zeta_inj >= 0.0) || !(d->zeta_f >= 0.0) || !std::isfinite(d->zeta_inj) ||
      !std::isfinite(d->zeta_f)) {
    err = "penalty weights must be finite and >= 0";
    return IBP_E_INVALID_ARG;
  }
  for (int l = 0; l < L; ++l) {
    const int a = d->line_from[l], b = d->line_to[l];
    if (a < 0 || a >= N || b < 0 || b >= N || a == b) {
      err = "line " + std::to_string(l) + ": endpoint out of range or self loop";
      return IBP_E_INVALID_ARG;
    }
    if (!(d->line_b[l] > 0.0) || !std::isfinite(d->line_b[l])) {
      err = "line " + std::to_string(l) + ": susceptance must be finite and > 0";
      return IBP_E_INVALID_ARG;
    }
    if (!(d->fmax_base[l] > 0.0) || !(d->fmax_ctg[l] > 0.0) || !(d->fmax_base[l] < 1e37) ||
        !(d->fmax_ctg[l] < 1e37)) {
      err = "line " + std::to_string(l) + ": flow limits must be in (0, 1e37)";
      return IBP_E_INVALID_ARG;
    }
  }
  for (int g = 0; g < G; ++g)
    if (d->gen_bus[g] < 0 || d->gen_bus[g] >= N || !std::isfinite(d->gen_cost[g])) {
      err = "generator " + std::to_string(g) + ": bus out of range or cost not finite";
      return IBP_E_INVALID_ARG;
    }
  for (int j = 0; j < D; ++j)
    if (d->load_bus[j] < 0 || d->load_bus[j] >= N || !std::isfinite(d->load_value[j])) {
      err = "load " + std::to_string(j) + ": bus out of range or value not finite";
      return IBP_E_INVALID_ARG;
    }
  if (d->ctg_line && d->n_ctg < 0) {
    err = "n_ctg < 0";
    return IBP_E_INVALID_ARG;
  }
  if (d->seg_ptr) {
    const int X = G + D;
    if (d->seg_ptr[0] != 0) {
      err = "seg_ptr[0] must be 0";
      return IBP_E_INVALID_ARG;
    }
    for (int j = 0; j < X; ++j)
      if (d->seg_ptr[j + 1] < d->seg_ptr[j]) {
        err = "seg_ptr must be non-decreasing";
        return IBP_E_INVALID_ARG;
      }
    const int S = d->seg_ptr[X];
    if (S > 0 && (!d->seg_a || !d->seg_b || !d->seg_U)) {
      err = "seg_a, seg_b and seg_U are required when curves have segments";
      return IBP_E_INVALID_ARG;
    }
    for (int i = 0; i < S; ++i)
      if (!std::isfinite(d->seg_a[i]) || !std::isfinite(d->seg_b[i]) || std::isnan(d->seg_U[i]) ||
          d->seg_U[i] == -std::numeric_limits<double>::infinity()) {
        err = "segment " + std::to_string(i) + ": slope and shift must be finite, cap finite or +inf";
        return IBP_E_INVALID_ARG;
      }
    net.seg_ptr.assign(d->seg_ptr, d->seg_ptr + X + 1);
    net.seg_a.assign(d->seg_a, d->seg_a + S);
    net.seg_b.assign(d->seg_b, d->seg_b + S);
    net.seg_U.assign(d->seg_U, d->seg_U + S);
  }

  net.N = N;
  net.L = L;
  net.G = G;
  net.D = D;
  net.slack = d->slack_bus;
  net.line_from.assign(d->line_from, d->line_from + L);
  net.line_to.assign(d->line_to, d->line_to + L);
  net.line_b.assign(d->line_b, d->line_b + L);
  net.fmax_base.assign(d->fmax_base, d->fmax_base + L);
  net.fmax_ctg.assign(d->fmax_ctg, d->fmax_ctg + L);
  net.gen_bus.assign(d->gen_bus, d->gen_bus + G);
  net.gen_cost.assign(d->gen_cost, d->gen_cost + G);
  net.load_bus.assign(d->load_bus, d->load_bus + D);
  net.load_value.assign(d->load_value, d->load_value + D);
  net.zeta_inj = d->zeta_inj;
  net.zeta_f = d->zeta_f;

  // connectivity (breadth-first from the slack)
  {
    std::vector<int> head(N + 1, 0), adj(2 * L);
    for (int l = 0; l < L; ++l) {
      head[net.line_from[l] + 1]++;
      head[net.line_to[l] + 1]++;
    }
    for (int n = 0; n < N; ++n) head[n + 1] += head[n];
    std::vector<int> fill(head.begin(), head.end() - 1);
    for (int l = 0; l < L; ++l) {
      adj[fill[net.line_from[l]]++] = net.line_to[l];
      adj[fill[net.line_to[l]]++] = net.line_from[l];
    }
    std::vector<uint8_t> seen(N, 0);
    std::vector<int> q{net.slack};
    seen[net.slack] = 1;
    for (size_t h = 0; h < q.size(); ++h)
      for (int e = head[q[h]]; e < head[q[h] + 1]; ++e)
        if (!seen[adj[e]]) {
          seen[adj[e]] = 1;
          q.push_back(adj[e]);
        }
    if ((int)q.size() != N) {
      err = "network is not connected (" + std::to_string(N - (int)q.size()) +
            " buses unreachable from the slack)";
      return IBP_E_DISCONNECTED;
    }
  }

  // contingency set
  std::vector<uint8_t> bridge = find_bridges(N, net.line_from, net.line_to);
  if (d->ctg_line) {
    std::vector<uint8_t> used(L, 0);
    for (int k = 0; k < d->n_ctg; ++k) {
      const int c = d->ctg_line[k];
      if (c < 0 || c >= L || used[c]) {
        err = "ctg_line[" + std::to_string(k) + "] out of range or repeated";
        return IBP_E_INVALID_ARG;
      }
      used[c] = 1;
      if (bridge[c]) {
        err = "outage of line " + std::to_string(c) + " islands the network";
        return IBP_E_ISLANDING_CTG;
      }
      net.ctg_line.push_back(c);
    }
  } else {
    for (int l = 0; l < L; ++l)
      if (!bridge[l]) net.ctg_line.push_back(l);
  }
  net.K = (int)net.ctg_line.size();
  net.ctg_of_line.assign(L, -1);
  for (int k = 0; k < net.K; ++k) net.ctg_of_line[net.ctg_line[k]] = k;

  // reduced admittance (dense, row-major), slack row/column removed
  const int64_t n = N - 1;
  auto red = [&](int bus) -> int64_t { return bus == net.slack ? -1 : (bus < net.slack ? bus : bus - 1); };
  std::vector<double> A;
  try {
    A.assign((size_t)n * n, 0.0);
  } catch (...) {
    err = "host allocation of the reduced admittance failed";
    return IBP_E_OUT_OF_MEMORY;
  }
  for (int l = 0; l < L; ++l) {
    const int64_t a = red(net.line_from[l]), b = red(net.line_to[l]);
    const double y = net.line_b[l];
    if (a >= 0) A[a * n + a] += y;
    if (b >= 0) A[b * n + b] += y;
    if (a >= 0 && b >= 0) {
      A[a * n + b] -= y;
      A[b * n + a] -= y;
    }
  }
  std::vector<double> Bsparse_diag(n);  // keep the diagonal for the residual check
  for (int64_t i = 0; i < n; ++i) Bsparse_diag[i] = A[i * n + i];

  if (!cholesky_lower(A.data(), n)) {
    err = "reduced admittance matrix is not positive definite";
    return IBP_E_DISCONNECTED;
  }
  std::vector<double> inv;
  spd_inverse_from_cholesky(A.data(), n, inv);
  std::vector<double>().swap(A);

  // PTDF rows
  net.phi.assign((size_t)L * N, 0.0);
  parallel_for(L, 64, [&](int64_t a, int64_t b) {
    for (int64_t l = a; l < b; ++l) {
      const int64_t fa = red(net.line_from[l]), fb = red(net.line_to[l]);
      const double y = net.line_b[l];
      double* row = net.phi.data() + l * N;
      for (int bus = 0; bus < N; ++bus) {
        const int64_t m = red(bus);
        if (m < 0) continue;
        const double x1 = fa >= 0 ? inv[fa * n + m] : 0.0;
        const double x2 = fb >= 0 ? inv[fb * n + m] : 0.0;
        row[bus] = y * (x1 - x2);
      }
    }
  });

  // a-posteriori PTDF error: residual R = Phi Y_B - Y_D E over non-slack columns,
  // row l:  R[l, m] = sum_j b_j (Phi[l, from_j] - Phi[l, to_j]) E[j, m] - b_l E[l, m].
  // Phi_r - Phi_exact = R Y_Br^{-1}, so per row |Phi_r - Phi_exact| <= ||R_l||_1 max|Y_Br^{-1}|.
  // max|Y_Br^{-1}| is bounded without trusting the computed inverse: Y_Br^{-1}
  // is symmetric positive definite, so its largest entry is on the diagonal,
  // and (Y_Br^{-1})_ii is the effective resistance between bus i and the slack
  // in the network of conductances b; removing every line off one path can
  // only raise it (Rayleigh monotonicity), so it is at most the resistance
  // sum_j 1/b_j of the least-resistance path from the slack (Dijkstra).
  const double inv_max = max_path_resistance(net);
  std::vector<double>().swap(inv);
  net.phi_err.assign(L, 0.0);
  {
    // adjacency lists for the residual
    std::vector<int> head(N + 1, 0), adj_line(2 * L);
    for (int l = 0; l < L; ++l) {
      head[net.line_from[l] + 1]++;
      head[net.line_to[l] + 1]++;
    }
    for (int b = 0; b < N; ++b) head[b + 1] += head[b];
    std::vector<int> fill(head.begin(), head.end() - 1);
    for (int l = 0; l < L; ++l) {
      adj_line[fill[net.line_from[l]]++] = l;
      adj_line[fill[net.line_to[l]]++] = l;
    }
    const double u64 = std::ldexp(1.0, -53);
    parallel_for(L, 64, [&](int64_t a, int64_t b) {
      for (int64_t l = a; l < b; ++l) {
        const double* row = net.phi.data() + l * N;
        // residual entries in 80-bit extended precision (64-bit significand),
        // so that the rounding of forming them is negligible next to their size
        double r1 = 0.0, fp = 0.0;
        const double uext = std::ldexp(1.0, -64);
        for (int m = 0; m < N; ++m) {
          if (m == net.slack) continue;
          long double s = 0.0L;
          double sa = 0.0;
          const int deg = head[m + 1] - head[m];
          for (int e = head[m]; e < head[m + 1]; ++e) {
            const int j = adj_line[e];
            const long double fj = (long double)net.line_b[j] *
                                   ((long double)row[net.line_from[j]] - (long double)row[net.line_to[j]]);
            s += (net.line_from[j] == m) ? fj : -fj;
            sa += std::fabs((double)fj);
          }
          if (net.line_from[l] == m) s -= net.line_b[l];
          if (net.line_to[l] == m) s += net.line_b[l];
          // |computed - exact residual| <= gamma_{deg+4} (sum |f_j| + b_l) in extended precision
          r1 += std::fabs((double)s);
          fp += 2.0 * (deg + 4) * uext * (sa + net.line_b[l]);
        }
        r1 *= 1.0 + 4.0 * N * u64;
        // residual plus the rounding error of forming it, times the bound on max|Y_Br^{-1}|
        const double bound = (r1 + fp) * inv_max;
        net.phi_err[l] = bound + 1e-300;
      }
    });
    net.phi_err_max = 0.0;
    for (int l = 0; l < L; ++l) net.phi_err_max = std::max(net.phi_err_max, net.phi_err[l]);
  }

  // outage factors, row k = outage of line c(k):  H[l, c] / (1 - H[c, c])
  const int K = net.K;
  net.one_m_hcc.assign(K, 0.0);
  net.min_one_m_hcc = 1.0;
  for (int k = 0; k < K; ++k) {
    const int c = net.ctg_line[k];
    const double hcc = net.phi[(size_t)c * N + net.line_from[c]] - net.phi[(size_t)c * N + net.line_to[c]];
    net.one_m_hcc[k] = 1.0 - hcc;
    net.min_one_m_hcc = std::min(net.min_one_m_hcc, 1.0 - hcc);
    if (!(1.0 - hcc >= 1e-6)) {
      err = "outage of line " + std::to_string(c) + " is ill-conditioned (1 - H_cc = " +
            std::to_string(1.0 - hcc) + ")";
      return IBP_E_ILL_CONDITIONED;
    }
  }
  try {
    net.lodf.assign((size_t)K * L, 0.0);
  } catch (...) {
    err = "host allocation of the outage factors failed";
    return IBP_E_OUT_OF_MEMORY;
  }
  // blocked over lines so that the PTDF rows being read stay in cache
  const int64_t LB = 32;
  parallel_for((L + LB - 1) / LB, 1, [&](int64_t a, int64_t b) {
    for (int64_t blk = a; blk < b; ++blk) {
      const int64_t l0 = blk * LB, l1 = std::min<int64_t>(L, l0 + LB);
      for (int k = 0; k < K; ++k) {
        const int c = net.ctg_line[k];
        const int fc = net.line_from[c], tc = net.line_to[c];
        const double den = net.one_m_hcc[k];
        double* out = net.lodf.data() + (size_t)k * L;
        for (int64_t l = l0; l < l1; ++l) {
          const double* row = net.phi.data() + l * N;
          out[l] = (row[fc] - row[tc]) / den;
        }
      }
    }
  });
  net.build_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return IBP_OK;
}

}  // namespace ibp
