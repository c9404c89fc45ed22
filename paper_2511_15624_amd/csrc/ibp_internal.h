// Internal declarations shared by the host construction, the C ABI and the
// kernel launchers of libibp.  Not installed; the public interface is
// include/ibp.h.
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/ibp.h"

namespace ibp {

// Float64 network factors built on the host (the "a0" setup step).
struct HostNet {
  int N = 0, L = 0, K = 0, G = 0, D = 0, slack = 0;
  std::vector<int32_t> line_from, line_to;
  std::vector<double> line_b, fmax_base, fmax_ctg;
  std::vector<int32_t> gen_bus, load_bus;
  std::vector<double> gen_cost, load_value;
  double zeta_inj = 0, zeta_f = 0;
  std::vector<int32_t> seg_ptr;            // [X + 1], empty for linear costs only
  std::vector<double> seg_a, seg_b, seg_U; // piecewise-linear curve segments

  std::vector<int32_t> ctg_line;     // [K] outaged line of each contingency
  std::vector<int32_t> ctg_of_line;  // [L] contingency index of a line, -1 if none
  std::vector<double> phi;           // [L x N] row-major, slack column zero
  std::vector<double> lodf;          // [K x L] row-major (row k = outage k)
  std::vector<double> one_m_hcc;     // [K] 1 - H_cc
  std::vector<double> phi_err;       // [L] bound on |phi64 - phi_exact| in row l
  double phi_err_max = 0;
  double min_one_m_hcc = 1;
  double build_seconds = 0;
};

// Validates the description and runs the float64 construction.  Returns
// IBP_OK or an error code with a message in `err`.
ibp_status build_host(const ibp_network_desc* d, HostNet& net, std::string& err);

// Bridge (islanding line) mask by an iterative low-link depth-first search.
std::vector<uint8_t> find_bridges(int N, const std::vector<int32_t>& from,
                                  const std::vector<int32_t>& to);

// Simple thread pool style parallel loop over [0, n).
void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& body);

}  // namespace ibp
