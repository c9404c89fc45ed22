/* A plain C99 caller of the C ABI in include/ibp.h (no C++ and no Python):
 * builds the hand-derived 3-bus triangle of tests/golden/three_bus.json and
 * prints what the library returns, one value per line, for the test that
 * compares it with the fixture.
 *
 *   three_bus host    host-only handle: query, outage list, exported factors
 *   three_bus device  handle on device 0: workspace size, forward bounds of
 *                     the fixture's box, and the chord-relaxation lower bound
 *
 * Exit status 0 on success, 1 on a library error (message on stderr). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "ibp.h"

#define CHECK(call)                                                          \
  do {                                                                       \
    ibp_status st_ = (call);                                                 \
    if (st_ != IBP_OK) {                                                     \
      fprintf(stderr, "%s -> %d: %s\n", #call, (int)st_, ibp_last_error()); \
      return 1;                                                              \
    }                                                                        \
  } while (0)

#define HCHECK(call)                                           \
  do {                                                         \
    if ((call) != hipSuccess) {                                \
      fprintf(stderr, "%s failed\n", #call);                   \
      return 1;                                                \
    }                                                          \
  } while (0)

static int host_mode(const ibp_network_desc* d) {
  ibp_network* net = NULL;
  ibp_network_info info;
  int32_t ctg[3];
  double ptdf[9], lodf[9];
  int i;
  CHECK(ibp_build_network(d, IBP_DEVICE_HOST_ONLY, &net));
  CHECK(ibp_network_query(net, &info));
  printf("n_bus %d\nn_line %d\nn_ctg %d\nn_input %d\n", info.n_bus, info.n_line, info.n_ctg, info.n_input);
  CHECK(ibp_network_ctg_lines(net, ctg));
  for (i = 0; i < info.n_ctg; ++i) printf("ctg %d %d\n", i, ctg[i]);
  CHECK(ibp_network_export(net, ptdf, lodf));
  for (i = 0; i < 9; ++i) printf("ptdf %d %d %.17g\n", i / 3, i % 3, ptdf[i]);
  for (i = 0; i < 3 * info.n_ctg; ++i) printf("lodf %d %d %.17g\n", i / 3, i % 3, lodf[i]);
  /* a compute call on a host-only handle is refused */
  printf("host_compute_status %d\n", (int)ibp_bound_boxes(net, 1, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, 0));
  ibp_free_network(net);
  return 0;
}

static int device_mode(const ibp_network_desc* d) {
  ibp_network* net = NULL;
  const float lo[2] = {0.0f, 1.0f}, hi[2] = {2.0f, 1.0f};
  float *dlo = NULL, *dhi = NULL;
  double *dout = NULL, out[4];
  void* ws = NULL;
  size_t bytes, bytes_c;
  CHECK(ibp_build_network(d, 0, &net));
  bytes = ibp_workspace_bytes(net, 1, IBP_F_NONE);
  bytes_c = ibp_workspace_bytes(net, 1, IBP_F_CROWN);
  printf("workspace %zu\nworkspace_crown %zu\n", bytes, bytes_c);
  if (bytes == 0 || bytes_c < bytes) return 1;
  HCHECK(hipMalloc((void**)&dlo, sizeof lo));
  HCHECK(hipMalloc((void**)&dhi, sizeof hi));
  HCHECK(hipMalloc((void**)&dout, sizeof out));
  HCHECK(hipMalloc(&ws, bytes_c));
  HCHECK(hipMemcpy(dlo, lo, sizeof lo, hipMemcpyHostToDevice));
  HCHECK(hipMemcpy(dhi, hi, sizeof hi, hipMemcpyHostToDevice));
  /* null stream: the calls are ordered with the copies around them */
  CHECK(ibp_bound_boxes(net, 1, dlo, dhi, dout, dout + 1, NULL, ws, bytes, NULL, IBP_F_NONE));
  CHECK(ibp_crown_lower_boxes(net, 1, dlo, dhi, dout + 2, dout + 3, NULL, NULL, ws, bytes_c, NULL, IBP_F_NONE));
  HCHECK(hipMemcpy(out, dout, sizeof out, hipMemcpyDeviceToHost));
  printf("f_lo %.17g\nf_hi %.17g\nchord_f_lo %.17g\nchord_f_hi %.17g\n", out[0], out[1], out[2], out[3]);
  /* a workspace one byte short is refused before any device work */
  printf("short_workspace_status %d\n",
         (int)ibp_bound_boxes(net, 1, dlo, dhi, dout, dout + 1, NULL, ws, bytes - 1, NULL, IBP_F_NONE));
  HCHECK(hipFree(ws));
  HCHECK(hipFree(dout));
  HCHECK(hipFree(dhi));
  HCHECK(hipFree(dlo));
  ibp_free_network(net);
  return 0;
}

int main(int argc, char** argv) {
  const int32_t from[3] = {0, 1, 0}, to[3] = {1, 2, 2};
  const double b[3] = {1.0, 1.0, 1.0}, fmax[3] = {0.1, 0.1, 0.1};
  const int32_t gen_bus[1] = {1}, load_bus[1] = {2};
  const double cost[1] = {10.0}, value[1] = {50.0};
  ibp_network_desc d;
  memset(&d, 0, sizeof d);
  d.n_bus = 3;
  d.n_line = 3;
  d.slack_bus = 0;
  d.line_from = from;
  d.line_to = to;
  d.line_b = b;
  d.fmax_base = fmax;
  d.fmax_ctg = fmax;
  d.n_gen = 1;
  d.gen_bus = gen_bus;
  d.gen_cost = cost;
  d.n_load = 1;
  d.load_bus = load_bus;
  d.load_value = value;
  d.zeta_inj = 100.0;
  d.zeta_f = 10.0;
  d.ctg_line = NULL;
  if (argc == 2 && strcmp(argv[1], "host") == 0) return host_mode(&d);
  if (argc == 2 && strcmp(argv[1], "device") == 0) return device_mode(&d);
  fprintf(stderr, "usage: %s host|device\n", argv[0]);
  return 2;
}
