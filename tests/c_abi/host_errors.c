/* Host-side paths of the C ABI for a sanitizer build (AddressSanitizer,
 * UndefinedBehaviorSanitizer, LeakSanitizer at exit): valid host-only builds
 * of generated networks (with and without an outage list and curves), export
 * and free, and every argument or network error the host can detect, each
 * printed as "<case> <status>" for the test to compare.  Needs no GPU: no
 * call here reaches the HIP runtime.  Exit status 0 unless a valid build
 * fails. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ibp.h"

typedef struct {
  int32_t n, l;
  int32_t *from, *to, *gbus, *dbus, *ctg, *seg_ptr;
  double *b, *fb, *fc, *cost, *value, *sa, *sb, *su;
} owned;

/* a ring of n buses with a chord every 7 buses (no bridges), one generator per
 * 5 buses, one load per 3 */
static void make_ring(owned* o, ibp_network_desc* d, int32_t n) {
  int32_t l = 0, i, g = 0, j = 0, nc = 0, k;
  memset(o, 0, sizeof *o);
  o->n = n;
  o->from = malloc(sizeof(int32_t) * 2 * n);
  o->to = malloc(sizeof(int32_t) * 2 * n);
  o->b = malloc(sizeof(double) * 2 * n);
  for (i = 0; i < n; ++i) {
    o->from[l] = i;
    o->to[l] = (i + 1) % n;
    o->b[l++] = 1.0 + 0.1 * (i % 5);
  }
  for (i = 0; i + 7 < n; i += 7) {
    o->from[l] = i;
    o->to[l] = i + 7;
    o->b[l++] = 2.0;
  }
  o->l = l;
  o->fb = malloc(sizeof(double) * l);
  o->fc = malloc(sizeof(double) * l);
  for (i = 0; i < l; ++i) o->fb[i] = o->fc[i] = 0.5 + 0.01 * i;
  o->gbus = malloc(sizeof(int32_t) * n);
  o->dbus = malloc(sizeof(int32_t) * n);
  o->cost = malloc(sizeof(double) * n);
  o->value = malloc(sizeof(double) * n);
  for (i = 0; i < n; i += 5) {
    o->gbus[g] = i;
    o->cost[g++] = 10.0 + i;
  }
  for (i = 1; i < n; i += 3) {
    o->dbus[j] = i;
    o->value[j++] = 40.0 + i;
  }
  o->ctg = malloc(sizeof(int32_t) * l);
  for (i = 0; i < l; i += 2) o->ctg[nc++] = i;
  /* two segments per device */
  o->seg_ptr = malloc(sizeof(int32_t) * (g + j + 1));
  o->sa = malloc(sizeof(double) * 2 * (g + j));
  o->sb = malloc(sizeof(double) * 2 * (g + j));
  o->su = malloc(sizeof(double) * 2 * (g + j));
  for (k = 0; k <= g + j; ++k) o->seg_ptr[k] = 2 * k;
  for (k = 0; k < g + j; ++k) {
    o->sa[2 * k] = 0.0;
    o->sb[2 * k] = 20.0;
    o->su[2 * k] = 1.0;
    o->sa[2 * k + 1] = 20.0;
    o->sb[2 * k + 1] = 10.0;
    o->su[2 * k + 1] = 1e30;
  }
  memset(d, 0, sizeof *d);
  d->n_bus = n;
  d->n_line = l;
  d->slack_bus = 0;
  d->line_from = o->from;
  d->line_to = o->to;
  d->line_b = o->b;
  d->fmax_base = o->fb;
  d->fmax_ctg = o->fc;
  d->n_gen = g;
  d->gen_bus = o->gbus;
  d->gen_cost = o->cost;
  d->n_load = j;
  d->load_bus = o->dbus;
  d->load_value = o->value;
  d->zeta_inj = 100.0;
  d->zeta_f = 10.0;
  d->n_ctg = nc;
  d->ctg_line = o->ctg;
}

static void release(owned* o) {
  free(o->from);
  free(o->to);
  free(o->b);
  free(o->fb);
  free(o->fc);
  free(o->gbus);
  free(o->dbus);
  free(o->cost);
  free(o->value);
  free(o->ctg);
  free(o->seg_ptr);
  free(o->sa);
  free(o->sb);
  free(o->su);
}

static int report(const char* what, ibp_status st) {
  printf("%s %d\n", what, (int)st);
  return (int)st;
}

static int valid_builds(void) {
  owned o;
  ibp_network_desc d;
  ibp_network* net = NULL;
  ibp_network_info info;
  double *ptdf, *lodf;
  int32_t* ctg;
  int32_t tiles[7];
  int rep, nc;
  make_ring(&o, &d, 150);
  nc = d.n_ctg;
  for (rep = 0; rep < 4; ++rep) {
    /* 0: listed outages; 1: NULL list, every non-bridge line; 2: listed
     * outages and curves; 3: an empty list (no outages) */
    d.ctg_line = rep == 1 ? NULL : o.ctg;
    d.n_ctg = rep == 1 || rep == 3 ? 0 : nc;
    if (rep == 2) {
      d.seg_ptr = o.seg_ptr;
      d.seg_a = o.sa;
      d.seg_b = o.sb;
      d.seg_U = o.su;
    }
    if (report("valid_build", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, &net)) != 0) return 1;
    if (report("query", ibp_network_query(net, &info)) != 0) return 1;
    printf("sizes %d %d %d %d\n", info.n_bus, info.n_line, info.n_ctg, info.n_input);
    ptdf = malloc(sizeof(double) * (size_t)info.n_line * info.n_bus);
    lodf = malloc(sizeof(double) * (size_t)(info.n_ctg ? info.n_ctg : 1) * info.n_line);
    ctg = malloc(sizeof(int32_t) * (size_t)(info.n_ctg ? info.n_ctg : 1));
    report("export", ibp_network_export(net, ptdf, lodf));
    report("ctg_lines", ibp_network_ctg_lines(net, ctg));
    report("host_bound", ibp_bound_boxes(net, 1, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, 0));
    report("host_noalloc", ibp_bound_boxes_noalloc(net, 1, NULL, NULL, NULL, NULL, NULL, NULL, 0));
    report("host_backward", ibp_bound_backward(net, 1, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, 0));
    report("host_timing", ibp_set_kernel_timing(net, 1));
    report("host_autotune", ibp_autotune_batched(net, 8, NULL, NULL, NULL, 0, NULL, NULL));
    report("tile_get", ibp_get_tile(net, tiles));
    report("tile_bad", ibp_set_tile_batched(net, 3, 0, 0, 1, 0));
    printf("host_workspace %zu\n", ibp_workspace_bytes(net, 4, IBP_F_NONE));
    free(ptdf);
    free(lodf);
    free(ctg);
    ibp_free_network(net);
    net = NULL;
  }
  release(&o);
  return 0;
}

static void invalid_builds(void) {
  owned o;
  ibp_network_desc d;
  ibp_network* net = NULL;
  int32_t saved;
  double sb;
  make_ring(&o, &d, 40);
  report("null_desc", ibp_build_network(NULL, IBP_DEVICE_HOST_ONLY, &net));
  report("null_out", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, NULL));
  report("bad_device", ibp_build_network(&d, -7, &net));
  saved = o.to[3];
  o.to[3] = 40;
  report("bus_out_of_range", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, &net));
  o.to[3] = o.from[3];
  report("self_loop", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, &net));
  o.to[3] = saved;
  sb = o.b[5];
  o.b[5] = 0.0;
  report("zero_susceptance", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, &net));
  o.b[5] = sb;
  d.zeta_f = -1.0;
  report("negative_zeta", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, &net));
  d.zeta_f = 10.0;
  d.slack_bus = 40;
  report("bad_slack", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, &net));
  d.slack_bus = 0;
  saved = o.gbus[1];
  o.gbus[1] = -1;
  report("bad_gen_bus", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, &net));
  o.gbus[1] = saved;
  saved = o.ctg[2];
  o.ctg[2] = o.l;
  report("bad_ctg_index", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, &net));
  o.ctg[2] = saved;
  /* the ring without its chords, minus one ring line: a path whose lines
   * are all bridges; listing one as an outage islands the network */
  d.n_line = o.n - 1;
  d.n_ctg = 1;
  report("islanding_outage", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, &net));
  /* two components: lines that never touch the last bus */
  d.n_line = o.n - 2;
  d.n_ctg = 0;
  d.ctg_line = NULL;
  report("disconnected", ibp_build_network(&d, IBP_DEVICE_HOST_ONLY, &net));
  printf("last_error_nonempty %d\n", ibp_last_error()[0] != 0);
  report("query_null", ibp_network_query(NULL, NULL));
  report("export_null", ibp_network_export(NULL, NULL, NULL));
  report("tile_null", ibp_set_tile_batched(NULL, 4, 0, 0, 1, 0));
  report("split_bad", ibp_split_select(-1, NULL, 0, NULL, 0, NULL, NULL, NULL, NULL, NULL, NULL, NULL));
  report("split_empty", ibp_split_select(0, NULL, 4, NULL, 3, NULL, NULL, NULL, NULL, NULL, NULL, NULL));
  report("split_null", ibp_split_select(4, NULL, 4, NULL, 3, NULL, NULL, NULL, NULL, NULL, NULL, NULL));
  report("probe_null", ibp_read_probe(NULL, 4, NULL, NULL));
  printf("workspace_null %zu\n", ibp_workspace_bytes(NULL, 4, IBP_F_NONE));
  ibp_free_network(NULL);
  release(&o);
}

int main(void) {
  if (valid_builds() != 0) return 1;
  invalid_builds();
  return 0;
}
