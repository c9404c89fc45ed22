#!/usr/bin/env python3
"""Benchmark of IBP through the SC-DCOPF graph on one MI355X.

Default workload: the large single-box form (8316 buses, 14000 lines, 1500
generators, 5000 flexible loads, 8000 N-1 outages, the whole admissible box),
float32 factors with outward padding.  One step = one call of
ibp_bound_boxes (box preparation, base flows, the full outage sweep and the
objective interval) with the box already resident in device memory.

Prints ONE JSON line:
  metric/value/unit      box x contingency x line interval evaluations per second
  roofline               the dominant kernel's algorithmic bytes / its mean
                         duration (HIP events on the launch stream) vs 8 TB/s
  step_roofline          the same for the whole step (PTDF + outage factors)
  cpu_baseline           the FP64 CPU oracle on the same box (host cores)
  bound_gap_vs_fp64      relative distance of the GPU bounds to the oracle's
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def _threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return 1


def cpu_baseline(net, lo, hi):
    """FP64 oracle on the same box, timed on the host (bound evaluation only)."""
    import oracle
    t0 = time.perf_counter()
    fac = oracle.factors(net)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = oracle.ibp(net, lo, hi, fac)
    t = time.perf_counter() - t0
    return r, t, t_build, int(fac["K"])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    from paper_2511_15624_amd import ibp, synth

    name = "c8316"
    net = synth.make_config(name)
    lo, hi = synth.full_box(net)
    t0 = time.perf_counter()
    n = ibp.Network(net, device=0)
    t_setup = time.perf_counter() - t0
    N, L, K = n.n_bus, n.n_line, n.n_ctg
    B = 1
    tlo = torch.from_numpy(lo[None].copy()).cuda()
    thi = torch.from_numpy(hi[None].copy()).cuda()
    ws = ibp.Workspace(n)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        f_lo, f_hi = ibp.ibp_bound_boxes(n, tlo, thi, ws=ws)
    torch.cuda.synchronize()

    # timed region: K steps between events on the launch stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        f_lo, f_hi = ibp.ibp_bound_boxes(n, tlo, thi, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    # kernel pass: the same steps again with the library recording a HIP event
    # pair around every kernel it queues on this stream (the events add gaps
    # between kernels, so the step time above is taken without them)
    n.set_kernel_timing(True)
    _ = n.kernel_times()
    for _ in range(args.steps):
        ibp.ibp_bound_boxes(n, tlo, thi, ws=ws)
    torch.cuda.synchronize()
    kt = n.kernel_times()
    n.set_kernel_timing(False)
    ms_step = ms_total / args.steps
    evals = B * K * L
    value = evals / (ms_step * 1e-3)

    # algorithmic bytes per launch: each float32 factor read once per box
    bytes_k = {"base_flows": 4.0 * L * N * B, "outage_sweep": 4.0 * L * K * B}
    avg = {k: v[0] / v[1] for k, v in kt.items()}
    dom = max(bytes_k, key=lambda k: avg.get(k, 0.0))
    achieved = bytes_k[dom] / (avg[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "mean_us": round(avg[dom] * 1e3, 2), "algorithmic_bytes": bytes_k[dom]}
    step_bytes = sum(bytes_k.values())
    step_gbs = step_bytes / (ms_step * 1e-3) / 1e9
    out = {
        "metric": "box·contingency·line interval evals/sec",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "large single box: 8316 buses, 14000 lines, 8000 N-1 outages, "
                               "1500 generators, 5000 flexible loads, whole admissible box",
                   "n_bus": N, "n_line": L, "n_ctg": K, "n_box": B, "seed": 4},
        "roofline": roof,
        "step_roofline": {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                          "algorithmic_bytes": step_bytes},
        "kernel_us": {k: round(v * 1e3, 2) for k, v in avg.items()},
        "setup_s": round(t_setup, 2),
    }
    g_lo, g_hi = float(f_lo.cpu()[0]), float(f_hi.cpu()[0])
    if not args.no_cpu_baseline:
        r, t_cpu, t_build, k_or = cpu_baseline(net, lo, hi)
        out["cpu_baseline"] = {"value": evals / t_cpu, "unit": "evals/s", "cores": _threads(),
                               "kind": "oracle",
                               "sample": f"the full single box ({K} outages x {L} lines), FP64 "
                                         f"numpy; {t_cpu:.2f} s; factor construction "
                                         f"{t_build:.1f} s not timed; elementwise stages single-threaded"}
        den_lo = max(abs(r["f_lo"]), 1.0)
        den_hi = max(abs(r["f_hi"]), 1.0)
        out["bound_gap_vs_fp64"] = {
            "encloses": bool(g_lo <= r["f_lo"] and g_hi >= r["f_hi"]),
            "lo_rel": (r["f_lo"] - g_lo) / den_lo,
            "hi_rel": (g_hi - r["f_hi"]) / den_hi,
            "gpu": [g_lo, g_hi], "oracle": [r["f_lo"], r["f_hi"]],
        }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
