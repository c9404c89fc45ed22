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
  bound_gap_vs_fp64      relative distance of the GPU bounds to the oracle's, on
                         the headline box and on samples of the sub-box workloads
  paper_context          the paper's own timing (other hardware), for context
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
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "ibp_traffic_c8316_single_box.json")
# kernel-name prefixes in rocprofv3 records (the template argument is the tile
# the network chose)
KERNEL_NAMES = {"base_flows": "ibp::k2_base_flows<", "outage_sweep": "ibp::k3_contingency<"}
ALGO_BYTES = {"base_flows": 465696000, "outage_sweep": 448000000}


def _record_kernel(kernels: dict, kernel: str):
    """The record entry of `kernel` (one instantiation per profiled run)."""
    names = [k for k in kernels if k.startswith(KERNEL_NAMES[kernel])]
    return kernels[names[0]] if len(names) == 1 else None


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter record
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's readings), or None when
    the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
        m = hashlib.sha256()
        for p in rec["sources"]:
            with open(os.path.join(ROOT, p), "rb") as g:
                m.update(g.read())
        if m.hexdigest()[:16] != rec["source_sha256_16"]:
            return None
        k = _record_kernel(rec["kernels"], kernel)
        return k["fetch_bytes"] + k["write_bytes"]
    except Exception:
        return None


def write_traffic_record(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """Turns four rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE of the bound,
    and of --calibrate-copy) into the committed record read by measured_traffic
    and a short markdown summary beside it."""
    import csv
    import hashlib

    def read(d):
        rows = {}
        for fn in os.listdir(d):
            if fn.endswith("counter_collection.csv"):
                with open(os.path.join(d, fn)) as f:
                    for r in csv.DictReader(f):
                        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
                        rows.setdefault(name, []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in rows.items()}

    fetch, write = read(fetch_dir), read(write_dir)
    cf = read(copy_fetch_dir)["__amd_rocclr_copyBuffer"]
    cw = read(copy_write_dir)["__amd_rocclr_copyBuffer"]
    fs, wsc = (1 << 30) / (cf * 1024), (1 << 30) / (cw * 1024)
    sources = ["paper_2511_15624_amd/csrc/ibp_forward.hip", "paper_2511_15624_amd/csrc/ibp_devfun.h"]
    m = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as g:
            m.update(g.read())
    kern = {}
    for k in sorted(fetch):
        if not k.startswith("ibp::"):
            continue
        algo = next((ALGO_BYTES[n] for n, pre in KERNEL_NAMES.items() if k.startswith(pre)), None)
        kern[k] = {"fetch_kib": fetch[k], "write_kib": write.get(k, 0.0), "fetch_bytes": fetch[k] * 1024 * fs,
                   "write_bytes": write.get(k, 0.0) * 1024 * wsc, "algorithmic_bytes": algo}
    rec = {"workload": "8316 buses, 14000 lines, 8000 outages, single whole box", "fetch_scale": fs,
           "write_scale": wsc, "source_sha256_16": m.hexdigest()[:16], "sources": sources, "kernels": kern}
    with open(TRAFFIC_RECORD, "w") as f:
        json.dump(rec, f, indent=1)
    # the summary repeats the commands with the output folders this record was made from
    rel = [os.path.relpath(os.path.abspath(d), ROOT) for d in (fetch_dir, write_dir, copy_fetch_dir, copy_write_dir)]
    cmd = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc {c} --output-format csv -d <repo>/{d} "
           "-o run -- python3 <repo>/bench.py {a}")
    lines = ["# HBM traffic counters: forward bound, 8316-bus single box", "",
             "Commands (repository root on one MI355X; each counter in a run of its own):", "", "```",
             cmd.format(c="FETCH_SIZE", d=rel[0], a="--steps 3 --warmup 1 --no-cpu-baseline --no-extras"),
             cmd.format(c="WRITE_SIZE", d=rel[1], a="--steps 3 --warmup 1 --no-cpu-baseline --no-extras"),
             cmd.format(c="FETCH_SIZE", d=rel[2], a="--calibrate-copy"),
             cmd.format(c="WRITE_SIZE", d=rel[3], a="--calibrate-copy"),
             "python3 bench.py --traffic-record " + " ".join(rel), "```", "",
             f"Calibration: a 1 GiB device copy (`__amd_rocclr_copyBuffer`) reads {cf:.1f} KiB FETCH_SIZE and "
             f"{cw:.1f} KiB WRITE_SIZE per dispatch,",
             f"so bytes = FETCH_SIZE KiB x 1024 x {fs:.4f} and WRITE_SIZE KiB x 1024 x {wsc:.4f}.", "",
             "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | read bytes (scaled) | written bytes | algorithmic bytes "
             "| traffic / algorithmic |", "|---|---|---|---|---|---|---|"]
    for k, v in kern.items():
        a = v["algorithmic_bytes"]
        ratio = f"{(v['fetch_bytes'] + v['write_bytes']) / a:.4f}" if a else "-"
        lines.append(f"| {k} | {v['fetch_kib']:.1f} | {v['write_kib']:.1f} | {v['fetch_bytes']:.4g} | "
                     f"{v['write_bytes']:.4g} | {a if a else '-'} | {ratio} |")
    lines += ["", "Kernel sources hashed for staleness: " + ", ".join(sources) + f" -> {rec['source_sha256_16']}."]
    with open(TRAFFIC_RECORD[:-5] + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    print(TRAFFIC_RECORD)
    return 0


def _threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return 1


def host_info():
    """Host cores, BLAS threads and CPU model, recorded beside the oracle's timings."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_count": os.cpu_count(), "cpus_available": avail, "blas_threads": _threads(), "cpu_model": model}


def cpu_baseline(net, lo, hi, min_seconds=10.0, max_runs=12):
    """FP64 oracle on the same box, timed on the host (bound evaluation only):
    repeated until about min_seconds of work (at most max_runs runs); returns
    the mean time per run and the run count."""
    import oracle
    t0 = time.perf_counter()
    fac = oracle.factors(net)
    t_build = time.perf_counter() - t0
    runs, total = 0, 0.0
    while runs < max_runs and (runs == 0 or total < min_seconds):
        t0 = time.perf_counter()
        r = oracle.ibp(net, lo, hi, fac)
        total += time.perf_counter() - t0
        runs += 1
    return r, total / runs, t_build, fac, runs


def cpu_batched_sample(synth, n_sample=4):
    """FP64 oracle on a seeded sample of the 2000-bus period boxes, per box
    (bound evaluation only); returns (evals per box, seconds per box, factors)."""
    import oracle
    net3 = synth.make_config("c2000")
    fac = oracle.factors(net3)
    lo, hi, _ = synth.period_boxes(net3, 18, 1024, seed=31)
    idx = np.random.default_rng(3).choice(lo.shape[0], n_sample, replace=False)
    t0 = time.perf_counter()
    for b in idx:
        oracle.ibp(net3, lo[b], hi[b], fac)
    t = (time.perf_counter() - t0) / n_sample
    return int(fac["K"]) * len(net3["line_from"]), t, fac


def sub_box_gaps(torch, ibp, synth, n3, net3, fac3, n4, net4, fac4):
    """Distance of the GPU bounds to the FP64 oracle's on seeded samples of the
    sub-box workloads, each computed in the launch configuration timed above
    (one call over every box of the workload): relative to max(|f|, 1 $), to
    the term scale T (|S| + zeta_inj I + zeta_f (Fb + Fc) of that side), to the
    error budget of the float32 padding rules (the largest gap they allow) and
    to the floor that any method reading float32 factors must leave."""
    from concurrent.futures import ThreadPoolExecutor

    from tests.error_budget import budget

    def gpu(n, lo, hi):
        f_lo, f_hi = ibp.ibp_bound_boxes(n, torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda())
        torch.cuda.synchronize()
        return f_lo.cpu().numpy(), f_hi.cpu().numpy()

    rng = np.random.default_rng(2024)
    lo3, hi3, _ = synth.period_boxes(net3, 18, 1024, seed=31)
    lo5, hi5 = synth.sub_boxes(net3, 4096, seed=51)
    lo4, hi4 = synth.sub_boxes(net4, 256, seed=41)
    cases = [("2000 buses, 18 periods x 1024 sub-boxes (one call)", n3, net3, fac3, lo3, hi3, 48),
             ("2000 buses, 4096 sub-boxes (one call)", n3, net3, fac3, lo5, hi5, 16),
             ("8316 buses, 256 sub-boxes (one call)", n4, net4, fac4, lo4, hi4, 8)]
    out = []
    with ThreadPoolExecutor(max_workers=8) as ex:
        for what, n, net, fac, lo, hi, k in cases:
            g_lo, g_hi = gpu(n, lo, hi)
            idx = np.sort(rng.choice(lo.shape[0], k, replace=False))
            pe = float(n.info.phi_abs_err)
            t0 = time.perf_counter()
            bus = list(ex.map(lambda b: budget(net, fac, lo[b], hi[b], pe), idx))
            secs = time.perf_counter() - t0
            rows = []
            for b, bu in zip(idx, bus):
                r = bu["r"]
                glo, ghi = r["f_lo"] - g_lo[b], g_hi[b] - r["f_hi"]
                flo, fhi = max(abs(r["f_lo"]), 1.0), max(abs(r["f_hi"]), 1.0)
                rows.append([glo, ghi, glo / flo, ghi / fhi, glo / bu["T_lo"], ghi / bu["T_hi"],
                             glo / bu["lo"], ghi / bu["hi"], glo / bu["floor_lo"], ghi / bu["floor_hi"],
                             bu["lo"] / flo, bu["hi"] / fhi, bu["floor_lo"] / flo, bu["floor_hi"] / fhi])
            a = np.array(rows)

            def mm(j):
                return {"max": float(a[:, j].max()), "median": float(np.median(a[:, j]))}

            out.append({"workload": what, "boxes_sampled": int(k), "oracle_seconds": round(secs, 1),
                        "encloses": bool(np.all(a[:, 0] >= 0) and np.all(a[:, 1] >= 0)),
                        "lo_rel_f": mm(2), "hi_rel_f": mm(3), "lo_rel_T": mm(4), "hi_rel_T": mm(5),
                        "over_1e-5_of_f": {"lo": int(np.sum(a[:, 2] > 1e-5)), "hi": int(np.sum(a[:, 3] > 1e-5))},
                        "gap_over_budget": {"lo": mm(6), "hi": mm(7)},
                        "gap_over_floor": {"lo": mm(8), "hi": mm(9)},
                        "budget_over_1e-5_of_f": {"lo": int(np.sum(a[:, 10] > 1e-5)),
                                                  "hi": int(np.sum(a[:, 11] > 1e-5))},
                        "floor_over_1e-5_of_f": {"lo": int(np.sum(a[:, 12] > 1e-5)),
                                                 "hi": int(np.sum(a[:, 13] > 1e-5))}})
    return out


def hbm_probe(torch, ibp):
    """Measured device bandwidth: torch copy_ of 1 GiB (bytes read + written)
    and the library's streaming-read probe over 1 GiB (the sweeps' load
    pattern), 10 times each."""
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    part = torch.empty(2048, dtype=torch.float32, device="cuda")
    ms_copy = _time(torch, lambda: y.copy_(x), 10)
    ms_read = _time(torch, lambda: ibp.ibp_read_probe(x, part), 10)
    del x, y
    torch.cuda.empty_cache()
    return {"copy_gbs": round(2 * (1 << 30) / (ms_copy * 1e-3) / 1e9, 1),
            "read_gbs": round((1 << 30) / (ms_read * 1e-3) / 1e9, 1),
            "note": "torch copy_ of 1 GiB (read + written bytes); ibp_read_probe over 1 GiB (read bytes)"}


def alu_probe(torch, ibp):
    """Measured float32 FMA issue rate: the library's probe (eight chains per
    lane, 2^19 lanes, 16384 steps), with every operand in a vector register and
    with one in a scalar register, 10 calls each."""
    out = torch.empty(ibp.ALU_PROBE_LANES, dtype=torch.float32, device="cuda")
    iters = 16384
    ops = ibp.ALU_PROBE_LANES * 8 * iters
    ms_v = _time(torch, lambda: ibp.ibp_alu_probe(out, iters, False), 10)
    ms_s = _time(torch, lambda: ibp.ibp_alu_probe(out, iters, True), 10)
    return {"fma_vector_operands_ops_per_s": ops / (ms_v * 1e-3), "fma_scalar_operand_ops_per_s": ops / (ms_s * 1e-3),
            "frac_of_valu_peak": round(ops / (ms_v * 1e-3) / VALU_PEAK, 4),
            "note": "lane FMAs per second of ibp_alu_probe; VALU_PEAK is 256 CUs x 128 float32 lanes per clock "
                    "x 2.4 GHz, which FMAs with all-vector-register operands reach (one scalar-register operand: "
                    "half the rate)"}


VALU_PEAK = 78.6e12  # float32 VALU lane-ops/s: 256 CUs x 128 lanes/clock x 2.4 GHz (FMA = one op)
MFMA_F64_PEAK = 78.6e12  # float64 dense matrix FLOP/s of MI355X
MFMA_F32_PEAK = 157.3e12  # float32 dense matrix FLOP/s of MI355X
VALU_PEAK_SOURCE = ("MI355X float32 vector peak 157.3 TFLOP/s with an FMA counted once: 256 CUs x 128 lanes per "
                    "clock x 2.4 GHz; the box-tiled sweep's counters show 0.414 wave instructions per SIMD per "
                    "cycle, above what 16 lanes per clock allow (profiles/ibp_batched_counters_c2000.md), and "
                    "the FMA probe's measured rate is reported beside it (alu_probe)")
OPS_PER_EVAL = 9.25  # VALU ops per box-outage-line evaluation in the outage sweep (from the ISA)
# VALU ops per element of the chord-relaxation sweep: post-outage centre and
# the two interval ends (5), the clipped lower end (3), the slope and its
# quantisation (8), the intercept and its padding (4), the value bound (6),
# activity, selects and sign (5), the fixed-point line totals (4) and the
# outage's four sums with the factor product (8)
CHORD_OPS_PER_ELEM = 43.0
# VALU ops per box-outage-line element of the screened backward sweep (the
# gradient of f_hi alone), on the elements of the lines its screen marks: the
# post-outage centre and radius (2 fma), the activity and sign tests (2
# compares), the selected factor and its sign (2 selects) and the two
# outage-side accumulations; the line side is counted from the compare masks on
# the scalar unit.  The compiled step issues 163 vector instructions per 16
# elements (the rest is loop and counter overhead).
OPS_PER_BWD_EVAL = 8.0
# VALU ops per factor and tile of the backward's line screen (multiply, max)
OPS_PER_SCREEN_EVAL = 2.0


def _time(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _tuned(torch, ibp, net, tlo, thi, ws, ev, ms_default):
    """Autotunes the box-tiled tiles on this very call, times the tuned call,
    then puts the default tiles back so later figures use the same code."""
    keep = net.tiles()
    t0 = time.perf_counter()
    tiles, _ = ibp.ibp_autotune_batched(net, tlo, thi)
    tune_s = time.perf_counter() - t0
    ms = _time(torch, lambda: ibp.ibp_bound_boxes(net, tlo, thi, ws=ws), 3)
    net.set_tile_batched(keep["k3_bt"], keep["k3_rows"], keep["k3_xcd"], keep["k2_mfma"], keep["k2_by"])
    net.set_screen_upper(keep["screen_upper"])
    names = ("k3_bt", "k3_rows", "k3_xcd", "k2_mfma", "k2_by", "screen_upper")
    return {"tiles": {k: tiles[k] for k in names}, "default_tiles": {k: keep[k] for k in names},
            "ms_per_call": ms, "value": ev / (ms * 1e-3), "speedup_vs_default": ms_default / ms,
            "tune_seconds": round(tune_s, 3)}


def extras(torch, ibp, synth, n4, net4):
    """Batched, backward and splitting throughput next to the per-box (plain) form."""
    res = {}
    # latency of one whole box on the small networks (one C-ABI call each)
    lat = {}
    for name in ("tiny", "c500"):
        netx = synth.make_config(name)
        nx = ibp.Network(netx, device=0)
        lx, hx = synth.full_box(netx)
        tl, th = torch.from_numpy(lx[None].copy()).cuda(), torch.from_numpy(hx[None].copy()).cuda()
        wsx = ibp.Workspace(nx)
        buf, _ = wsx.get(1)
        o_lo = torch.empty(1, dtype=torch.float64, device="cuda")
        o_hi = torch.empty(1, dtype=torch.float64, device="cuda")
        import ctypes
        cargs = (nx.handle, 1, ctypes.c_void_p(tl.data_ptr()), ctypes.c_void_p(th.data_ptr()),
                 ctypes.c_void_p(o_lo.data_ptr()), ctypes.c_void_p(o_hi.data_ptr()), ctypes.c_void_p(),
                 ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), 0)
        call = ibp.load_library().ibp_bound_boxes
        lat[name + "_us"] = round(_time(torch, lambda: ibp._check(call(*cargs)), 200) * 1e3, 2)
        nx.close()
    res["latency"] = {"workload": "whole box, one C-ABI call, back to back: 14 buses / 19 outages and "
                                  "500 buses / 590 outages",
                      **lat}
    # batched: 2000-bus network, 18 periods x 1024 sub-boxes in one call
    net3 = synth.make_config("c2000")
    n3 = ibp.Network(net3, device=0)
    lo, hi, _ = synth.period_boxes(net3, 18, 1024, seed=31)
    tlo, thi = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    ws = ibp.Workspace(n3)
    ms = _time(torch, lambda: ibp.ibp_bound_boxes(n3, tlo, thi, ws=ws), 3)
    ev = lo.shape[0] * n3.n_ctg * n3.n_line
    sub = 1024
    ms_p = _time(torch, lambda: ibp.ibp_bound_boxes(n3, tlo[:sub], thi[:sub], ws=ws, flags=ibp.IBP_F_PLAIN), 1)
    ev_p = sub * n3.n_ctg * n3.n_line
    n3.set_kernel_timing(True)
    n3.kernel_times()
    ibp.ibp_bound_boxes(n3, tlo, thi, ws=ws)
    kt = n3.kernel_times()
    n3.set_kernel_timing(False)
    sweep_ms = kt.get("batched_outage_sweep", (float("nan"), 1))[0]
    res["batched"] = {
        "workload": f"2000 buses, {n3.n_line} lines, {n3.n_ctg} outages, 18 periods x 1024 sub-boxes = "
                    f"{lo.shape[0]} boxes in one call",
        "value": ev / (ms * 1e-3), "unit": "evals/s", "ms_per_call": ms,
        "plain_value": ev_p / (ms_p * 1e-3), "plain_sample": f"first {sub} boxes, per-box kernels",
        "speedup_vs_plain": (ev / ms) / (ev_p / ms_p),
        "kernel_ms": {k: round(v[0], 3) for k, v in kt.items()},
        "roofline": {"bound": "alu", "kernel": "batched_outage_sweep",
                     "achieved": ev * OPS_PER_EVAL / (sweep_ms * 1e-3), "peak": VALU_PEAK, "unit": "ops/s",
                     "peak_source": VALU_PEAK_SOURCE,
                     "frac": ev * OPS_PER_EVAL / (sweep_ms * 1e-3) / VALU_PEAK,
                     "ops_per_eval": OPS_PER_EVAL},
    }
    res["batched"]["tuned"] = _tuned(torch, ibp, n3, tlo, thi, ws, ev, ms)
    # the same call with the upper-penalty line screen (IBP_F_SCREEN_UPPER):
    # both penalty sums over the lines that can hold an active penalty
    scr = ibp.IBP_F_SCREEN_UPPER
    ms_s = _time(torch, lambda: ibp.ibp_bound_boxes(n3, tlo, thi, ws=ws, flags=scr), 3)
    n3.set_kernel_timing(True)
    n3.kernel_times()
    ibp.ibp_bound_boxes(n3, tlo, thi, ws=ws, flags=scr)
    kts = n3.kernel_times()
    n3.set_kernel_timing(False)
    res["batched"]["screened"] = {"flags": "IBP_F_SCREEN_UPPER", "ms_per_call": ms_s, "value": ev / (ms_s * 1e-3),
                                  "speedup_vs_default": ms / ms_s,
                                  "kernel_ms": {k: round(v[0], 3) for k, v in kts.items()},
                                  "note": "bounds equal the default call's within float32 summation order "
                                          "(1e-6 relative), both certified"}
    # the base flows of the same call on the float64 matrix cores: 2 products
    # (centre, radius) x 2 flops x lines x buses x boxes
    bf_ms = kt.get("batched_base_flows", (float("nan"), 1))[0]
    bf_flops = 4.0 * n3.n_line * n3.n_bus * lo.shape[0]
    res["batched"]["roofline_base_flows"] = {
        "bound": "mfma", "kernel": "batched_base_flows", "achieved": bf_flops / (bf_ms * 1e-3),
        "peak": MFMA_F64_PEAK, "unit": "FLOP/s", "frac": bf_flops / (bf_ms * 1e-3) / MFMA_F64_PEAK,
        "flops": bf_flops}
    # batched on the large network: 256 sub-boxes
    blo, bhi = synth.sub_boxes(net4, 256, seed=41)
    t4l, t4h = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    ws4 = ibp.Workspace(n4)
    ms4 = _time(torch, lambda: ibp.ibp_bound_boxes(n4, t4l, t4h, ws=ws4), 3)
    ms4p = _time(torch, lambda: ibp.ibp_bound_boxes(n4, t4l, t4h, ws=ws4, flags=ibp.IBP_F_PLAIN), 1)
    ev4 = 256 * n4.n_ctg * n4.n_line
    res["batched_large"] = {"workload": "8316 buses, 256 sub-boxes", "value": ev4 / (ms4 * 1e-3),
                            "unit": "evals/s", "ms_per_call": ms4, "plain_value": ev4 / (ms4p * 1e-3),
                            "speedup_vs_plain": ms4p / ms4,
                            "tuned": _tuned(torch, ibp, n4, t4l, t4h, ws4, ev4, ms4)}
    ms4s = _time(torch, lambda: ibp.ibp_bound_boxes(n4, t4l, t4h, ws=ws4, flags=ibp.IBP_F_SCREEN_UPPER), 3)
    res["batched_large"]["screened"] = {"flags": "IBP_F_SCREEN_UPPER", "ms_per_call": ms4s,
                                        "value": ev4 / (ms4s * 1e-3), "speedup_vs_default": ms4 / ms4s}
    # backward: 2000-bus network, 4096 sub-boxes of period 0
    blo, bhi = synth.sub_boxes(net3, 4096, seed=51)
    t5l, t5h = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
    g0 = torch.zeros(4096, dtype=torch.float64, device="cuda")
    g1 = torch.ones(4096, dtype=torch.float64, device="cuda")
    wsb = ibp.Workspace(n3)
    msf = _time(torch, lambda: ibp.ibp_bound_boxes(n3, t5l, t5h, ws=wsb), 3)
    msb = _time(torch, lambda: ibp.ibp_bound_backward(n3, t5l, t5h, None, g1, ws=wsb,
                                                       flags=ibp.IBP_F_UPPER_ONLY), 3)
    msb2 = _time(torch, lambda: ibp.ibp_bound_backward(n3, t5l, t5h, g0, g1, ws=wsb), 3)
    sub = 256
    msbp = _time(torch, lambda: ibp.ibp_bound_backward(n3, t5l[:sub], t5h[:sub], None, g1[:sub], ws=wsb,
                                                        flags=ibp.IBP_F_PLAIN | ibp.IBP_F_UPPER_ONLY), 1)
    ev5 = 4096 * n3.n_ctg * n3.n_line
    # the differentiation form as a training loop runs it: the upper bound, then
    # its gradient on the same boxes, with and without reusing the forward's
    # intermediates
    up = ibp.IBP_F_UPPER_ONLY
    wsf = ibp.Workspace(n3)

    def fwd_bwd(keep):
        ibp.ibp_bound_boxes(n3, t5l, t5h, ws=wsf, flags=up | (ibp.IBP_F_KEEP_PREP if keep else 0))
        ibp.ibp_bound_backward(n3, t5l, t5h, None, g1, ws=wsf, flags=up | (ibp.IBP_F_REUSE_PREP if keep else 0))

    ms_fb_keep = _time(torch, lambda: fwd_bwd(True), 3)
    ms_fb = _time(torch, lambda: fwd_bwd(False), 3)
    n3.set_kernel_timing(True)
    n3.kernel_times()
    for _ in range(3):
        ibp.ibp_bound_backward(n3, t5l, t5h, None, g1, ws=wsb, flags=ibp.IBP_F_UPPER_ONLY)
    ktb = {k: v[0] / 3 for k, v in n3.kernel_times().items()}
    n3.set_kernel_timing(False)
    marked, pairs = ibp.ibp_backward_screen_lines(n3, 4096, wsb)
    # the same call with every line swept (IBP_TILE=k5s=0 keeps the dense sweep)
    os.environ["IBP_TILE"] = "k5s=0"
    n3d = ibp.Network(net3, device=0)
    os.environ.pop("IBP_TILE")
    msbd = _time(torch, lambda: ibp.ibp_bound_backward(n3d, t5l, t5h, None, g1, ws=wsb,
                                                        flags=ibp.IBP_F_UPPER_ONLY), 3)
    n3d.close()
    k5_ev = marked * n3.n_ctg * 4  # elements the screened sweep evaluates (4 boxes per tile)
    k5s_ms = ktb.get("backward_line_screen", float("nan"))
    k5s_ops = OPS_PER_SCREEN_EVAL * n3.n_ctg * n3.n_line * (pairs // n3.n_line)
    k5_ms = ktb.get("backward_outage_sweep", float("nan"))
    k6_ms = ktb.get("backward_ptdf_t", float("nan"))
    k6_fma = 2.0 * n3.n_bus * n3.n_line * 4096
    res["backward"] = {"workload": "2000 buses, 4096 sub-boxes: d(f_hi)/d(box endpoints), one-sided call",
                       "value": ev5 / (msb * 1e-3), "unit": "evals/s", "ms_backward": msb,
                       "ms_backward_two_sided_weights": msb2,
                       "ms_backward_dense_sweep": msbd,
                       "screen": {"marked_tile_lines": marked, "tile_lines": pairs,
                                  "marked_fraction": marked / pairs,
                                  "note": "per tile of 4 boxes, the lines on which some outage can make the lower "
                                          "penalty active; only those are swept (value counts every element of "
                                          "the map, as the dense sweep evaluates them)"},
                       "ms_forward": msf, "plain_value": sub * n3.n_ctg * n3.n_line / (msbp * 1e-3),
                       "plain_sample": f"first {sub} boxes, per-box kernels",
                       "kernel_ms": {k: round(v, 3) for k, v in ktb.items()},
                       "forward_then_backward": {
                           "workload": "upper bound then its gradient on the same 4096 boxes (one-sided calls)",
                           "ms_reusing_forward_intermediates": ms_fb_keep, "ms_recomputing": ms_fb,
                           "value": ev5 / (ms_fb_keep * 1e-3), "unit": "evals/s (each element forward and back)"},
                       "roofline": {"bound": "alu", "kernel": "backward_outage_sweep",
                                    "achieved": k5_ev * OPS_PER_BWD_EVAL / (k5_ms * 1e-3), "peak": VALU_PEAK,
                                    "peak_source": VALU_PEAK_SOURCE,
                                    "unit": "ops/s", "frac": k5_ev * OPS_PER_BWD_EVAL / (k5_ms * 1e-3) / VALU_PEAK,
                                    "ops_per_eval": OPS_PER_BWD_EVAL, "evals": k5_ev},
                       "roofline_screen": {"bound": "alu", "kernel": "backward_line_screen",
                                           "achieved": k5s_ops / (k5s_ms * 1e-3), "peak": VALU_PEAK,
                                           "unit": "ops/s", "frac": k5s_ops / (k5s_ms * 1e-3) / VALU_PEAK,
                                           "ops": k5s_ops},
                       "roofline_ptdf_t": {"bound": "mfma", "kernel": "backward_ptdf_t",
                                           "achieved": 2.0 * k6_fma / (k6_ms * 1e-3), "peak": MFMA_F32_PEAK,
                                           "unit": "FLOP/s", "frac": 2.0 * k6_fma / (k6_ms * 1e-3) / MFMA_F32_PEAK,
                                           "flops": 2.0 * k6_fma}}
    # piecewise-linear cost and value curves (1-4 segments per device) on the
    # single large box and on the batched workload, beside the linear-cost runs
    lo4, hi4 = synth.full_box(net4)
    s4l, s4h = torch.from_numpy(lo4[None].copy()).cuda(), torch.from_numpy(hi4[None].copy()).cuda()
    ws1 = ibp.Workspace(n4)
    ms_lin = _time(torch, lambda: ibp.ibp_bound_boxes(n4, s4l, s4h, ws=ws1), 50)
    n4c = ibp.Network(synth.with_pwl_costs(net4, seed=9), device=0)
    ms_cur = _time(torch, lambda: ibp.ibp_bound_boxes(n4c, s4l, s4h, ws=ws1), 50)
    n4c.set_kernel_timing(True)
    n4c.kernel_times()
    for _ in range(10):
        ibp.ibp_bound_boxes(n4c, s4l, s4h, ws=ws1)
    kt4 = n4c.kernel_times()
    n4c.set_kernel_timing(False)
    n4c.close()
    n3c = ibp.Network(synth.with_pwl_costs(net3, seed=10), device=0)
    ms3c = _time(torch, lambda: ibp.ibp_bound_boxes(n3c, tlo, thi, ws=ws), 3)
    n3c.close()
    ev1 = n4.n_ctg * n4.n_line
    res["curves"] = {
        "workload": "piecewise-linear cost/value curves, 1-4 segments per device: the large single box, "
                    "and 18 periods x 1024 sub-boxes on the 2000-bus network",
        "single_box_value": ev1 / (ms_cur * 1e-3), "unit": "evals/s", "single_box_ms": ms_cur,
        "single_box_ms_linear_costs": ms_lin,
        "single_box_kernel_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in kt4.items()},
        "batched_value": ev / (ms3c * 1e-3), "batched_ms": ms3c, "batched_ms_linear_costs": ms,
    }
    # linear-relaxation upper bound: the large single box, and 1024 sub-boxes of
    # the 2000-bus network; time and tightening of f_hi against IBP alone
    wsc = ibp.Workspace(n4)
    ms_c1 = _time(torch, lambda: ibp.ibp_crown_bound_boxes(n4, s4l, s4h, ws=wsc), 20)
    n4.set_kernel_timing(True)
    n4.kernel_times()
    for _ in range(5):
        _, c_hi1, c_only1 = ibp.ibp_crown_bound_boxes(n4, s4l, s4h, crown=True, ws=wsc)
    ktc = n4.kernel_times()
    n4.set_kernel_timing(False)
    i_lo1, i_hi1 = ibp.ibp_bound_boxes(n4, s4l, s4h, ws=ws1)
    c3l, c3h = tlo[:1024].contiguous(), thi[:1024].contiguous()
    ws3c = ibp.Workspace(n3)
    ms_c3 = _time(torch, lambda: ibp.ibp_crown_bound_boxes(n3, c3l, c3h, ws=ws3c), 2)
    ms_i3 = _time(torch, lambda: ibp.ibp_bound_boxes(n3, c3l, c3h, ws=ws3c), 2)
    _, c_hi3 = ibp.ibp_crown_bound_boxes(n3, c3l, c3h, ws=ws3c)
    _, i_hi3 = ibp.ibp_bound_boxes(n3, c3l, c3h, ws=ws3c)
    tight3 = ((i_hi3 - c_hi3) / i_hi3.abs()).cpu()
    ms_r3 = _time(torch, lambda: ibp.ibp_crown_bound_boxes(n3, c3l, c3h, ws=ws3c, ref_iters=4), 1)
    _, r_hi3 = ibp.ibp_crown_bound_boxes(n3, c3l, c3h, ws=ws3c, ref_iters=4)
    tightr = ((i_hi3 - r_hi3) / i_hi3.abs()).cpu()
    res["crown"] = {
        "workload": "linear-relaxation upper bound: the large single box; 1024 sub-boxes (2000 buses)",
        "single_box_ms": ms_c1, "single_box_ms_ibp_only": ms_lin,
        "single_box_value": ev1 / (ms_c1 * 1e-3), "unit": "evals/s",
        "single_box_kernel_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in ktc.items()},
        "single_box_f_hi_ibp": float(i_hi1[0]), "single_box_f_hi_crown": float(c_only1[0]),
        "batch_ms": ms_c3, "batch_ms_ibp_only": ms_i3,
        "batch_value": 1024 * n3.n_ctg * n3.n_line / (ms_c3 * 1e-3),
        "batch_f_hi_tightening_mean": float(tight3.mean()), "batch_f_hi_tightening_max": float(tight3.max()),
        "batch_ms_4_reference_points": ms_r3,
        "batch_f_hi_tightening_mean_4_reference_points": float(tightr.mean()),
        "batch_f_hi_tightening_max_4_reference_points": float(tightr.max()),
    }
    # chord-relaxation lower bound: the same two workloads; time and tightening
    # of f_lo against IBP alone
    ms_l1 = _time(torch, lambda: ibp.ibp_crown_lower_boxes(n4, s4l, s4h, ws=wsc), 20)
    n4.set_kernel_timing(True)
    n4.kernel_times()
    for _ in range(5):
        _, _, l_only1 = ibp.ibp_crown_lower_boxes(n4, s4l, s4h, crown=True, ws=wsc)
    ktl = n4.kernel_times()
    n4.set_kernel_timing(False)
    ms_l3 = _time(torch, lambda: ibp.ibp_crown_lower_boxes(n3, c3l, c3h, ws=ws3c), 2)
    ms_i3l = _time(torch, lambda: ibp.ibp_bound_boxes(n3, c3l, c3h, ws=ws3c, flags=ibp.IBP_F_LOWER_ONLY), 2)
    ms_l3o = _time(torch, lambda: ibp.ibp_crown_lower_boxes(n3, c3l, c3h, ws=ws3c, flags=ibp.IBP_F_LOWER_ONLY), 2)
    l_lo3, _ = ibp.ibp_crown_lower_boxes(n3, c3l, c3h, ws=ws3c)
    i_lo3, _ = ibp.ibp_bound_boxes(n3, c3l, c3h, ws=ws3c)
    tightl = ((l_lo3 - i_lo3) / i_lo3.abs()).cpu()
    n3.set_kernel_timing(True)
    n3.kernel_times()
    ibp.ibp_crown_lower_boxes(n3, c3l, c3h, ws=ws3c)
    ktl3 = n3.kernel_times()
    n3.set_kernel_timing(False)
    # per call (the box-tiled call's timer slot also holds its small zeroing kernel)
    sw1 = ktl["crown_outage_sweep"][0] / 5
    sw3 = ktl3["crown_outage_sweep"][0]
    e3 = 1024 * n3.n_ctg * n3.n_line
    res["crown_lower"] = {
        "workload": "chord-relaxation lower bound: the large single box; 1024 sub-boxes (2000 buses)",
        "roofline_chord_sweep": {
            "bound": "alu", "kernel": "crown_outage_sweep", "peak": VALU_PEAK, "unit": "ops/s",
            "peak_source": VALU_PEAK_SOURCE, "ops_per_element": CHORD_OPS_PER_ELEM,
            "single_box": {"ms": sw1, "achieved": ev1 * CHORD_OPS_PER_ELEM / (sw1 * 1e-3),
                           "frac": ev1 * CHORD_OPS_PER_ELEM / (sw1 * 1e-3) / VALU_PEAK},
            "batch": {"ms": sw3, "achieved": e3 * CHORD_OPS_PER_ELEM / (sw3 * 1e-3),
                      "frac": e3 * CHORD_OPS_PER_ELEM / (sw3 * 1e-3) / VALU_PEAK}},
        "single_box_ms": ms_l1, "single_box_ms_ibp_only": ms_lin,
        "single_box_value": ev1 / (ms_l1 * 1e-3), "unit": "evals/s",
        "single_box_kernel_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in ktl.items()},
        "single_box_f_lo_ibp": float(i_lo1[0]), "single_box_f_lo_chord": float(l_only1[0]),
        "batch_ms": ms_l3, "batch_ms_lower_only": ms_l3o, "batch_ms_ibp_lower_only": ms_i3l,
        "batch_value": 1024 * n3.n_ctg * n3.n_line / (ms_l3 * 1e-3),
        "batch_f_lo_tightening_mean": float(tightl.mean()), "batch_f_lo_tightening_max": float(tightl.max()),
    }
    # splitting: 4096 roots, 10 rounds of gradient-ranked bisection
    from paper_2511_15624_amd.split import BoxSplitter
    sp = BoxSplitter(n3, t5l, t5h, rounds=10)
    torch.cuda.synchronize()
    gap0 = float(sp.gap().sum())
    hist = sp.run(10)
    gap10, secs = hist[-1][:2]
    # the same loop with every line swept by its one-sided calls (no screens)
    os.environ["IBP_TILE"] = "k3s=0,k5s=0"
    n3d = ibp.Network(net3, device=0)
    os.environ.pop("IBP_TILE")
    spd = BoxSplitter(n3d, t5l, t5h, rounds=10)
    torch.cuda.synchronize()
    gap10d, secsd = spd.run(10)[-1][:2]
    n3d.close()
    res["splitting"] = {"workload": "2000 buses, 4096 root boxes, 10 rounds (2 children + 2 centre points "
                                    "per root per round)",
                        "gap_reduction_per_s": (gap0 - gap10) / secs, "unit": "$/s",
                        "total_gap_before": gap0, "total_gap_after": gap10, "seconds": secs,
                        "relative_gap_reduction": (gap0 - gap10) / gap0,
                        "dense_sweeps": {"seconds": secsd, "gap_reduction_per_s": (gap0 - gap10d) / secsd,
                                         "note": "IBP_TILE=k3s=0,k5s=0: the one-sided calls sweep every line"}}
    # branch and bound with screening: 4096 instances on the 14-bus network
    # (boxes of 30-90% of each range at seeded positions; the 2000-bus
    # sub-boxes above are all certified max f < 0 by IBP alone), statuses from
    # IBP at the roots, from the relaxation at the roots, and after up to 40
    # rounds on the open roots
    from paper_2511_15624_amd.split import BranchAndBound
    nett = synth.make_config("tiny")
    nt = ibp.Network(nett, device=0)
    lo_t, hi_t = synth.full_box(nett)
    span = hi_t.astype(float) - lo_t
    rng = np.random.default_rng(77)
    w = rng.uniform(0.3, 0.9, (4096, 1))
    a = lo_t[None, :] + rng.random((4096, lo_t.size)) * span[None, :] * (1 - w)
    tl = torch.from_numpy(synth.round_down_f32(a).astype(np.float32)).cuda()
    th = torch.from_numpy(synth.round_up_f32(a + w * span[None, :]).astype(np.float32)).cuda()
    c_ibp = BranchAndBound(nt, tl, th, rounds=40, relax=False).counts()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bb = BranchAndBound(nt, tl, th, rounds=40, relax=True)
    c_root = bb.counts()
    hist = bb.run(40)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    t0 = time.perf_counter()
    bbr = BranchAndBound(nt, tl, th, rounds=40, relax=True, ref_iters=4)
    c_root_r = bbr.counts()
    hist_r = bbr.run(40)
    torch.cuda.synchronize()
    secs_r = time.perf_counter() - t0
    res["branch_and_bound"] = {
        "workload": "14-bus network, 4096 instance boxes; screening for max f < 0 / >= 0; relaxation bounds "
                    "and vertex points; up to 40 rounds on the open roots",
        "statuses_ibp_roots": c_ibp, "statuses_relaxation_roots": c_root, "statuses_final": bb.counts(),
        "rounds_run": len(hist), "open_per_round": [h[2] for h in hist], "seconds": secs,
        "with_4_reference_points": {"statuses_roots": c_root_r, "statuses_final": bbr.counts(),
                                    "rounds_run": len(hist_r), "open_per_round": [h[2] for h in hist_r],
                                    "seconds": secs_r},
    }
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched / backward / splitting measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--batched-only", type=int, default=0, metavar="CALLS",
                    help="only run the batched call (2000 buses, 18 x 1024 sub-boxes) CALLS times after one "
                         "warm-up call; for profiler runs")
    ap.add_argument("--probes-only", action="store_true",
                    help="only run the read-bandwidth and FMA issue-rate probes; for profiler runs")
    ap.add_argument("--backward-only", type=int, default=0, metavar="CALLS",
                    help="only run the one-sided backward (2000 buses, 4096 sub-boxes, gradient of f_hi) CALLS "
                         "times after one warm-up call, and print its per-kernel times; for profiler runs")
    ap.add_argument("--chord-only", type=int, default=0, metavar="CALLS",
                    help="only run the chord-relaxation lower bound (8316 buses, one whole box; 2000 buses, 1024 "
                         "sub-boxes, lower side only) CALLS times each after one warm-up call, and print the "
                         "relaxation sweep's times; for profiler runs")
    ap.add_argument("--traffic-record", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write the HBM traffic record from four rocprofv3 --pmc output folders (no GPU)")
    args = ap.parse_args(argv)
    if args.traffic_record:
        return write_traffic_record(*args.traffic_record)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(boxes would be split across GPUs with the factors replicated). Run with --gpus 1.",
              file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.calibrate_copy:
        # 1 GiB read + 1 GiB written per copy: divides the profiler's FETCH_SIZE /
        # WRITE_SIZE readings into bytes
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "copies": 5}), flush=True)
        return 0
    from paper_2511_15624_amd import ibp, synth
    if args.batched_only:
        net3 = synth.make_config("c2000")
        n3 = ibp.Network(net3, device=0)
        lo3, hi3, _ = synth.period_boxes(net3, 18, 1024, seed=31)
        tlo3, thi3 = torch.from_numpy(lo3).cuda(), torch.from_numpy(hi3).cuda()
        ws3 = ibp.Workspace(n3)
        ibp.ibp_bound_boxes(n3, tlo3, thi3, ws=ws3)
        ms3 = _time(torch, lambda: ibp.ibp_bound_boxes(n3, tlo3, thi3, ws=ws3), args.batched_only)
        print(json.dumps({"workload": "2000 buses, 18 x 1024 sub-boxes", "calls": args.batched_only,
                          "ms_per_call": ms3}), flush=True)
        return 0

    if args.probes_only:
        print(json.dumps({"hbm_probe": hbm_probe(torch, ibp), "alu_probe": alu_probe(torch, ibp)}), flush=True)
        return 0

    if args.chord_only:
        res = {}
        for name, nb in (("c8316", 0), ("c2000", 1024)):
            netc = synth.make_config(name)
            nc = ibp.Network(netc, device=0)
            if nb:
                lo_, hi_ = synth.sub_boxes(netc, nb, seed=61)
            else:
                lo_, hi_ = (a[None].copy() for a in synth.full_box(netc))
            tl, th = torch.from_numpy(lo_).cuda(), torch.from_numpy(hi_).cuda()
            wsc = ibp.Workspace(nc)
            fl = ibp.IBP_F_LOWER_ONLY if nb else 0
            call = lambda: ibp.ibp_crown_lower_boxes(nc, tl, th, ws=wsc, flags=fl)  # noqa: E731
            call()
            nc.set_kernel_timing(True)
            nc.kernel_times()
            for _ in range(args.chord_only):
                call()
            kt = nc.kernel_times()
            nc.set_kernel_timing(False)
            res[name] = {k: v[0] / args.chord_only for k, v in kt.items()}  # per call
            nc.close()
        print(json.dumps({"workload": "chord relaxation: 8316 buses one whole box; 2000 buses 1024 sub-boxes",
                          "calls": args.chord_only, "kernel_ms": res}), flush=True)
        return 0

    if args.backward_only:
        net3 = synth.make_config("c2000")
        n3 = ibp.Network(net3, device=0)
        blo, bhi = synth.sub_boxes(net3, 4096, seed=51)
        t5l, t5h = torch.from_numpy(blo).cuda(), torch.from_numpy(bhi).cuda()
        g1 = torch.ones(4096, dtype=torch.float64, device="cuda")
        wsb = ibp.Workspace(n3)
        call = lambda: ibp.ibp_bound_backward(n3, t5l, t5h, None, g1, ws=wsb, flags=ibp.IBP_F_UPPER_ONLY)  # noqa: E731
        call()
        ms = _time(torch, call, args.backward_only)
        n3.set_kernel_timing(True)
        n3.kernel_times()
        for _ in range(args.backward_only):
            call()
        kt = n3.kernel_times()
        print(json.dumps({"workload": "2000 buses, 4096 sub-boxes, backward of f_hi", "calls": args.backward_only,
                          "ms_per_call": ms, "kernel_ms": {k: v[0] / v[1] for k, v in kt.items()}}), flush=True)
        return 0

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

    # outputs and workspace allocated once; each step is one C-ABI call
    # (ibp_bound_boxes) on the current stream, so host-side Python work does
    # not pace the device
    f_lo = torch.empty(B, dtype=torch.float64, device="cuda")
    f_hi = torch.empty(B, dtype=torch.float64, device="cuda")
    buf, _ = ws.get(B)
    lib = ibp.load_library()
    import ctypes
    cargs = (n.handle, B, ctypes.c_void_p(tlo.data_ptr()), ctypes.c_void_p(thi.data_ptr()),
             ctypes.c_void_p(f_lo.data_ptr()), ctypes.c_void_p(f_hi.data_ptr()), ctypes.c_void_p(),
             ctypes.c_void_p(buf.data_ptr()), buf.numel(), ctypes.c_void_p(stream.cuda_stream), 0)
    call = lib.ibp_bound_boxes
    for _ in range(args.warmup):
        ibp._check(call(*cargs))
    torch.cuda.synchronize()

    # timed region: K steps between events on the launch stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    status = [call(*cargs) for _ in range(args.steps)]
    e1.record(stream)
    torch.cuda.synchronize()
    if any(status):
        ibp._check(next(st for st in status if st))
    ms_total = e0.elapsed_time(e1)
    # kernel pass: the same steps again with the library timing every kernel it
    # queues on this stream (HIP events recorded by the dispatches of the
    # single-box kernels themselves; the step time above is taken without them)
    n.set_kernel_timing(True)
    _ = n.kernel_times()
    for _ in range(args.steps):
        ibp._check(call(*cargs))
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
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
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
    probe = hbm_probe(torch, ibp)
    out["hbm_probe"] = probe
    out["alu_probe"] = alu_probe(torch, ibp)
    # every ALU roofline also against the probe's measured FMA rate
    rate = out["alu_probe"]["fma_vector_operands_ops_per_s"]

    def _frac_of_probe(d):
        if isinstance(d, dict):
            if d.get("bound") == "alu":
                for sub in [d] + [v for v in d.values() if isinstance(v, dict) and "achieved" in v]:
                    if "achieved" in sub:
                        sub["frac_of_alu_probe"] = round(sub["achieved"] / rate, 4)
            for v in d.values():
                _frac_of_probe(v)

    roof["frac_of_read_probe"] = round(achieved / probe["read_gbs"], 4)
    out["step_roofline"]["frac_of_read_probe"] = round(step_gbs / probe["read_gbs"], 4)
    if not args.no_extras:
        out.update(extras(torch, ibp, synth, n, net))
    _frac_of_probe(out)
    out["paper_context"] = {
        "figure": "mean IBP runtime per time index reaching 23.8 s on the largest instance (8316 buses, 11972 "
                  "lines, 6289 N-1 outages), alpha,beta-CROWN on an NVIDIA H200, graph construction included; "
                  "about 6289 x 11972 / 23.8 = 3.2e6 outage x line evaluations/s (derived, not printed)",
        "source": "Sec. IV-B, Fig. 3; sizes in Table I",
        "note": "context only: other hardware, software, instances and precision",
    }
    if not args.no_cpu_baseline:
        r, t_cpu, t_build, fac4, runs = cpu_baseline(net, lo, hi)
        hinfo = host_info()
        out["cpu_baseline"] = {"value": evals / t_cpu, "unit": "evals/s", "cores": hinfo["blas_threads"],
                               "kind": "oracle",
                               "sample": f"the full single box ({K} outages x {L} lines), FP64 "
                                         f"numpy; {t_cpu:.2f} s per box, mean of {runs} runs; factor construction "
                                         f"{t_build:.1f} s not timed; matrix products on the BLAS threads "
                                         f"(cores), elementwise stages single-threaded",
                               "host": hinfo}
        if not args.no_extras:
            ev3, t3, fac3 = cpu_batched_sample(synth)
            n_b3 = out["batched"]["ms_per_call"]
            out["cpu_baseline"]["batched_sample"] = {
                "value": ev3 / t3, "unit": "evals/s", "seconds_per_box": t3,
                "sample": "4 seeded boxes of the 2000-bus 18 x 1024 period set, FP64 numpy, per box; the "
                          "18432-box call extrapolates to " + f"{t3 * 18432:.0f} s on the host against "
                          f"{n_b3:.1f} ms on the GPU"}
        den_lo = max(abs(r["f_lo"]), 1.0)
        den_hi = max(abs(r["f_hi"]), 1.0)
        out["bound_gap_vs_fp64"] = {
            "encloses": bool(g_lo <= r["f_lo"] and g_hi >= r["f_hi"]),
            "lo_rel": (r["f_lo"] - g_lo) / den_lo,
            "hi_rel": (g_hi - r["f_hi"]) / den_hi,
            "gpu": [g_lo, g_hi], "oracle": [r["f_lo"], r["f_hi"]],
        }
        if not args.no_extras:
            net3 = synth.make_config("c2000")
            n3 = ibp.Network(net3, device=0)
            out["bound_gap_vs_fp64"]["sub_boxes"] = sub_box_gaps(torch, ibp, synth, n3, net3, fac3, n, net, fac4)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
