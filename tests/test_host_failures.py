"""Host failure paths of the C ABI (no GPU): a construction that runs out of
memory returns IBP_E_OUT_OF_MEMORY with a message, leaks nothing, and leaves
the library usable; no C++ exception crosses the boundary.

The failure is real, not simulated: a child process caps its own address
space (RLIMIT_AS) a few tens of MB above what it already maps, then builds the
2000-bus network host-only, whose dense factors need about 160 MB.  Under the
cap, allocations of the factors fail and so do thread starts (each reserves
its stack), which exercises the builder's worker pool too.  Repeated failed
builds must not grow the process (no leak), and a build after the cap is
lifted must give the same factors as one before it."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import json, os, resource, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_2511_15624_amd import ibp, synth

_libc = __import__("ctypes").CDLL("libc.so.6")


def status():
    # freed heap memory goes back to the system first (glibc keeps it otherwise)
    _libc.malloc_trim(0)
    out = {}
    with open("/proc/self/status") as f:
        for line in f:
            k, _, v = line.partition(":")
            if k in ("VmSize", "VmRSS"):
                out[k] = int(v.split()[0]) * 1024
    return out

def ptdf(h):
    p, _ = h.export()
    h.close()
    return p

net = synth.make_config("c2000")
ibp.load_library()
ref = ptdf(ibp.Network(net, device=ibp.IBP_DEVICE_HOST_ONLY))
soft, hard = resource.getrlimit(resource.RLIMIT_AS)
res = {"margins": {}}
for margin_mb in (8, 48, 120, 160, 512):
    before = status()
    resource.setrlimit(resource.RLIMIT_AS, (before["VmSize"] + (margin_mb << 20), hard))
    codes = []
    for i in range(8):
        if i == 2:
            warm = status()
        try:
            ibp.Network(net, device=ibp.IBP_DEVICE_HOST_ONLY).close()
            codes.append("IBP_OK")
        except ibp.IBPError as e:
            codes.append(e.name)
            res.setdefault("message", str(e))
    after = status()
    resource.setrlimit(resource.RLIMIT_AS, (soft, hard))
    before = warm
    res["margins"][margin_mb] = {"codes": codes, "rss_growth": after["VmRSS"] - before["VmRSS"],
                                 "vm_growth": after["VmSize"] - before["VmSize"]}
res["same_after"] = bool(np.array_equal(ptdf(ibp.Network(net, device=ibp.IBP_DEVICE_HOST_ONLY)), ref))
print(json.dumps(res))
'''


@pytest.mark.parametrize("threads", ["1", "8"])
def test_out_of_memory_during_construction(threads):
    # one malloc arena: worker threads would otherwise map 64 MB arenas of
    # address space (not memory) whenever they start, which would read as growth
    env = dict(os.environ, IBP_HOST_THREADS=threads, MALLOC_ARENA_MAX="1")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    codes = [c for m in res["margins"].values() for c in m["codes"]]
    assert set(codes) <= {"IBP_OK", "IBP_E_OUT_OF_MEMORY"}, codes
    # the tightest cap fails every build, the loosest lets every one through
    assert set(res["margins"]["8"]["codes"]) == {"IBP_E_OUT_OF_MEMORY"}, res
    assert set(res["margins"]["512"]["codes"]) == {"IBP_OK"}, res
    assert "alloc" in res["message"] or "resource" in res["message"], res["message"]
    for margin, m in res["margins"].items():
        # after two warm-up attempts, six more failed (or successful) builds
        # leave the resident size as it was (a leaked factor matrix would add
        # tens of MB per build; the address space may keep freed heap pages)
        assert m["rss_growth"] < (16 << 20) and m["vm_growth"] < (64 << 20), (margin, m)
    assert res["same_after"]
