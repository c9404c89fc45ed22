"""The host side of the C ABI under AddressSanitizer, UndefinedBehaviorSanitizer
and LeakSanitizer (no GPU): the library is rebuilt with the sanitizers on its
host code (device code as usual), and two plain C programs drive it --
tests/c_abi/three_bus.c in host mode and tests/c_abi/host_errors.c, which
builds generated networks host-only (with and without outage lists and curves)
and runs every argument and network error the host detects.  Any sanitizer
report fails the run; the printed statuses are checked against the header's
error contract."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2511_15624_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = "/opt/rocm"
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
SAN = ["address", "undefined"]

OK, INVALID, DISCONNECTED, ISLANDING, HOST_ONLY = 0, 1, 2, 3, 8


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-2000:] + r.stderr[-4000:]
    return r


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("ROCm clang is not available")
    out = tmp_path_factory.mktemp("asan")
    hipcc = build._hipcc()
    host_san = []
    for s in SAN:  # sanitizers on the host pass only
        host_san += ["-Xarch_host", f"-fsanitize={s}"]
    host_san += ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
    jobs, objs = [], []
    for src in build.HIP_SOURCES:
        obj = str(out / (src + ".o"))
        objs.append(obj)
        jobs.append([hipcc, *build.hip_flags(), *host_san, "-c", os.path.join(build.CSRC, src), "-o", obj])
    for src in build.HOST_SOURCES:
        obj = str(out / (src + ".o"))
        objs.append(obj)
        jobs.append([CLANG + "++", "-O1", "-g", "-std=c++17", "-fPIC", "-mavx2", "-mfma", "-pthread",
                     "-fsanitize=" + ",".join(SAN), "-fno-omit-frame-pointer",
                     "-c", os.path.join(build.CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(_run, jobs))
    lib = str(out / "libibp_san.so")
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={build.ARCH}", "-pthread", *host_san, "-o", lib, *objs])
    exes = {}
    for prog in ("three_bus", "host_errors"):
        exe = str(out / prog)
        _run([CLANG, "-std=c99", "-Wall", "-Wextra", "-Werror", "-g", "-fsanitize=" + ",".join(SAN),
              "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
              "-I", os.path.join(ROCM, "include"), os.path.join(ROOT, "tests", "c_abi", prog + ".c"),
              "-o", exe, lib, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
              f"-Wl,-rpath,{out}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"])
        exes[prog] = exe
    return exes


def _san_env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=24"
    env["HIP_VISIBLE_DEVICES"] = ""
    return env


def _statuses(stdout):
    vals = {}
    for line in stdout.splitlines():
        key, *rest = line.split()
        vals.setdefault(key, []).append(rest)
    return vals


def test_three_bus_host_mode_is_clean(sanitized):
    r = subprocess.run([sanitized["three_bus"], "host"], capture_output=True, text=True, timeout=300,
                       env=_san_env())
    assert r.returncode == 0, r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr, r.stderr[-4000:]
    v = _statuses(r.stdout)
    assert v["n_bus"] == [["3"]] and v["host_compute_status"] == [[str(HOST_ONLY)]]


def test_host_errors_are_reported_and_clean(sanitized):
    r = subprocess.run([sanitized["host_errors"]], capture_output=True, text=True, timeout=600, env=_san_env())
    assert r.returncode == 0, r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    v = _statuses(r.stdout)
    first = {k: int(x[0][0]) for k, x in v.items() if len(x[0]) == 1 and x[0][0].lstrip("-").isdigit()}
    # four valid host-only builds, each with its queries
    assert [int(x[0]) for x in v["valid_build"]] == [OK] * 4
    assert [x for x in v["sizes"]] == [["150", "171", "86", "80"], ["150", "171", "171", "80"],
                                       ["150", "171", "86", "80"], ["150", "171", "0", "80"]]
    for key in ("query", "export", "ctg_lines", "tile_get"):
        assert [int(x[0]) for x in v[key]] == [OK] * 4, key
    for key in ("host_bound", "host_noalloc", "host_backward", "host_timing", "host_autotune"):
        assert [int(x[0]) for x in v[key]] == [HOST_ONLY] * 4, key
    assert [int(x[0]) for x in v["tile_bad"]] == [INVALID] * 4
    assert [int(x[0]) for x in v["host_workspace"]] == [0] * 4
    for key in ("null_desc", "null_out", "bad_device", "bus_out_of_range", "self_loop", "zero_susceptance",
                "negative_zeta", "bad_slack", "bad_gen_bus", "bad_ctg_index", "query_null", "export_null",
                "tile_null", "split_bad", "split_null", "probe_null"):
        assert first[key] == INVALID, (key, first[key])
    assert first["islanding_outage"] == ISLANDING
    assert first["disconnected"] == DISCONNECTED
    assert first["split_empty"] == OK
    assert first["last_error_nonempty"] == 1
    assert first["workspace_null"] == 0
