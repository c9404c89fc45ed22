"""The C ABI used from a plain C99 program (tests/c_abi/three_bus.c), with no
C++ and no Python between the caller and libibp.so: include/ibp.h compiles as
C99 with warnings as errors, and the program's results for the hand-derived
3-bus triangle match tests/golden/three_bus.json (factors exact to 1e-12; the
GPU bounds enclose the exact IBP interval within the 1e-5 bar).  The device
run is a child process of the test."""
import json
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2511_15624_amd")
ROCM = "/opt/rocm"


def _golden():
    with open(os.path.join(ROOT, "tests", "golden", "three_bus.json")) as f:
        g = json.load(f)

    def num(x):
        return np.array([[float(Fraction(v)) for v in row] for row in x]) if isinstance(x[0], list) \
            else np.array([float(Fraction(v)) for v in x])
    return g, num


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    if not os.path.exists(os.path.join(LIBDIR, "libibp.so")):
        pytest.fail("libibp.so is missing: build it first")
    out = str(tmp_path_factory.mktemp("c_abi") / "three_bus")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c_abi", "three_bus.c"), "-o", out,
           "-L", LIBDIR, "-l:libibp.so", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def _run(exe, mode):
    r = subprocess.run([exe, mode], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    vals = {}
    for line in r.stdout.splitlines():
        key, *rest = line.split()
        vals.setdefault(key, []).append([float(x) for x in rest])
    return vals


def test_header_is_c99_and_host_path_matches_the_fixture(exe):
    g, num = _golden()
    v = _run(exe, "host")
    assert v["n_bus"] == [[3.0]] and v["n_line"] == [[3.0]] and v["n_ctg"] == [[3.0]] and v["n_input"] == [[2.0]]
    assert [int(c[1]) for c in v["ctg"]] == g["ctg_line"]
    ptdf = np.zeros((3, 3))
    for i, j, x in v["ptdf"]:
        ptdf[int(i), int(j)] = x
    assert np.allclose(ptdf, num(g["ptdf"]), rtol=0, atol=1e-12)
    lodf = np.zeros((3, 3))
    for k, l, x in v["lodf"]:
        lodf[int(k), int(l)] = x
    # row k of the export is the distribution column of outage k
    assert np.allclose(lodf, num(g["lodf_columns"]), rtol=0, atol=1e-12)
    assert v["host_compute_status"] == [[8.0]]          # IBP_E_HOST_ONLY


@pytest.mark.gpu
def test_device_path_encloses_the_fixture(exe):
    g, num = _golden()
    v = _run(exe, "device")
    f_lo, f_hi = v["f_lo"][0][0], v["f_hi"][0][0]
    e_lo, e_hi = num(g["f"])
    S, I, Fb, Fc = num(g["S"]), num(g["I"]), num(g["Fb"]), num(g["Fc"])
    zi, zf = g["network"]["zeta_inj"], g["network"]["zeta_f"]
    scale_lo = max(abs(e_lo), abs(S[0]) + zi * I[1] + zf * (Fb[1] + Fc[1]), 1.0)
    scale_hi = max(abs(e_hi), abs(S[1]) + zi * I[0] + zf * (Fb[0] + Fc[0]), 1.0)
    assert f_lo <= e_lo and (e_lo - f_lo) / scale_lo <= 1e-5
    assert f_hi >= e_hi and (f_hi - e_hi) / scale_hi <= 1e-5
    # the lower-bound call: IBP's f_hi, and an f_lo between IBP's and the true
    # minimum (f is concave in the one free input, so the minimum is at an end)
    c_lo, c_hi = v["chord_f_lo"][0][0], v["chord_f_hi"][0][0]
    net = dict(g["network"], line_from=np.array(g["network"]["line_from"], np.int32),
               line_to=np.array(g["network"]["line_to"], np.int32))
    for k in ("line_b", "fmax_base", "fmax_ctg", "gen_cost", "load_value", "gen_pmin", "gen_pmax",
              "load_dmin", "load_dmax"):
        net[k] = np.array(net[k], float)
    net["gen_bus"] = np.array(net["gen_bus"], np.int32)
    net["load_bus"] = np.array(net["load_bus"], np.int32)
    fac = oracle.factors(net)
    ends = oracle.point_eval_many(net, np.array([g["box_lo"], g["box_hi"]], float), fac["ctg"])
    assert c_hi == f_hi
    assert f_lo <= c_lo <= ends.min()
    assert v["short_workspace_status"] == [[7.0]]       # IBP_E_WORKSPACE
