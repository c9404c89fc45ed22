"""Thin ctypes binding of libibp (include/ibp.h): argument marshalling only.

Every step of the bound computation runs in the HIP library; PyTorch is used
for device memory (tensors whose pointers are handed to the library) and for
the stream the kernels are queued on.  There is no fallback: if the library
is missing the calls raise.

Python names mirror the C entry points: ``ibp_build_network``,
``ibp_bound_boxes``, ``ibp_bound_backward``.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibp.so")

IBP_DEVICE_HOST_ONLY = -1
IBP_F_NONE = 0
IBP_F_PLAIN = 1
IBP_F_AUTOTUNE = 2
IBP_F_BACKWARD = 4
IBP_F_CROWN = 8
IBP_F_CROWN_REF = 16
IBP_F_UPPER_ONLY = 32   # only f_hi is needed (f_lo = -inf)
IBP_F_LOWER_ONLY = 64   # only f_lo is needed (f_hi valid but looser)
IBP_F_KEEP_PREP = 128   # forward: leave the intermediates for a backward on the same boxes
IBP_F_REUSE_PREP = 256  # backward: take them instead of recomputing
IBP_F_SCREEN_UPPER = 512  # calls bounding f_lo: screen the upper penalties (narrow boxes, points)

STATUS = {
    0: "IBP_OK",
    1: "IBP_E_INVALID_ARG",
    2: "IBP_E_DISCONNECTED",
    3: "IBP_E_ISLANDING_CTG",
    4: "IBP_E_ILL_CONDITIONED",
    5: "IBP_E_OUT_OF_MEMORY",
    6: "IBP_E_DEVICE",
    7: "IBP_E_WORKSPACE",
    8: "IBP_E_HOST_ONLY",
}

EXPORTED = [
    "ibp_build_network",
    "ibp_network_query",
    "ibp_network_ctg_lines",
    "ibp_network_export",
    "ibp_free_network",
    "ibp_workspace_bytes",
    "ibp_bound_boxes",
    "ibp_bound_boxes_noalloc",
    "ibp_backward_screen_lines",
    "ibp_bound_backward",
    "ibp_crown_bound_boxes",
    "ibp_crown_lower_boxes",
    "ibp_set_kernel_timing",
    "ibp_kernel_times",
    "ibp_set_tile",
    "ibp_autotune",
    "ibp_set_tile_batched",
    "ibp_get_tile",
    "ibp_set_screen_upper",
    "ibp_get_screen_upper",
    "ibp_autotune_batched",
    "ibp_split_select",
    "ibp_split_bisect",
    "ibp_split_update",
    "ibp_split_screen",
    "ibp_read_probe",
    "ibp_alu_probe",
    "ibp_last_error",
]

KERNEL_IDS = ["box_prep", "base_flows", "outage_sweep", "finalize", "line_epilogue", "batched_base_flows",
              "batched_outage_sweep", "backward_outage_sweep", "backward_ptdf_t", "backward_endpoints",
              "crown_outage_sweep", "crown_ptdf_t", "crown_inputs", "backward_line_terms",
              "backward_line_screen", "forward_line_screen"]


TILE_FIELDS = ("k2_nc", "k3_kc", "k3_bt", "k3_rows", "k3_xcd", "k2_mfma", "k2_by")


class IBPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class NetworkDesc(ctypes.Structure):
    _fields_ = [
        ("n_bus", ctypes.c_int32),
        ("n_line", ctypes.c_int32),
        ("slack_bus", ctypes.c_int32),
        ("line_from", ctypes.POINTER(ctypes.c_int32)),
        ("line_to", ctypes.POINTER(ctypes.c_int32)),
        ("line_b", ctypes.POINTER(ctypes.c_double)),
        ("fmax_base", ctypes.POINTER(ctypes.c_double)),
        ("fmax_ctg", ctypes.POINTER(ctypes.c_double)),
        ("n_gen", ctypes.c_int32),
        ("gen_bus", ctypes.POINTER(ctypes.c_int32)),
        ("gen_cost", ctypes.POINTER(ctypes.c_double)),
        ("n_load", ctypes.c_int32),
        ("load_bus", ctypes.POINTER(ctypes.c_int32)),
        ("load_value", ctypes.POINTER(ctypes.c_double)),
        ("zeta_inj", ctypes.c_double),
        ("zeta_f", ctypes.c_double),
        ("n_ctg", ctypes.c_int32),
        ("ctg_line", ctypes.POINTER(ctypes.c_int32)),
        ("seg_ptr", ctypes.POINTER(ctypes.c_int32)),
        ("seg_a", ctypes.POINTER(ctypes.c_double)),
        ("seg_b", ctypes.POINTER(ctypes.c_double)),
        ("seg_U", ctypes.POINTER(ctypes.c_double)),
    ]


class NetworkInfo(ctypes.Structure):
    _fields_ = [
        ("n_bus", ctypes.c_int32),
        ("n_line", ctypes.c_int32),
        ("n_ctg", ctypes.c_int32),
        ("n_gen", ctypes.c_int32),
        ("n_load", ctypes.c_int32),
        ("n_input", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("min_one_minus_hcc", ctypes.c_double),
        ("phi_abs_err", ctypes.c_double),
        ("device_bytes", ctypes.c_size_t),
        ("build_seconds", ctypes.c_double),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libibp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: run `python -m paper_2511_15624_amd.build`")
    # PyTorch ships its own HIP runtime with the same soname as the system one;
    # whichever is loaded first serves the whole process.  Load torch's first so
    # that the tensors handed to the library and its kernels share one runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, sz, i64, u32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_uint32
    i32 = ctypes.c_int32
    lib.ibp_build_network.argtypes = [ctypes.POINTER(NetworkDesc), ctypes.c_int, ctypes.POINTER(vp)]
    lib.ibp_build_network.restype = ctypes.c_int
    lib.ibp_network_query.argtypes = [vp, ctypes.POINTER(NetworkInfo)]
    lib.ibp_network_query.restype = ctypes.c_int
    lib.ibp_network_ctg_lines.argtypes = [vp, vp]
    lib.ibp_network_ctg_lines.restype = ctypes.c_int
    lib.ibp_network_export.argtypes = [vp, vp, vp]
    lib.ibp_network_export.restype = ctypes.c_int
    lib.ibp_free_network.argtypes = [vp]
    lib.ibp_free_network.restype = None
    lib.ibp_workspace_bytes.argtypes = [vp, i64, u32]
    lib.ibp_workspace_bytes.restype = sz
    lib.ibp_bound_boxes.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, sz, vp, u32]
    lib.ibp_bound_boxes.restype = ctypes.c_int
    lib.ibp_bound_boxes_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, u32]
    lib.ibp_bound_boxes_noalloc.restype = ctypes.c_int
    lib.ibp_bound_backward.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp, u32]
    lib.ibp_bound_backward.restype = ctypes.c_int
    lib.ibp_backward_screen_lines.argtypes = [vp, i64, vp, sz, vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.ibp_backward_screen_lines.restype = ctypes.c_int
    lib.ibp_crown_bound_boxes.argtypes = [vp, i64, vp, vp, i32, vp, vp, vp, vp, vp, sz, vp, u32]
    lib.ibp_crown_bound_boxes.restype = ctypes.c_int
    lib.ibp_crown_lower_boxes.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp, u32]
    lib.ibp_crown_lower_boxes.restype = ctypes.c_int
    lib.ibp_set_kernel_timing.argtypes = [vp, ctypes.c_int]
    lib.ibp_set_kernel_timing.restype = ctypes.c_int
    lib.ibp_kernel_times.argtypes = [vp, ctypes.c_int32, vp, vp]
    lib.ibp_kernel_times.restype = ctypes.c_int
    lib.ibp_set_tile.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    lib.ibp_set_tile.restype = ctypes.c_int
    lib.ibp_autotune.argtypes = [vp, i64, vp, vp, vp, sz, vp, vp]
    lib.ibp_autotune.restype = ctypes.c_int
    lib.ibp_set_tile_batched.argtypes = [vp, i32, i32, i32, i32, i32]
    lib.ibp_set_tile_batched.restype = ctypes.c_int
    lib.ibp_get_tile.argtypes = [vp, vp]
    lib.ibp_get_tile.restype = ctypes.c_int
    lib.ibp_set_screen_upper.argtypes = [vp, i32]
    lib.ibp_set_screen_upper.restype = ctypes.c_int
    lib.ibp_get_screen_upper.argtypes = [vp, vp]
    lib.ibp_get_screen_upper.restype = ctypes.c_int
    lib.ibp_autotune_batched.argtypes = [vp, i64, vp, vp, vp, sz, vp, vp]
    lib.ibp_autotune_batched.restype = ctypes.c_int
    lib.ibp_split_select.argtypes = [i64, vp, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.ibp_split_select.restype = ctypes.c_int
    lib.ibp_split_bisect.argtypes = [i64, vp, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.ibp_split_bisect.restype = ctypes.c_int
    lib.ibp_split_update.argtypes = [i64, vp, i32, vp, vp, vp, i32, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.ibp_split_update.restype = ctypes.c_int
    lib.ibp_split_screen.argtypes = [i64, vp, vp, ctypes.c_double, vp, vp, vp, vp]
    lib.ibp_split_screen.restype = ctypes.c_int
    lib.ibp_read_probe.argtypes = [vp, i64, vp, vp]
    lib.ibp_read_probe.restype = ctypes.c_int
    lib.ibp_alu_probe.argtypes = [vp, i64, i32, vp]
    lib.ibp_alu_probe.restype = ctypes.c_int
    lib.ibp_last_error.argtypes = []
    lib.ibp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise IBPError(status, load_library().ibp_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Network:
    """Owns an ``ibp_network*``.  ``net`` is a dict of numpy arrays (see synth)."""

    def __init__(self, net: dict, device: int = 0):
        lib = load_library()
        self._keep = {}

        def arr(key, dtype):
            a = np.ascontiguousarray(np.asarray(net[key]), dtype=dtype)
            self._keep[key] = a
            return a

        lf, lt = arr("line_from", np.int32), arr("line_to", np.int32)
        lb = arr("line_b", np.float64)
        fb, fc = arr("fmax_base", np.float64), arr("fmax_ctg", np.float64)
        gb, gc = arr("gen_bus", np.int32), arr("gen_cost", np.float64)
        db, dv = arr("load_bus", np.int32), arr("load_value", np.float64)
        d = NetworkDesc()
        d.n_bus = int(net["n_bus"])
        d.n_line = lf.size
        d.slack_bus = int(net["slack_bus"])
        d.line_from, d.line_to = _ptr(lf, ctypes.c_int32), _ptr(lt, ctypes.c_int32)
        d.line_b = _ptr(lb, ctypes.c_double)
        d.fmax_base, d.fmax_ctg = _ptr(fb, ctypes.c_double), _ptr(fc, ctypes.c_double)
        d.n_gen, d.gen_bus, d.gen_cost = gb.size, _ptr(gb, ctypes.c_int32), _ptr(gc, ctypes.c_double)
        d.n_load, d.load_bus, d.load_value = db.size, _ptr(db, ctypes.c_int32), _ptr(dv, ctypes.c_double)
        d.zeta_inj = float(net["zeta_inj"])
        d.zeta_f = float(net["zeta_f"])
        if net.get("ctg_line") is not None:
            cl = arr("ctg_line", np.int32)
            d.n_ctg = cl.size
            d.ctg_line = _ptr(cl, ctypes.c_int32)
        else:
            d.n_ctg = 0
            d.ctg_line = ctypes.POINTER(ctypes.c_int32)()
        if net.get("seg_ptr") is not None:
            # piecewise-linear curves: the C side cannot see array lengths
            sp_ = arr("seg_ptr", np.int32)
            sa, sb, su = arr("seg_a", np.float64), arr("seg_b", np.float64), arr("seg_U", np.float64)
            if sp_.size != gb.size + db.size + 1 or not (sa.size == sb.size == su.size == int(sp_[-1])):
                raise IBPError(1, "seg_ptr needs G + D + 1 entries and seg_a/b/U seg_ptr[-1] each")
            d.seg_ptr = _ptr(sp_, ctypes.c_int32)
            d.seg_a, d.seg_b, d.seg_U = (_ptr(a, ctypes.c_double) for a in (sa, sb, su))
        h = ctypes.c_void_p()
        _check(lib.ibp_build_network(ctypes.byref(d), int(device), ctypes.byref(h)))
        self._h = h
        self._keep = None
        info = NetworkInfo()
        _check(lib.ibp_network_query(h, ctypes.byref(info)))
        self.info = info
        self.n_bus, self.n_line, self.n_ctg = info.n_bus, info.n_line, info.n_ctg
        self.n_gen, self.n_load, self.n_input = info.n_gen, info.n_load, info.n_input
        self.device = info.device

    @property
    def handle(self):
        return self._h

    def ctg_lines(self) -> np.ndarray:
        out = np.zeros(self.n_ctg, np.int32)
        _check(load_library().ibp_network_ctg_lines(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def export(self):
        ptdf = np.zeros((self.n_line, self.n_bus))
        lodf = np.zeros((self.n_ctg, self.n_line))
        _check(load_library().ibp_network_export(self._h, ptdf.ctypes.data_as(ctypes.c_void_p),
                                                 lodf.ctypes.data_as(ctypes.c_void_p)))
        return ptdf, lodf

    def workspace_bytes(self, n_box: int, flags: int = 0) -> int:
        return int(load_library().ibp_workspace_bytes(self._h, int(n_box), int(flags)))

    def set_kernel_timing(self, enable: bool):
        _check(load_library().ibp_set_kernel_timing(self._h, int(bool(enable))))

    def kernel_times(self) -> dict:
        """{kernel name: (total_ms, launches)} since the last read."""
        n = len(KERNEL_IDS)
        ms = np.zeros(n)
        cnt = np.zeros(n, np.int64)
        _check(load_library().ibp_kernel_times(self._h, n, ms.ctypes.data_as(ctypes.c_void_p),
                                               cnt.ctypes.data_as(ctypes.c_void_p)))
        return {KERNEL_IDS[i]: (float(ms[i]), int(cnt[i])) for i in range(n) if cnt[i] > 0}

    def set_tile(self, k2_nc: int, k3_kc: int):
        _check(load_library().ibp_set_tile(self._h, int(k2_nc), int(k3_kc)))

    def set_tile_batched(self, k3_bt: int, k3_rows: int, k3_xcd: int, k2_mfma: int, k2_by: int):
        _check(load_library().ibp_set_tile_batched(self._h, int(k3_bt), int(k3_rows), int(k3_xcd), int(k2_mfma),
                                                   int(k2_by)))

    def tiles(self) -> dict:
        out = np.zeros(7, np.int32)
        _check(load_library().ibp_get_tile(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        t = dict(zip(TILE_FIELDS, (int(v) for v in out)))
        t["screen_upper"] = int(self.screen_upper())
        return t

    def set_screen_upper(self, on: bool):
        _check(load_library().ibp_set_screen_upper(self._h, int(bool(on))))

    def screen_upper(self) -> bool:
        out = ctypes.c_int32(0)
        _check(load_library().ibp_get_screen_upper(self._h, ctypes.byref(out)))
        return bool(out.value)

    def close(self):
        if getattr(self, "_h", None):
            load_library().ibp_free_network(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ibp_build_network(net: dict, device: int = 0) -> Network:
    return Network(net, device)


# ---------------------------------------------------------------- torch helpers

def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _on(stream):
    """Makes `stream` current for the allocations and the call: memory the
    call's kernels use then belongs to the stream they run on, so the caching
    allocator cannot hand it out while they still run."""
    return contextlib.nullcontext() if stream is None else _torch().cuda.stream(stream)


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()


class Workspace:
    """Grow-only device workspace (a uint8 tensor) for one network."""

    def __init__(self, net: Network):
        self.net = net
        self.buf = None

    def get(self, n_box: int, flags: int = 0):
        """The buffer (grown to the call's size) for a call on the current stream."""
        torch = _torch()
        need = self.net.workspace_bytes(n_box, flags)
        if self.buf is None or self.buf.numel() < need:
            self.buf = torch.empty(max(need, 256), dtype=torch.uint8, device=f"cuda:{self.net.device}")
        else:
            # used on this stream too: a later free must wait for its work
            self.buf.record_stream(torch.cuda.current_stream(self.buf.device))
        return self.buf, need


def _check_boxes(net: Network, lo, hi):
    torch = _torch()
    if lo.dtype != torch.float32 or hi.dtype != torch.float32:
        raise TypeError("box endpoints must be float32")
    if lo.shape != hi.shape or lo.dim() != 2 or lo.shape[1] != net.n_input:
        raise ValueError(f"boxes must be [n_box, {net.n_input}]")
    if not (lo.is_cuda and hi.is_cuda):
        raise ValueError("boxes must be device tensors")
    return lo.contiguous(), hi.contiguous()


def ibp_bound_boxes(net: Network, lo, hi, terms: bool = False, flags: int = 0, ws: Workspace = None,
                    stream=None):
    """Bounds [f_lo, f_hi] (float64 device tensors) for float32 device boxes [n_box, X].

    ``stream``: the kernels run there (default: the current stream); outputs
    and a temporary workspace are then allocated on that stream.  The boxes
    must be ready on it (the caller orders that), and the outputs are ready
    once it has run them."""
    torch = _torch()
    lo, hi = _check_boxes(net, lo, hi)
    n = lo.shape[0]
    with _on(stream):
        f_lo = torch.empty(n, dtype=torch.float64, device=lo.device)
        f_hi = torch.empty(n, dtype=torch.float64, device=lo.device)
        t = torch.empty((n, 8), dtype=torch.float64, device=lo.device) if terms else None
        ws = ws or Workspace(net)
        buf, need = ws.get(n, flags)
        _check(load_library().ibp_bound_boxes(net.handle, n, _dev_ptr(lo), _dev_ptr(hi), _dev_ptr(f_lo),
                                              _dev_ptr(f_hi), _dev_ptr(t), _dev_ptr(buf), buf.numel(),
                                              _stream_ptr(stream), flags))
    return (f_lo, f_hi, t) if terms else (f_lo, f_hi)


IBP_NOALLOC_SCRATCH_BYTES = 32 << 20


def ibp_bound_boxes_noalloc(net: Network, lo, hi, f_lo, f_hi, terms=None, flags: int = 0, stream=None):
    """ibp_bound_boxes on the library's own scratch array: fills the caller's
    float64 device tensors f_lo, f_hi [n_box] (and terms [n_box, 8] if given);
    no workspace is allocated here or in the library."""
    torch = _torch()
    lo, hi = _check_boxes(net, lo, hi)
    n = lo.shape[0]
    for name, t, shape in (("f_lo", f_lo, (n,)), ("f_hi", f_hi, (n,)), ("terms", terms, (n, 8))):
        if t is None and name == "terms":
            continue
        if (t is None or t.dtype != torch.float64 or tuple(t.shape) != shape or not t.is_contiguous()
                or t.device != lo.device):
            raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {shape}")
    _check(load_library().ibp_bound_boxes_noalloc(net.handle, n, _dev_ptr(lo), _dev_ptr(hi), _dev_ptr(f_lo),
                                                  _dev_ptr(f_hi), _dev_ptr(terms), _stream_ptr(stream), flags))


def ibp_bound_backward(net: Network, lo, hi, g_lo, g_hi, flags: int = 0, ws: Workspace = None,
                       stream=None):
    """d(g_lo . f_lo + g_hi . f_hi) / d(lo, hi) as float64 device tensors [n_box, X].
    With flags IBP_F_UPPER_ONLY (IBP_F_LOWER_ONLY) g_lo (g_hi) is not read and may be None."""
    torch = _torch()
    lo, hi = _check_boxes(net, lo, hi)
    n = lo.shape[0]
    if g_lo is None and not flags & IBP_F_UPPER_ONLY or g_hi is None and not flags & IBP_F_LOWER_ONLY:
        raise ValueError("g_lo / g_hi may be None only with the matching one-sided flag")
    with _on(stream):
        g_lo = None if flags & IBP_F_UPPER_ONLY else g_lo.to(device=lo.device, dtype=torch.float64).contiguous()
        g_hi = None if flags & IBP_F_LOWER_ONLY else g_hi.to(device=lo.device, dtype=torch.float64).contiguous()
        d_lo = torch.empty((n, net.n_input), dtype=torch.float64, device=lo.device)
        d_hi = torch.empty((n, net.n_input), dtype=torch.float64, device=lo.device)
        ws = ws or Workspace(net)
        buf, need = ws.get(n, flags | IBP_F_BACKWARD)
        _check(load_library().ibp_bound_backward(net.handle, n, _dev_ptr(lo), _dev_ptr(hi), _dev_ptr(g_lo),
                                                 _dev_ptr(g_hi), _dev_ptr(d_lo), _dev_ptr(d_hi),
                                                 _dev_ptr(buf), buf.numel(), _stream_ptr(stream), flags))
    return d_lo, d_hi


def ibp_backward_screen_lines(net: Network, n_box: int, ws: Workspace, stream=None):
    """(marked, all) (tile, line) pairs of the screened sweep of the last
    IBP_F_UPPER_ONLY backward call on ``ws`` with ``n_box`` boxes."""
    marked, pairs = ctypes.c_int64(0), ctypes.c_int64(0)
    with _on(stream):
        _check(load_library().ibp_backward_screen_lines(net.handle, int(n_box), _dev_ptr(ws.buf), ws.buf.numel(),
                                                        _stream_ptr(stream), ctypes.byref(marked),
                                                        ctypes.byref(pairs)))
    return marked.value, pairs.value


def ibp_crown_bound_boxes(net: Network, lo, hi, crown: bool = False, flags: int = 0, ws: Workspace = None,
                          stream=None, vertex=None, ref_iters: int = 0):
    """IBP bounds with f_hi tightened by the linear relaxation of the penalties:
    (f_lo, f_hi) or, with crown=True, (f_lo, f_hi, smallest relaxation bound).
    ``ref_iters``: further relaxations with slopes taken at reference points.
    ``vertex``: optional float32 device tensor [n_box, X] that receives the box
    vertex maximising the last relaxation's linear part."""
    torch = _torch()
    lo, hi = _check_boxes(net, lo, hi)
    n = lo.shape[0]
    if vertex is not None and (vertex.dtype != torch.float32 or tuple(vertex.shape) != tuple(lo.shape)
                               or not vertex.is_contiguous() or vertex.device != lo.device):
        raise ValueError("vertex must be a contiguous float32 device tensor shaped like the boxes")
    with _on(stream):
        f_lo = torch.empty(n, dtype=torch.float64, device=lo.device)
        f_hi = torch.empty(n, dtype=torch.float64, device=lo.device)
        c = torch.empty(n, dtype=torch.float64, device=lo.device) if crown else None
        ws = ws or Workspace(net)
        buf, need = ws.get(n, flags | IBP_F_CROWN | (IBP_F_CROWN_REF if ref_iters > 0 else 0))
        _check(load_library().ibp_crown_bound_boxes(net.handle, n, _dev_ptr(lo), _dev_ptr(hi), int(ref_iters),
                                                    _dev_ptr(f_lo), _dev_ptr(f_hi), _dev_ptr(c), _dev_ptr(vertex),
                                                    _dev_ptr(buf), buf.numel(), _stream_ptr(stream), flags))
    return (f_lo, f_hi, c) if crown else (f_lo, f_hi)


def ibp_crown_lower_boxes(net: Network, lo, hi, crown: bool = False, flags: int = 0, ws: Workspace = None,
                          stream=None, vertex=None):
    """IBP bounds with f_lo tightened by the chord relaxation of the penalties:
    (f_lo, f_hi) or, with crown=True, (f_lo, f_hi, relaxation bound alone).
    ``vertex``: optional float32 device tensor [n_box, X] that receives the box
    vertex minimising the relaxation's linear part."""
    torch = _torch()
    lo, hi = _check_boxes(net, lo, hi)
    n = lo.shape[0]
    if vertex is not None and (vertex.dtype != torch.float32 or tuple(vertex.shape) != tuple(lo.shape)
                               or not vertex.is_contiguous() or vertex.device != lo.device):
        raise ValueError("vertex must be a contiguous float32 device tensor shaped like the boxes")
    with _on(stream):
        f_lo = torch.empty(n, dtype=torch.float64, device=lo.device)
        f_hi = torch.empty(n, dtype=torch.float64, device=lo.device)
        c = torch.empty(n, dtype=torch.float64, device=lo.device) if crown else None
        ws = ws or Workspace(net)
        buf, need = ws.get(n, flags | IBP_F_CROWN)
        _check(load_library().ibp_crown_lower_boxes(net.handle, n, _dev_ptr(lo), _dev_ptr(hi), _dev_ptr(f_lo),
                                                    _dev_ptr(f_hi), _dev_ptr(c), _dev_ptr(vertex),
                                                    _dev_ptr(buf), buf.numel(), _stream_ptr(stream), flags))
    return (f_lo, f_hi, c) if crown else (f_lo, f_hi)


def ibp_read_probe(src, partial, stream=None):
    """Streams a contiguous 16-byte aligned device tensor with the load pattern
    of the HBM-bound sweeps; writes 2048 float32 partial sums into `partial`."""
    torch = _torch()
    if not (src.is_cuda and src.is_contiguous() and src.numel() * src.element_size() >= 16):
        raise ValueError("src must be a contiguous device tensor of at least 16 bytes")
    if partial.dtype != torch.float32 or partial.numel() < 2048 or not partial.is_cuda:
        raise ValueError("partial must be a float32 device tensor with 2048 entries")
    n4 = src.numel() * src.element_size() // 16
    _check(load_library().ibp_read_probe(_dev_ptr(src), n4, _dev_ptr(partial), _stream_ptr(stream)))


ALU_PROBE_LANES = 524288


def ibp_alu_probe(out, iters: int, scalar_operand: bool = False, stream=None):
    """Float32 FMA issue-rate probe: eight FMA chains per lane over 2^19 lanes
    for `iters` steps; writes each lane's chain sum (16.0 once iters >= 64)
    into `out` (float32 device tensor of 2^19 entries)."""
    torch = _torch()
    if out.dtype != torch.float32 or out.numel() < ALU_PROBE_LANES or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 device tensor with 524288 entries")
    _check(load_library().ibp_alu_probe(_dev_ptr(out), int(iters), int(bool(scalar_operand)), _stream_ptr(stream)))


def ibp_autotune(net: Network, lo, hi, stream=None):
    """Times every tile pair on these device boxes and keeps the fastest; returns it."""
    torch = _torch()
    lo, hi = _check_boxes(net, lo, hi)
    n = lo.shape[0]
    need = net.workspace_bytes(n, IBP_F_AUTOTUNE)
    chosen = np.zeros(2, np.int32)
    with _on(stream):
        buf = torch.empty(max(need, 256), dtype=torch.uint8, device=lo.device)
        _check(load_library().ibp_autotune(net.handle, n, _dev_ptr(lo), _dev_ptr(hi), _dev_ptr(buf), buf.numel(),
                                           _stream_ptr(stream), chosen.ctypes.data_as(ctypes.c_void_p)))
    return int(chosen[0]), int(chosen[1])


def _tile_cache_key(net: Network, n_box: int) -> str:
    """(device name, buses, lines, outages, box-count bucket): the box count is
    rounded up to a power of two, as tiles depend on the batch's size class."""
    name = _torch().cuda.get_device_name(net.device)
    bucket = 1 << max(0, int(n_box - 1).bit_length())
    return f"{name}|N{net.n_bus}|L{net.n_line}|K{net.n_ctg}|B{bucket}"


def ibp_autotune_batched(net: Network, lo, hi, stream=None, cache: str = None):
    """Box-tiled tiles for calls like this one: times the candidates on these
    device boxes (at least 4) and keeps the fastest.  With ``cache`` (a JSON
    file path), tiles found before for the same device, network sizes and box
    bucket are set without timing, and new ones are added to the file.
    Returns (tiles dict, True if taken from the cache)."""
    import json as _json
    torch = _torch()
    lo, hi = _check_boxes(net, lo, hi)
    n = lo.shape[0]
    key = _tile_cache_key(net, n)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = _json.load(f)
        if key in table:
            v = table[key]
            net.set_tile_batched(v["k3_bt"], v["k3_rows"], v["k3_xcd"], v["k2_mfma"], v["k2_by"])
            net.set_screen_upper(v.get("screen_upper", 0))
            return net.tiles(), True
    need = net.workspace_bytes(n, IBP_F_AUTOTUNE)
    chosen = np.zeros(5, np.int32)
    with _on(stream):
        buf = torch.empty(max(need, 256), dtype=torch.uint8, device=lo.device)
        _check(load_library().ibp_autotune_batched(net.handle, n, _dev_ptr(lo), _dev_ptr(hi), _dev_ptr(buf),
                                                   buf.numel(), _stream_ptr(stream),
                                                   chosen.ctypes.data_as(ctypes.c_void_p)))
    tiles = net.tiles()
    if cache:
        table[key] = {k: tiles[k] for k in ("k3_bt", "k3_rows", "k3_xcd", "k2_mfma", "k2_by", "screen_upper")}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            _json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return tiles, False
