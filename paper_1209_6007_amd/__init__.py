"""shatterbc: exact betweenness centrality on MI355X (gfx950).

Thin ctypes binding of the C interface in include/shatterbc.h.  Every function
named ``sbc_*`` here marshals its arguments and calls the C function of the
same name; all computation happens in libshatterbc.so (host preprocessing in
C++, traversal in HIP kernels).  There is no Python or CPU fallback: if the
library is missing, importing the binding's functions raises.

PyTorch is used only for device memory and streams (``betweenness_device``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshatterbc.so")


def kernel_source_hash() -> str:
    """Hash of the sources that decide what a launch does (device code, and
    the host code that orders and batches its work); counter results are
    tied to it."""
    import hashlib

    h = hashlib.sha256()
    for f in ("kernel_types.hpp", "kernels_dev.hpp", "kernels.hip", "prep.cpp", "runtime.hip"):
        with open(os.path.join(_HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]

SBC_OK = 0
SBC_SANITIZE = 1
SBC_PLAIN = 0
SBC_COMPRESSED = 1
SBC_UNORDERED = 2
SBC_DETERMINISTIC = 4

STATUS = {
    0: "SBC_OK", -1: "SBC_E_INVALID_ARG", -2: "SBC_E_NOT_SYMMETRIC", -3: "SBC_E_SELF_LOOP",
    -4: "SBC_E_DUP_EDGE", -5: "SBC_E_INDEX_RANGE", -6: "SBC_E_TOO_LARGE", -7: "SBC_E_OOM",
    -8: "SBC_E_DEVICE", -9: "SBC_E_SIGMA_OVERFLOW", -10: "SBC_E_CANCELLED", -11: "SBC_E_NOT_READY",
    -12: "SBC_E_NO_DEVICE",
}


class SbcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class PrepStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "n", "m", "components", "stripped", "blocks", "bridges", "twin_classes", "twins_merged",
        "tiny_pieces", "pieces", "piece_vertices", "piece_arcs")] + [
        ("work_teps", ctypes.c_double), ("ms_degree1", ctypes.c_double), ("ms_shatter", ctypes.c_double),
        ("ms_twins", ctypes.c_double), ("ms_pack", ctypes.c_double), ("side_vertices", ctypes.c_int64),
        ("side_pieces", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RunStats(ctypes.Structure):
    _fields_ = [("ms_device", ctypes.c_double), ("ms_traverse", ctypes.c_double), ("ms_mapback", ctypes.c_double),
                ("ms_host", ctypes.c_double), ("teps", ctypes.c_double), ("algo_bytes", ctypes.c_double),
                ("items", ctypes.c_int64), ("batched_sources", ctypes.c_int64), ("lds_sources", ctypes.c_int64),
                ("global_sources", ctypes.c_int64), ("overflow", ctypes.c_int32),
                ("ms_class", ctypes.c_double * 5), ("bytes_class", ctypes.c_double * 5),
                ("teps_class", ctypes.c_double * 5), ("grid_class", ctypes.c_int32 * 5),
                ("items_class", ctypes.c_int32 * 5)]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if isinstance(v, ctypes.Array) else v
        return out


class JobStats(ctypes.Structure):
    _fields_ = [("submit_to_start_ms", ctypes.c_double), ("start_to_done_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("teps", ctypes.c_double), ("footprint_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FarStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "components", "stripped", "blocks", "bridges", "pieces",
                                               "piece_vertices", "piece_arcs")] + [("ms_prep", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FarRunStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("ms_kernel", "ms_device_total", "ms_finish", "ms_total", "teps")] + \
               [(k, ctypes.c_int64) for k in ("items", "grid", "waves")] + [("flags", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "sbc_status_string": ([ctypes.c_int32], ctypes.c_char_p),
    "sbc_last_error": ([], ctypes.c_char_p),
    "sbc_version": ([], ctypes.c_char_p),
    "sbc_context_create": ([ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int32),
    "sbc_context_destroy": ([_vp], ctypes.c_int32),
    "sbc_context_set_param": ([_vp, ctypes.c_char_p, ctypes.c_int64], ctypes.c_int32),
    "sbc_context_get_param": ([_vp, ctypes.c_char_p, _i64p], ctypes.c_int32),
    "sbc_context_device_name": ([_vp, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int32),
    "sbc_graph_create": ([ctypes.c_int32, _i32p, _i32p, ctypes.c_uint32, ctypes.POINTER(_vp)], ctypes.c_int32),
    "sbc_graph_destroy": ([_vp], ctypes.c_int32),
    "sbc_graph_info": ([_vp, _i32p, _i64p], ctypes.c_int32),
    "sbc_graph_preprocess": ([_vp, ctypes.c_char_p, ctypes.POINTER(PrepStats)], ctypes.c_int32),
    "sbc_graph_export_sizes": ([_vp, _i64p, _i64p, _i64p, _i64p], ctypes.c_int32),
    "sbc_graph_export": ([_vp, _i32p, _i32p, _i32p, _i32p, _i32p, _f64p, _f64p, _i32p, _i32p], ctypes.c_int32),
    "sbc_graph_export_side": ([_vp, _i32p], ctypes.c_int32),
    "sbc_plan_create": ([_vp, _vp, ctypes.c_uint32, ctypes.POINTER(_vp)], ctypes.c_int32),
    "sbc_plan_destroy": ([_vp], ctypes.c_int32),
    "sbc_plan_execute": ([_vp, _vp, _vp], ctypes.c_int32),
    "sbc_plan_sync": ([_vp, ctypes.POINTER(RunStats)], ctypes.c_int32),
    "sbc_plan_result": ([_vp, _f64p], ctypes.c_int32),
    "sbc_plan_use_graph": ([_vp, ctypes.c_int], ctypes.c_int32),
    "sbc_plan_phase_profile": ([_vp, _f64p, ctypes.c_int32], ctypes.c_int32),
    "sbc_plan_team_layout": ([_vp, _i32p, _i32p, ctypes.c_int32, _i32p], ctypes.c_int32),
    "sbc_betweenness": ([_vp, _vp, ctypes.c_uint32, _f64p, ctypes.POINTER(RunStats)], ctypes.c_int32),
    "sbc_betweenness_device": ([_vp, _vp, ctypes.c_uint32, _vp, _vp, ctypes.POINTER(RunStats)], ctypes.c_int32),
    "sbc_betweenness_sources": ([_vp, _vp, ctypes.c_int64, _i32p, _f64p, ctypes.POINTER(RunStats)], ctypes.c_int32),
    "sbc_piece_bc": ([_vp, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p, ctypes.c_int, _f64p,
                      ctypes.POINTER(RunStats)], ctypes.c_int32),
    "sbc_single_source": ([_vp, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p, ctypes.c_int32, _i32p, _f64p, _f64p],
                          ctypes.c_int32),
    "sbc_sources_state": ([_vp, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p, ctypes.c_int32, _i32p, ctypes.c_int,
                           _i32p, _f64p, _f64p], ctypes.c_int32),
    "sbc_piece_bc_noalloc": ([_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
                             ctypes.c_int32),
    "sbc_copy_bandwidth": ([_vp, ctypes.c_size_t, ctypes.c_int, _f64p], ctypes.c_int32),
    "sbc_far_create": ([_vp, ctypes.c_char_p, ctypes.POINTER(_vp), ctypes.POINTER(FarStats)], ctypes.c_int32),
    "sbc_far_destroy": ([_vp], ctypes.c_int32),
    "sbc_far_info": ([_vp, _i32p, _i64p, _i64p], ctypes.c_int32),
    "sbc_far_export": ([_vp, _i32p, _i32p, _i32p, _i32p, _i32p], ctypes.c_int32),
    "sbc_far_finish": ([_vp, _i64p, _i64p, _f64p], ctypes.c_int32),
    "sbc_far_run": ([_vp, _vp, _i64p, _i64p, _f64p, ctypes.POINTER(FarRunStats)], ctypes.c_int32),
    "sbc_server_create": ([_vp, ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_vp)], ctypes.c_int32),
    "sbc_server_destroy": ([_vp], ctypes.c_int32),
    "sbc_server_submit": ([_vp, _vp, ctypes.c_uint32, ctypes.POINTER(_vp)], ctypes.c_int32),
    "sbc_job_poll": ([_vp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int32),
    "sbc_job_wait": ([_vp, _f64p, ctypes.POINTER(JobStats)], ctypes.c_int32),
    "sbc_job_release": ([_vp], ctypes.c_int32),
}

EXPORTED = tuple(_SIGS)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int):
    if rc != SBC_OK:
        raise SbcError(rc, lib().sbc_last_error().decode(errors="replace"))


def _i32(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _mode(mode) -> int:
    if isinstance(mode, int):
        return mode
    m = {"plain": SBC_PLAIN, "compressed": SBC_COMPRESSED}[mode.split("+")[0]]
    if "unordered" in mode:
        m |= SBC_UNORDERED
    if "deterministic" in mode:
        m |= SBC_DETERMINISTIC
    return m


# ------------------------------------------------------------------ wrappers

def sbc_version() -> str:
    return lib().sbc_version().decode()


def sbc_context_create(device: int = 0):
    h = _vp()
    _check(lib().sbc_context_create(device, ctypes.byref(h)))
    return h


def sbc_context_destroy(ctx):
    _check(lib().sbc_context_destroy(ctx))


def sbc_context_set_param(ctx, key: str, value: int):
    _check(lib().sbc_context_set_param(ctx, key.encode(), int(value)))


def sbc_context_get_param(ctx, key: str) -> int:
    v = ctypes.c_int64()
    _check(lib().sbc_context_get_param(ctx, key.encode(), ctypes.byref(v)))
    return v.value


def sbc_context_device_name(ctx) -> str:
    buf = ctypes.create_string_buffer(256)
    _check(lib().sbc_context_device_name(ctx, buf, 256))
    return buf.value.decode()


def sbc_graph_create(n: int, row_ptr, col, flags: int = 0):
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    h = _vp()
    _check(lib().sbc_graph_create(int(n), rpp, clp, flags, ctypes.byref(h)))
    return h


def sbc_graph_destroy(g):
    _check(lib().sbc_graph_destroy(g))


def sbc_graph_info(g):
    n = ctypes.c_int32()
    a = ctypes.c_int64()
    _check(lib().sbc_graph_info(g, ctypes.byref(n), ctypes.byref(a)))
    return n.value, a.value


def sbc_graph_preprocess(g, ops: str = "dai") -> dict:
    st = PrepStats()
    _check(lib().sbc_graph_preprocess(g, ops.encode(), ctypes.byref(st)))
    return st.as_dict()


def sbc_graph_export(g) -> dict:
    P, V, A, M = (ctypes.c_int64() for _ in range(4))
    _check(lib().sbc_graph_export_sizes(g, ctypes.byref(P), ctypes.byref(V), ctypes.byref(A), ctypes.byref(M)))
    n, _ = sbc_graph_info(g)
    out = {
        "vtx_off": np.zeros(P.value + 1, np.int32), "row": np.zeros(V.value + 1, np.int32),
        "col": np.zeros(max(A.value, 1), np.int32), "reach": np.zeros(max(V.value, 1), np.int32),
        "ident": np.zeros(max(V.value, 1), np.int32), "corr": np.zeros(max(V.value, 1), np.float64),
        "bcx": np.zeros(max(n, 1), np.float64), "map_off": np.zeros(n + 1, np.int32),
        "map_idx": np.zeros(max(M.value, 1), np.int32),
    }
    p = {k: v.ctypes.data_as(_f64p if v.dtype == np.float64 else _i32p) for k, v in out.items()}
    _check(lib().sbc_graph_export(g, p["vtx_off"], p["row"], p["col"], p["reach"], p["ident"], p["corr"], p["bcx"],
                                  p["map_off"], p["map_idx"]))
    nside = np.zeros(max(P.value, 1), np.int32)
    _check(lib().sbc_graph_export_side(g, nside.ctypes.data_as(_i32p)))
    out["nside"] = nside[:P.value]
    out["col"] = out["col"][:A.value]
    for k in ("reach", "ident", "corr"):
        out[k] = out[k][:V.value]
    out["bcx"] = out["bcx"][:n]
    out["map_idx"] = out["map_idx"][:M.value]
    return out


def sbc_plan_create(ctx, g, mode=SBC_COMPRESSED):
    h = _vp()
    _check(lib().sbc_plan_create(ctx, g, _mode(mode), ctypes.byref(h)))
    return h


def sbc_plan_destroy(plan):
    _check(lib().sbc_plan_destroy(plan))


def sbc_plan_execute(plan, bc_dev_ptr=None, stream=None):
    _check(lib().sbc_plan_execute(plan, _vp(bc_dev_ptr) if bc_dev_ptr else None, _vp(stream) if stream else None))


def sbc_plan_sync(plan) -> dict:
    st = RunStats()
    _check(lib().sbc_plan_sync(plan, ctypes.byref(st)))
    return st.as_dict()


def sbc_plan_result(plan, n: int) -> np.ndarray:
    out = np.zeros(max(n, 1), np.float64)
    _check(lib().sbc_plan_result(plan, out.ctypes.data_as(_f64p)))
    return out[:n]


PHASE_NAMES = ("fetch_ms", "fwd_discover_ms", "fwd_count_ms", "fwd_count_split_ms", "fwd_retire_ms",
               "backward_ms", "backward_split_ms", "restore_ms", "items", "levels", "entries", "team_sync_ms")


def sbc_plan_phase_profile(plan) -> dict:
    out = np.zeros(len(PHASE_NAMES), np.float64)
    _check(lib().sbc_plan_phase_profile(plan, out.ctypes.data_as(_f64p), len(PHASE_NAMES)))
    return dict(zip(PHASE_NAMES, out.tolist()))


def sbc_plan_team_layout(plan, cap: int = 64):
    """(sizes, xcc_masks) of the team kernel's teams in the last execution."""
    sizes = np.zeros(cap, np.int32)
    masks = np.zeros(cap, np.int32)
    nt = np.zeros(1, np.int32)
    _check(lib().sbc_plan_team_layout(plan, sizes.ctypes.data_as(_i32p), masks.ctypes.data_as(_i32p), cap,
                                      nt.ctypes.data_as(_i32p)))
    k = min(int(nt[0]), cap)
    return sizes[:k].copy(), masks[:k].copy()


def sbc_plan_use_graph(plan, enable: bool = True):
    _check(lib().sbc_plan_use_graph(plan, 1 if enable else 0))


def sbc_betweenness(ctx, g, mode=SBC_COMPRESSED, with_stats: bool = False):
    n, _ = sbc_graph_info(g)
    out = np.zeros(max(n, 1), np.float64)
    st = RunStats()
    _check(lib().sbc_betweenness(ctx, g, _mode(mode), out.ctypes.data_as(_f64p), ctypes.byref(st)))
    return (out[:n], st.as_dict()) if with_stats else out[:n]


def sbc_betweenness_device(ctx, g, mode, bc_dev_ptr: int, stream: int | None = None) -> dict:
    st = RunStats()
    _check(lib().sbc_betweenness_device(ctx, g, _mode(mode), _vp(bc_dev_ptr), _vp(stream) if stream else None,
                                        ctypes.byref(st)))
    return st.as_dict()


def sbc_betweenness_sources(ctx, g, sources, with_stats: bool = False):
    n, _ = sbc_graph_info(g)
    sv, svp = _i32(sources)
    out = np.zeros(max(n, 1), np.float64)
    st = RunStats()
    _check(lib().sbc_betweenness_sources(ctx, g, len(sv), svp, out.ctypes.data_as(_f64p), ctypes.byref(st)))
    return (out[:n], st.as_dict()) if with_stats else out[:n]


def sbc_piece_bc(ctx, n, row_ptr, col, reach=None, ident=None, kernel: int = 0, with_stats: bool = False):
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    re, rep = _i32(reach)
    idn, idp = _i32(ident)
    out = np.zeros(max(n, 1), np.float64)
    st = RunStats()
    _check(lib().sbc_piece_bc(ctx, int(n), rpp, clp, rep, idp, int(kernel), out.ctypes.data_as(_f64p),
                              ctypes.byref(st)))
    return (out[:n], st.as_dict()) if with_stats else out[:n]


def sbc_single_source(ctx, n, row_ptr, col, s: int, reach=None, ident=None):
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    re, rep = _i32(reach)
    idn, idp = _i32(ident)
    dist = np.zeros(n, np.int32)
    sig = np.zeros(n, np.float64)
    dl = np.zeros(n, np.float64)
    _check(lib().sbc_single_source(ctx, int(n), rpp, clp, rep, idp, int(s), dist.ctypes.data_as(_i32p),
                                   sig.ctypes.data_as(_f64p), dl.ctypes.data_as(_f64p)))
    return dist, sig, dl


def sbc_sources_state(ctx, n, row_ptr, col, sources, kernel: int = 0, reach=None, ident=None):
    """(dist, sigma, delta), each [len(sources), n]: row k belongs to sources[k]."""
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    re, rep = _i32(reach)
    idn, idp = _i32(ident)
    sv, svp = _i32(sources)
    k = len(sv)
    dist = np.zeros((k, n), np.int32)
    sig = np.zeros((k, n), np.float64)
    dl = np.zeros((k, n), np.float64)
    _check(lib().sbc_sources_state(ctx, int(n), rpp, clp, rep, idp, k, svp, int(kernel),
                                   dist.ctypes.data_as(_i32p), sig.ctypes.data_as(_f64p), dl.ctypes.data_as(_f64p)))
    return dist, sig, dl


def sbc_piece_bc_noalloc(ctx, n: int, arcs: int, row_ptr_dev: int, col_dev: int, reach_dev, ident_dev,
                         bc_dev: int, flags_dev=None, stream=None):
    """Device-pointer arguments (integers); see include/shatterbc.h."""
    _check(lib().sbc_piece_bc_noalloc(ctx, int(n), int(arcs), _vp(row_ptr_dev), _vp(col_dev),
                                      _vp(reach_dev) if reach_dev else None, _vp(ident_dev) if ident_dev else None,
                                      _vp(bc_dev), _vp(flags_dev) if flags_dev else None,
                                      _vp(stream) if stream else None))


def sbc_copy_bandwidth(ctx, nbytes: int = 1 << 30, reps: int = 10) -> float:
    g = ctypes.c_double()
    _check(lib().sbc_copy_bandwidth(ctx, int(nbytes), int(reps), ctypes.byref(g)))
    return g.value


def sbc_server_create(ctx, slots: int = 4, hbm_budget_bytes: int = 0):
    h = _vp()
    _check(lib().sbc_server_create(ctx, int(slots), int(hbm_budget_bytes), ctypes.byref(h)))
    return h


def sbc_server_destroy(server):
    _check(lib().sbc_server_destroy(server))


def sbc_server_submit(server, g, mode=SBC_COMPRESSED):
    h = _vp()
    _check(lib().sbc_server_submit(server, g, _mode(mode), ctypes.byref(h)))
    return h


def sbc_job_poll(job) -> bool:
    d = ctypes.c_int()
    _check(lib().sbc_job_poll(job, ctypes.byref(d)))
    return bool(d.value)


def sbc_job_wait(job, n: int):
    out = np.zeros(max(n, 1), np.float64)
    st = JobStats()
    _check(lib().sbc_job_wait(job, out.ctypes.data_as(_f64p), ctypes.byref(st)))
    return out[:n], st.as_dict()


def sbc_job_release(job):
    _check(lib().sbc_job_release(job))


# ------------------------------------------------------------ conveniences

class Context:
    """Owns an sbc_context (device binding and tuning knobs)."""

    def __init__(self, device: int = 0, params: dict | None = None):
        self.h = sbc_context_create(device)
        for k, v in (params or {}).items():
            sbc_context_set_param(self.h, k, v)

    def close(self):
        if self.h:
            sbc_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sbc_far_create(g, ops: str = "oda"):
    """Prepares graph handle g for farness; returns (handle, stats dict)."""
    h = _vp()
    st = FarStats()
    _check(lib().sbc_far_create(g, ops.encode(), ctypes.byref(h), ctypes.byref(st)))
    return h, st.as_dict()


def sbc_far_destroy(f):
    _check(lib().sbc_far_destroy(f))


def sbc_far_export(f) -> dict:
    P, V, A = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().sbc_far_info(f, ctypes.byref(P), ctypes.byref(V), ctypes.byref(A)))
    out = {"vtx_off": np.zeros(P.value + 1, np.int32), "row": np.zeros(V.value + 1, np.int32),
           "col": np.zeros(max(A.value, 1), np.int32), "reach": np.zeros(max(V.value, 1), np.int32),
           "orig": np.zeros(max(V.value, 1), np.int32)}
    _check(lib().sbc_far_export(f, *(out[k].ctypes.data_as(_i32p) for k in ("vtx_off", "row", "col", "reach", "orig"))))
    out["col"] = out["col"][:A.value]
    out["reach"] = out["reach"][:V.value]
    out["orig"] = out["orig"][:V.value]
    return out


def sbc_far_finish(f, n: int, piece_sums):
    """Host pass only: (farness int64[n], closeness f64[n]) from per-piece sums."""
    w = np.ascontiguousarray(piece_sums, dtype=np.int64)
    far = np.zeros(max(n, 1), np.int64)
    clo = np.zeros(max(n, 1), np.float64)
    _check(lib().sbc_far_finish(f, w.ctypes.data_as(_i64p) if w.size else None, far.ctypes.data_as(_i64p),
                                clo.ctypes.data_as(_f64p)))
    return far[:n], clo[:n]


def sbc_far_run(ctx, f, n: int, with_piece_sums: bool = False):
    """Device sums and host pass: (farness, closeness, stats[, piece_sums])."""
    P, V, A = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().sbc_far_info(f, ctypes.byref(P), ctypes.byref(V), ctypes.byref(A)))
    w = np.zeros(max(V.value, 1), np.int64)
    far = np.zeros(max(n, 1), np.int64)
    clo = np.zeros(max(n, 1), np.float64)
    st = FarRunStats()
    _check(lib().sbc_far_run(ctx, f, w.ctypes.data_as(_i64p) if with_piece_sums else None,
                             far.ctypes.data_as(_i64p), clo.ctypes.data_as(_f64p), ctypes.byref(st)))
    if with_piece_sums:
        return far[:n], clo[:n], st.as_dict(), w[:V.value]
    return far[:n], clo[:n], st.as_dict()


def closeness(n, row_ptr, col, ops: str = "oda", device: int = 0, ctx: Context | None = None):
    """Farness (int64) and closeness ((component size - 1) / farness) of a CSR graph."""
    own = ctx is None
    ctx = ctx or Context(device)
    g = Graph(n, row_ptr, col)
    f = None
    try:
        f, _ = sbc_far_create(g.h, ops)
        far, clo, _ = sbc_far_run(ctx.h, f, n)
        return far, clo
    finally:
        if f:
            sbc_far_destroy(f)
        g.close()
        if own:
            ctx.close()


class Graph:
    """Owns an sbc_graph (host copy of a CSR graph and its preprocessing)."""

    def __init__(self, n, row_ptr, col, sanitize: bool = False):
        self.n = int(n)
        self.h = sbc_graph_create(n, row_ptr, col, SBC_SANITIZE if sanitize else 0)

    def preprocess(self, ops: str = "dai") -> dict:
        return sbc_graph_preprocess(self.h, ops)

    def close(self):
        if self.h:
            sbc_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def betweenness(n, row_ptr, col, mode: str = "compressed", ops: str = "dai", device: int = 0,
                ctx: Context | None = None) -> np.ndarray:
    """Exact betweenness (ordered pairs unless mode has '+unordered') of a CSR graph."""
    own = ctx is None
    ctx = ctx or Context(device)
    g = Graph(n, row_ptr, col)
    try:
        if mode.startswith("compressed"):
            g.preprocess(ops)
        return sbc_betweenness(ctx.h, g.h, _mode(mode))
    finally:
        g.close()
        if own:
            ctx.close()


def betweenness_device(n, row_ptr, col, mode: str = "compressed", ops: str = "dai", ctx: Context | None = None):
    """Same, with the result in a torch.float64 tensor on the current device and stream."""
    import torch

    own = ctx is None
    ctx = ctx or Context(torch.cuda.current_device())
    g = Graph(n, row_ptr, col)
    try:
        if mode.startswith("compressed"):
            g.preprocess(ops)
        out = torch.empty(max(int(n), 1), dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        sbc_betweenness_device(ctx.h, g.h, _mode(mode), out.data_ptr(), stream)
        return out[: int(n)]
    finally:
        g.close()
        if own:
            ctx.close()
