"""Betweenness oracle -- TEST INFRASTRUCTURE ONLY.

Plain CPU implementations used to check the GPU library.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import this package.
It shares no code with ``paper_1209_6007_amd`` and never imports it.

* ``bc_plain``        Algorithm 1 (Bc-Org, Section 2.1) in C, FP64.
* ``bc_weighted``     Algorithm 2 (Bc-Reach, Section 3.2.1) with the
                      identical-vertex weights of Section 3.3.3, in C, FP64.
* ``bc_classes``      ``bc_weighted`` for piece vertices standing for ident[v]
                      identical vertices whose reaches (possibly different)
                      sum to reach[v].
* ``single_source``   per-source levels / path counts / dependencies.
* ``bc_pieces``       ``bc_weighted`` on every piece of a packed set of pieces.
* ``bc_side``         Algorithm 3 (Bfs-Side, Section 3.3.2) for side vertices
                      removed one after another.
* ``farness`` / ``farness_pieces``  sum of shortest-path distances (weighted
                      by a per-vertex weight), one breadth-first search per
                      vertex, exact int64: the plain definition behind
                      closeness centrality, the measure the paper names as
                      the next one to shatter (Sections 1 and 5).
* ``brute.bc_bruteforce`` Eq. (1) evaluated pair by pair (tiny graphs).

All scores are over ordered pairs, unnormalised (Eq. (1)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.oracle_bc_plain.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int64, i32p, ctypes.c_int, f64p]
        lib.oracle_bc_plain.restype = ctypes.c_int
        lib.oracle_bc_weighted.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, ctypes.c_int64, i32p,
                                           ctypes.c_int, f64p]
        lib.oracle_bc_weighted.restype = ctypes.c_int
        lib.oracle_single_source.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, ctypes.c_int32, i32p,
                                             f64p, f64p]
        lib.oracle_single_source.restype = ctypes.c_int
        lib.oracle_bc_pieces.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, i32p, ctypes.c_int, f64p]
        lib.oracle_bc_pieces.restype = ctypes.c_int
        lib.oracle_bc_side.argtypes = [ctypes.c_int32, i32p, i32p, i32p, ctypes.c_int64, i32p, ctypes.c_int, f64p]
        lib.oracle_bc_side.restype = ctypes.c_int
        lib.oracle_bc_classes.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, ctypes.c_int, f64p]
        lib.oracle_bc_classes.restype = ctypes.c_int
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_farness_pieces.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, ctypes.c_int, i64p]
        lib.oracle_farness_pieces.restype = ctypes.c_int
        lib.oracle_farness_sources.argtypes = [ctypes.c_int32, i32p, i32p, i32p, ctypes.c_int64, i32p, ctypes.c_int,
                                               i64p]
        lib.oracle_farness_sources.restype = ctypes.c_int
        _lib = lib
    return _lib


def _i32(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


def bc_plain(n, row_ptr, col, sources=None, threads: int | None = None) -> np.ndarray:
    """Algorithm 1 over all sources (or the given source subset)."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    sv, svp = _i32(sources)
    out = np.zeros(max(n, 1), dtype=np.float64)
    nsrc = 0 if sources is None else len(sv)
    rc = lib.oracle_bc_plain(int(n), rpp, clp, nsrc, svp, threads or default_threads(),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise RuntimeError(f"oracle_bc_plain failed: {rc}")
    return out[:n]


def bc_weighted(n, row_ptr, col, reach=None, ident=None, sources=None, threads: int | None = None) -> np.ndarray:
    """Algorithm 2 with reach and identical-vertex weights; returns bc'."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    re, rep = _i32(reach)
    idn, idp = _i32(ident)
    sv, svp = _i32(sources)
    out = np.zeros(max(n, 1), dtype=np.float64)
    nsrc = 0 if sources is None else len(sv)
    rc = lib.oracle_bc_weighted(int(n), rpp, clp, rep, idp, nsrc, svp, threads or default_threads(),
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise RuntimeError(f"oracle_bc_weighted failed: {rc}")
    return out[:n]


def bc_classes(n, row_ptr, col, reach_sum, ident, threads: int | None = None) -> np.ndarray:
    """Algorithm 2 with identical-vertex weights where piece vertex v stands
    for ident[v] members whose reaches sum to reach_sum[v]; returns bc' (the
    members' common part: the dependency starts at their mean reach minus one)."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    re, rep = _i32(reach_sum)
    idn, idp = _i32(ident)
    out = np.zeros(max(n, 1), dtype=np.float64)
    rc = lib.oracle_bc_classes(int(n), rpp, clp, rep, idp, threads or default_threads(),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise RuntimeError(f"oracle_bc_classes failed: {rc}")
    return out[:n]


def single_source(n, row_ptr, col, s: int, reach=None, ident=None):
    """Returns (dist int32 with -1 unreachable, sigma f64, delta f64) for source s."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    re, rep = _i32(reach)
    idn, idp = _i32(ident)
    dist = np.zeros(n, dtype=np.int32)
    sig = np.zeros(n, dtype=np.float64)
    dl = np.zeros(n, dtype=np.float64)
    rc = lib.oracle_single_source(int(n), rpp, clp, rep, idp, int(s),
                                  dist.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  dl.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise RuntimeError(f"oracle_single_source failed: {rc}")
    return dist, sig, dl


def bc_pieces(vtx_off, row, col, reach=None, ident=None, threads: int | None = None) -> np.ndarray:
    """bc_weighted of every piece of a packed set (piece p owns packed vertices
    vtx_off[p]..vtx_off[p+1]-1; row holds absolute arc offsets into col, col
    piece-local ids); returns bc' per packed vertex."""
    lib = _load()
    vo, vop = _i32(vtx_off)
    rw, rwp = _i32(row)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    re, rep = _i32(reach)
    idn, idp = _i32(ident)
    P = len(vo) - 1
    V = int(vo[-1]) if P > 0 else 0
    out = np.zeros(max(V, 1), dtype=np.float64)
    rc = lib.oracle_bc_pieces(int(P), vop, rwp, clp, rep, idp, threads or default_threads(),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise RuntimeError(f"oracle_bc_pieces failed: {rc}")
    return out[:V]


def bc_side(n, row_ptr, col, reach, sides, threads: int | None = None) -> np.ndarray:
    """Algorithm 3 for the side vertices `sides`, removed in that order from
    the attributed graph (row_ptr, col, reach): bc' contributions per vertex."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    re, rep = _i32(reach if reach is not None else np.ones(n, np.int32))
    sv, svp = _i32(sides)
    out = np.zeros(max(n, 1), dtype=np.float64)
    rc = lib.oracle_bc_side(int(n), rpp, clp, rep, len(sv), svp, threads or default_threads(),
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise RuntimeError(f"oracle_bc_side failed: {rc}")
    return out[:n]


def farness_pieces(vtx_off, row, col, weight=None, threads: int | None = None) -> np.ndarray:
    """For every packed vertex x of every piece (layout as in bc_pieces): the
    sum over the vertices y of x's piece reachable from x of
    weight[y] * dist(x, y), int64 (weight None: all ones)."""
    lib = _load()
    vo, vop = _i32(vtx_off)
    rw, rwp = _i32(row)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    wt, wtp = _i32(weight)
    P = len(vo) - 1
    V = int(vo[-1]) if P > 0 else 0
    out = np.zeros(max(V, 1), dtype=np.int64)
    rc = lib.oracle_farness_pieces(int(P), vop, rwp, clp, wtp, threads or default_threads(),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise RuntimeError(f"oracle_farness_pieces failed: {rc}")
    return out[:V]


def farness(n, row_ptr, col, weight=None, sources=None, threads: int | None = None) -> np.ndarray:
    """Sum of shortest-path distances from every vertex (or from each of
    `sources`, in that order) to the vertices it reaches (weighted by
    weight[y] when given), int64."""
    if sources is None:
        if n == 0:
            return np.zeros(0, dtype=np.int64)
        return farness_pieces(np.array([0, n], np.int32), row_ptr, col, weight, threads)
    lib = _load()
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    wt, wtp = _i32(weight)
    sv, svp = _i32(sources)
    out = np.zeros(max(len(sv), 1), dtype=np.int64)
    rc = lib.oracle_farness_sources(int(n), rpp, clp, wtp, len(sv), svp, threads or default_threads(),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise RuntimeError(f"oracle_farness_sources failed: {rc}")
    return out[:len(sv)]


def bc(g, sources=None, threads=None) -> np.ndarray:
    """Convenience: Algorithm 1 on a graphgen.Graph-like object (n, row_ptr, col)."""
    return bc_plain(g.n, g.row_ptr, g.col, sources=sources, threads=threads)
