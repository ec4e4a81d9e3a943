"""CPU oracle for the Canonical Hub Labeling -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product library never links or calls it.

Thin ctypes wrapper over ``chl_oracle.c`` (plain C, built with gcc). See the
header of that file for what each function computes and which passage of the
paper it follows. All labels are returned in input vertex ids; hubs are given
by their rank position (0 = most important).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_DEFINITION = 0
MODE_PLANT = 1          # Algorithm 3 with early termination
MODE_PLANT_FULL = 2     # Algorithm 3 without early termination


def build(src=_SRC, out=_LIB, extra=()):
    """Compile the oracle with gcc into a shared library."""
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", *extra, src, "-o", out]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def load(path=None):
    """Load (building first if absent) the oracle library."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    lib_path = path or _LIB
    if not os.path.exists(lib_path) or (path is None and os.path.getmtime(lib_path) < os.path.getmtime(_SRC)):
        build(out=lib_path)
    lib = C.CDLL(lib_path)
    vp = C.c_void_p
    lib.oracle_run_roots.restype = vp
    lib.oracle_run_roots.argtypes = [C.c_int32, vp, vp, vp, vp, vp, C.c_int64, C.c_int, C.c_int]
    lib.oracle_run_roots_levels.restype = vp
    lib.oracle_run_roots_levels.argtypes = [C.c_int32, vp, vp, vp, vp, vp, C.c_int64, vp, C.c_int32,
                                            C.c_int32, C.c_int32, C.c_int]
    lib.oracle_run_count.restype = C.c_int64
    lib.oracle_run_count.argtypes = [vp, C.c_int64]
    lib.oracle_run_total.restype = C.c_int64
    lib.oracle_run_total.argtypes = [vp]
    lib.oracle_run_labels.argtypes = [vp, C.c_int64, vp, vp]
    lib.oracle_run_stats.argtypes = [vp, vp]
    lib.oracle_run_assemble.argtypes = [vp, vp, vp, vp]
    lib.oracle_run_free.argtypes = [vp]
    lib.oracle_query.argtypes = [vp, vp, vp, vp, C.c_int64, vp]
    lib.oracle_sssp.argtypes = [C.c_int32, vp, vp, vp, C.c_int32, vp]
    lib.oracle_query2.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_int64, vp]
    lib.oracle_parents.argtypes = [C.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.oracle_paths.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int64, vp, vp, vp]
    if path is None:
        _lib = lib
    return lib


def _graph_args(row_ptr, col, w, order):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    return row_ptr, col, w, order


class Labels:
    """Assembled labeling: offsets[n+1], hub_pos[L] (rank positions), dist[L] (int64)."""

    def __init__(self, offsets, hub_pos, dist, stats=None):
        self.offsets, self.hub_pos, self.dist, self.stats = offsets, hub_pos, dist, stats

    @property
    def n(self):
        return len(self.offsets) - 1

    @property
    def total(self):
        return int(self.offsets[-1])

    def of(self, v):
        a, b = self.offsets[v], self.offsets[v + 1]
        return list(zip(self.hub_pos[a:b].tolist(), self.dist[a:b].tolist()))


def chl(row_ptr, col, w, order, mode=MODE_PLANT, threads=None, lib=None):
    """Complete CHL of the graph under the ranking ``order`` (order[0] most
    important). Returns ``Labels`` with per-root stats [n_roots, 4] =
    (settled, arcs, labels, early) indexed by root rank position."""
    lib = lib or load()
    row_ptr, col, w, order = _graph_args(row_ptr, col, w, order)
    n = len(row_ptr) - 1
    threads = threads or min(16, os.cpu_count() or 1)
    h = lib.oracle_run_roots(n, row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data,
                             order.ctypes.data, None, 0, mode, threads)
    try:
        total = lib.oracle_run_total(h)
        offsets = np.zeros(n + 1, dtype=np.int64)
        hub = np.zeros(max(total, 1), dtype=np.int32)
        dist = np.zeros(max(total, 1), dtype=np.int64)
        lib.oracle_run_assemble(h, offsets.ctypes.data, hub.ctypes.data, dist.ctypes.data)
        stats = np.zeros((n, 4), dtype=np.int64)
        lib.oracle_run_stats(h, stats.ctypes.data)
    finally:
        lib.oracle_run_free(h)
    return Labels(offsets, hub[:total], dist[:total], stats)


def _assemble(lib, h, n):
    try:
        total = lib.oracle_run_total(h)
        offsets = np.zeros(n + 1, dtype=np.int64)
        hub = np.zeros(max(total, 1), dtype=np.int32)
        dist = np.zeros(max(total, 1), dtype=np.int64)
        lib.oracle_run_assemble(h, offsets.ctypes.data, hub.ctypes.data, dist.ctypes.data)
        stats = np.zeros((n, 4), dtype=np.int64)
        lib.oracle_run_stats(h, stats.ctypes.data)
    finally:
        lib.oracle_run_free(h)
    return Labels(offsets, hub[:total], dist[:total], stats)


def chl_pruned(row_ptr, col, w, order, eta=None, grown=None, levels=None, pmain=None, threads=None,
               lib=None, half=0):
    """Complete CHL by PLaNT trees with rank-prefix pruning (Section 4.3),
    grown in levels: ``levels`` = [g_0, g_1, ...]: roots [0, g_0) unpruned,
    level [g_{j-1}, g_j) pruned by the labels of hubs [0, g_{j-1}), and every
    later root pruned by hubs [0, pmain). ``eta, grown`` is the one-level
    case (levels=[grown], pmain=eta). Same labels as chl(); different work
    counts (stats, indexed by root rank position). half > 0: the graph is the
    combined graph of a directed graph (see combined_directed) with
    half = its vertex count."""
    lib = lib or load()
    if levels is None:
        levels, pmain = [grown], eta
    row_ptr, col, w, order = _graph_args(row_ptr, col, w, order)
    n = len(row_ptr) - 1
    lv = np.ascontiguousarray(levels, dtype=np.int32)
    threads = threads or min(16, os.cpu_count() or 1)
    h = lib.oracle_run_roots_levels(n, row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data,
                                    order.ctypes.data, None, 0, lv.ctypes.data, len(lv), int(pmain), int(half),
                                    threads)
    return _assemble(lib, h, n)


def chl_pruned_roots(row_ptr, col, w, order, root_pos, levels, pmain, threads=None, lib=None, half=0):
    """Work statistics [len(root_pos), 4] = (settled, arcs, labels, early) of
    the pruned trees of the given roots (rank positions) under the level
    schedule of chl_pruned; only the levels up to the largest requested root
    and the requested later roots are grown."""
    lib = lib or load()
    row_ptr, col, w, order = _graph_args(row_ptr, col, w, order)
    n = len(row_ptr) - 1
    lv = np.ascontiguousarray(levels, dtype=np.int32)
    rp = np.ascontiguousarray(root_pos, dtype=np.int32)
    threads = threads or min(16, os.cpu_count() or 1)
    h = lib.oracle_run_roots_levels(n, row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data,
                                    order.ctypes.data, rp.ctypes.data, len(rp), lv.ctypes.data, len(lv),
                                    int(pmain), int(half), threads)
    try:
        stats = np.zeros((len(rp), 4), dtype=np.int64)
        lib.oracle_run_stats(h, stats.ctypes.data)
    finally:
        lib.oracle_run_free(h)
    return stats


def roots(row_ptr, col, w, order, root_pos, mode=MODE_PLANT, threads=None, lib=None):
    """Labels of selected roots (given by rank position). Returns a list of
    (vertices int32, dists int64) sorted by vertex, one per root, and stats
    [len(root_pos), 4]."""
    lib = lib or load()
    row_ptr, col, w, order = _graph_args(row_ptr, col, w, order)
    n = len(row_ptr) - 1
    rp = np.ascontiguousarray(root_pos, dtype=np.int32)
    threads = threads or min(16, os.cpu_count() or 1)
    h = lib.oracle_run_roots(n, row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data,
                             order.ctypes.data, rp.ctypes.data, len(rp), mode, threads)
    out = []
    try:
        for t in range(len(rp)):
            c = lib.oracle_run_count(h, t)
            v = np.zeros(max(c, 1), dtype=np.int32)
            d = np.zeros(max(c, 1), dtype=np.int64)
            lib.oracle_run_labels(h, t, v.ctypes.data, d.ctypes.data)
            v, d = v[:c], d[:c]
            s = np.argsort(v, kind="stable")
            out.append((v[s], d[s]))
        stats = np.zeros((len(rp), 4), dtype=np.int64)
        lib.oracle_run_stats(h, stats.ctypes.data)
    finally:
        lib.oracle_run_free(h)
    return out, stats


def query(labels, pairs, lib=None):
    """Distances for int32 pairs [q, 2] by the sorted-list merge; -1 if no common hub."""
    lib = lib or load()
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    out = np.zeros(len(pairs), dtype=np.int64)
    off = np.ascontiguousarray(labels.offsets, dtype=np.int64)
    hub = np.ascontiguousarray(labels.hub_pos, dtype=np.int32)
    dist = np.ascontiguousarray(labels.dist, dtype=np.int64)
    lib.oracle_query(off.ctypes.data, hub.ctypes.data, dist.ctypes.data,
                     pairs.ctypes.data, len(pairs), out.ctypes.data)
    return out


def sssp(row_ptr, col, w, src, lib=None):
    """Dijkstra distances from src (int64, -1 unreachable)."""
    lib = lib or load()
    row_ptr, col, w, _ = _graph_args(row_ptr, col, w, np.zeros(1, np.int32))
    n = len(row_ptr) - 1
    out = np.zeros(n, dtype=np.int64)
    lib.oracle_sssp(n, row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data, int(src), out.ctypes.data)
    return out


def parents(labels, row_ptr, col, w, lib=None):
    """Per label of ``labels`` (same order): the parent vertex (input id; the
    smallest-id neighbour that is the next vertex of a shortest path towards
    the hub; -1 for a hub's own label) and the position of the parent's label
    of the same hub within the parent's list. Returns (parent, slot) int32."""
    lib = lib or load()
    row_ptr, col, w, _ = _graph_args(row_ptr, col, w, np.zeros(1, np.int32))
    off = np.ascontiguousarray(labels.offsets, dtype=np.int64)
    hub = np.ascontiguousarray(labels.hub_pos, dtype=np.int32)
    dist = np.ascontiguousarray(labels.dist, dtype=np.int64)
    total = int(off[-1])
    par = np.zeros(max(total, 1), dtype=np.int32)
    slot = np.zeros(max(total, 1), dtype=np.int32)
    lib.oracle_parents(len(off) - 1, row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data, off.ctypes.data,
                       hub.ctypes.data, dist.ctypes.data, par.ctypes.data, slot.ctypes.data)
    return par[:total], slot[:total]


def paths(labels, parent, slot, pairs, lib=None):
    """Shortest paths for int32 pairs [q, 2]: (hops int64[q], -1 when
    disconnected; path_off int64[q+1]; path int32[path_off[q]]), pair k's
    vertices being path[path_off[k]:path_off[k+1]], u first, v last."""
    lib = lib or load()
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    q = len(pairs)
    off = np.ascontiguousarray(labels.offsets, dtype=np.int64)
    hub = np.ascontiguousarray(labels.hub_pos, dtype=np.int32)
    dist = np.ascontiguousarray(labels.dist, dtype=np.int64)
    par = np.ascontiguousarray(parent, dtype=np.int32)
    sl = np.ascontiguousarray(slot, dtype=np.int32)
    hops = np.zeros(max(q, 1), dtype=np.int64)
    lib.oracle_paths(off.ctypes.data, hub.ctypes.data, dist.ctypes.data, par.ctypes.data, sl.ctypes.data,
                     pairs.ctypes.data, q, hops.ctypes.data, None, None)
    hops = hops[:q]
    path_off = np.zeros(q + 1, dtype=np.int64)
    np.cumsum(np.where(hops >= 0, hops + 1, 0), out=path_off[1:])
    path = np.zeros(max(int(path_off[-1]), 1), dtype=np.int32)
    lib.oracle_paths(off.ctypes.data, hub.ctypes.data, dist.ctypes.data, par.ctypes.data, sl.ctypes.data,
                     pairs.ctypes.data, q, hops.ctypes.data, path_off.ctypes.data, path.ctypes.data)
    return hops, path_off, path[:int(path_off[-1])]


def _transpose(row_ptr, col, w):
    """CSR of the reversed graph: row v lists the arcs u -> v as (u, w)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = len(row_ptr) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    dst = np.asarray(col, dtype=np.int64)
    p = np.lexsort((src, dst))
    trow = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(dst, minlength=n), out=trow[1:])
    return trow, src[p].astype(np.int32), np.asarray(w, dtype=np.int32)[p]


def chl_directed(row_ptr, col, w, order, mode=MODE_PLANT, threads=None, lib=None):
    """CHL of a directed graph given by its out-arc CSR (footnote of Section
    1): (L_out, L_in). L_in(v) holds (h, d(h, v)) from the trees grown along
    the arcs; L_out(v) holds (h, d(v, h)) from the trees grown on the
    reversed graph. Only the PLaNT modes apply (the definition form needs a
    symmetric graph)."""
    assert mode in (MODE_PLANT, MODE_PLANT_FULL)
    lab_in = chl(row_ptr, col, w, order, mode=mode, threads=threads, lib=lib)
    trow, tcol, tw = _transpose(row_ptr, col, w)
    lab_out = chl(trow, tcol, tw, order, mode=mode, threads=threads, lib=lib)
    return lab_out, lab_in


def query_directed(lab_out, lab_in, pairs, lib=None):
    """d(u, v) for int32 pairs [q, 2] from L_out(u) and L_in(v); -1 if none."""
    lib = lib or load()
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    out = np.zeros(len(pairs), dtype=np.int64)
    a = [np.ascontiguousarray(x, dtype=t) for x, t in ((lab_out.offsets, np.int64), (lab_out.hub_pos, np.int32),
                                                      (lab_out.dist, np.int64), (lab_in.offsets, np.int64),
                                                      (lab_in.hub_pos, np.int32), (lab_in.dist, np.int64))]
    lib.oracle_query2(*(x.ctypes.data for x in a), pairs.ctypes.data, len(pairs), out.ctypes.data)
    return out


def combined_directed(row_ptr, col, w, order):
    """The combined graph of a directed graph: the graph on ids [0, n), its
    reversal on [n, 2n), ranking interleaved (v at rank position 2 pos(v), its
    reversed copy at 2 pos(v) + 1). Its labels on [0, n) are the in-labels,
    on [n, 2n) the out-labels, each with hub position // 2."""
    row_ptr, col, w, order = _graph_args(row_ptr, col, w, order)
    n = len(row_ptr) - 1
    trow, tcol, tw = _transpose(row_ptr, col, w)
    row2 = np.concatenate([row_ptr, row_ptr[-1] + trow[1:]])
    col2 = np.concatenate([col, tcol + n]).astype(np.int32)
    w2 = np.concatenate([w, tw]).astype(np.int32)
    order2 = np.empty(2 * n, dtype=np.int32)
    order2[0::2] = order
    order2[1::2] = order + n
    return row2, col2, w2, order2


def split_combined(lab, n):
    """(L_out, L_in) from a labeling of the combined graph."""
    off = lab.offsets
    tin = int(off[n])
    lin = Labels(off[:n + 1].copy(), lab.hub_pos[:tin] // 2, lab.dist[:tin])
    lout = Labels(off[n:] - tin, lab.hub_pos[tin:] // 2, lab.dist[tin:])
    return lout, lin
