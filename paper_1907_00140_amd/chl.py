"""Python binding of libchl.so (include/chl.h): argument marshalling only.

Every step of the build and of the queries runs in the HIP library; this
module turns torch tensors into device pointers, passes the current HIP
stream, and wraps the returned handle. Device memory for the library comes
from torch's caching allocator through the chl_allocator callbacks (or from
hipMalloc with ``allocator="hip"``).
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchl.so")

CHL_OK = 0
ERRORS = {
    -1: "CHL_ERR_INVALID_ARG", -2: "CHL_ERR_OOM", -3: "CHL_ERR_HIP",
    -4: "CHL_ERR_DIST_OVERFLOW", -5: "CHL_ERR_NO_DEVICE", -6: "CHL_ERR_BUSY",
}
MODE_BATCHED, MODE_PLAIN = 0, 1
NOALLOC_MAX_PAIRS = 1 << 20     # CHL_NOALLOC_MAX_PAIRS


class ChlError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {ERRORS.get(code, code)} ({code})")


class CGraph(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_arcs", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("w", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class CAllocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class CBuildOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("roots_in_flight", C.c_int32), ("wg_size", C.c_int32),
                ("delta", C.c_int64), ("early_term", C.c_int32), ("stats", C.c_int32),
                ("autotune", C.c_int32), ("root_count", C.c_int32), ("root_begin", C.c_int32),
                ("root_stride", C.c_int32), ("prune_hubs", C.c_int32), ("team_wgs", C.c_int32),
                ("group_levels", C.c_int32), ("small_trees", C.c_int32), ("hybrid_psi", C.c_int32)]


class CStats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in (
        "n", "labels", "settled", "arcs", "early_trees", "key_bits", "roots_in_flight",
        "wg_size", "delta", "prune_hubs", "prefix_roots", "launches", "clock_khz")] + [(f, C.c_double) for f in (
            "tree_ms", "prefix_ms", "kernel_ms")] + [("kernel_launches", C.c_int64)] + [
        (f, C.c_double) for f in ("assemble_ms", "prep_ms", "tune_ms")] + [
        ("levels", C.c_int64), ("level_end", C.c_int64 * 16), ("level_ms", C.c_double * 16),
        ("level_teams", C.c_int64 * 16), ("small_trees", C.c_int64), ("hybrid_switch", C.c_int64),
        ("hybrid_psi", C.c_double), ("hybrid_supersteps", C.c_int64), ("hybrid_emitted", C.c_int64),
        ("hybrid_removed", C.c_int64), ("hybrid_clean_ms", C.c_double)]


class CServerOpts(C.Structure):
    _fields_ = [("mem_budget", C.c_size_t), ("max_batch", C.c_int32), ("build_streams", C.c_int32),
                ("build_wg", C.c_int32), ("reserved", C.c_int32)]


_lib = None
_lib_lock = threading.Lock()


def load(path=LIB_PATH):
    """Load libchl.so; raises if it has not been built (no fallback path)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with "
                              "`python -m paper_1907_00140_amd.build` (hipcc, gfx950)")
        lib = C.CDLL(path)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "chl_error_string": (C.c_char_p, [C.c_int]),
            "chl_build_opts_default": (None, [vp]),
            "chl_build": (C.c_int, [vp, vp, vp, vp, vp, vp]),
            "chl_labels_info": (C.c_int, [vp, vp, vp]),
            "chl_build_directed": (C.c_int, [vp, vp, vp, vp, vp, vp]),
            "chl_labels_directed": (C.c_int, [vp, vp]),
            "chl_labels_export_in": (C.c_int, [vp, vp, vp, vp, C.c_int, vp]),
            "chl_labels_export": (C.c_int, [vp, vp, vp, vp, C.c_int, vp]),
            "chl_labels_hub_vertex": (C.c_int, [vp, vp, C.c_int, vp]),
            "chl_query": (C.c_int, [vp, vp, i64, vp, vp]),
            "chl_labels_parents": (C.c_int, [vp, vp, vp, vp, vp]),
            "chl_microbench_atomic_min": (C.c_int, [vp, i64, C.c_int, i64, vp, vp, vp]),
            "chl_query_path_hops": (C.c_int, [vp, vp, vp, vp, i64, vp, vp, vp]),
            "chl_query_paths": (C.c_int, [vp, vp, vp, vp, i64, vp, vp, vp]),
            "chl_query_path_hops_noalloc": (C.c_int, [vp, vp, vp, vp, i64, vp, vp, vp]),
            "chl_build_stats": (C.c_int, [vp, vp, vp, C.c_int, vp]),
            "chl_labels_free": (None, [vp]),
            "chl_server_opts_default": (None, [vp]),
            "chl_server_create": (C.c_int, [vp, vp, vp]),
            "chl_server_add_labels": (C.c_int, [vp, vp, vp]),
            "chl_server_submit_queries": (C.c_int, [vp, i32, vp, vp, i64, vp, vp]),
            "chl_server_submit_build": (C.c_int, [vp, i32, i64, vp, vp, vp, vp, C.c_double, vp, vp, vp]),
            "chl_server_build_footprint": (C.c_size_t, [vp, i32, i64]),
            "chl_server_budget_peak": (C.c_size_t, [vp]),
            "chl_server_trace": (C.c_int, [vp, vp, i64, vp]),
            "chl_server_start": (C.c_int, [vp]),
            "chl_server_wait": (C.c_int, [vp]),
            "chl_server_labels": (vp, [vp, i32]),
            "chl_server_destroy": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        return lib


def _check(code, what):
    if code != CHL_OK:
        raise ChlError(code, what)


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class TorchAllocator:
    """chl_allocator backed by torch's caching allocator (device memory and
    its accounting stay with torch)."""

    def __init__(self, device=None, cap=None):
        """cap: refuse (return NULL for) an allocation that would take the
        live bytes past `cap` (None: no limit)."""
        self.device = torch.device(device or "cuda")
        self._live = {}
        self._mu = threading.Lock()
        self.calls = 0          # number of allocations made through this allocator
        self.cap = cap

        def _alloc(nbytes, ctx):
            # (an exception must not escape a ctypes callback: its return
            # value would then be undefined)
            try:
                if self.cap is not None and self.live_bytes + int(nbytes) > self.cap:
                    return None
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
                p = t.data_ptr()
                with self._mu:
                    self._live[p] = t
                    self.calls += 1
                return p
            except Exception:
                return None

        def _free(ptr, ctx):
            with self._mu:
                self._live.pop(ptr, None)

        self._a = ALLOC_FN(_alloc)
        self._f = FREE_FN(_free)
        self.c = CAllocator(self._a, self._f, None)

    @property
    def live_bytes(self):
        with self._mu:
            return sum(t.numel() for t in self._live.values())


_default_alloc = None


def default_allocator():
    global _default_alloc
    if _default_alloc is None:
        _default_alloc = TorchAllocator()
    return _default_alloc


def _dev(x, dtype):
    """Marshal an array-like to a contiguous device tensor of dtype."""
    if isinstance(x, torch.Tensor):
        t = x.to(device="cuda", dtype=dtype)
    else:
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(x))).to(device="cuda", dtype=dtype)
    return t.contiguous()


class Labels:
    """Handle of a device-resident canonical labeling."""

    def __init__(self, handle, allocator):
        self._h = C.c_void_p(handle)
        self._alloc = allocator        # keeps the callbacks alive
        self.lib = load()

    @property
    def handle(self):
        return self._h

    def info(self):
        n = C.c_int32()
        total = C.c_int64()
        _check(self.lib.chl_labels_info(self._h, C.byref(n), C.byref(total)), "chl_labels_info")
        return n.value, total.value

    def export(self, device="cpu", stream=None):
        """(offsets int64[n+1], hub_pos int32[L], dist int32[L]) as tensors."""
        n, total = self.info()
        on_host = str(device) == "cpu"
        kw = dict(device=device)
        if on_host:
            off = np.zeros(n + 1, np.int64)
            hub = np.zeros(max(total, 1), np.int32)
            dist = np.zeros(max(total, 1), np.int32)
            _check(self.lib.chl_labels_export(self._h, off.ctypes.data, hub.ctypes.data, dist.ctypes.data,
                                              1, _stream_ptr(stream)), "chl_labels_export")
            return torch.from_numpy(off), torch.from_numpy(hub[:total]), torch.from_numpy(dist[:total])
        off = torch.empty(n + 1, dtype=torch.int64, **kw)
        hub = torch.empty(max(total, 1), dtype=torch.int32, **kw)
        dist = torch.empty(max(total, 1), dtype=torch.int32, **kw)
        _check(self.lib.chl_labels_export(self._h, off.data_ptr(), hub.data_ptr(), dist.data_ptr(), 0,
                                          _stream_ptr(stream)), "chl_labels_export")
        return off, hub[:total], dist[:total]

    @property
    def directed(self):
        return self.lib.chl_labels_directed(self._h, None) == 1

    def export_in(self, device="cpu", stream=None):
        """In-labels of a directed labeling, laid out as export()."""
        n, _ = self.info()
        tot = C.c_int64()
        self.lib.chl_labels_directed(self._h, C.byref(tot))
        total = tot.value
        if str(device) == "cpu":
            off = np.zeros(n + 1, np.int64)
            hub = np.zeros(max(total, 1), np.int32)
            dist = np.zeros(max(total, 1), np.int32)
            _check(self.lib.chl_labels_export_in(self._h, off.ctypes.data, hub.ctypes.data, dist.ctypes.data, 1,
                                                 _stream_ptr(stream)), "chl_labels_export_in")
            return torch.from_numpy(off), torch.from_numpy(hub[:total]), torch.from_numpy(dist[:total])
        off = torch.empty(n + 1, dtype=torch.int64, device=device)
        hub = torch.empty(max(total, 1), dtype=torch.int32, device=device)
        dist = torch.empty(max(total, 1), dtype=torch.int32, device=device)
        _check(self.lib.chl_labels_export_in(self._h, off.data_ptr(), hub.data_ptr(), dist.data_ptr(), 0,
                                             _stream_ptr(stream)), "chl_labels_export_in")
        return off, hub[:total], dist[:total]

    def offsets(self, stream=None):
        """offsets int64[n+1] (by input id) on the host, without the label arrays."""
        n, _ = self.info()
        off = np.zeros(n + 1, np.int64)
        _check(self.lib.chl_labels_export(self._h, off.ctypes.data, None, None, 1, _stream_ptr(stream)),
               "chl_labels_export")
        return off

    def hub_vertex(self, device="cpu", stream=None):
        """Input id of the vertex at each hub rank position (int32[n]), as a
        host tensor or, with device="cuda", a device tensor."""
        n, _ = self.info()
        if device == "cpu":
            out = np.zeros(n, np.int32)
            _check(self.lib.chl_labels_hub_vertex(self._h, out.ctypes.data, 1, _stream_ptr(stream)),
                   "chl_labels_hub_vertex")
            return torch.from_numpy(out)
        out = torch.empty(n, dtype=torch.int32, device=device)
        _check(self.lib.chl_labels_hub_vertex(self._h, out.data_ptr(), 0, _stream_ptr(stream)),
               "chl_labels_hub_vertex")
        (stream or torch.cuda.current_stream()).synchronize()
        return out

    def query(self, pairs, out=None, stream=None):
        """Distances for pairs [q, 2] (input ids) as an int64 device tensor."""
        p = _dev(pairs, torch.int32).reshape(-1, 2)
        q = p.shape[0]
        if out is None:
            out = torch.empty(max(q, 1), dtype=torch.int64, device="cuda")
        _check(self.lib.chl_query(self._h, p.data_ptr(), q, out.data_ptr(), _stream_ptr(stream)), "chl_query")
        return out[:q]

    def parents(self, row_ptr, col, w, stream=None):
        """Per label (export order): the next vertex towards its hub on a
        shortest path (smallest input id among the candidates; -1 for a hub's
        own label) and the position of that vertex's label of the same hub in
        its list. g = the CSR the labeling was built from. Returns (parent,
        slot) int32 device tensors."""
        rp = _dev(row_ptr, torch.int64)
        cl = _dev(col, torch.int32)
        ww = _dev(w, torch.int32)
        n, total = self.info()
        g = CGraph(rp.numel() - 1, cl.numel(), rp.data_ptr(), cl.data_ptr() if cl.numel() else None,
                   ww.data_ptr() if ww.numel() else None)
        par = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
        slot = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
        _check(self.lib.chl_labels_parents(self._h, C.byref(g), par.data_ptr(), slot.data_ptr(),
                                           _stream_ptr(stream)), "chl_labels_parents")
        return par[:total], slot[:total]

    def path_hops(self, pairs, parent, slot, stream=None, noalloc=False, out=None):
        """(hops int64[q], path_off int64[q+1]) device tensors for pairs [q, 2].
        noalloc=True calls chl_query_path_hops_noalloc (no device memory taken
        from the labeling's allocator; q <= NOALLOC_MAX_PAIRS); out = (hops,
        path_off) caller tensors to fill."""
        p = _dev(pairs, torch.int32).reshape(-1, 2)
        q = p.shape[0]
        if out is None:
            hops = torch.empty(max(q, 1), dtype=torch.int64, device="cuda")
            off = torch.empty(q + 1, dtype=torch.int64, device="cuda")
        else:
            hops, off = out
        f = self.lib.chl_query_path_hops_noalloc if noalloc else self.lib.chl_query_path_hops
        _check(f(self._h, parent.data_ptr(), slot.data_ptr(), p.data_ptr(), q, hops.data_ptr(), off.data_ptr(),
                 _stream_ptr(stream)), "chl_query_path_hops_noalloc" if noalloc else "chl_query_path_hops")
        return hops[:q], off[:q + 1]

    def paths(self, pairs, parent, slot, stream=None):
        """Shortest paths for pairs [q, 2]: (hops int64[q], path_off
        int64[q+1], path int32[path_off[q]]) device tensors; pair k's vertices
        are path[path_off[k]:path_off[k+1]], u first and v last."""
        p = _dev(pairs, torch.int32).reshape(-1, 2)
        q = p.shape[0]
        hops, off = self.path_hops(p, parent, slot, stream)
        total = int(off[q].item())
        path = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
        _check(self.lib.chl_query_paths(self._h, parent.data_ptr(), slot.data_ptr(), p.data_ptr(), q,
                                        off.data_ptr(), path.data_ptr(), _stream_ptr(stream)), "chl_query_paths")
        return hops, off, path[:total]

    def stats(self, per_root=False):
        s = CStats()
        pr = None
        ptr = None
        if per_root:
            n, _ = self.info()
            pr = np.zeros((n, 6), np.int64)
            ptr = pr.ctypes.data
        _check(self.lib.chl_build_stats(self._h, C.byref(s), ptr, 1, _stream_ptr()), "chl_build_stats")
        d = {f: getattr(s, f) for f, _ in CStats._fields_}
        nl = int(s.levels)
        for f in ("level_end", "level_ms", "level_teams"):
            d[f] = list(d[f])[:nl]
        if per_root:
            d["per_root"] = pr
        return d

    def free(self):
        if self._h:
            self.lib.chl_labels_free(self._h)
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build(row_ptr, col, w, order, mode="batched", roots_in_flight=0, wg_size=0, delta=0,
          early_term=True, stats=True, autotune=True, roots=None, prune_hubs=0, team_wgs=0,
          stream=None, allocator="torch", directed=False, groups=True, small=None, hybrid_psi=0):
    """chl_build over a symmetric CSR (row_ptr int64, col int32, w int32) and a
    ranking order (order[0] most important). roots = (begin, count, stride)
    restricts the build to those root rank positions. directed=True: the CSR
    holds the out-arcs of a directed graph (chl_build_directed). hybrid_psi > 0:
    the Hybrid construction with that switching threshold. Returns Labels."""
    lib = load()
    rp = _dev(row_ptr, torch.int64)
    cl = _dev(col, torch.int32)
    ww = _dev(w, torch.int32)
    od = _dev(order, torch.int32)
    n = rp.numel() - 1
    g = CGraph(n, cl.numel(), rp.data_ptr(), cl.data_ptr() if cl.numel() else None,
               ww.data_ptr() if ww.numel() else None)
    o = CBuildOpts()
    lib.chl_build_opts_default(C.byref(o))
    o.mode = MODE_PLAIN if mode == "plain" else MODE_BATCHED
    o.roots_in_flight = int(roots_in_flight)
    o.wg_size = int(wg_size)
    o.delta = int(delta)
    o.early_term = 1 if early_term else 0
    o.stats = 1 if stats else 0
    o.autotune = 1 if autotune else 0
    if roots is not None:
        o.root_begin, o.root_count, o.root_stride = (int(x) for x in roots)
    o.prune_hubs = int(prune_hubs)
    o.team_wgs = int(team_wgs)
    o.group_levels = 0 if groups else -1
    o.small_trees = 0 if small is None else (1 if small else -1)
    o.hybrid_psi = int(hybrid_psi)
    al = allocator if isinstance(allocator, TorchAllocator) else default_allocator() if allocator == "torch" else None
    out = C.c_void_p()
    f = lib.chl_build_directed if directed else lib.chl_build
    code = f(C.byref(g), od.data_ptr(), C.byref(o), C.byref(al.c) if al else None, _stream_ptr(stream),
             C.byref(out))
    _check(code, "chl_build_directed" if directed else "chl_build")
    return Labels(out.value, al)


def microbench_atomic_min(words, key_bits=32, ops=1 << 28, stream=None):
    """Random atomic minima on a device array of `words` keys: (ops done, ms)."""
    lib = load()
    buf = torch.empty(int(words) * (key_bits // 8), dtype=torch.uint8, device="cuda")
    done, ms = C.c_int64(), C.c_double()
    _check(lib.chl_microbench_atomic_min(buf.data_ptr(), int(words), int(key_bits), int(ops), C.byref(done),
                                         C.byref(ms), _stream_ptr(stream)), "chl_microbench_atomic_min")
    return done.value, ms.value
