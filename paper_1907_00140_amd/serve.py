"""Python binding of the continuous-batching server of libchl.so
(chl_server_* in include/chl.h): argument marshalling only. The dispatch
loop, batching, admission and timing all run in the library's C++ thread."""
from __future__ import annotations

import ctypes as C

import numpy as np

from .chl import CServerOpts, Labels, _check, load


class BuildTicket:
    """Result slots of one submitted build (valid after Server.wait)."""

    def __init__(self, arrays):
        self._arrays = arrays          # host arrays must outlive the request
        self.gid = C.c_int32(-1)
        self.lat = C.c_double(0.0)
        self.status = C.c_int32(0)


class QueryTicket:
    def __init__(self, pairs, t, out, lat):
        self.pairs, self.t, self.out, self.lat = pairs, t, out, lat


class Server:
    def __init__(self, mem_budget=16 << 30, max_batch=1 << 16, build_streams=2, build_wg=128, allocator=None):
        """allocator: a chl.TorchAllocator for the builds' device memory (None:
        the stream-ordered pools of the build streams)."""
        self.lib = load()
        self._alloc = allocator
        o = CServerOpts()
        self.lib.chl_server_opts_default(C.byref(o))
        o.mem_budget = int(mem_budget)
        o.max_batch = int(max_batch)
        o.build_streams = int(build_streams)
        o.build_wg = int(build_wg)
        h = C.c_void_p()
        _check(self.lib.chl_server_create(C.byref(o), C.byref(allocator.c) if allocator is not None else None,
                                          C.byref(h)), "chl_server_create")
        self._h = h
        self._keep = []

    def add_labels(self, labels: Labels) -> int:
        gid = C.c_int32()
        _check(self.lib.chl_server_add_labels(self._h, labels.handle, C.byref(gid)), "chl_server_add_labels")
        self._keep.append(labels)
        return gid.value

    def submit_queries(self, gid, pairs, t_arrival) -> QueryTicket:
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        t = np.ascontiguousarray(t_arrival, dtype=np.float64)
        q = len(pairs)
        out = np.zeros(max(q, 1), np.int64)
        lat = np.zeros(max(q, 1), np.float64)
        _check(self.lib.chl_server_submit_queries(self._h, int(gid), pairs.ctypes.data, t.ctypes.data, q,
                                                  out.ctypes.data, lat.ctypes.data), "chl_server_submit_queries")
        tk = QueryTicket(pairs, t, out[:q], lat[:q])
        self._keep.append(tk)
        return tk

    def submit_build(self, row_ptr, col, w, order, t_arrival) -> BuildTicket:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        w = np.ascontiguousarray(w, dtype=np.int32)
        order = np.ascontiguousarray(order, dtype=np.int32)
        tk = BuildTicket((row_ptr, col, w, order))
        _check(self.lib.chl_server_submit_build(
            self._h, len(row_ptr) - 1, len(col), row_ptr.ctypes.data, col.ctypes.data if len(col) else None,
            w.ctypes.data if len(w) else None, order.ctypes.data, float(t_arrival), C.byref(tk.gid),
            C.byref(tk.lat), C.byref(tk.status)), "chl_server_submit_build")
        self._keep.append(tk)
        return tk

    def footprint(self, n, n_arcs) -> int:
        return int(self.lib.chl_server_build_footprint(self._h, int(n), int(n_arcs)))

    def budget_peak(self) -> int:
        return int(self.lib.chl_server_budget_peak(self._h))

    def trace(self):
        """Rows (kind, t0, t1, t2, size) of the last run: kind 0 = query batch
        (earliest arrival, queued, completed, queries), 1 = build (arrival,
        admitted, completed, vertices)."""
        n = C.c_int64()
        _check(self.lib.chl_server_trace(self._h, None, 0, C.byref(n)), "chl_server_trace")
        rows = np.zeros((max(n.value, 1), 5), np.float64)
        _check(self.lib.chl_server_trace(self._h, rows.ctypes.data, n.value, C.byref(n)), "chl_server_trace")
        return rows[:n.value]

    def start(self):
        _check(self.lib.chl_server_start(self._h), "chl_server_start")

    def wait(self):
        _check(self.lib.chl_server_wait(self._h), "chl_server_wait")

    def labels(self, gid) -> Labels:
        """A borrowed view of a server-owned labeling (do not free)."""
        p = self.lib.chl_server_labels(self._h, int(gid))
        if not p:
            raise KeyError(gid)
        L = Labels(p, None)
        L.free = lambda: None          # owned by the server
        return L

    def close(self):
        if self._h:
            self.lib.chl_server_destroy(self._h)
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def open_loop(server_factory, resident, query_sets, rate, builds=(), seed=0):
    """Run one open-loop experiment: `resident` is a list of Labels, query_sets
    a list of pair arrays (one per resident labeling), all interleaved as one
    Poisson stream at `rate` queries/s; `builds` a list of (config dict,
    arrival time). Returns (per-set results, per-set latencies, build tickets,
    wall seconds)."""
    import graphgen as gg
    srv = server_factory()
    gids = [srv.add_labels(L) for L in resident]
    total = sum(len(p) for p in query_sets)
    t = gg.poisson_arrivals(total, rate, seed)
    owner = np.repeat(np.arange(len(query_sets)), [len(p) for p in query_sets])
    np.random.default_rng(seed + 1).shuffle(owner)
    tickets = []
    for i, pairs in enumerate(query_sets):
        tickets.append(srv.submit_queries(gids[i], pairs, t[owner == i]))
    btk = [srv.submit_build(c["row_ptr"], c["col"], c["w"], c["order"], ta) for c, ta in builds]
    import time
    t0 = time.perf_counter()
    srv.start()
    srv.wait()
    wall = time.perf_counter() - t0
    return srv, tickets, btk, wall
