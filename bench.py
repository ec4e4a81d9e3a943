"""Benchmark of the PLaNT CHL build and distance queries on one MI355X.

One step = the whole hot path over one batch of synthetic input: chl_build of
the complete canonical labeling of the R-MAT scale-16 graph (validation, rank
renumbering, the batched persistent tree kernel, label assembly) followed by
chl_query on its 10^6 query pairs. Inputs (CSR, ranking, pairs) are resident
in device memory before the timed region starts.

value = build GTEPS = arcs scanned by the reference Dijkstra trees (counted
by the CPU oracle with early termination) / build time / 1e9.

Prints one JSON line. Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "rmat16"
COUNTS = os.path.join(ROOT, "tests", "golden", "workload_counts.json")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_tree_rmat16.json")
# the tree kernel and the host code that picks its launches: byte counters
# taken for other sources no longer describe the kernel
TREE_SRC = [os.path.join(ROOT, "paper_1907_00140_amd", "csrc", f) for f in ("tree.hip", "api.cpp")]


def src_sha():
    h = hashlib.sha256()
    for f in TREE_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def serve_measure(chl, gg, c, row, col, w, order, stream, qout, q):
    """Open-loop serving on the resident labeling: saturation throughput of
    the server path, then a Poisson stream at half of it with two label
    builds of other graphs arriving meanwhile."""
    import numpy as np
    from paper_1907_00140_amd import serve
    L = chl.build(row, col, w, order, stream=stream)
    sp = np.concatenate([c["pairs"], c["pairs"]])
    mk = lambda: serve.Server(mem_budget=32 << 30, max_batch=1 << 16, build_streams=2, build_wg=128)
    srv = mk()
    gid = srv.add_labels(L)
    tk = srv.submit_queries(gid, sp, np.zeros(len(sp)))
    t1 = time.perf_counter()
    srv.start()
    srv.wait()
    sat_qps = len(sp) / (time.perf_counter() - t1)
    srv.close()
    rate = 0.5 * sat_qps
    span = len(sp) / rate
    blds = [(gg.make_config("rmat12_0"), 0.2 * span), (gg.make_config("rmat13_1"), 0.5 * span)]
    srv, tks, btk, wall = serve.open_loop(mk, [L], [sp], rate, builds=blds, seed=11)
    lat = tks[0].lat
    assert np.array_equal(tks[0].out[:q], qout.cpu().numpy())
    serving = {"resident": "R-MAT scale 16 labeling", "queries": int(len(sp)),
           "saturated_qps": round(sat_qps, 1), "rate_qps": round(rate, 1),
           "achieved_qps": round(len(sp) / float(np.max(tks[0].t + lat)), 1),
           "p50_us": round(float(np.percentile(lat, 50)) * 1e6, 2),
           "p99_us": round(float(np.percentile(lat, 99)) * 1e6, 2),
           "builds": [{"graph": nm, "status": int(b.status.value), "latency_s": round(b.lat.value, 4)}
                      for (cc, _), b, nm in zip(blds, btk, ("rmat12_0", "rmat13_1"))]}
    srv.close()
    L.free()

    return serving


def serve_full(chl, gg, stream):
    """The serving experiment at full size: the labelings of the R-MAT
    scale-16 and the 1024x1024 diagonal-grid workloads resident, 10^7
    uniform query pairs (half on each graph, in one Poisson stream) at 0.25,
    0.5 and 0.9 of the server path's saturated rate, with 16 build requests
    (R-MAT scales 10..16, seeds 500+i, weights [1,1000]) arriving over the
    stream and admitted by HBM footprint. Every answer is checked against a
    direct chl_query of the same labeling, every build against the same build
    run alone."""
    import numpy as np
    import torch
    from paper_1907_00140_amd import serve
    dev = torch.device("cuda:0")
    names = ("rmat16", "grid1024d")
    res, qsets, direct = [], [], []
    for k, nm in enumerate(names):
        c = gg.make_config(nm)
        d = [torch.from_numpy(c[f]).to(dev) for f in ("row_ptr", "col", "w", "order")]
        t1 = time.perf_counter()
        L = chl.build(*d, stream=stream)
        torch.cuda.synchronize()
        print("serve-full: built %s in %.2f s" % (nm, time.perf_counter() - t1), file=sys.stderr, flush=True)
        pairs = gg.query_pairs(c["n"], 5_000_000, 702 + k)
        direct.append(L.query(torch.from_numpy(pairs).to(dev), stream=stream).cpu().numpy())
        res.append(L)
        qsets.append(pairs)
        del d
    mk = lambda: serve.Server(mem_budget=64 << 30, max_batch=1 << 16, build_streams=2, build_wg=128)
    # saturation: every query due at time 0
    srv = mk()
    gids = [srv.add_labels(L) for L in res]
    tks = [srv.submit_queries(g, p, np.zeros(len(p))) for g, p in zip(gids, qsets)]
    t1 = time.perf_counter()
    srv.start()
    srv.wait()
    sat = sum(len(p) for p in qsets) / (time.perf_counter() - t1)
    for tk, ref in zip(tks, direct):
        assert np.array_equal(tk.out, ref)
    srv.close()
    print("serve-full: saturated %.3g queries/s" % sat, file=sys.stderr, flush=True)
    bcfg = [gg.make_config("rmat%d_%d" % (10 + i % 7, i)) for i in range(16)]
    alone = []
    for c in bcfg:
        Lb = chl.build(c["row_ptr"], c["col"], c["w"], c["order"], stream=stream)
        alone.append([x.numpy() for x in Lb.export("cpu")])
        Lb.free()
    out = {"resident": list(names), "queries": int(sum(len(p) for p in qsets)), "saturated_qps": round(sat, 1),
           "rates": []}
    for f in (0.25, 0.5, 0.9):
        rate = f * sat
        span = sum(len(p) for p in qsets) / rate
        tb = gg.poisson_arrivals(16, 16 / span, 900 + int(100 * f))
        srv, tks, btk, wall = serve.open_loop(mk, res, qsets, rate, builds=list(zip(bcfg, tb)), seed=int(100 * f))
        for tk, ref in zip(tks, direct):
            assert np.array_equal(tk.out, ref), "served answers differ from chl_query"
        for b, ref in zip(btk, alone):
            assert b.status.value == 0, "build request failed: %d" % b.status.value
            got = [x.numpy() for x in srv.labels(b.gid.value).export("cpu")]
            assert all(np.array_equal(x, y) for x, y in zip(got, ref)), "served build differs from alone"
        lat = np.concatenate([tk.lat for tk in tks])
        tend = max(float(np.max(tk.t + tk.lat)) for tk in tks)
        blat = np.array([b.lat.value for b in btk])
        out["rates"].append({"fraction": f, "rate_qps": round(rate, 1),
                             "achieved_qps": round(len(lat) / tend, 1),
                             "p50_us": round(float(np.percentile(lat, 50)) * 1e6, 2),
                             "p99_us": round(float(np.percentile(lat, 99)) * 1e6, 2),
                             "per_graph_p99_us": [round(float(np.percentile(tk.lat, 99)) * 1e6, 2) for tk in tks],
                             "build_latency_s": {"p50": round(float(np.median(blat)), 4),
                                                 "max": round(float(blat.max()), 4)},
                             "wall_s": round(wall, 3)})
        srv.close()
        print("serve-full:", json.dumps(out["rates"][-1]), file=sys.stderr, flush=True)
    for L in res:
        L.free()
    return out


def paths_measure(chl, L, c, d, pairs, stream, reps=3):
    """Shortest-path extension on a resident labeling: the parents kernel
    (one launch; HIP events on the build stream, median of reps) against
    its algorithmic bytes, and path queries (hop counts + path vertices) for
    the given device pairs. Algorithmic bytes of the parents kernel: 4 per
    lookup of a label's hub in a neighbour's list (sum over v of
    deg(v) * |L_v| lookups), 16 per label (its hub and distance read, its
    parent and slot written), 8 per arc and 32 per vertex (row and label
    offsets)."""
    import numpy as np
    import torch
    row, col, w = d[0], d[1], d[2]
    off = L.offsets()
    deg = np.diff(c["row_ptr"])
    lab = np.diff(off)
    lookups = int((deg * lab).sum())
    total = int(off[-1])
    alg = 4 * lookups + 16 * total + 8 * int(len(c["col"])) + 32 * int(c["n"])
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        par, slot = L.parents(row, col, w, stream=stream)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    pm = float(np.median(ms))
    L.paths(pairs[:1000], par, slot, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hops, poff, path = L.paths(pairs, par, slot, stream=stream)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t1
    h = hops.cpu().numpy()
    conn = h >= 0
    achieved = alg / (pm / 1e3) / 1e9
    r = {"parents_ms": round(pm, 3), "parents_alg_bytes": alg, "lookups": lookups,
         "parents_roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(achieved / HBM_PEAK_GBS, 5)},
         "path_pairs": int(len(h)), "path_s": round(ts, 5), "paths_per_s": round(len(h) / ts, 1),
         "connected": int(conn.sum()), "mean_hops": round(float(h[conn].mean()), 2) if conn.any() else None,
         "max_hops": int(h.max()), "path_vertices": int(poff[-1].item())}
    del par, slot, hops, poff, path
    return r


def directed_measure(chl, gg, stream, reps=3):
    """Directed R-MAT scale 16 (the generator's samples read as arcs): the
    complete out- and in-labels (chl_build_directed: one build over the graph
    and its reversal, rank-prefix pruning across the two directions) timed
    after one untimed build that tunes, and 10^6 queries. GTEPS = arcs
    scanned by the oracle's unpruned early-terminating trees in both
    directions (tests/golden/workload_counts.json) / build time, the same
    convention as the undirected line."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    name = "rmat16dir"
    c = gg.make_config(name)
    d = [torch.from_numpy(c[f]).to(dev) for f in ("row_ptr", "col", "w", "order")]
    pairs = torch.from_numpy(c["pairs"]).to(dev)
    L = chl.build(*d, directed=True, stream=stream)
    torch.cuda.synchronize()
    L.free()
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L = chl.build(*d, directed=True, stream=stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        st = L.stats()
        if len(times) < reps:
            L.free()
    qo = L.query(pairs, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.query(pairs, out=qo, stream=stream)
    torch.cuda.synchronize()
    qs = len(c["pairs"]) / (time.perf_counter() - t1)
    L.free()
    b = float(np.median(times))
    wc = json.load(open(COUNTS)).get(name, {})
    r = {"workload": "directed R-MAT scale 16 (65,536 vertices, %d arcs), int32 weights [1,1000], "
                     "total-degree rank; out- and in-labels + 10^6 uniform queries" % c["m"],
         "build_s": round(b, 4), "build_s_runs": [round(t, 4) for t in times], "labels": st["labels"],
         "gpu_arcs": st["arcs"], "queries_per_s": round(qs, 1),
         "roots_in_flight": st["roots_in_flight"], "wg_size": st["wg_size"], "delta": st["delta"],
         "prune_hubs_combined": st["prune_hubs"],
         "phases_ms": {"prep": round(st["prep_ms"], 2), "prefix": round(st["prefix_ms"], 2),
                       "main": round(st["tree_ms"], 2), "assemble": round(st["assemble_ms"], 2)}}
    if "arcs" in wc:
        r["gteps"] = round(wc["arcs"] / b / 1e9, 4)
        r["oracle_arcs"] = wc["arcs"]
        r["gpu_arcs_per_unpruned_oracle_arc"] = round(st["arcs"] / wc["arcs"], 4)
        assert st["labels"] == wc["labels"], "label count differs from the oracle's"
    # the oracle's trees under the same pruning schedule on the combined graph
    lv = next((v for v in wc.values() if isinstance(v, dict) and v.get("grown") == st["prefix_roots"]
               and v.get("pmain") == st["prune_hubs"]), None)
    if lv is not None:
        a = lv["head"]["arcs"] + lv["rest"]["arcs"]
        r["method_gteps"] = round(a / b / 1e9, 4)
        r["oracle_arcs_method"] = a
        r["work_inflation"] = round(st["arcs"] / a, 3)
    print("directed:", json.dumps(r), file=sys.stderr, flush=True)
    return r


def large_workloads(chl, gg, stream):
    """The other workloads: the 64x64 grid (10^4 queries), the 1024x1024 grid
    with 5% diagonal shortcuts and R-MAT scale 20 (10^6 queries each). Full
    labeling resident in HBM (median of 3 builds after one untimed build that
    also tunes), label-size histogram (log2 bins of |L_v|), early-termination
    rate, exploration per label, queries/s, and for the grids the plain
    one-root-per-launch form estimated from head roots and rank-stratified
    roots (64 + 256 on the small grid, 16 + 64 on the large one)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    out = {}
    for nm in ("grid64", "grid1024d", "rmat20"):
        c = gg.make_config(nm)
        d = [torch.from_numpy(c[f]).to(dev) for f in ("row_ptr", "col", "w", "order")]
        pairs = torch.from_numpy(c["pairs"]).to(dev)
        L = chl.build(*d, stream=stream)
        torch.cuda.synchronize()
        L.free()
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L = chl.build(*d, stream=stream)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            if len(times) < 3:
                L.free()
        tb = float(np.median(times))
        st = L.stats()
        off = L.offsets()
        sizes = np.diff(off)
        bins = np.bincount(np.floor(np.log2(np.maximum(sizes, 1))).astype(np.int64))
        qo = L.query(pairs, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        qo = L.query(pairs, out=qo, stream=stream)
        torch.cuda.synchronize()
        qs = len(c["pairs"]) / (time.perf_counter() - t1)
        npath = 10_000 if nm.startswith("grid") else len(c["pairs"])
        pth = paths_measure(chl, L, c, d, pairs[:npath], stream)
        L.free()
        r = {"n": c["n"], "edges": c["m"], "build_s": round(tb, 4), "build_s_runs": [round(t, 4) for t in times],
             "labels": st["labels"], "als": round(st["labels"] / c["n"], 2), "max_label_size": int(sizes.max()),
             "label_size_hist_log2": {"[%d,%d)" % (1 << k, 2 << k): int(v) for k, v in enumerate(bins) if v},
             "early_termination_rate": round(st["early_trees"] / c["n"], 4),
             "settled_per_tree": round(st["settled"] / c["n"], 1),
             "explored_per_label": round(st["settled"] / max(1, st["labels"]), 2),
             "gpu_arcs": st["arcs"], "gpu_arcs_per_s": round(st["arcs"] / tb, 1),
             "prune_hubs": st["prune_hubs"], "roots_in_flight": st["roots_in_flight"], "wg_size": st["wg_size"],
             "delta": st["delta"], "key_bits": st["key_bits"],
             "phases_ms": {"prep": round(st["prep_ms"], 1), "prefix": round(st["prefix_ms"], 1),
                           "main": round(st["tree_ms"], 1), "assemble": round(st["assemble_ms"], 1)},
             "queries_per_s": round(qs, 1), "paths": pth}
        wc = json.load(open(COUNTS)).get(nm, {})
        if "arcs" in wc:
            r["gteps"] = round(wc["arcs"] / tb / 1e9, 4)
            r["oracle_arcs_unpruned"] = wc["arcs"]
        lv = next((v for v in wc.values() if isinstance(v, dict) and v.get("grown") == st["prefix_roots"]
                   and v.get("pmain") == st["prune_hubs"]), None)
        if lv is not None:
            a = lv["head"]["arcs"] + lv["rest"]["arcs"]
            r["method_gteps"] = round(a / tb / 1e9, 4)
            r["work_inflation"] = round(st["arcs"] / a, 3)
        elif st["prune_hubs"] == 0 and "arcs" in wc:
            r["work_inflation"] = round(st["arcs"] / wc["arcs"], 3)
        if nm.startswith("grid"):
            n = c["n"]
            H, NS = (64, 256) if n < 100_000 else (16, 64)
            stride = (n - H) // NS
            tp = []
            for roots in ((0, H, 1), (H, NS, stride)):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                Lp = chl.build(*d, mode="plain", roots=roots, stream=stream)
                torch.cuda.synchronize()
                tp.append(time.perf_counter() - t1)
                Lp.free()
            r["plain_form"] = {"build_s_est": round(tp[0] + tp[1] * stride, 3),
                               "method": "%d head roots + %d rank-stratified roots (stride %d), "
                                         "sum = head + sample * stride" % (H, NS, stride)}
        out[nm] = r
        print("large:", nm, json.dumps(r), file=sys.stderr, flush=True)
        del d, pairs
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form estimate")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-directed", action="store_true", help="skip the directed-graph measurement")
    ap.add_argument("--no-paths", action="store_true", help="skip the shortest-path measurement")
    ap.add_argument("--no-atomic-ceiling", action="store_true", help="skip the atomic-minimum microbenchmark")
    ap.add_argument("--large", action="store_true",
                    help="also build the other workloads (64x64 grid, 1024x1024 diagonal grid, R-MAT 20) "
                         "and report them in a 'large' object")
    ap.add_argument("--serve-full", action="store_true",
                    help="also run the full-size serving experiment (two resident labelings, 10^7 queries "
                         "at three rates, 16 builds); adds a 'serving_full' object")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(every tree is independent; see the sharding design in the docs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen as gg
    from paper_1907_00140_amd import chl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    c = gg.make_config(WORKLOAD)
    counts = json.load(open(COUNTS))[WORKLOAD]
    A, S, Lc = counts["arcs"], counts["settled"], counts["labels"]
    row = torch.from_numpy(c["row_ptr"]).to(dev)
    col = torch.from_numpy(c["col"]).to(dev)
    w = torch.from_numpy(c["w"]).to(dev)
    order = torch.from_numpy(c["order"]).to(dev)
    pairs = torch.from_numpy(c["pairs"]).to(dev)
    q = pairs.shape[0]
    qout = torch.empty(q, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        L = chl.build(row, col, w, order, stream=stream)
        L.query(pairs, out=qout, stream=stream)
        return L

    for _ in range(args.warmup):
        L = step()
        assert L.info()[1] == Lc, "label count differs from the oracle's"
        L.free()
    torch.cuda.synchronize()
    build_ms, query_ms, kernel_ms, klaunch, stats = [], [], [], [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tb = time.perf_counter()
        L = chl.build(row, col, w, order, stream=stream)
        torch.cuda.synchronize()
        tq = time.perf_counter()
        L.query(pairs, out=qout, stream=stream)
        torch.cuda.synchronize()
        te = time.perf_counter()
        build_ms.append((tq - tb) * 1e3)
        query_ms.append((te - tq) * 1e3)
        stats = L.stats(per_root=True)
        per_root = stats.pop("per_root")
        gpu_arcs = int(per_root[:, 1].sum())
        kernel_ms.append(stats["kernel_ms"])
        klaunch.append(stats["kernel_launches"])
        L.free()
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    b_s = float(np.median(build_ms)) / 1e3
    gteps = A / b_s / 1e9
    qps = q / (float(np.median(query_ms)) / 1e3)

    # roofline of the dominant kernels, the tree kernels (teams for the first
    # levels, the batched kernel for the others and the main phase): every
    # production launch of one build, timed with events on the build stream
    # inside the library.
    # Algorithmic bytes = 16 per scanned arc + 16 per settled vertex + 8 per
    # label, with the units counted by the oracle's trees under the same
    # pruning configuration (tests/golden/workload_counts.json)
    g, pm = stats["prefix_roots"], stats["prune_hubs"]
    if g == 0:
        cfg = None
        units = {"arcs": A, "settled": S, "labels": Lc}
    else:
        cfg = next((v for k, v in counts.items() if isinstance(v, dict) and v.get("grown") == g
                    and v.get("pmain") == pm), None)
        if cfg is None:
            sys.exit("no oracle work counts for a %d-hub prefix grown over %d roots: run "
                     "python -m oracle.workload_counts %s" % (pm, g, WORKLOAD))
        units = {k: cfg["head"][k] + cfg["rest"][k] for k in ("arcs", "settled", "labels")}
    nl = max(1, int(np.median(klaunch)))
    alg_bytes = (16 * units["arcs"] + 16 * units["settled"] + 8 * units["labels"]) / nl
    per_launch_ms = float(np.median(kernel_ms)) / nl
    achieved = alg_bytes / (per_launch_ms / 1e3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC):
        tr = json.load(open(TRAFFIC))
        if tr.get("tree_src_sha") == src_sha():
            traffic = tr.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "tree kernels k_tree_team + k_tree_batched (every production launch of a build: team levels, wide levels, main phase)",
                "kernel_ms": round(per_launch_ms, 3), "launches_per_build": nl,
                "alg_bytes_per_launch": alg_bytes,
                "units_per_build": units}

    # shortest-path extension on the resident labeling (outside the timed
    # steps: an extra build)
    paths = None
    if not args.no_paths:
        L = chl.build(row, col, w, order, stream=stream)
        paths = paths_measure(chl, L, c, (row, col, w), pairs, stream)
        L.free()

    directed = None if args.no_directed else directed_measure(chl, gg, stream)

    # end to end from host memory: upload of the CSR and the ranking, the
    # build, and the labeling copied back to host memory (the timed steps
    # above start with the inputs resident in HBM)
    e2e = None
    if not args.no_paths:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hd = [torch.from_numpy(c[f]).to(dev) for f in ("row_ptr", "col", "w", "order")]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        Le = chl.build(*hd, stream=stream)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        Le.export("cpu")
        t4 = time.perf_counter()
        Le.free()
        del hd
        e2e = {"upload_ms": round((t2 - t1) * 1e3, 3), "build_ms": round((t3 - t2) * 1e3, 3),
               "download_ms": round((t4 - t3) * 1e3, 3), "total_ms": round((t4 - t1) * 1e3, 3),
               "gteps_end_to_end": round(A / (t4 - t1) / 1e9, 4),
               "note": "pageable host arrays (numpy) -> device, chl_build, chl_labels_export to host"}

    # ceiling of the relaxation's memory operation: random atomic minima on
    # an array of the main phase's slot keys (roots in flight x n keys)
    atomics = None
    if not args.no_atomic_ceiling:
        kb = int(stats["key_bits"])
        words = int(stats["roots_in_flight"]) * c["n"]
        chl.microbench_atomic_min(words, kb, ops=1 << 24)
        rates = []
        for _ in range(3):
            done, ams = chl.microbench_atomic_min(words, kb, ops=1 << 28)
            rates.append(done / (ams / 1e3))
        build_kernel_s = per_launch_ms * nl / 1e3
        relax = gpu_arcs / build_kernel_s
        atomics = {"ceiling_atomic_min_per_s": round(max(rates), 1), "array_bytes": words * kb // 8, "key_bits": kb,
                   "tree_relaxations_per_s": round(relax, 1), "frac": round(relax / max(rates), 5),
                   "note": "relaxations = arcs relaxed by the tree kernels of one build (a key load and at most one "
                           "atomic minimum each) / their summed launch time; ceiling = best of 3 runs of 2^28 random "
                           "atomic minima (chl_microbench_atomic_min)"}

    # the same batched build without the common label table (PLaNT trees
    # alone, Section 4.2), for reference
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Lu = chl.build(row, col, w, order, prune_hubs=-1, stream=stream)
    torch.cuda.synchronize()
    unpruned_s = time.perf_counter() - t1
    unpruned_arcs = Lu.stats()["arcs"]
    Lu.free()
    # the unpruned build is tuned on its first call; time it again
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Lu = chl.build(row, col, w, order, prune_hubs=-1, stream=stream)
    torch.cuda.synchronize()
    unpruned_s = time.perf_counter() - t1
    Lu.free()

    # plain form (one root per cooperative launch, the whole device on one
    # tree): time the 64 head roots and a rank-stratified sample of 256 of
    # the others; the sum over the rest is estimated as sample time * stride
    n = c["n"]
    H, NS = 64, 256
    stride = (n - H) // NS
    tp = []
    for roots in ((0, H, 1), (H, NS, stride)) if not args.no_plain else ():
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Lp = chl.build(row, col, w, order, mode="plain", roots=roots, stream=stream)
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t1)
        Lp.free()
    plain_est_s = tp[0] + tp[1] * stride if tp else None

    # open-loop serving on the resident labeling: saturation throughput of the
    # server path, then a Poisson stream at half of it with two label builds
    # of other graphs arriving meanwhile
    serving = {"p50_us": None, "p99_us": None}
    if not args.no_serve:
        serving = serve_measure(chl, gg, c, row, col, w, order, stream, qout, q)

    large = large_workloads(chl, gg, stream) if args.large else None
    serving_full = serve_full(chl, gg, stream) if args.serve_full else None

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        tc = time.perf_counter()
        lab = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"], mode=oracle.MODE_PLANT, threads=threads)
        ct = time.perf_counter() - tc
        assert lab.total == Lc
        tq = time.perf_counter()
        qo = oracle.query(lab, c["pairs"])
        tq = time.perf_counter() - tq
        assert np.array_equal(qo, qout.cpu().numpy())
        model = next((l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")), "?")
        cpu = {"value": round(A / ct / 1e9, 4), "unit": "GTEPS", "cores": threads, "kind": "oracle",
               "sample": "full R-MAT scale-16 labeling (all 65,536 roots), %.1f s" % ct,
               "queries_per_s_1_thread": round(len(c["pairs"]) / tq, 1),
               "host": {"cpu": model, "nproc": os.cpu_count()}}

    out = {
        "metric": "CHL build time (s) + GTEPS; PPSD queries/s with p50/p99 latency, 1 MI355X",
        "value": round(gteps, 4), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total_s / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "R-MAT scale 16 (65,536 vertices, %d edges), int32 weights [1,1000], degree rank; "
                               "full canonical labeling + 10^6 uniform queries" % c["m"],
                   "mode": "batched", "roots_in_flight": stats["roots_in_flight"], "wg_size": stats["wg_size"],
                   "delta": stats["delta"], "key_bits": stats["key_bits"], "prune_hubs": stats["prune_hubs"]},
        "build_s": round(b_s, 4), "queries_per_s": round(qps, 1), "labels": Lc,
        "p50_us": serving["p50_us"], "p99_us": serving["p99_us"],
        "batched_unpruned": {"build_s": round(unpruned_s, 4), "gteps": round(A / unpruned_s / 1e9, 4),
                             "gpu_arcs": unpruned_arcs},
        "plain_form": None if plain_est_s is None else {
            "build_s_est": round(plain_est_s, 3), "gteps_est": round(A / plain_est_s / 1e9, 4),
            "method": "64 head roots + 256 rank-stratified roots (stride %d), sum = head + sample * stride" % stride},
        "serving": serving,
        "gpu_arcs": gpu_arcs,
        "oracle_arcs_unpruned": A,
        "oracle_arcs_method": units["arcs"],
        "method_gteps": round(units["arcs"] / b_s / 1e9, 4),
        "work_inflation": round(gpu_arcs / max(1, units["arcs"]), 3),
        "phases_ms": {"prep": round(stats["prep_ms"], 3), "prefix": round(stats["prefix_ms"], 3),
                      "main": round(stats["tree_ms"], 3), "assemble": round(stats["assemble_ms"], 3)},
        "roofline": roofline, "atomics": atomics, "cpu_baseline": cpu, "end_to_end": e2e,
        "paths": paths,
        "directed": directed,
    }
    if serving_full is not None:
        out["serving_full"] = serving_full
    if large is not None:
        out["large"] = large
    print(json.dumps(out))


if __name__ == "__main__":
    main()
