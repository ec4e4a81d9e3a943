"""Benchmark of the PLaNT CHL build and distance queries on one MI355X.

One step = the whole hot path over one batch of synthetic input: chl_build of
the complete canonical labeling of R-MAT scale 20 (1,048,576 vertices, the
largest single-GPU workload: validation, rank renumbering, the rank-prefix
pruning levels, the batched main phase, label assembly) followed by
chl_query on its 10^6 query pairs. Inputs (CSR, ranking, pairs) are resident
in device memory before the timed region starts.

value = method GTEPS = arcs scanned by the oracle's trees under the same
build schedule (the rank-prefix levels the build reports; counts in
tests/golden/workload_counts.json, keyed by that schedule) / median build
time / 1e9. The arcs of the oracle's unpruned trees, which the method never
scans, appear only in separately named fields.

The same run also measures the other workloads (64x64 grid, R-MAT 16,
1024x1024 grid with shortcuts), the full serving experiment (labelings of
R-MAT 16 and the large grid resident, 10^7 Poisson queries at three rates,
twice each, 16 build requests), directed R-MAT 16, the Hybrid construction
against PLaNT trees alone, shortest paths, the plain one-root-per-launch form,
an atomic-minimum reference and the CPU oracle.

Prints one JSON line. Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       [--sections headline,workloads,serving,directed,hybrid,paths,atomics,cpu]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "rmat20"
COUNTS = os.path.join(ROOT, "tests", "golden", "workload_counts.json")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_tree_%s.json")
# the tree kernels and the host code that picks their launches: byte counters
# taken for other sources no longer describe the kernels
TREE_SRC = [os.path.join(ROOT, "paper_1907_00140_amd", "csrc", f) for f in ("tree.hip", "api.cpp")]
SECTIONS = ("headline", "workloads", "serving", "directed", "hybrid", "paths", "atomics", "cpu")
NAMES = {
    "grid64": "64x64 grid (4,096 vertices, 8,064 edges), int32 weights [1,100], degree rank",
    "rmat16": "R-MAT scale 16 (65,536 vertices, %d edges), int32 weights [1,1000], degree rank",
    "grid1024d": "1024x1024 grid + 5%% diagonal shortcuts (1,048,576 vertices, %d edges), int32 weights "
                 "[1,10000], degree rank",
    "rmat20": "R-MAT scale 20 (1,048,576 vertices, %d edges), int32 weights [1,65536], degree rank",
}


def wname(name, m):
    return NAMES[name] % m if "%d" in NAMES[name] else NAMES[name]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def src_sha():
    h = hashlib.sha256()
    for f in TREE_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def schedule_key(st):
    return "%s/%d" % (",".join(str(int(b)) for b in st["level_end"]), int(st["prune_hubs"]))


def method_units(counts, name, st):
    """The oracle's work units (arcs, settled, labels) under the schedule the
    build ran, or None when that schedule was not counted."""
    e = counts.get(name, {}).get("schedules", {}).get(schedule_key(st))
    if e is None:
        return None
    return {k: e["head"][k] + e["rest"][k] for k in ("arcs", "settled", "labels")}


def alg_bytes(u):
    """Algorithmic bytes of the tree phase: 16 per scanned arc (8 B arc + 8 B
    key access), 16 per settled vertex (row offsets + key), 8 per label."""
    return 16 * u["arcs"] + 16 * u["settled"] + 8 * u["labels"]


def dev_inputs(c, dev):
    import torch
    return [torch.from_numpy(c[f]).to(dev) for f in ("row_ptr", "col", "w", "order")]


def timed_builds(chl, d, reps, stream, **kw):
    """Median host time of `reps` builds (the caller has built once to tune);
    returns (median s, runs, stats of the last, its labels handle)."""
    import numpy as np
    import torch
    times, L, st = [], None, None
    for i in range(reps):
        if L is not None:
            L.free()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L = chl.build(*d, stream=stream, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
    st = L.stats(per_root=not kw.get("directed", False))
    return float(np.median(times)), times, st, L


def label_shape(L, st, n):
    """Label-size histogram (log2 bins of |L_v|), early-termination rate and
    the exploration overhead Psi (vertex relaxations per label) over windows
    of 64 consecutive roots (the paper's measure over recent trees)."""
    import numpy as np
    sizes = np.diff(L.offsets())
    bins = np.bincount(np.floor(np.log2(np.maximum(sizes, 1))).astype(np.int64))
    pr = st["per_root"]
    k = 64
    m = (len(pr) // k) * k
    psi = pr[:m, 0].reshape(-1, k).sum(1) / np.maximum(1, pr[:m, 2].reshape(-1, k).sum(1))
    return {"label_size_hist_log2": {"[%d,%d)" % (1 << i, 2 << i): int(v) for i, v in enumerate(bins) if v},
            "max_label_size": int(sizes.max()), "als": round(float(sizes.mean()), 2),
            "early_termination_rate": round(st["early_trees"] / n, 4),
            "settled_per_tree": round(st["settled"] / n, 1),
            "psi_64_root_windows": {"mean": round(float(psi.mean()), 2),
                                    "p50": round(float(np.percentile(psi, 50)), 2),
                                    "p99": round(float(np.percentile(psi, 99)), 2),
                                    "max": round(float(psi.max()), 2),
                                    "note": "GPU vertex relaxations / labels per window of 64 consecutive roots"}}


def level_table(counts, name, st):
    """Per pruning level: roots, workgroups per tree, device time and the
    oracle's work under the same schedule (algorithmic GB/s per level)."""
    e = counts.get(name, {}).get("schedules", {}).get(schedule_key(st))
    rows = []
    lo = 0
    for i, (end, ms, tw) in enumerate(zip(st["level_end"], st["level_ms"], st["level_teams"])):
        r = {"roots": [lo, int(end)], "team_wgs": int(tw), "ms": round(ms, 3)}
        if "per_root" in st:
            r["gpu_arcs"] = int(st["per_root"][lo:int(end), 1].sum())
        if e is not None and i < len(e["levels"]):
            u = e["levels"][i][2]
            r["oracle_arcs"] = u["arcs"]
            r["alg_gbs"] = round(alg_bytes(u) / (ms / 1e3) / 1e9, 1) if ms > 0 else None
        rows.append(r)
        lo = int(end)
    if "per_root" in st and st["level_end"]:
        r = {"roots": [lo, int(st["n"])], "main_phase": True, "gpu_arcs": int(st["per_root"][lo:, 1].sum())}
        if e is not None:
            r["oracle_arcs"] = e["rest"]["arcs"]
        rows.append(r)
    return rows


def queries_per_s(L, pairs, stream, reps=3):
    import numpy as np
    import torch
    qo = L.query(pairs, stream=stream)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.query(pairs, out=qo, stream=stream)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t1)
    return pairs.shape[0] / float(np.median(ts)), qo


def plain_form(chl, d, n, head, strata, stream, full=False):
    """The plain one-root-per-launch form (the whole device grows one tree per
    cooperative launch, unpruned): measured outright when `full` (every root
    grown, in 8 consecutive root ranges so that each range reports when it
    ends; the time is the sum of the 8 builds, their labels add up to the
    complete labeling's), else the `head` first roots plus `strata`
    rank-stratified roots, the rest extrapolated as sample time * stride."""
    import torch
    if full:
        parts = 8
        step = (n + parts - 1) // parts
        total, labels = 0.0, 0
        for lo in range(0, n, step):
            cnt = min(step, n - lo)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            Lp = chl.build(*d, mode="plain", roots=(lo, cnt, 1), stream=stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            total += dt
            labels += Lp.info()[1]
            Lp.free()
            say("plain form: roots [%d, %d) in %.1f s" % (lo, lo + cnt, dt))
        return {"build_s": round(total, 3), "labels": labels,
                "method": "complete build, measured: every root grown, in 8 consecutive root ranges timed one "
                          "after the other"}
    stride = (n - head) // strata
    tp = []
    for roots in ((0, head, 1), (head, strata, stride)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Lp = chl.build(*d, mode="plain", roots=roots, stream=stream)
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t1)
        Lp.free()
    return {"build_s_est": round(tp[0] + tp[1] * stride, 3),
            "method": "estimate: %d head roots (%.3f s) + %d rank-stratified roots (stride %d, %.3f s) x stride"
                      % (head, tp[0], strata, stride, tp[1])}


def headline(chl, gg, counts, args, dev, stream):
    """R-MAT scale 20: warmup builds (the first tunes), then exactly K timed
    steps of build + 10^6 queries, each bracketed by device synchronisation."""
    import numpy as np
    import torch
    c = gg.make_config(WORKLOAD)
    d = dev_inputs(c, dev)
    pairs = torch.from_numpy(c["pairs"]).to(dev)
    qout = torch.empty(pairs.shape[0], dtype=torch.int64, device=dev)
    for _ in range(args.warmup):
        L = chl.build(*d, stream=stream)
        L.query(pairs, out=qout, stream=stream)
        L.free()
    torch.cuda.synchronize()
    build_ms, query_ms, kern, st, L = [], [], [], None, None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if L is not None:
            L.free()
        tb = time.perf_counter()
        L = chl.build(*d, stream=stream)
        torch.cuda.synchronize()
        tq = time.perf_counter()
        L.query(pairs, out=qout, stream=stream)
        torch.cuda.synchronize()
        te = time.perf_counter()
        build_ms.append((tq - tb) * 1e3)
        query_ms.append((te - tq) * 1e3)
        s = L.stats()
        kern.append((s["kernel_ms"], s["kernel_launches"]))
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    st = L.stats(per_root=True)
    b_s = float(np.median(build_ms)) / 1e3
    units = method_units(counts, WORKLOAD, st)
    if units is None:
        sys.exit("no oracle work counts for the schedule %s of %s: run python tests/golden/make_workload_counts.py "
                 "%s --schedule %s" % (schedule_key(st), WORKLOAD, WORKLOAD, schedule_key(st)))
    assert st["labels"] == units["labels"], "label count differs from the oracle's"
    gpu_arcs = int(st["per_root"][:, 1].sum())
    # roofline of the dominant kernels, the tree kernels (teams for the first
    # levels, tree groups for the levels of 64 to 256 roots, the batched kernel
    # for the wider levels and the main phase):
    # every production launch of a build, timed with HIP events on the build
    # stream inside the library
    kms = float(np.median([k[0] for k in kern]))
    nl = int(np.median([k[1] for k in kern]))
    per_launch_ms = kms / nl
    ab = alg_bytes(units) / nl
    achieved = ab / (per_launch_ms / 1e3) / 1e9
    traffic = None
    tf = TRAFFIC % WORKLOAD
    if os.path.exists(tf):
        tr = json.load(open(tf))
        if tr.get("tree_src_sha") == src_sha() and tr.get("schedule") == schedule_key(st):
            traffic = tr.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "tree kernels k_tree_team + k_tree_group + k_tree_batched (every production launch of a "
                          "build: team levels, group levels, wide levels, main phase)",
                "kernel_ms": round(per_launch_ms, 3), "launches_per_build": nl, "alg_bytes_per_launch": ab,
                "units_per_build": units}
    qps = pairs.shape[0] / (float(np.median(query_ms)) / 1e3)
    oracle_unpruned = counts.get(WORKLOAD, {}).get("unpruned")
    h = {"c": c, "d": d, "pairs": pairs, "qout": qout, "L": L, "st": st,
         "line": {"value": round(units["arcs"] / b_s / 1e9, 4), "ms_per_step": round(total_s / args.steps * 1e3, 3),
                  "build_s": round(b_s, 4), "build_s_runs": [round(x / 1e3, 4) for x in build_ms],
                  "queries_per_s": round(qps, 1), "labels": int(st["labels"]),
                  "oracle_arcs_method": units["arcs"], "gpu_arcs": gpu_arcs,
                  "work_inflation": round(gpu_arcs / max(1, units["arcs"]), 3),
                  "schedule": schedule_key(st), "key_bits": int(st["key_bits"]),
                  "phases_ms": {"prep": round(st["prep_ms"], 3), "prefix": round(st["prefix_ms"], 3),
                                "main": round(st["tree_ms"], 3), "assemble": round(st["assemble_ms"], 3)},
                  "levels": level_table(counts, WORKLOAD, st),
                  "unpruned_equivalent_gteps": (round(oracle_unpruned["arcs"] / b_s / 1e9, 2)
                                                if oracle_unpruned else None),
                  "roofline": roofline}}
    h["line"].update(label_shape(L, st, c["n"]))
    return h


def workload(chl, gg, counts, name, dev, stream, reps, plain=None):
    """One of the other workloads: median of `reps` builds after one that
    tunes, 10^6 (10^4 for the small grid) queries, method GTEPS."""
    import torch
    c = gg.make_config(name)
    d = dev_inputs(c, dev)
    pairs = torch.from_numpy(c["pairs"]).to(dev)
    L = chl.build(*d, stream=stream)
    torch.cuda.synchronize()
    L.free()
    b, runs, st, L = timed_builds(chl, d, reps, stream)
    qps, _ = queries_per_s(L, pairs, stream)
    units = method_units(counts, name, st)
    r = {"workload": wname(name, c["m"]), "n": c["n"], "edges": c["m"],
         "build_s": round(b, 4), "build_s_runs": [round(t, 4) for t in runs], "labels": int(st["labels"]),
         "queries": int(pairs.shape[0]), "queries_per_s": round(qps, 1), "schedule": schedule_key(st),
         "key_bits": int(st["key_bits"]), "roots_in_flight": st["roots_in_flight"], "wg_size": st["wg_size"],
         "delta": st["delta"], "gpu_arcs": int(st["arcs"]),
         "phases_ms": {"prep": round(st["prep_ms"], 2), "prefix": round(st["prefix_ms"], 2),
                       "main": round(st["tree_ms"], 2), "assemble": round(st["assemble_ms"], 2)},
         "kernel_ms": round(st["kernel_ms"], 3), "kernel_launches": int(st["kernel_launches"])}
    if units is not None:
        assert st["labels"] == units["labels"], "%s: label count differs from the oracle's" % name
        r["method_gteps"] = round(units["arcs"] / b / 1e9, 4)
        r["oracle_arcs_method"] = units["arcs"]
        r["work_inflation"] = round(st["arcs"] / max(1, units["arcs"]), 3)
        ab = alg_bytes(units)
        r["tree_alg_gbs"] = round(ab / (st["kernel_ms"] / 1e3) / 1e9, 2)
        r["tree_hbm_frac"] = round(ab / (st["kernel_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 5)
    up = counts.get(name, {}).get("unpruned")
    if up is not None:
        r["unpruned_equivalent_gteps"] = round(up["arcs"] / b / 1e9, 2)
    r["levels"] = level_table(counts, name, st)
    r.update(label_shape(L, st, c["n"]))
    if plain is not None:
        r["plain_form"] = plain_form(chl, d, c["n"], plain[0], plain[1], stream, full=plain[2])
        p = r["plain_form"]
        if "labels" in p:
            assert p["labels"] == st["labels"], "%s: the plain form's labels differ in number" % name
        if name.startswith("rmat"):
            # like for like: the plain form grows unpruned trees, so it is set
            # beside the batched form without rank-prefix pruning as well
            Lu = chl.build(*d, stream=stream, prune_hubs=-1)
            Lu.free()
            bu, _, _, Lu = timed_builds(chl, d, 2, stream, prune_hubs=-1)
            Lu.free()
            p["batched_unpruned_s"] = round(bu, 4)
            p["unpruned_batched_speedup"] = round(p.get("build_s", p.get("build_s_est")) / bu, 1)
        ps = p.get("build_s", p.get("build_s_est"))
        r["plain_form"]["batched_speedup"] = round(ps / b, 1)
    say("workload", name, json.dumps({k: v for k, v in r.items() if k not in ("levels",)}))
    return r, L, c


def serve_full(chl, gg, stream, resident, reps=2):
    """The serving workload: the labelings of R-MAT 16 and of the 1024x1024
    grid resident, 10^7 uniform query pairs (half on each graph, one Poisson
    stream) at 0.25, 0.5 and 0.9 of the server path's saturated rate, each
    rate run `reps` times, with 16 build requests (R-MAT scales 10..16, seeds
    500+i, weights [1,1000]) arriving over the stream and admitted by HBM
    footprint. Every answer is checked against a direct chl_query of the same
    labeling, every served build against the same build alone."""
    import numpy as np
    import torch
    from paper_1907_00140_amd import serve
    dev = torch.device("cuda:0")
    qsets, direct = [], []
    for k, (c, L) in enumerate(resident):
        pairs = gg.query_pairs(c["n"], 5_000_000, 702 + k)
        direct.append(L.query(torch.from_numpy(pairs).to(dev), stream=stream).cpu().numpy())
        qsets.append(pairs)
    res = [L for _, L in resident]
    mk = lambda: serve.Server(mem_budget=64 << 30, max_batch=1 << 16, build_streams=2, build_wg=128)
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
    say("serving: saturated %.3g queries/s" % sat)
    bcfg = [gg.make_config("rmat%d_%d" % (10 + i % 7, i)) for i in range(16)]
    alone = []
    for c in bcfg:
        Lb = chl.build(c["row_ptr"], c["col"], c["w"], c["order"], stream=stream)
        alone.append([x.numpy() for x in Lb.export("cpu")])
        Lb.free()
    out = {"resident": ["rmat16", "grid1024d"], "queries": int(sum(len(p) for p in qsets)),
           "saturated_qps": round(sat, 1), "builds": len(bcfg), "rates": []}
    for f in (0.25, 0.5, 0.9):
        rate = f * sat
        span = sum(len(p) for p in qsets) / rate
        row = {"fraction": f, "rate_qps": round(rate, 1), "runs": []}
        for rep in range(reps):
            tb = gg.poisson_arrivals(16, 16 / span, 900 + int(100 * f) + 7 * rep)
            srv, tks, btk, wall = serve.open_loop(mk, res, qsets, rate, builds=list(zip(bcfg, tb)),
                                                  seed=int(100 * f) + 1000 * rep)
            for tk, ref in zip(tks, direct):
                assert np.array_equal(tk.out, ref), "served answers differ from chl_query"
            for b, ref in zip(btk, alone):
                assert b.status.value == 0, "build request failed: %d" % b.status.value
                got = [x.numpy() for x in srv.labels(b.gid.value).export("cpu")]
                assert all(np.array_equal(x, y) for x, y in zip(got, ref)), "served build differs from alone"
            lat = np.concatenate([tk.lat for tk in tks])
            tend = max(float(np.max(tk.t + tk.lat)) for tk in tks)
            blat = np.array([b.lat.value for b in btk])
            tr = srv.trace()
            qb, bb = tr[tr[:, 0] == 0], tr[tr[:, 0] == 1]
            dev_ms = (qb[:, 3] - qb[:, 2]) * 1e3
            wait_ms = (qb[:, 2] - qb[:, 1]) * 1e3
            slow = dev_ms > 1.0
            # a slow batch overlapped a build when some build ran (admitted,
            # not yet complete) while the batch was on the device
            ov = np.array([bool(((bb[:, 2] < b[3]) & (bb[:, 3] > b[2])).any()) for b in qb[slow]]) \
                if slow.any() and len(bb) else np.zeros(int(slow.sum()), bool)
            anatomy = {"batches": int(len(qb)),
                       "device_ms": {"p50": round(float(np.percentile(dev_ms, 50)), 3),
                                     "p99": round(float(np.percentile(dev_ms, 99)), 3),
                                     "max": round(float(dev_ms.max()), 3)},
                       "dispatch_wait_ms": {"p50": round(float(np.percentile(wait_ms, 50)), 3),
                                            "p99": round(float(np.percentile(wait_ms, 99)), 3),
                                            "max": round(float(wait_ms.max()), 3)},
                       "batches_over_1ms_on_device": int(slow.sum()),
                       "of_which_during_a_build": int(ov.sum())}
            row["runs"].append({"achieved_qps": round(len(lat) / tend, 1),
                                "p50_us": round(float(np.percentile(lat, 50)) * 1e6, 2),
                                "p99_us": round(float(np.percentile(lat, 99)) * 1e6, 2),
                                "p999_us": round(float(np.percentile(lat, 99.9)) * 1e6, 2),
                                "per_graph_p99_us": [round(float(np.percentile(tk.lat, 99)) * 1e6, 2) for tk in tks],
                                "build_latency_s": {"p50": round(float(np.median(blat)), 4),
                                                    "max": round(float(blat.max()), 4)},
                                "batch_anatomy": anatomy,
                                "wall_s": round(wall, 3)})
            srv.close()
            say("serving:", f, json.dumps(row["runs"][-1]))
        out["rates"].append(row)
    return out


def directed_measure(chl, gg, counts, stream, reps=3):
    """Directed R-MAT scale 16 (the generator's samples read as arcs): out-
    and in-labels in one build (chl_build_directed), median of `reps` builds
    after one that tunes, and 10^6 queries. method GTEPS = arcs of the
    oracle's trees on the combined graph under the same schedule / time."""
    import torch
    dev = torch.device("cuda:0")
    name = "rmat16dir"
    c = gg.make_config(name)
    d = dev_inputs(c, dev)
    pairs = torch.from_numpy(c["pairs"]).to(dev)
    L = chl.build(*d, directed=True, stream=stream)
    torch.cuda.synchronize()
    L.free()
    b, runs, st, L = timed_builds(chl, d, reps, stream, directed=True)
    qps, _ = queries_per_s(L, pairs, stream)
    L.free()
    r = {"workload": "directed R-MAT scale 16 (65,536 vertices, %d arcs), int32 weights [1,1000], total-degree "
                     "rank; out- and in-labels + 10^6 uniform queries" % c["m"],
         "build_s": round(b, 4), "build_s_runs": [round(t, 4) for t in runs], "labels": int(st["labels"]),
         "gpu_arcs": int(st["arcs"]), "queries_per_s": round(qps, 1), "schedule": schedule_key(st)}
    units = method_units(counts, name, st)
    if units is not None:
        r["method_gteps"] = round(units["arcs"] / b / 1e9, 4)
        r["oracle_arcs_method"] = units["arcs"]
        r["work_inflation"] = round(st["arcs"] / units["arcs"], 3)
    up = counts.get(name, {}).get("unpruned")
    if up is not None:
        r["unpruned_equivalent_gteps"] = round(up["arcs"] / b / 1e9, 2)
    say("directed:", json.dumps(r))
    return r


def hybrid_measure(chl, gg, stream, reps=2, psi_th=100):
    """The Hybrid construction (Section 4.2.1, Psi_th = 100 as the paper sets
    for scale-free graphs) against PLaNT trees for every root, on R-MAT scale
    16 under two rankings where the trees explore far more than they label:
    a random ranking (seed 77), rank-prefix pruning at its default, and the
    degree ranking with rank-prefix pruning off (the paper's PLaNT). Median
    of `reps` builds each after one that tunes; the two labelings must be
    equal (compared on the device)."""
    import torch
    dev = torch.device("cuda:0")
    c = gg.make_config("rmat16")
    out = []
    for rank, kw in (("random rank (seed 77)", {}), ("degree rank, rank-prefix pruning off", {"prune_hubs": -1})):
        order = gg.random_rank(c["n"], 77) if rank.startswith("random") else c["order"]
        d = dev_inputs(dict(c, order=order), dev)
        r = {"workload": "R-MAT scale 16 (65,536 vertices, %d edges), %s" % (c["m"], rank), "psi_th": psi_th}
        labs = []
        for name, extra in (("plant", {}), ("hybrid", {"hybrid_psi": psi_th})):
            L = chl.build(*d, stream=stream, **kw, **extra)
            torch.cuda.synchronize()
            L.free()
            b, runs, st, L = timed_builds(chl, d, reps, stream, **kw, **extra)
            r[name + "_build_s"] = round(b, 4)
            r[name + "_build_s_runs"] = [round(t, 4) for t in runs]
            r[name + "_vertex_relaxations"] = int(st["settled"])
            r[name + "_arcs"] = int(st["arcs"])
            if name == "hybrid":
                r.update({"switch_root": int(st["hybrid_switch"]), "psi_at_switch": round(st["hybrid_psi"], 1),
                          "supersteps": int(st["hybrid_supersteps"]), "pruned_tree_labels": int(st["hybrid_emitted"]),
                          "cleaned_away": int(st["hybrid_removed"]), "clean_ms": round(st["hybrid_clean_ms"], 2)})
            r["labels"] = int(st["labels"])
            labs.append(L.export(dev, stream=stream))
            torch.cuda.synchronize()
            L.free()
        r["same_labels"] = all(bool(torch.equal(x, y)) for x, y in zip(*labs))
        assert r["same_labels"], "the Hybrid labeling differs from PLaNT's"
        r["speedup"] = round(r["plant_build_s"] / r["hybrid_build_s"], 2)
        del labs, d
        say("hybrid:", json.dumps(r))
        out.append(r)
    return out


def paths_measure(chl, L, c, d, pairs, stream, reps=3):
    """Shortest-path extension on a resident labeling: the parents kernel
    (HIP events on the build stream, median of reps) against its algorithmic
    bytes, and path queries (hop counts + path vertices). Algorithmic bytes of
    the parents kernel: 4 per lookup of a label's hub in a neighbour's list
    (sum over v of deg(v) * |L_v|), 16 per label (hub and distance read,
    parent and slot written), 8 per arc and 32 per vertex."""
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


def atomic_ceiling(chl, st, n, gpu_arcs, kernel_s):
    """Ceiling of the relaxation's memory operation: random atomic minima on
    an array of the main phase's slot keys (roots in flight x n keys)."""
    kb = int(st["key_bits"])
    words = int(st["roots_in_flight"]) * n
    chl.microbench_atomic_min(words, kb, ops=1 << 24)
    rates = []
    for _ in range(3):
        done, ams = chl.microbench_atomic_min(words, kb, ops=1 << 28)
        rates.append(done / (ams / 1e3))
    relax = gpu_arcs / kernel_s
    return {"ceiling_atomic_min_per_s": round(max(rates), 1), "array_bytes": words * kb // 8, "key_bits": kb,
            "tree_relaxations_per_s": round(relax, 1), "frac": round(relax / max(rates), 5),
            "note": "relaxations = arcs relaxed by the tree kernels of one build (a key load and at most one atomic "
                    "minimum each) / their summed launch time; ceiling = best of 3 runs of 2^28 random atomic minima"}


def cpu_baseline(gg, counts, qout_c2=None, c2=None):
    """The oracle on the host cores, on a bounded sample of the headline
    workload: its pruned PLaNT trees (the method the GPU runs) of the roots at
    rank positions [0, 64) of R-MAT scale 20 under the build's first three
    levels ([0, 16) unpruned, [16, 32) and [32, 64) pruned by the complete
    labels of the levels before), i.e. the largest trees of the build. Also
    the CPU query rate: the oracle's sorted-list merge on the R-MAT 16
    labeling, 10^6 pairs split over all threads."""
    import numpy as np
    import oracle
    threads = min(16, os.cpu_count() or 1)
    c = gg.make_config(WORKLOAD)
    lv = [16, 32, 64]
    t = time.perf_counter()
    stats = oracle.chl_pruned_roots(c["row_ptr"], c["col"], c["w"], c["order"], list(range(64)), levels=lv,
                                    pmain=64, threads=threads)
    ct = time.perf_counter() - t
    arcs = int(stats[:, 1].sum())
    e = counts.get(WORKLOAD, {}).get("schedules", {})
    full = next((v for v in e.values() if v["bounds"][:3] == lv), None)
    if full is not None:
        want = sum(x[2]["arcs"] for x in full["levels"][:3])
        assert arcs == want, "oracle sample arcs %d != counted %d" % (arcs, want)
    model = next((l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")), "?")
    r = {"value": round(arcs / ct / 1e9, 4), "unit": "GTEPS", "cores": threads, "kind": "oracle",
         "sample": "pruned PLaNT trees (oracle.chl_pruned) of the 64 most important roots of R-MAT scale 20 under "
                   "the levels [0,16),[16,32),[32,64): %d arcs, %d labels in %.1f s" % (arcs, int(stats[:, 2].sum()), ct),
         "host": {"cpu": model, "nproc": os.cpu_count()}}
    if c2 is not None:
        lab = oracle.chl_pruned(c2["row_ptr"], c2["col"], c2["w"], c2["order"], levels=[16, 128, 1024], pmain=1024,
                                threads=threads)
        pairs = c2["pairs"]
        chunks = np.array_split(pairs, threads)
        t = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            qo = np.concatenate(list(ex.map(lambda p: oracle.query(lab, p), chunks)))
        tq = time.perf_counter() - t
        if qout_c2 is not None:
            assert np.array_equal(qo, qout_c2), "oracle queries differ from the GPU's"
        r["queries_per_s"] = round(len(pairs) / tq, 1)
        r["queries_sample"] = "R-MAT 16 labeling, 10^6 uniform pairs, sorted-list merge on %d threads" % threads
    return r


def main():
    global WORKLOAD
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma list of " + ",".join(SECTIONS) + " (headline always runs)")
    ap.add_argument("--plain-full", default="",
                    help="workload whose plain one-root-per-launch form is measured outright (e.g. rmat16; takes "
                         "minutes); the others are estimated from root samples")
    ap.add_argument("--headline", default=WORKLOAD, choices=sorted(NAMES),
                    help="workload of the timed steps (default: R-MAT scale 20; others for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(every tree is independent; see the sharding design in the docs)", file=sys.stderr)
        sys.exit(2)
    sec = set(s for s in args.sections.split(",") if s) | {"headline"}

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
    counts = json.load(open(COUNTS))
    stream = torch.cuda.current_stream()
    WORKLOAD = args.headline
    chl.load()
    # where the library is mapped (stack addresses in a profiler's or a
    # crash report can then be attributed to it)
    with open("/proc/self/maps") as f:
        segs = [l.split()[0] for l in f if l.rstrip().endswith("libchl.so")]
    if segs:
        say("libchl.so mapped at %s-%s" % (segs[0].split("-")[0], segs[-1].split("-")[1]))

    say("headline: %s, %d warmup + %d steps" % (WORKLOAD, args.warmup, args.steps))
    H = headline(chl, gg, counts, args, dev, stream)
    line = H["line"]
    say("headline:", json.dumps({k: line[k] for k in ("value", "build_s", "queries_per_s", "schedule")}))

    # the plain one-root-per-launch form on the headline workload: the
    # unpruned tree of each root grown by the whole device, estimated from
    # the 16 most important roots and 64 rank-stratified ones
    plain4 = None
    if "workloads" in sec:
        plain4 = plain_form(chl, H["d"], H["c"]["n"], 16, 64, stream, full=args.plain_full == WORKLOAD)
        ps = plain4.get("build_s", plain4.get("build_s_est"))
        plain4["batched_speedup"] = round(ps / line["build_s"], 1)

    paths = None
    if "paths" in sec:
        paths = paths_measure(chl, H["L"], H["c"], H["d"], H["pairs"], stream)
    atomics = None
    if "atomics" in sec:
        atomics = atomic_ceiling(chl, H["st"], H["c"]["n"], line["gpu_arcs"],
                                 line["roofline"]["kernel_ms"] * line["roofline"]["launches_per_build"] / 1e3)
    H["L"].free()
    del H["d"], H["pairs"]

    others, keep = {}, {}
    if "workloads" in sec or "serving" in sec:
        plan = [("grid64", 5, (64, 256)), ("rmat16", 5, (64, 256)), ("grid1024d", 3, (16, 64))]
        for name, reps, pl in plan:
            if "workloads" not in sec and name == "grid64":
                continue
            full = args.plain_full == name
            r, L, c = workload(chl, gg, counts, name, dev, stream, reps,
                               plain=(pl[0], pl[1], full) if "workloads" in sec else None)
            others[name] = r
            if name in ("rmat16", "grid1024d") and "serving" in sec:
                keep[name] = (c, L)
            else:
                L.free()
    serving = None
    if "serving" in sec:
        serving = serve_full(chl, gg, stream, [keep["rmat16"], keep["grid1024d"]])
    qout_c2 = None
    c2 = None
    if "rmat16" in keep:
        c2 = keep["rmat16"][0]
        qout_c2 = keep["rmat16"][1].query(c2["pairs"], stream=stream).cpu().numpy()
    for c, L in keep.values():
        L.free()
    directed = directed_measure(chl, gg, counts, stream) if "directed" in sec else None
    hybrid = hybrid_measure(chl, gg, stream) if "hybrid" in sec else None
    cpu = cpu_baseline(gg, counts, qout_c2, c2 if c2 is not None else gg.make_config("rmat16")) \
        if "cpu" in sec and WORKLOAD == "rmat20" else None

    p50 = p99 = None
    if serving is not None:
        mid = serving["rates"][1]["runs"]
        p50 = round(sum(r["p50_us"] for r in mid) / len(mid), 2)
        p99 = round(max(r["p99_us"] for r in mid), 2)
    out = {
        "metric": "CHL build time (s) + GTEPS; PPSD queries/s with p50/p99 latency, 1 MI355X",
        "value": line["value"], "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": line["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64" if line["key_bits"] == 64 else "u32", "data": "synthetic",
        "config": {"workload": wname(WORKLOAD, H["c"]["m"]) + "; complete canonical labeling (chl_build, "
                               "batched form, rank-prefix pruning) + 10^6 uniform queries per step",
                   "mode": "batched", "schedule": line["schedule"],
                   "roots_in_flight": H["st"]["roots_in_flight"], "wg_size": H["st"]["wg_size"],
                   "delta": H["st"]["delta"], "key_bits": line["key_bits"], "prune_hubs": H["st"]["prune_hubs"]},
        "value_definition": "method GTEPS: arcs scanned by the oracle's PLaNT trees under the build's own "
                            "rank-prefix schedule / median build time",
        "p50_us": p50, "p99_us": p99,
        "roofline": line.pop("roofline"), "cpu_baseline": cpu,
    }
    for k, v in line.items():
        if k not in ("value", "ms_per_step"):
            out[k] = v
    out["plain_form"] = plain4
    out["workloads"] = others or None
    out["serving"] = serving
    out["directed"] = directed
    out["hybrid"] = hybrid
    out["paths"] = paths
    out["atomics"] = atomics
    print(json.dumps(out))


if __name__ == "__main__":
    main()
