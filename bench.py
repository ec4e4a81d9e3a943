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
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_tree_batched_rmat16.json")
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form estimate")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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

    # roofline of the dominant kernel, the batched tree kernel: all its
    # production launches of one build (the prefix levels and the main
    # phase), timed with events on the build stream inside the library.
    # Algorithmic bytes = 16 per scanned arc + 16 per settled vertex + 8 per
    # label, with the units counted by the oracle's trees under the same
    # pruning configuration (tests/golden/workload_counts.json)
    g, pm = stats["prefix_roots"], stats["prune_hubs"]
    if g == 0:
        cfg = None
        units = {"arcs": A, "settled": S, "labels": Lc}
    else:
        cfg = next(v for k, v in counts.items() if isinstance(v, dict) and v.get("grown") == g
                   and v.get("pmain") == pm)
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
                "kernel": "k_tree_batched (production launches: prefix levels + main phase)",
                "kernel_ms": round(per_launch_ms, 3), "launches_per_build": nl,
                "alg_bytes_per_launch": alg_bytes,
                "units_per_build": units}

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

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        tc = time.perf_counter()
        lab = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"], mode=oracle.MODE_PLANT, threads=threads)
        ct = time.perf_counter() - tc
        assert lab.total == Lc
        cpu = {"value": round(A / ct / 1e9, 4), "unit": "GTEPS", "cores": threads, "kind": "oracle",
               "sample": "full R-MAT scale-16 labeling (all 65,536 roots), %.1f s" % ct}

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
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
