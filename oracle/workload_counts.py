"""Write tests/golden/workload_counts.json: the oracle's work counts (arcs
scanned A, vertices settled S, labels L) of the early-terminating trees of
every root, for the named workloads. These are the algorithmic work units of
the build (used for GTEPS and the roofline's algorithmic bytes). Calls only
the oracle and the input generators.

Usage: python -m oracle.workload_counts [--pruned-only | --no-levels] [name ...]
(directed workloads, e.g. rmat16dir: both directions, unpruned)
(--pruned-only skips the unpruned trees, whose count takes hours on the
million-vertex R-MAT graph; --no-levels skips the pruned trees, which the
build does not use on grids and whose prefix queries over grid-sized label
sets take hours.)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "workload_counts.json")


def _sums(st, lo, hi):
    """Work totals of the roots at rank positions [lo, hi)."""
    return {"arcs": int(st[lo:hi, 1].sum()), "settled": int(st[lo:hi, 0].sum()),
            "labels": int(st[lo:hi, 2].sum()), "early_trees": int(st[lo:hi, 3].sum())}


LEVELS = [16, 128, 1024, 4096]
LEVEL0 = 16
LEVEL_LABELS_X2 = 1 << 21


def level_bounds(labels_per_root, gmax, first=None):
    """The pruning-level schedule of the batched build: roots [0, 16) first;
    after a level whose roots have at least 2^21 labels in total the next
    level is twice as large a prefix, else eight times, up to gmax; `first`,
    when given, is the factor of the first pruned level instead (4 for a
    directed build's combined graph). Labels per root do not depend on the
    schedule, so any run's counts fix it."""
    g = min(LEVEL0, gmax)
    lv = [g]
    lab = int(labels_per_root[0:g].sum())
    while g < gmax:
        f = first if first and g == LEVEL0 else (2 if lab >= LEVEL_LABELS_X2 else 8)
        g2 = min(gmax, f * g)
        lab = int(labels_per_root[g:g2].sum())
        lv.append(g2)
        g = g2
    return lv


def counts_directed(name, threads=None):
    """Directed workloads: the unpruned early-terminating trees of every root
    along the arcs (in-labels) and on the reversed graph (out-labels); the
    totals add both ("in" and "out" keep each)."""
    c = gg.make_config(name)
    n = int(c["n"])
    out = {"n": n, "m": int(c["m"]), "threads": threads or min(16, os.cpu_count() or 1), "directed": True}
    t = time.time()
    lo, li = oracle.chl_directed(c["row_ptr"], c["col"], c["w"], c["order"], threads=threads)
    out["oracle_s"] = round(time.time() - t, 2)
    out["out"], out["in"] = _sums(lo.stats, 0, n), _sums(li.stats, 0, n)
    for k in ("arcs", "settled", "labels", "early_trees"):
        out[k] = out["out"][k] + out["in"][k]
    # the library's directed build: one build over the combined graph (the
    # graph and its reversal, 2n vertices, ranks interleaved) with the
    # rank-prefix levels of the undirected build
    r2, c2, w2, o2 = oracle.combined_directed(c["row_ptr"], c["col"], c["w"], c["order"])
    n2 = 2 * n
    gmax = min(LEVELS[-1], max(64, n2 // 64), n2 // 2)
    lv = [g for g in LEVELS if g < gmax] + [gmax]
    t = time.time()
    p = oracle.chl_pruned(r2, c2, w2, o2, levels=lv, pmain=lv[-1], half=n, threads=threads)
    lv2 = level_bounds(p.stats[:, 2], gmax, first=4)
    if lv2 != lv:
        lv = lv2
        p = oracle.chl_pruned(r2, c2, w2, o2, levels=lv, pmain=lv[-1], half=n, threads=threads)
    assert p.total == out["labels"]
    out["oracle_pruned_s"] = round(time.time() - t, 2)
    out["levels%d" % lv[-1]] = {"grown": lv[-1], "pmain": lv[-1], "head": _sums(p.stats, 0, lv[-1]),
                                "rest": _sums(p.stats, lv[-1], n2), "bounds": lv, "combined": True,
                                "levels": [[a, b, _sums(p.stats, a, b)] for a, b in zip([0] + lv[:-1], lv)]}
    return out


def counts(name, threads=None, pruned_only=False, levels=True):
    """Unpruned totals, and the work split (roots grown before the main
    phase / main phase) of each configuration the library's batched build
    can run: no pruning ("unpruned"), the 16 unpruned probe-level roots
    followed by unpruned trees ("split16"), and pruning in the levels of
    level_bounds() up to the build's default prefix, min(4096, max(64, n/64),
    n/2) hubs, with the main phase pruned by that whole prefix
    ("levels<prefix>")."""
    c = gg.make_config(name)
    n = int(c["n"])
    out = {"n": n, "m": int(c["m"]), "threads": threads or min(16, os.cpu_count() or 1)}
    lab = None
    if not pruned_only:
        t = time.time()
        lab = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"], mode=oracle.MODE_PLANT, threads=threads)
        out["oracle_s"] = round(time.time() - t, 2)
        st = lab.stats
        out.update(_sums(st, 0, n))
        out["split16"] = {"grown": 16, "pmain": 0, "head": _sums(st, 0, 16), "rest": _sums(st, 16, n)}
    gmax = min(LEVELS[-1], max(64, n // 64), n // 2)
    lv = [g for g in LEVELS if g < gmax] + [gmax]
    if lv and levels:
        t = time.time()
        p = oracle.chl_pruned(c["row_ptr"], c["col"], c["w"], c["order"], levels=lv, pmain=lv[-1], threads=threads)
        lv2 = level_bounds(p.stats[:, 2], gmax, first=4)
        if lv2 != lv:
            lv = lv2
            p = oracle.chl_pruned(c["row_ptr"], c["col"], c["w"], c["order"], levels=lv, pmain=lv[-1],
                                  threads=threads)
        if lab is not None:
            assert p.total == lab.total
        else:
            out["labels"] = int(p.total)
            out["oracle_pruned_s"] = round(time.time() - t, 2)
        out["levels%d" % lv[-1]] = {"grown": lv[-1], "pmain": lv[-1], "head": _sums(p.stats, 0, lv[-1]),
                                    "rest": _sums(p.stats, lv[-1], n), "bounds": lv,
                                    "levels": [[a, b, _sums(p.stats, a, b)] for a, b in zip([0] + lv[:-1], lv)]}
    return out


if __name__ == "__main__":
    args = sys.argv[1:]
    pruned_only = "--pruned-only" in args
    levels = "--no-levels" not in args
    names = [a for a in args if not a.startswith("--")] or ["grid64", "rmat16"]
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for nm in names:
        if gg.make_config(nm).get("directed"):
            data[nm] = counts_directed(nm)
        else:
            data[nm] = counts(nm, pruned_only=pruned_only, levels=levels)
        print(nm, data[nm], flush=True)
    json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
