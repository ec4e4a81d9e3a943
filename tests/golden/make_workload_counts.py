"""Write tests/golden/workload_counts.json: the oracle's work counts of a
workload's trees (arcs scanned A, vertices settled S, labels L, trees that
stopped early), the algorithmic work units behind GTEPS and the roofline's
algorithmic bytes. Calls only the oracle and the input generators.

Counts are kept per build schedule, under the key "<b0,b1,...,bL>/<p>":
roots [0, b0) grow unpruned, each level [b_{j-1}, b_j) is pruned by the
complete labels of the hubs [0, b_{j-1}) (rank-prefix pruning, Section 4.3),
and the main phase's roots [bL, n) by the hubs [0, p). "/0" means every tree
unpruned; "16/0" the first 16 roots as a level of their own, then unpruned
trees (what a build runs when its probe drops pruning). The labels never
depend on the schedule; the work does. A benchmark looks the counts up by the
schedule its build reports (chl_stats: level_end, prune_hubs), so counts of
another schedule are never used by mistake.

    python tests/golden/make_workload_counts.py NAME [--unpruned]
           [--schedule 16,32,64/64] [--default]

--unpruned counts the unpruned trees of every root (also giving "/0" and
"16/0"); --schedule counts the pruned trees under that schedule; --default
counts the schedule that the library's default build takes (the policy below
mirrors the library's: roots [0, 16) first, then each level 8 times the
prefix, or 2 and 4 times in turn after levels whose roots emitted 2^21 labels
or more, or 4 times for the first pruned level of a directed build's combined
graph, up
to min(8192, max(64, n/64), n/2) hubs). Directed workloads are counted on
their combined graph (the graph and its reversal, ranks interleaved), as the
library builds them.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "workload_counts.json")

LEVEL0 = 16
LEVEL_LABELS_X2 = 1 << 21


def schedule_key(bounds, pmain):
    return "%s/%d" % (",".join(str(int(b)) for b in bounds), int(pmain))


def level_bounds(labels_per_root, gmax, first=None):
    """Level ends of the default schedule for a prefix of gmax hubs, from the
    labels per root (which do not depend on the schedule, so any complete
    run's counts fix it)."""
    g = min(LEVEL0, gmax)
    lv = [g]
    lab = int(labels_per_root[0:g].sum())
    last_f = 0
    while g < gmax:
        if first and g == LEVEL0:
            f = first
        elif lab >= LEVEL_LABELS_X2:
            f = 4 if last_f == 2 else 2
        else:
            f = 8
        last_f = f
        g2 = min(gmax, f * g)
        lab = int(labels_per_root[g:g2].sum())
        lv.append(g2)
        g = g2
    return lv


def default_prefix(n):
    return min(8192, max(64, n // 64), n // 2)


def _sums(st, lo, hi):
    return {"arcs": int(st[lo:hi, 1].sum()), "settled": int(st[lo:hi, 0].sum()),
            "labels": int(st[lo:hi, 2].sum()), "early_trees": int(st[lo:hi, 3].sum())}


def _entry(st, bounds, pmain, n):
    lo = [0] + list(bounds[:-1])
    end = bounds[-1] if bounds else 0
    return {"bounds": list(bounds), "pmain": int(pmain), "head": _sums(st, 0, end), "rest": _sums(st, end, n),
            "levels": [[a, b, _sums(st, a, b)] for a, b in zip(lo, bounds)]}


def _graph(name):
    c = gg.make_config(name)
    if c.get("directed"):
        r2, c2, w2, o2 = oracle.combined_directed(c["row_ptr"], c["col"], c["w"], c["order"])
        return c, (r2, c2, w2, o2), int(c["n"])
    return c, (c["row_ptr"], c["col"], c["w"], c["order"]), 0


def count(name, data, unpruned=False, schedules=(), default=False, threads=None):
    c, g, half = _graph(name)
    n = len(g[0]) - 1
    ent = data.setdefault(name, {})
    ent.update({"n": int(c["n"]), "m": int(c["m"]), "threads": threads or min(16, os.cpu_count() or 1)})
    if half:
        ent["directed"] = True
        ent["combined_n"] = n
    sch = ent.setdefault("schedules", {})
    lab_per_root = None
    if unpruned:
        t = time.time()
        lab = oracle.chl(*g, mode=oracle.MODE_PLANT, threads=threads)
        ent["oracle_s"] = round(time.time() - t, 2)
        ent["unpruned"] = _sums(lab.stats, 0, n)
        sch[schedule_key([], 0)] = _entry(lab.stats, [], 0, n)
        sch[schedule_key([16], 0)] = _entry(lab.stats, [16], 0, n)
        lab_per_root = lab.stats[:, 2]
    todo = [tuple(s) for s in schedules]
    if default:
        gmax = default_prefix(n)
        if lab_per_root is None:
            # the default schedule depends on labels per root: a first run
            # under any schedule gives them
            b0 = level_bounds(np.zeros(n, dtype=np.int64), gmax, first=4 if half else None)
            p = oracle.chl_pruned(*g, levels=b0, pmain=b0[-1], half=half, threads=threads)
            lab_per_root = p.stats[:, 2]
            b1 = level_bounds(lab_per_root, gmax, first=4 if half else None)
            if b1 == b0:
                sch[schedule_key(b0, b0[-1])] = _entry(p.stats, b0, b0[-1], n)
                ent["labels"] = int(p.total)
            else:
                todo.append((tuple(b1), b1[-1]))
        else:
            b1 = level_bounds(lab_per_root, gmax, first=4 if half else None)
            todo.append((tuple(b1), b1[-1]))
    for bounds, pmain in todo:
        t = time.time()
        p = oracle.chl_pruned(*g, levels=list(bounds), pmain=pmain, half=half, threads=threads)
        e = _entry(p.stats, list(bounds), pmain, n)
        e["oracle_s"] = round(time.time() - t, 2)
        sch[schedule_key(bounds, pmain)] = e
        ent["labels"] = int(p.total)
        print(name, schedule_key(bounds, pmain), e["head"], e["rest"], flush=True)
    return ent


def lookup(data, name, bounds, pmain):
    """Work units (arcs, settled, labels) of a workload's trees under a build
    schedule, or None when that schedule was not counted."""
    e = data.get(name, {}).get("schedules", {}).get(schedule_key(bounds, pmain))
    if e is None:
        return None
    return {k: e["head"][k] + e["rest"][k] for k in ("arcs", "settled", "labels", "early_trees")}


def _parse_schedule(s):
    b, p = s.split("/")
    return tuple(int(x) for x in b.split(",") if x), int(p)


if __name__ == "__main__":
    args = sys.argv[1:]
    names = [a for a in args if not a.startswith("--") and "/" not in a]
    sch = [_parse_schedule(args[i + 1]) for i, a in enumerate(args) if a == "--schedule"]
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for nm in names:
        count(nm, data, unpruned="--unpruned" in args, schedules=sch, default="--default" in args)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
