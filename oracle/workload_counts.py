"""Write tests/golden/workload_counts.json: the oracle's work counts (arcs
scanned A, vertices settled S, labels L) of the early-terminating trees of
every root, for the named workloads. These are the algorithmic work units of
the build (used for GTEPS and the roofline's algorithmic bytes). Calls only
the oracle and the input generators.

Usage: python -m oracle.workload_counts [name ...]
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


def counts(name, threads=None):
    c = gg.make_config(name)
    t = time.time()
    lab = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"], mode=oracle.MODE_PLANT, threads=threads)
    el = time.time() - t
    st = lab.stats
    return {"n": int(c["n"]), "m": int(c["m"]), "arcs": int(st[:, 1].sum()), "settled": int(st[:, 0].sum()),
            "labels": int(lab.total), "early_trees": int(st[:, 3].sum()), "oracle_s": round(el, 2),
            "threads": threads or min(16, os.cpu_count() or 1)}


if __name__ == "__main__":
    names = sys.argv[1:] or ["grid64", "rmat16"]
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for nm in names:
        data[nm] = counts(nm)
        print(nm, data[nm], flush=True)
    json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
