"""Write tests/golden/digest_<workload>.json: commutative digests of the
oracle's complete canonical labeling of a million-vertex workload (see
tests/digest.py), which the GPU parity tests compare with a complete default
build. Calls only the oracle and the input generators.

    python tests/golden/make_digests.py grid1024d        # oracle.chl, PLaNT trees
    python tests/golden/make_digests.py rmat20           # oracle.chl_pruned
    python tests/golden/make_digests.py rmat20 --crosscheck
    python tests/golden/make_digests.py serving          # the 16 serving build graphs

grid1024d is labelled by the oracle's unpruned PLaNT trees (Algorithm 3 with
early termination; about 5 minutes on 8 threads, 31 GB of host memory at the
peak). For rmat20 the unpruned trees take hours, so its labels come from
oracle.chl_pruned (PLaNT trees with rank-prefix pruning, Section 4.3), whose
equality with the definition is pinned by the brute-force tests; the level
schedule passed to it only splits the work and does not change a label.
--crosscheck additionally grows the unpruned trees of the root sample that is
not in the first 1024 (the stratified roots, each alone, oracle.roots) and
requires their labels to equal the pruned run's.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import digest  # noqa: E402
import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

# a level schedule for the pruned oracle (roots [0, 16) unpruned, then each
# level pruned by the complete labels of the levels before it)
PRUNED_LEVELS = {"rmat20": [16, 32, 64, 128, 256, 512, 1024, 2048, 4096]}


SERVING_BUILDS = ["rmat%d_%d" % (10 + i % 7, i) for i in range(16)]


def serving_bundle():
    """digest_serving_builds.json: the 16 build requests of the serving
    workload (R-MAT scales 10-16, seeds 500+i), each labelled by oracle.chl."""
    out = {}
    for nm in SERVING_BUILDS:
        c = gg.make_config(nm)
        t = time.time()
        lab = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"], mode=oracle.MODE_PLANT)
        s = digest.summary(lab.offsets, lab.hub_pos, lab.dist)
        s["source"] = "oracle.chl (PLaNT trees, Algorithm 3 with early termination)"
        out[nm] = s
        print("%s: %d labels, %.1f s" % (nm, lab.total, time.time() - t), flush=True)
    path = os.path.join(HERE, "digest_serving_builds.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")
    print("wrote", path, flush=True)


def main(argv):
    names = [a for a in argv if not a.startswith("--")]
    cross = "--crosscheck" in argv
    if "serving" in names:
        serving_bundle()
        names = [a for a in names if a != "serving"]
    for nm in names:
        c = gg.make_config(nm)
        t = time.time()
        if nm in PRUNED_LEVELS:
            lv = PRUNED_LEVELS[nm]
            lab = oracle.chl_pruned(c["row_ptr"], c["col"], c["w"], c["order"], levels=lv, pmain=lv[-1])
            how = "oracle.chl_pruned (PLaNT trees, rank-prefix pruning, levels %s)" % lv
        else:
            lab = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"], mode=oracle.MODE_PLANT)
            how = "oracle.chl (PLaNT trees, Algorithm 3 with early termination)"
        ts = time.time() - t
        print("%s: %d labels in %.1f s" % (nm, lab.total, ts), flush=True)
        t = time.time()
        s = digest.summary(lab.offsets, lab.hub_pos, lab.dist)
        print("%s: digests in %.1f s" % (nm, time.time() - t), flush=True)
        s["workload"] = nm
        s["source"] = how
        s["oracle_s"] = round(ts, 1)
        s["threads"] = min(16, os.cpu_count() or 1)
        if cross:
            roots = [r for r in s["roots"] if r >= 1024]
            t = time.time()
            got, _ = oracle.roots(c["row_ptr"], c["col"], c["w"], c["order"], roots)
            pos = {r: i for i, r in enumerate(s["roots"])}
            for r, (v, d) in zip(roots, got):
                tsum = digest.root_tag(r, v, d)
                i = pos[r]
                assert len(v) == s["root_labels"][i] and tsum == s["root_tags"][i], "root %d differs" % r
            s["crosscheck"] = ("unpruned PLaNT trees of the %d sampled roots at rank position >= 1024 "
                               "(oracle.roots) equal the pruned run's, %.1f s" % (len(roots), time.time() - t))
            print(nm, s["crosscheck"], flush=True)
        out = os.path.join(HERE, "digest_%s.json" % nm)
        with open(out, "w") as f:
            json.dump(s, f, separators=(",", ":"))
            f.write("\n")
        print("wrote", out, flush=True)
        del lab


if __name__ == "__main__":
    main(sys.argv[1:])
