"""Parity at full size: complete default builds of the million-vertex
workloads, the 64-bit-key path through every kernel of the build schedule,
and the serving workload's build graphs, against the oracle.

The complete labelings of the 1024x1024 grid with shortcuts (1.28e9 labels)
and of R-MAT scale 20 are compared through commutative digests (tests/
digest.py) of the oracle's labels, written by tests/golden/make_digests.py:
per block of 1024 vertex ids the label count and the sum of the labels'
tags, the same per block of 1024 hub rank positions, and the count and tag
sum of each of the top 1000 roots and of 1000 rank-stratified roots. Trees
are independent (Section 4.2), so a root's labels in a complete build are
the labels of that root alone; the top roots are the largest trees, grown
by the team and wide-level kernels under rank-prefix pruning (Section 4.3).
"""
import json
import os
import sys

import numpy as np
import pytest

import digest
import graphgen as gg
import oracle
from gpu_util import assert_same_labels, gpu_labels

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a device"
    from paper_1907_00140_amd import chl
    chl.load()


def _golden(name):
    with open(os.path.join(GOLDEN, "digest_%s.json" % name)) as f:
        return json.load(f)


def _check_sorted(off, hub):
    """Every L_v strictly increasing in hub rank position (unique hubs)."""
    first = np.zeros(len(hub), bool)
    first[off[:-1][np.diff(off) > 0]] = True
    assert (np.diff(hub.astype(np.int64))[~first[1:]] > 0).all(), "a label list is not strictly increasing"


def _digest_check(L, want, where):
    off, hub, dist = (t.numpy() for t in L.export("cpu"))
    _say(where, "exported", int(off[-1]), "labels")
    _check_sorted(off, hub)
    got = digest.summary(off, hub, dist, roots=want["roots"])
    bad = digest.compare(got, want)
    assert not bad, "%s: %d mismatches, first: %s" % (where, len(bad), bad[:8])
    assert got["label_size_hist_log2"] == want["label_size_hist_log2"]
    assert got["max_label_size"] == want["max_label_size"]
    return got


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,kw", [("rmat20", {}), ("rmat20", {"team_wgs": 2, "groups": False}),
                                     ("grid1024d", {})],
                         ids=["rmat20", "rmat20-team2", "grid1024d"])
def test_full_build_digests(name, kw):
    """The complete default build (validation, renumbering, every pruning
    level, team launches, the main phase, assembly; 64-bit keys) equals the
    oracle's labeling block by block and root by root."""
    from paper_1907_00140_amd import chl
    want = _golden(name)
    c = gg.make_config(name)
    _say(name, kw, "build")
    L = chl.build(c["row_ptr"], c["col"], c["w"], c["order"], **kw)
    st = L.stats()
    _say(name, "levels", st["level_end"], "teams", st["level_teams"], "key bits", st["key_bits"])
    assert st["key_bits"] == 64
    assert st["labels"] == want["total"]
    if name == "rmat20":
        assert st["levels"] >= 2 and st["prune_hubs"] > 0
        if kw.get("groups", True):
            assert any(t < 0 for t in st["level_teams"]), st["level_teams"]     # groups of 16 trees
        else:
            assert any(t > 1 for t in st["level_teams"]), st["level_teams"]     # teams
    _digest_check(L, want, name)
    L.free()


_REF = {}


def _ref(name):
    if name not in _REF:
        c = gg.make_config(name)
        _REF[name] = (c, oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"]))
    return _REF[name]


@pytest.mark.parametrize("team,prune,groups", [(0, 0, True), (2, 0, False), (16, 1024, False), (1, 1024, True),
                                              (0, 1024, True)])
def test_u64_keys_levels_rmat14(team, prune, groups):
    """R-MAT 14 with weights up to 2^18: (n - 1) * w_max >= 2^31, so the
    build takes 64-bit keys through the team levels, the wide levels (more
    trees than team slots: a 1024-hub prefix has the level [128, 1024)) and
    the main phase (all pruned but the first level); labels and labels per
    root equal the oracle's."""
    c, ref = _ref("rmat14s11w18")
    _say("u64 rmat14", team, prune, groups)
    L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"], team_wgs=team, prune_hubs=prune,
                                   groups=groups)
    st = L.stats(per_root=True)
    _say("levels", st["level_end"], "teams", st["level_teams"], "prune", st["prune_hubs"])
    lt = st["level_teams"]
    assert st["key_bits"] == 64
    assert st["levels"] >= 3 and st["prune_hubs"] > 0
    if team == 1:
        assert all(t == 1 for t in lt)
    elif groups:
        assert any(t < 0 for t in lt), "no group launch"
    else:
        assert any(t > 1 for t in lt), "no team launch"
    if prune == 1024 and not groups:
        assert any(t == 1 for t in lt[1:]), "no wide (batched) pruned level"
    assert_same_labels(off, hub, dist, ref, "u64 team=%d" % team)
    assert np.array_equal(st["per_root"][:, 2], ref.stats[:, 2])
    q = L.query(c["pairs"]).cpu().numpy()
    assert np.array_equal(q, oracle.query(ref, c["pairs"]))
    L.free()


SERVING_BUILDS = ["rmat%d_%d" % (10 + i % 7, i) for i in range(16)]


@pytest.mark.timeout(600)
def test_serving_build_graphs():
    """The 16 build requests of the serving workload (R-MAT scales 10-16,
    seeds 500+i, weights [1,1000]), each built alone with the default
    options, equal the oracle's labelings."""
    from paper_1907_00140_amd import chl
    with open(os.path.join(GOLDEN, "digest_serving_builds.json")) as f:
        want = json.load(f)
    for nm in SERVING_BUILDS:
        c = gg.make_config(nm)
        _say("serving build", nm)
        L = chl.build(c["row_ptr"], c["col"], c["w"], c["order"])
        _digest_check(L, want[nm], nm)
        L.free()


@pytest.mark.timeout(600)
def test_served_builds_with_resident_rmat16():
    """Builds of scales 13-16 submitted to a server that holds the R-MAT 16
    labeling and answers a Poisson stream of its queries meanwhile: every
    served build equals the oracle's labeling, every served answer equals a
    direct chl_query."""
    from paper_1907_00140_amd import chl, serve
    with open(os.path.join(GOLDEN, "digest_serving_builds.json")) as f:
        want = json.load(f)
    c = gg.make_config("rmat16")
    L = chl.build(c["row_ptr"], c["col"], c["w"], c["order"])
    pairs = c["pairs"][:400_000]
    direct = L.query(pairs).cpu().numpy()
    names = [nm for nm in SERVING_BUILDS if int(nm[4:].split("_")[0]) >= 13]
    builds = [(gg.make_config(nm), 0.002 + 0.004 * i) for i, nm in enumerate(names)]
    _say("served builds", names)
    srv, tks, btk, wall = serve.open_loop(
        lambda: serve.Server(mem_budget=16 << 30, max_batch=1 << 15, build_streams=2, build_wg=128),
        [L], [pairs], rate=2e7, builds=builds, seed=3)
    assert np.array_equal(tks[0].out, direct)
    for nm, tk in zip(names, btk):
        assert tk.status.value == 0, (nm, tk.status.value)
        _digest_check(srv.labels(tk.gid.value), want[nm], "served " + nm)
    _say("p50 %.1f us p99 %.1f us wall %.3f s" % (np.percentile(tks[0].lat, 50) * 1e6,
                                                    np.percentile(tks[0].lat, 99) * 1e6, wall))
    srv.close()
    L.free()


def test_hub_vertex_map():
    """chl_labels_hub_vertex returns the ranking: hub_pos p is the input id
    order[p] (host and device outputs)."""
    import torch
    c = gg.make_config("rmat12s9")
    L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"])
    hv = L.hub_vertex()
    assert np.array_equal(np.asarray(hv), c["order"])
    dev = L.hub_vertex(device="cuda")
    assert isinstance(dev, torch.Tensor) and dev.is_cuda
    assert np.array_equal(dev.cpu().numpy(), c["order"])
    # every vertex's self label (pos(v), 0) maps back to v
    v = np.repeat(np.arange(c["n"]), np.diff(off))
    self_lab = dist == 0
    assert np.array_equal(c["order"][hub[self_lab]], v[self_lab])
    L.free()


def test_capped_allocator_oom():
    """An allocator that refuses memory past a cap: chl_build returns
    CHL_ERR_OOM (or succeeds when the cap is large enough) and gives back
    every byte it took; a build that succeeds equals the oracle."""
    from paper_1907_00140_amd import chl
    c, ref = _ref("rmat12s9")
    seen = set()
    for cap in (1 << 12, 1 << 16, 1 << 20, 4 << 20, 16 << 20, 64 << 20, 1 << 40):
        al = chl.TorchAllocator(cap=cap)
        try:
            L = chl.build(c["row_ptr"], c["col"], c["w"], c["order"], allocator=al)
        except chl.ChlError as e:
            assert e.code == -2, (cap, e.code)
            seen.add("oom")
        else:
            seen.add("ok")
            off, hub, dist = (t.numpy() for t in L.export("cpu"))
            assert_same_labels(off, hub, dist, ref, "cap %d" % cap)
            L.free()
        assert al.live_bytes == 0, "cap %d: %d bytes not returned" % (cap, al.live_bytes)
    assert seen == {"oom", "ok"}
