"""HIP build and queries against the CPU oracle, bit-exact, through the C-ABI.

Labels are unique for a graph and a ranking (the canonical labeling), so
every comparison is an exact equality of offsets, hubs and distances.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
import pins
from gpu_util import assert_same_labels, gpu_labels, per_root_from_export

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a device"
    from paper_1907_00140_amd import chl
    chl.load()


@pytest.mark.parametrize("name", ["fig1_example.txt", "reading1_counterexample.txt"])
@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_golden_ties(name, mode):
    _say("golden", name, mode)
    n, order, edges, want = pins.load_golden(name)
    row, col, w = pins.csr_from_edges(n, edges)
    L, off, hub, dist = gpu_labels(row, col, w, order, mode=mode, delta=1, autotune=False)
    ref = oracle.chl(row, col, w, order)
    assert_same_labels(off, hub, dist, ref, name)
    got = {v: list(zip(hub[off[v]:off[v + 1]].tolist(), dist[off[v]:off[v + 1]].tolist())) for v in range(n)}
    assert got == want


@pytest.mark.parametrize("seed", range(24))
def test_random_small(seed):
    """Random multigraphs with few distinct weights (many ties), ragged sizes."""
    g = np.random.default_rng(seed)
    n = int(g.integers(2, 300))
    m = int(g.integers(n // 2, 3 * n))
    wmax = int(g.integers(1, 6))
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, wmax + 1, m))]
    row, col, w = pins.csr_from_edges(n, e)
    order = gg.random_rank(n, seed) if seed % 2 else gg.degree_rank(row, seed)
    _say("random_small", seed, n, m, wmax)
    ref = oracle.chl(row, col, w, order)
    for kw in (dict(mode="batched", delta=1 + seed % 4, roots_in_flight=1 + seed % 7, wg_size=256, autotune=False),
               dict(mode="batched", delta=1000, wg_size=512, autotune=False, prune_hubs=-1),
               dict(mode="batched", delta=3, wg_size=1024, autotune=False, prune_hubs=4 * (1 + seed % 16)),
               dict(mode="batched", delta=2 + seed % 5, autotune=False, team_wgs=2 + seed % 15),
               dict(mode="batched", delta=1 + seed % 5, autotune=False, team_wgs=2 + seed % 15, groups=False),
               dict(mode="plain", delta=2, autotune=False)):
        L, off, hub, dist = gpu_labels(row, col, w, order, **kw)
        assert_same_labels(off, hub, dist, ref, str(kw))


@pytest.mark.parametrize("seed", range(6))
def test_groups_random(seed):
    """Levels grown as groups of 16 trees with vertex-major keys, on random
    multigraphs with few distinct weights (many ties) and random or degree
    ranks: a prefix of up to 1024 hubs puts 112 trees in the level [16, 128),
    which runs as 7 groups (with early termination and without, and with
    ragged group counts from odd prefix sizes)."""
    g = np.random.default_rng(100 + seed)
    n = int(g.integers(300, 2500))
    m = int(g.integers(n, 4 * n))
    wmax = int(g.integers(1, 8))
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, wmax + 1, m))]
    row, col, w = pins.csr_from_edges(n, e)
    order = gg.random_rank(n, seed) if seed % 2 else gg.degree_rank(row, seed)
    ref = oracle.chl(row, col, w, order)
    for kw in (dict(prune_hubs=min(1024, n // 2), autotune=False, delta=1 + seed % 3),
               dict(prune_hubs=min(500, n // 2), autotune=False, early_term=False, delta=2)):
        _say("groups random", seed, n, m, wmax, kw)
        L, off, hub, dist = gpu_labels(row, col, w, order, **kw)
        st = L.stats(per_root=True)
        assert any(t < 0 for t in st["level_teams"]), st["level_teams"]
        assert_same_labels(off, hub, dist, ref, str(kw))
        assert np.array_equal(st["per_root"][:, 2], ref.stats[:, 2])


@pytest.mark.parametrize("name,kw", [("rmat12s9", {}), ("rmat14s11", {"prune_hubs": 1024}),
                                     ("rmat14s11w18", {}), ("grid64", {"prune_hubs": -1}),
                                     ("grid128x128_5", {"prune_hubs": 256}), ("rmat10d3", {"directed": True})])
def test_small_trees(name, kw):
    """The main phase by the small-tree kernel (one wave per tree, its state
    in LDS; trees that outgrow it grown again by the batched kernel): the
    oracle's labels and labels per root, with and without early
    termination (grids: most trees outgrow LDS and take the fallback)."""
    c = gg.make_config(name)
    directed = kw.pop("directed", False)
    if directed:
        ro, ri = oracle.chl_directed(c["row_ptr"], c["col"], c["w"], c["order"])
    else:
        ref = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"])
    for early in (True, False):
        _say("small trees", name, kw, early)
        L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"], small=True, autotune=False,
                                       early_term=early, directed=directed, **kw)
        st = L.stats(per_root=not directed)
        assert st["small_trees"] > 0
        if directed:
            assert_same_labels(off, hub, dist, ro, "out")
            o2, h2, d2 = (t.numpy() for t in L.export_in("cpu"))
            assert_same_labels(o2, h2, d2, ri, "in")
        else:
            assert_same_labels(off, hub, dist, ref, "%s %s" % (kw, early))
            assert np.array_equal(st["per_root"][:, 2], ref.stats[:, 2])
        L.free()


def test_grid64_full():
    """64x64 grid workload: full labeling, both forms, plus its 10^4 queries."""
    c = gg.make_config("grid64")
    ref = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"])
    for kw in (dict(mode="batched"), dict(mode="batched", early_term=False, autotune=False),
               dict(mode="plain", autotune=False)):
        _say("grid64", kw)
        L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"], **kw)
        assert_same_labels(off, hub, dist, ref, str(kw))
    qref = oracle.query(ref, c["pairs"])
    q = L.query(c["pairs"]).cpu().numpy()
    assert np.array_equal(q, qref)
    assert np.array_equal(L.offsets(), ref.offsets)


@pytest.mark.parametrize("k,wg,delta,eta,team", [(1, 256, 1, -1, 0), (3, 512, 7, 16, 1), (64, 1024, 50, 64, 2),
                                                 (256, 256, 100, 4, 16), (1024, 512, 400, 32, 5),
                                                 (2048, 256, 10_000, -1, 0), (4096, 64, 300, 64, 0),
                                                 (1536, 128, 25, 16, 0)])
def test_parameter_invariance_rmat12(k, wg, delta, eta, team):
    """Every (roots in flight, workgroup size, bucket width, pruning hubs,
    workgroups per tree of the first levels) gives the same labels."""
    c = gg.make_config("rmat12s9")
    ref = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"])
    _say("invariance", k, wg, delta, eta, team)
    L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"], mode="batched",
                                   roots_in_flight=k, wg_size=wg, delta=delta, autotune=False,
                                   prune_hubs=eta if eta < 0 else 4 * (eta // 4 or 1), team_wgs=team)
    assert_same_labels(off, hub, dist, ref)
    st = L.stats(per_root=True)
    assert np.array_equal(st["per_root"][:, 2], ref.stats[:, 2])


@pytest.mark.parametrize("team", [1, 2, 3, 8, 16])
@pytest.mark.parametrize("groups", [False, True])
def test_team_sizes_rmat14(team, groups):
    """The first levels grown by teams of 1..16 workgroups per tree, or as
    groups of 16 trees per team (vertex-major keys): same labels and the same
    labels per root as the oracle; with early termination off as well."""
    c = gg.make_config("rmat14s11")
    ref = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"])
    for early in (True, False):
        _say("teams", team, "groups", groups, early)
        L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"], team_wgs=team,
                                       early_term=early, autotune=False, prune_hubs=1024, groups=groups)
        assert_same_labels(off, hub, dist, ref)
        st = L.stats(per_root=True)
        assert np.array_equal(st["per_root"][:, 2], ref.stats[:, 2])
        lt = st["level_teams"]
        if groups and team != 1:
            assert lt[1] < 0, lt                    # [16,128): 112 trees as groups of 16
        else:
            assert all(t > 0 for t in lt), lt


def test_team_grid():
    """Teams on a grid (unpruned first level only when the probe drops the
    pruning) give the oracle's labels; so do pruning levels without teams
    (256-thread workgroups), whose reordered roots fill the label pool and
    resume."""
    c = gg.make_config("grid128x128_5")
    ref = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"])
    for kw in (dict(team_wgs=4), dict(team_wgs=16, prune_hubs=256, autotune=False),
               dict(team_wgs=4, prune_hubs=256, autotune=False, groups=False),
               dict(prune_hubs=1024, wg_size=256, autotune=False)):
        _say("team grid", kw)
        L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"], **kw)
        assert_same_labels(off, hub, dist, ref)


def test_default_schedule_rmat14():
    """Default pruning on a 16,384-vertex R-MAT graph: a max(64, n/64) = 256-hub
    prefix grown in levels [0,16), [16,128), [128,256) (each level emits far
    fewer than 2^21 labels, so the prefix grows 8x), then the main phase:
    four production launches, and the oracle's labels."""
    c = gg.make_config("rmat14s11")
    ref = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"])
    _say("default schedule")
    L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"], autotune=False)
    assert_same_labels(off, hub, dist, ref)
    st = L.stats()
    assert st["prefix_roots"] == 256 and st["prune_hubs"] == 256
    assert st["kernel_launches"] == 4


def test_repeatable_rmat14():
    """Repeated builds give identical labels (no order-dependent races)."""
    c = gg.make_config("rmat14s11")
    ref = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"])
    for i in range(3):
        _say("repeat", i)
        L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"])
        assert_same_labels(off, hub, dist, ref)
    q = L.query(c["pairs"]).cpu().numpy()
    assert np.array_equal(q, oracle.query(ref, c["pairs"]))


def test_rmat16_full():
    """R-MAT scale 16 workload: full labeling bit-exact, and 10^6 queries."""
    c = gg.make_config("rmat16")
    _say("rmat16 oracle")
    ref = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"])
    _say("rmat16 gpu")
    L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"])
    assert_same_labels(off, hub, dist, ref)
    q = L.query(c["pairs"]).cpu().numpy()
    assert np.array_equal(q, oracle.query(ref, c["pairs"]))
    st = L.stats(per_root=True)
    assert st["labels"] == ref.total
    assert np.array_equal(st["per_root"][:, 2], ref.stats[:, 2])   # labels per root
    _say("rmat16 gpu, no pruning")
    L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"], prune_hubs=-1)
    assert_same_labels(off, hub, dist, ref)


def test_invalid_inputs():
    from paper_1907_00140_amd import chl
    row, col, w = pins.csr_from_edges(4, [(0, 1, 1), (1, 2, 2), (2, 3, 1)])
    order = np.arange(4, dtype=np.int32)
    bad = [
        (row, col, w, np.array([0, 1, 1, 3], np.int32)),        # not a permutation
        (row, col, w, np.array([0, 1, 2, 4], np.int32)),        # out of range
        (row, col, np.where(w == 2, 0, w).astype(np.int32), order),   # zero weight
        (row, col, np.where(w == 2, -3, w).astype(np.int32), order),  # negative weight
        (row, np.where(col == 3, 7, col).astype(np.int32), w, order),  # neighbour out of range
    ]
    # asymmetric: change one direction's weight
    w2 = w.copy()
    w2[0] = 5
    bad.append((row, col, w2, order))
    r2 = row.copy()
    r2[-1] += 1                                                  # row_ptr[n] != n_arcs
    bad.append((r2, col, w, order))
    for i, (r, c_, ww, o) in enumerate(bad):
        _say("invalid", i)
        with pytest.raises(chl.ChlError) as e:
            chl.build(r, c_, ww, o)
        assert e.value.code == -1
    # options out of range
    for kw in (dict(wg_size=96), dict(mode="plain", wg_size=64), dict(mode="plain", wg_size=1024),
               dict(team_wgs=17), dict(team_wgs=-1), dict(prune_hubs=8193), dict(roots_in_flight=-2)):
        with pytest.raises(chl.ChlError) as e:
            chl.build(row, col, w, order, **kw)
        assert e.value.code == -1, kw
    L = chl.build(row, col, w, order)
    with pytest.raises(chl.ChlError):
        L.query(np.array([[0, 4]], np.int32))
    assert L.query(np.zeros((0, 2), np.int32)).numel() == 0


def test_edge_cases():
    """Single vertex, isolated vertices, self-loops and parallel arcs."""
    from paper_1907_00140_amd import chl
    # one vertex, no arcs
    L = chl.build(np.array([0, 0], np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32),
                  np.array([0], np.int32))
    off, hub, dist = L.export("cpu")
    assert off.tolist() == [0, 1] and hub.tolist() == [0] and dist.tolist() == [0]
    assert L.query(np.array([[0, 0]], np.int32)).cpu().tolist() == [0]
    # self-loops and parallel arcs, plus an isolated vertex
    edges = [(0, 1, 5), (0, 1, 2), (1, 1, 3), (1, 2, 1), (2, 0, 9), (2, 0, 9)]
    row, col, w = pins.csr_from_edges(4, edges)
    order = np.array([2, 0, 3, 1], np.int32)
    ref = oracle.chl(row, col, w, order)
    L, off, hub, dist = gpu_labels(row, col, w, order, autotune=False, delta=1)
    assert_same_labels(off, hub, dist, ref)
    q = L.query(np.array([[0, 2], [3, 1], [3, 3], [1, 0]], np.int32)).cpu().tolist()
    assert q == [3, -1, 0, 2]


@pytest.mark.parametrize("rank", ["degree", "random"])
def test_trivial_roots(rank):
    """A main-phase root whose tree is the root alone (no arcs, or every
    neighbour outranks it) gets its single label (r, r, 0) without a tree:
    R-MAT 12 with 3000 isolated vertices added (under a random rank spread
    over every level and the main phase, under the degree rank all in the
    main phase). Labels and labels per root equal the oracle's; those roots
    report one settled vertex, no arcs relaxed, no early stop, one round and
    no tree time, and the others were grown by the tree kernels."""
    c = gg.make_config("rmat12s9")
    extra = 3000
    row = np.concatenate([c["row_ptr"], np.full(extra, c["row_ptr"][-1], np.int64)])
    n = len(row) - 1
    order = np.asarray(gg.random_rank(n, 11) if rank == "random" else gg.degree_rank(row, 11))
    _say("trivial roots", rank, n)
    ref = oracle.chl(row, c["col"], c["w"], order)
    L, off, hub, dist = gpu_labels(row, c["col"], c["w"], order)
    assert_same_labels(off, hub, dist, ref, "trivial " + rank)
    st = L.stats(per_root=True)
    pr = st["per_root"]
    assert np.array_equal(pr[:, 2], ref.stats[:, 2])
    start = int(st["prefix_roots"])
    # by rank position: no arcs, or the largest neighbour position below its own
    pos = np.empty(n, np.int64)
    pos[order] = np.arange(n)
    deg = np.diff(row)
    top = np.full(n, -1, np.int64)
    np.maximum.at(top, np.repeat(np.arange(n), deg), pos[c["col"]])
    arcless = (deg == 0)[order][start:]
    outranked = ((deg > 0) & (top < pos))[order][start:]
    _say("main-phase roots", n - start, "without arcs", int(arcless.sum()), "outranked", int(outranked.sum()))
    assert arcless.sum() >= (extra if rank == "degree" else extra // 2) and outranked.sum() > 0
    trivial = arcless | outranked
    m = pr[start:][trivial]
    assert np.all(m[:, 0] == 1) and np.all(m[:, 1] == 0) and np.all(m[:, 2] == 1)
    assert np.all(m[:, 3] == 0) and np.all(m[:, 4] == 1) and np.all(m[:, 5] == 0)
    assert np.all(pr[start:][~trivial, 5] > 0)
    L.free()
    # no arcs at all: every root is its own tree
    L = chl_build_empty(700)
    off, hub, dist = (t.numpy() for t in L.export("cpu"))
    assert np.array_equal(off, np.arange(701)) and np.array_equal(dist, np.zeros(700))
    assert L.stats()["labels"] == 700
    L.free()


def chl_build_empty(n):
    from paper_1907_00140_amd import chl
    return chl.build(np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32),
                     np.arange(n, dtype=np.int32)[::-1].copy())


def test_distance_overflow():
    """A label distance of 2^31 - 1 or more is an error; just below is fine."""
    from paper_1907_00140_amd import chl
    big = 2**30
    row, col, w = pins.csr_from_edges(3, [(0, 1, big), (1, 2, big - 2)])
    order = np.array([0, 1, 2], np.int32)
    L, off, hub, dist = gpu_labels(row, col, w, order, autotune=False, delta=1 << 20)
    assert dist.max() == 2 * big - 2
    row, col, w = pins.csr_from_edges(3, [(0, 1, big), (1, 2, big - 1)])
    with pytest.raises(chl.ChlError) as e:
        chl.build(row, col, w, order, autotune=False, delta=1 << 20)
    assert e.value.code == -4


def test_grid_large_sampled():
    """256x256 grid with diagonal shortcuts: per-root parity on the top roots
    and a rank-stratified sample (roots are independent, Section 4.2)."""
    c = gg.make_config("grid256x256_3")
    n = c["n"]
    roots = list(range(64)) + list(np.linspace(64, n - 1, 192).astype(int))
    _say("grid256 gpu")
    L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], c["order"])
    _say("grid256 oracle roots")
    want, _ = oracle.roots(c["row_ptr"], c["col"], c["w"], c["order"], roots)
    got = per_root_from_export(off, hub, dist, c["order"], roots)
    for r, (v, d) in zip(roots, want):
        gv, gd = got[int(r)]
        assert np.array_equal(gv, v) and np.array_equal(gd, d), r
    # every L_v strictly increasing in hub
    seg_first = np.zeros(len(hub), bool)
    seg_first[off[:-1][np.diff(off) > 0]] = True
    assert (np.diff(hub.astype(np.int64))[~seg_first[1:]] > 0).all()


def _sampled_roots_parity(name, head, strata):
    """Per-root parity on a full-size workload: the GPU builds only the head
    roots (largest trees) and a rank-stratified sample, with the same launch
    configuration as a full build; the oracle grows the same trees."""
    from paper_1907_00140_amd import chl
    c = gg.make_config(name)
    n = c["n"]
    stride = (n - head) // strata
    for begin, count, step in ((0, head, 1), (head, strata, stride)):
        roots = [begin + i * step for i in range(count)]
        _say(name, "gpu roots", begin, count, step)
        L = chl.build(c["row_ptr"], c["col"], c["w"], c["order"], roots=(begin, count, step))
        off, hub, dist = (t.numpy() for t in L.export("cpu"))
        assert L.info()[1] == len(hub)
        _say(name, "oracle roots")
        want, wst = oracle.roots(c["row_ptr"], c["col"], c["w"], c["order"], roots)
        got = per_root_from_export(off, hub, dist, c["order"], roots)
        assert sum(len(v) for v, _ in want) == len(hub)
        for r, (v, d) in zip(roots, want):
            gv, gd = got[int(r)]
            assert np.array_equal(gv, v) and np.array_equal(gd, d), (name, r)
        L.free()


def test_grid1024d_sampled_roots():
    _sampled_roots_parity("grid1024d", 48, 160)


def test_rmat20_sampled_roots():
    _sampled_roots_parity("rmat20", 24, 160)


def test_grid1024d_full_queries():
    """Complete labeling of the 1024x1024 grid with shortcuts: every L_v is
    strictly increasing in hub and holds its self label; queries from sampled
    sources equal Dijkstra distances (cover property at full size)."""
    import torch
    from paper_1907_00140_amd import chl
    c = gg.make_config("grid1024d")
    n = c["n"]
    _say("grid1024d full build")
    L = chl.build(c["row_ptr"], c["col"], c["w"], c["order"])
    off, hub, dist = L.export("cuda")
    pos = torch.empty(n, dtype=torch.int32, device="cuda")
    pos[torch.from_numpy(c["order"]).long().cuda()] = torch.arange(n, dtype=torch.int32, device="cuda")
    cnt = off[1:] - off[:-1]
    assert int(cnt.min()) >= 1
    first = torch.zeros(hub.numel(), dtype=torch.bool, device="cuda")
    first[off[:-1]] = True
    dh = hub[1:].long() - hub[:-1].long()
    assert bool((dh[~first[1:]] > 0).all())
    # the last entry of L_v is v itself at distance 0 (no hub ranks below v)
    last = off[1:] - 1
    assert bool((hub[last] == pos).all()) and bool((dist[last] == 0).all())
    g = np.random.default_rng(3)
    for s in g.choice(n, 6, replace=False):
        ref = oracle.sssp(c["row_ptr"], c["col"], c["w"], int(s))
        tgt = g.choice(n, 20000, replace=False).astype(np.int32)
        pairs = np.stack([np.full(len(tgt), s, np.int32), tgt], 1)
        q = L.query(pairs).cpu().numpy()
        assert np.array_equal(q, ref[tgt]), s
    L.free()


def test_microbench_atomic_min():
    """The measurement entry point runs, reports what it did, and leaves every
    key at or below its all-ones start."""
    import torch
    from paper_1907_00140_amd import chl
    lib = chl.load()
    import ctypes as C
    for kb in (32, 64):
        words = 1 << 20
        buf = torch.empty(words * kb // 8, dtype=torch.uint8, device="cuda")
        done, ms = C.c_int64(), C.c_double()
        rc = lib.chl_microbench_atomic_min(buf.data_ptr(), words, kb, 1 << 22, C.byref(done), C.byref(ms),
                                           C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0 and done.value >= 1 << 21 and ms.value > 0
        v = buf.view(torch.int32 if kb == 32 else torch.int64)
        assert (v != -1).sum().item() > words // 2        # most keys were lowered
    with pytest.raises(chl.ChlError):
        chl.microbench_atomic_min(16, key_bits=16)


def test_query_tiers_rmat20():
    """R-MAT 20 (48 labels per vertex on average): a batch of 70,000 pairs
    takes the two-tier query kernel with 32-lane groups; answers equal
    Dijkstra from the 20 sources, and equal the one-group-per-query kernel
    that smaller batches take."""
    import torch
    from paper_1907_00140_amd import chl
    c = gg.make_config("rmat20")
    row, col, w, order = c["row_ptr"], c["col"], c["w"], c["order"]
    n = len(row) - 1
    _say("query tiers rmat20")
    L = chl.build(row, col, w, order)
    g = np.random.default_rng(11)
    src = g.choice(np.nonzero(np.diff(row) > 0)[0], 20, replace=False)
    tgt = g.integers(0, n, (20, 3500))
    pairs = np.stack([np.repeat(src, 3500), tgt.ravel()], 1).astype(np.int32)
    q = L.query(torch.from_numpy(pairs).cuda()).cpu().numpy()
    for i, s in enumerate(src):
        ref = oracle.sssp(row, col, w, int(s))
        assert np.array_equal(q[i * 3500:(i + 1) * 3500], ref[tgt[i]]), int(s)
    parts = [L.query(torch.from_numpy(pairs[a:a + 30000]).cuda()).cpu().numpy() for a in range(0, len(pairs), 30000)]
    assert np.array_equal(np.concatenate(parts), q)


def test_query_long_lists_complete_graph():
    """K_3000 with unit weights (closed form: L_v = {(v, 0)} and (u, 1) for
    every u ranked above v, so the lowest ranked vertices hold ~3000 labels):
    label sizes, and queries between low-ranked vertices, whose lists exceed
    the LDS stage of the long-list query kernel, equal 1 (0 when u = v)."""
    from paper_1907_00140_amd import chl
    n = 3000
    row = np.arange(n + 1, dtype=np.int64) * (n - 1)
    col = np.broadcast_to(np.arange(n, dtype=np.int32), (n, n))[~np.eye(n, dtype=bool)].copy()
    w = np.ones(len(col), dtype=np.int32)
    order = gg.random_rank(n, 5)
    pos = pins.pos_of(order)
    _say("complete graph", n)
    L = chl.build(row, col, w, order)
    off, hub, dist = (t.numpy() for t in L.export("cpu"))
    assert np.array_equal(np.diff(off), pos + 1)
    low = order[-400:]
    g = np.random.default_rng(5)
    pairs = np.stack([g.choice(low, 5000), g.choice(low, 5000)], 1).astype(np.int32)
    pairs = np.concatenate([pairs, np.stack([g.integers(0, n, 5000), g.integers(0, n, 5000)], 1).astype(np.int32)])
    q = L.query(pairs).cpu().numpy()
    assert np.array_equal(q, (pairs[:, 0] != pairs[:, 1]).astype(np.int64))


def test_sort_tiers_two_hubs():
    """Rows and label lists of every length tier of the segmented sort: two
    hubs adjacent to 9000 leaves (rows of 9000 arcs; the hub ranked last
    holds 9003 labels) and vertices of degree 63 to 4097 around the 64-, 128-,
    256- and 8192-key tier bounds; labels bit-exact, queries equal the
    oracle's."""
    g = np.random.default_rng(7)
    nl = 9000
    degs = [63, 64, 65, 100, 128, 129, 200, 255, 256, 257, 1000, 4097]
    n = 2 + nl + len(degs)
    leaves = np.arange(2, 2 + nl)
    e = [(0, int(v), 1) for v in leaves] + [(1, int(v), 1) for v in leaves]
    for i, d in enumerate(degs):
        for u, w in zip(g.choice(leaves, d, replace=False), g.integers(1, 4, d)):
            e.append((2 + nl + i, int(u), int(w)))
    row, col, w = pins.csr_from_edges(n, e)
    order = np.concatenate([[0], g.permutation(np.arange(2, n)), [1]]).astype(np.int32)
    _say("sort tiers", n, len(col))
    ref = oracle.chl(row, col, w, order)
    assert np.diff(ref.offsets).max() > 8192 and np.diff(row).max() > 8192
    L, off, hub, dist = gpu_labels(row, col, w, order)
    assert_same_labels(off, hub, dist, ref)
    pairs = np.stack([g.integers(0, n, 20000), g.integers(0, n, 20000)], 1).astype(np.int32)
    assert np.array_equal(L.query(pairs).cpu().numpy(), oracle.query(ref, pairs))


@pytest.mark.parametrize("rank", ["degree", "random"])
def test_hashed_root_distances(rank):
    """Prefixes of 4096 hubs and more: the main phase holds each root's
    prefix distances in an LDS hash; roots with more prefix labels than it
    holds (most of them under a random ranking) are grown afterwards with the
    dense array. Labels and labels per root equal the oracle's."""
    c = gg.make_config("rmat14s11")
    order = c["order"] if rank == "degree" else gg.random_rank(c["n"], 5)
    _say("hashed root distances", rank)
    ref = oracle.chl(c["row_ptr"], c["col"], c["w"], order)
    # the batched kernel alone (not the small-tree kernel) grows the main phase
    L, off, hub, dist = gpu_labels(c["row_ptr"], c["col"], c["w"], order, prune_hubs=4096, small=False)
    assert_same_labels(off, hub, dist, ref, "hashed " + rank)
    st = L.stats(per_root=True)
    assert st["prune_hubs"] == 4096
    assert st["small_trees"] == 0
    assert np.array_equal(st["per_root"][:, 2], ref.stats[:, 2])
    # both paths ran: a main-phase root's prefix labels are its labels of the
    # hubs [0, 4096); the hash holds 512 of them (degree rank: at most 85
    # each, all hashed; random rank: 7,688 of the 12,288 roots have more)
    start = int(st["prefix_roots"])
    assert start == 4096
    cs = np.concatenate([[0], np.cumsum(ref.hub_pos < 4096)])
    per_v = cs[ref.offsets[1:]] - cs[ref.offsets[:-1]]
    over = int((per_v[np.asarray(order)[start:]] > 512).sum())
    _say("main-phase roots beyond the hash: %d of %d" % (over, c["n"] - start))
    assert over < c["n"] - start
    if rank == "random":
        assert over > 0
    L.free()
