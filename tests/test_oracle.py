"""The CPU oracle against what the paper and the mathematics fix: brute force
on tiny graphs, closed forms, the worked tie example and the counterexample
for the reading of Algorithm 3 (see tests/pins.py)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import pins


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


def test_fig1_example(lib):
    pins.check_golden(lib, "fig1_example.txt")


def test_reading1_counterexample(lib):
    pins.check_golden(lib, "reading1_counterexample.txt")
    n, order, edges, _ = pins.load_golden("reading1_counterexample.txt")
    row, col, w = pins.csr_from_edges(n, edges)
    lab = oracle.chl(row, col, w, order, lib=lib)
    # h = vertex 1, u = vertex 4: no label, distance 2 through x
    assert all(h != 1 for h, _ in lab.of(4))
    assert oracle.query(lab, np.array([[1, 4]], np.int32), lib=lib)[0] == 2


@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_ties(lib, seed):
    n = 12 + seed % 30
    lab, D, order = pins.check_bruteforce(lib, n, int(n * 1.6), 1 + seed % 3, seed)
    if seed % 4 == 0:
        pins.check_minimal(lib, lab, D, seed)


@pytest.mark.parametrize("seed", range(10))
def test_bruteforce_degree_rank(lib, seed):
    pins.check_bruteforce(lib, 50, 110, 4, 1000 + seed, rank="degree")


def test_bruteforce_disconnected(lib):
    # sparse: several components and isolated vertices
    for s in range(5):
        lab, D, _ = pins.check_bruteforce(lib, 40, 25, 5, 77 + s)
        assert (D >= pins.INF).any()


@pytest.mark.parametrize("seed", range(3))
def test_closed_forms(lib, seed):
    pins.check_path(lib, 20 + seed, seed)
    pins.check_star(lib, 9 + seed, seed)
    pins.check_complete(lib, 8 + seed, seed)
    pins.check_unit_grid(lib, 5 + seed, 6, seed)
    pins.check_even_cycle(lib, 4 + seed, seed)
    pins.check_tree(lib, 25 + seed, seed)


def test_sssp(lib):
    pins.check_sssp(lib, 3)


def test_top_root_is_full_dijkstra(lib):
    """The most important vertex outranks everybody, so its labels are the
    Dijkstra distances to its whole component."""
    c = gg.make_config("grid64")
    out, _ = oracle.roots(c["row_ptr"], c["col"], c["w"], c["order"], [0], lib=lib)
    v, d = out[0]
    ref = oracle.sssp(c["row_ptr"], c["col"], c["w"], int(c["order"][0]), lib=lib)
    assert np.array_equal(v, np.nonzero(ref >= 0)[0])
    assert np.array_equal(d, ref[ref >= 0])


def test_modes_agree_grid64(lib):
    c = gg.make_config("grid64")
    labs = pins.all_modes(c["row_ptr"], c["col"], c["w"], c["order"], lib)
    for l in labs[1:]:
        assert np.array_equal(l.offsets, labs[0].offsets)
        assert np.array_equal(l.hub_pos, labs[0].hub_pos)
        assert np.array_equal(l.dist, labs[0].dist)
    # early termination does strictly less work than the full trees
    assert labs[1].stats[:, 1].sum() < labs[2].stats[:, 1].sum()


def test_unique_witness_grid64(lib):
    """Lemma 2: for every label (h, d) in L_v the merge of L_v and L_h reaches
    d only at hub h (a second minimiser would be a higher-ranked vertex of
    SP_{v,h}). Checked on a sample of labels of the 64x64 grid."""
    c = gg.make_config("grid64")
    lab = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"], lib=lib)
    g = np.random.default_rng(5)
    for k in g.choice(lab.total, 3000, replace=False):
        v = int(np.searchsorted(lab.offsets, k, side="right") - 1)
        hp, d = int(lab.hub_pos[k]), int(lab.dist[k])
        h = int(c["order"][hp])
        Lv = dict(lab.of(v))
        Lh = dict(lab.of(h))
        mins = [x for x in Lv if x in Lh and Lv[x] + Lh[x] == d]
        assert mins == [hp]


def test_queries_match_dijkstra_grid64(lib):
    c = gg.make_config("grid64")
    lab = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"], lib=lib)
    pairs = c["pairs"][:2000]
    q = oracle.query(lab, pairs, lib=lib)
    for s in np.unique(pairs[:50, 0]):
        ref = oracle.sssp(c["row_ptr"], c["col"], c["w"], int(s), lib=lib)
        sel = pairs[:, 0] == s
        assert np.array_equal(q[sel], ref[pairs[sel, 1]])
    assert (q[pairs[:, 0] == pairs[:, 1]] == 0).all()


@pytest.mark.parametrize("seed", range(12))
def test_work_counts(lib, seed):
    pins.check_stats(lib, 18 + seed, 30 + 2 * seed, 1 + seed % 3, 300 + seed)


@pytest.mark.parametrize("seed", range(16))
def test_pruned_equals_definition(lib, seed):
    """Rank-prefix pruning (Section 4.3) leaves every label unchanged:
    brute force on random tie-heavy multigraphs, several prefix sizes."""
    g = np.random.default_rng(seed)
    n = 20 + seed * 3
    m = int(n * 1.8)
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, 2 + seed % 4, m))]
    row, col, w = pins.csr_from_edges(n, e)
    order = gg.random_rank(n, seed) if seed % 2 else gg.degree_rank(row, seed)
    want = pins.brute_labels(pins.floyd_warshall(n, row, col, w), order)
    for eta, grown in ((1, 1), (4, 4), (4, 9), (8, 8), (n, n)):
        lab = oracle.chl_pruned(row, col, w, order, eta, grown, threads=2, lib=lib)
        assert pins.oracle_labels(lab) == want, (eta, grown)


def test_pruned_work_grid64_rmat12(lib):
    """Same labels as the unpruned trees on larger graphs, with less work."""
    for name in ("grid64", "rmat12s9"):
        c = gg.make_config(name)
        ref = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"], lib=lib)
        for eta, grown in ((16, 16), (16, 64), (64, 64)):
            lab = oracle.chl_pruned(c["row_ptr"], c["col"], c["w"], c["order"], eta, grown, lib=lib)
            assert np.array_equal(lab.offsets, ref.offsets)
            assert np.array_equal(lab.hub_pos, ref.hub_pos)
            assert np.array_equal(lab.dist, ref.dist)
            assert np.array_equal(lab.stats[:, 2], ref.stats[:, 2])
            assert lab.stats[:, 1].sum() <= ref.stats[:, 1].sum()


@pytest.mark.parametrize("seed", range(10))
def test_levels_equal_definition(lib, seed):
    """Pruning in levels (each level pruned by the complete prefix below it)
    leaves every label unchanged."""
    g = np.random.default_rng(100 + seed)
    n = 30 + seed * 4
    m = int(n * 2)
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, 2 + seed % 3, m))]
    row, col, w = pins.csr_from_edges(n, e)
    order = gg.degree_rank(row, seed)
    want = pins.brute_labels(pins.floyd_warshall(n, row, col, w), order)
    for levels, pmain in (([2, 8], 8), ([1, 4, 16], 16), ([3, 9, 27], 9), ([4, 16], 0)):
        lab = oracle.chl_pruned(row, col, w, order, levels=levels, pmain=pmain, threads=2, lib=lib)
        assert pins.oracle_labels(lab) == want, (levels, pmain)


def test_level_schedule_rule():
    """The pruning-level schedule the work counts use: roots [0, 16) first,
    then a prefix 2x and 4x larger in turn after levels whose roots emitted
    >= 2^21 labels, else 8x larger, capped at the prefix size."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "make_workload_counts", os.path.join(os.path.dirname(__file__), "golden", "make_workload_counts.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    level_bounds = mod.level_bounds
    lab = np.zeros(70_000, np.int64)
    lab[:16] = 200_000          # 3.2 M labels: work-bound level -> x2
    lab[16:32] = 100_000        # 1.6 M labels -> x8
    assert level_bounds(lab, 4096) == [16, 32, 256, 2048, 4096]
    lab[16:32] = 200_000        # 3.2 M labels -> x4 after the x2
    lab[32:128] = 30_000        # 2.9 M labels -> x2 after the x4
    assert level_bounds(lab, 4096) == [16, 32, 128, 256, 2048, 4096]
    assert level_bounds(np.zeros(100, np.int64), 50) == [16, 50]
    assert level_bounds(np.zeros(100, np.int64), 8) == [8]
    # a directed build's first pruned level grows by 4
    assert level_bounds(np.zeros(4096, np.int64), 2048, first=4) == [16, 64, 512, 2048]


@pytest.mark.parametrize("seed", range(8))
def test_parents_and_paths_bruteforce(lib, seed):
    pins.check_paths_bruteforce(lib, 20 + 3 * seed, 30 + 6 * seed, 1 + seed % 3, 500 + seed)


def test_path_graph_walks(lib):
    for s in range(3):
        pins.check_path_graph_walks(lib, 15 + s, s)


def test_parents_grid64_against_dijkstra(lib):
    """grid64: for sampled hubs, every labelled vertex's parent is the
    smallest-id neighbour p with d(h,p) + w = d(h,v) (Dijkstra from h), and
    sampled paths are walks along arcs of the queried length."""
    c = gg.make_config("grid64")
    row, col, w, order = c["row_ptr"], c["col"], c["w"], c["order"]
    lab = oracle.chl(row, col, w, order, lib=lib)
    par, slot = oracle.parents(lab, row, col, w, lib=lib)
    for hp in (0, 1, 7, 100, 2000, 4095):
        h = int(order[hp])
        dh = oracle.sssp(row, col, w, h, lib=lib)
        vs = np.nonzero(np.diff(lab.offsets) > 0)[0]
        for v in vs:
            a, b = lab.offsets[v], lab.offsets[v + 1]
            i = a + np.searchsorted(lab.hub_pos[a:b], hp)
            if i == b or lab.hub_pos[i] != hp:
                continue
            nb = [(int(col[e]), int(w[e])) for e in range(row[v], row[v + 1])]
            want = min((p for p, x in nb if dh[p] + x == dh[v]), default=-1)
            assert par[i] == want
    pairs = c["pairs"][:300]
    hops, poff, path = oracle.paths(lab, par, slot, pairs, lib=lib)
    d = oracle.query(lab, pairs, lib=lib)
    wt = {(v, int(col[e])): int(w[e]) for v in range(len(row) - 1) for e in range(row[v], row[v + 1])}
    for k, (u, v) in enumerate(pairs.tolist()):
        P = path[poff[k]:poff[k + 1]].tolist()
        assert P[0] == u and P[-1] == v and len(P) == hops[k] + 1
        assert sum(wt[(P[t], P[t + 1])] for t in range(len(P) - 1)) == d[k]


@pytest.mark.parametrize("seed", range(8))
def test_directed_bruteforce(lib, seed):
    pins.check_directed_bruteforce(lib, 15 + 4 * seed, 30 + 12 * seed, 1 + seed % 4, 700 + seed)


def test_directed_closed_forms(lib):
    for s in range(3):
        pins.check_directed_cycle(lib, 7 + 3 * s, s)
        pins.check_symmetric_as_directed(lib, 30 + s, 60, s)


def test_directed_rmat10_queries_match_dijkstra(lib):
    """Directed R-MAT 10: queries from the two label sets equal Dijkstra over
    the arcs from sampled sources."""
    c = gg.make_config("rmat10d3")
    lo, li = oracle.chl_directed(c["row_ptr"], c["col"], c["w"], c["order"], lib=lib)
    pairs = c["pairs"][:3000]
    q = oracle.query_directed(lo, li, pairs, lib=lib)
    for s in np.unique(pairs[:40, 0]):
        ref = oracle.sssp(c["row_ptr"], c["col"], c["w"], int(s), lib=lib)
        sel = pairs[:, 0] == s
        assert np.array_equal(q[sel], ref[pairs[sel, 1]])


@pytest.mark.parametrize("seed", range(6))
def test_directed_pruned_levels(lib, seed):
    pins.check_directed_pruned(lib, 20 + 3 * seed, 60 + 10 * seed, 1 + seed % 3, 900 + seed)
