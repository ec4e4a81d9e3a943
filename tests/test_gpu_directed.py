"""Directed graphs on the GPU (chl_build_directed): out- and in-labels and
queries against the oracle, bit for bit, through the C-ABI.

Both label sets are canonical (fixed by the graph and the ranking), so every
comparison is an exact equality."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
import pins
from gpu_util import assert_same_labels

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


def _both(L):
    o = [t.numpy() for t in L.export("cpu")]
    i = [t.numpy() for t in L.export_in("cpu")]
    return o, i


def _check(row, col, w, order, pairs, where, **kw):
    from paper_1907_00140_amd import chl
    ref_out, ref_in = oracle.chl_directed(row, col, w, order)
    L = chl.build(row, col, w, order, directed=True, **kw)
    assert L.directed
    (oo, oh, od), (io, ih, idd) = _both(L)
    assert_same_labels(oo, oh, od, ref_out, where + " out")
    assert_same_labels(io, ih, idd, ref_in, where + " in")
    q = L.query(pairs).cpu().numpy()
    assert np.array_equal(q, oracle.query_directed(ref_out, ref_in, pairs)), where + ": queries differ"
    return L, ref_out, ref_in, q


def _all_pairs(n):
    uu, vv = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([uu.ravel(), vv.ravel()], 1).astype(np.int32)


@pytest.mark.parametrize("seed", range(16))
def test_random_small_directed(seed):
    """Random directed multigraphs (parallel arcs, loops, sinks, unreachable
    pairs) with few distinct weights; queries of all pairs also equal the
    Floyd-Warshall distances."""
    g = np.random.default_rng(2000 + seed)
    n = int(g.integers(2, 120))
    m = int(g.integers(n // 2, 4 * n))
    wmax = int(g.integers(1, 6))
    a = [(int(x), int(y), int(z)) for x, y, z in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, wmax + 1, m))]
    row, col, w = pins.csr_from_arcs(n, a)
    order = gg.random_rank(n, seed) if seed % 2 else gg.degree_rank_directed(row, col, seed)
    _say("random_small_directed", seed, n, m, wmax)
    kw = [dict(delta=1 + seed % 3, autotune=False), dict(), dict(wg_size=64, roots_in_flight=3, autotune=False),
          dict(mode="plain", autotune=False)][seed % 4]
    _, _, _, q = _check(row, col, w, order, _all_pairs(n), "seed %d" % seed, **kw)
    D = pins.floyd_warshall(n, row, col, w)
    assert np.array_equal(q.reshape(n, n), np.where(D >= pins.INF, -1, D))


def test_symmetric_graph_as_directed():
    """Both arcs of every edge given as a directed graph: both label sets
    equal the undirected labeling."""
    from paper_1907_00140_amd import chl
    c = gg.make_config("rmat12s9")
    ref = oracle.chl(c["row_ptr"], c["col"], c["w"], c["order"])
    L = chl.build(c["row_ptr"], c["col"], c["w"], c["order"], directed=True)
    (oo, oh, od), (io, ih, idd) = _both(L)
    assert_same_labels(oo, oh, od, ref, "out")
    assert_same_labels(io, ih, idd, ref, "in")


@pytest.mark.parametrize("name", ["rmat10d3", "rmat12d9"])
def test_directed_rmat_small(name):
    c = gg.make_config(name)
    _say("directed", name)
    _check(c["row_ptr"], c["col"], c["w"], c["order"], c["pairs"], name)


def test_directed_rmat16():
    """The benchmark's directed graph: both complete label sets, 10^5 queries."""
    c = gg.make_config("rmat16dir")
    _say("rmat16dir")
    L, ref_out, ref_in, _ = _check(c["row_ptr"], c["col"], c["w"], c["order"], c["pairs"][:100000], "rmat16dir")
    st = L.stats()
    assert st["labels"] == ref_out.total + ref_in.total


def test_directed_errors():
    import torch
    from paper_1907_00140_amd import chl
    # a sink (3), a source (0), an unreachable pair, a loop and parallel arcs
    arcs = [(0, 1, 2), (1, 2, 2), (0, 2, 5), (0, 2, 4), (2, 3, 1), (4, 4, 2), (4, 0, 1)]
    n = 5
    row, col, w = pins.csr_from_arcs(n, arcs)
    order = np.array([2, 0, 4, 1, 3], np.int32)
    pairs = np.array([[0, 3], [3, 0], [4, 3], [1, 1], [3, 4]], np.int32)
    L, _, _, q = _check(row, col, w, order, pairs, "small directed", autotune=False)
    assert q.tolist() == [5, -1, 6, 0, -1]
    # per-root statistics are not kept; parents and paths are for undirected labelings
    with pytest.raises(chl.ChlError):
        L.stats(per_root=True)
    with pytest.raises(chl.ChlError):
        L.parents(row, col, w)
    # export_in of an undirected labeling
    c = gg.make_config("rmat10s3")
    U = chl.build(c["row_ptr"], c["col"], c["w"], c["order"])
    assert not U.directed
    with pytest.raises(chl.ChlError):
        U.export_in("cpu")
    # an arc to a vertex out of range, a zero weight
    bad = col.copy()
    bad[0] = n
    with pytest.raises(chl.ChlError):
        chl.build(row, bad, w, order, directed=True)
    w0 = w.copy()
    w0[1] = 0
    with pytest.raises(chl.ChlError):
        chl.build(row, col, w0, order, directed=True)
    # an id out of range in a query
    with pytest.raises(chl.ChlError):
        L.query(torch.tensor([[0, n]], dtype=torch.int32))


def test_directed_in_server():
    """A directed labeling registered with the server: served answers equal
    chl_query's."""
    from paper_1907_00140_amd import chl, serve
    c = gg.make_config("rmat12d9")
    L = chl.build(c["row_ptr"], c["col"], c["w"], c["order"], directed=True)
    alone = L.query(c["pairs"]).cpu().numpy()
    srv, tickets, _, _ = serve.open_loop(
        lambda: serve.Server(mem_budget=1 << 30, max_batch=2048, build_streams=1, build_wg=64),
        [L], [c["pairs"]], rate=2e5, builds=[], seed=3)
    assert np.array_equal(tickets[0].out, alone)
    srv.close()


@pytest.mark.parametrize("kw", [dict(prune_hubs=-1), dict(prune_hubs=64), dict(prune_hubs=255, team_wgs=3),
                                dict(prune_hubs=1024, wg_size=128), dict(prune_hubs=1023, wg_size=128),
                                dict(autotune=False)])
def test_directed_pruning_invariance(kw):
    """Rank-prefix pruning across the two directions (d(h, x) from the
    out-labels, d(x, u) from the in-labels; odd prefix sizes included, with
    teams and with wide levels only, whose roots start in the order of their
    partners' prefix-label counts): the same label sets with every prefix
    and team size."""
    c = gg.make_config("rmat12d9")
    _say("directed pruning", kw)
    L, _, _, _ = _check(c["row_ptr"], c["col"], c["w"], c["order"], c["pairs"][:5000], str(kw), **kw)
    if kw.get("prune_hubs", 0) > 0:
        assert L.stats()["prune_hubs"] == kw["prune_hubs"]
