"""The Hybrid construction (Section 4.2.1): PLaNT trees until a window of
roots explores more than Psi_th vertices per label, then pruned trees with
rank queries in supersteps (Algorithm 1), each superstep cleaned by DQ_Clean
(Algorithm 2). Its output must be the CHL: equal, bit for bit, to the
oracle's labeling, with the same labels per root."""
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


def _check(row, col, w, order, tag, **kw):
    from paper_1907_00140_amd import chl
    ref = oracle.chl(row, col, w, order)
    L = chl.build(row, col, w, order, **kw)
    off, hub, dist = (x.numpy() for x in L.export("cpu"))
    assert_same_labels(off, hub, dist, ref, tag)
    st = L.stats(per_root=True)
    n = len(row) - 1
    assert np.array_equal(st["per_root"][:, 2], ref.stats[:, 2]), tag + ": labels per root differ"
    assert st["labels"] == ref.offsets[-1]
    sw = int(st["hybrid_switch"])
    assert 0 < sw <= n
    if sw < n:
        assert st["hybrid_supersteps"] >= 1 and st["hybrid_psi"] > kw["hybrid_psi"]
        # the pruned trees' labels, less the ones cleaned, are those of the roots [sw, n)
        assert st["hybrid_emitted"] - st["hybrid_removed"] == int(ref.stats[sw:, 2].sum()), tag
    else:
        assert st["hybrid_supersteps"] == 0 and st["hybrid_emitted"] == 0
    L.free()
    return st


@pytest.mark.parametrize("seed", range(10))
def test_hybrid_random_small(seed):
    """Random multigraphs with many ties, random or degree rank, a switch
    after the first window (Psi_th = 1) and supersteps of few roots."""
    g = np.random.default_rng(1000 + seed)
    n = int(g.integers(70, 900))
    m = int(g.integers(n, 4 * n))
    wmax = int(g.integers(1, 8))
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, wmax + 1, m))]
    row, col, w = pins.csr_from_edges(n, e)
    order = gg.random_rank(n, seed) if seed % 2 else gg.degree_rank(row, seed)
    _say("hybrid random_small", seed, n, m, wmax)
    st = _check(row, col, w, order, "hybrid random_small %d" % seed, hybrid_psi=1, roots_in_flight=1 + seed % 5,
                autotune=False, wg_size=256, prune_hubs=(-1, 0, 32)[seed % 3])
    _say("  switch", st["hybrid_switch"], "supersteps", st["hybrid_supersteps"], "removed", st["hybrid_removed"])


CASES = [
    # (workload, ranking, build options)
    ("rmat12s9", "random", dict(hybrid_psi=1, roots_in_flight=64, autotune=False)),
    ("rmat12s9", "degree", dict(hybrid_psi=20, prune_hubs=-1, roots_in_flight=64, autotune=False)),
    ("grid64", "degree", dict(hybrid_psi=5, roots_in_flight=32, autotune=False)),
    ("rmat14s11", "random", dict(hybrid_psi=5, roots_in_flight=128, autotune=False)),
    ("rmat14s11", "degree", dict(hybrid_psi=100, prune_hubs=-1, roots_in_flight=256, autotune=False)),
    ("rmat14s11w18", "degree", dict(hybrid_psi=2, prune_hubs=-1, roots_in_flight=256, autotune=False)),
    ("rmat12s9", "random", dict(hybrid_psi=1 << 30)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_hybrid_workloads(case):
    name, rank, kw = CASES[case]
    c = gg.make_config(name)
    order = gg.random_rank(c["n"], 77) if rank == "random" else c["order"]
    _say("hybrid", name, rank, kw)
    st = _check(c["row_ptr"], c["col"], c["w"], order, "hybrid %s %s" % (name, rank), **kw)
    _say("  switch %d of %d at psi %.1f, supersteps %d, emitted %d, removed %d, clean %.2f ms, key bits %d" % (
        st["hybrid_switch"], c["n"], st["hybrid_psi"], st["hybrid_supersteps"], st["hybrid_emitted"],
        st["hybrid_removed"], st["hybrid_clean_ms"], st["key_bits"]))
    if kw["hybrid_psi"] < 1 << 30:
        assert st["hybrid_switch"] < c["n"], "the threshold was never crossed"


def test_hybrid_invalid_options():
    from paper_1907_00140_amd import chl
    c = gg.make_config("rmat10d3")
    with pytest.raises(chl.ChlError) as e:
        chl.build(c["row_ptr"], c["col"], c["w"], c["order"], directed=True, hybrid_psi=100)
    assert e.value.code == -1
    c = gg.make_config("grid64")
    for kw in (dict(roots=(0, 10, 1)), dict(mode="plain")):
        with pytest.raises(chl.ChlError) as e:
            chl.build(c["row_ptr"], c["col"], c["w"], c["order"], hybrid_psi=100, **kw)
        assert e.value.code == -1
    with pytest.raises(chl.ChlError) as e:
        chl.build(c["row_ptr"], c["col"], c["w"], c["order"], hybrid_psi=-1)
    assert e.value.code == -1
