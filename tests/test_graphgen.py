"""Input generators: shapes, symmetry, determinism, rank validity."""
import numpy as np
import pytest

import graphgen as gg


def _check_csr(n, row, col, w):
    assert row[0] == 0 and np.all(np.diff(row) >= 0) and row[-1] == len(col) == len(w)
    src = np.repeat(np.arange(n), np.diff(row))
    assert (col != src).all()                                   # no self-loops
    key = src.astype(np.int64) * n + col
    assert len(np.unique(key)) == len(key)                      # no duplicates
    rev = col.astype(np.int64) * n + src
    a = np.argsort(key); b = np.argsort(rev)
    assert np.array_equal(key[a], rev[b]) and np.array_equal(w[a], w[b])  # symmetric


def test_grid64():
    c = gg.make_config("grid64")
    assert c["n"] == 4096 and c["m"] == 2 * 64 * 63
    deg = np.diff(c["row_ptr"])
    assert (deg == 2).sum() == 4 and (deg == 3).sum() == 248 and (deg == 4).sum() == 3844
    assert c["w"].min() >= 1 and c["w"].max() <= 100
    _check_csr(c["n"], c["row_ptr"], c["col"], c["w"])
    assert c["pairs"].shape == (10_000, 2)


def test_grid_diagonals():
    n, u, v, w = gg.grid_edges(128, 128, 1, 10_000, 3, diag_prob=0.05)
    base = 2 * 128 * 127
    extra = len(u) - base
    assert 0.03 * 127 * 128 < extra < 0.06 * 127 * 128
    r_u, c_u = np.divmod(u, 128); r_v, c_v = np.divmod(v, 128)
    diag = (r_v - r_u == 1) & (np.abs(c_v - c_u) == 1)
    assert diag.sum() == extra


def test_rmat_small():
    n, u, v, w = gg.rmat_edges(10, 8, *gg.RMAT_ABC, 5, 1, 1000)
    assert n == 1024 and (u < v).all() and len(u) < 8 * 1024
    row, col, ww = gg.to_csr(n, u, v, w)
    _check_csr(n, row, col, ww)
    deg = np.diff(row)
    assert deg.max() > 20 * max(1, np.median(deg))              # skewed degrees


def test_determinism():
    a = gg.make_config("rmat10_3")
    b = gg.make_config("rmat10_3")
    for k in ("row_ptr", "col", "w", "order", "pairs"):
        assert np.array_equal(a[k], b[k])
    c = gg.make_config("rmat10_4")
    assert not np.array_equal(a["col"], c["col"]) or not np.array_equal(a["w"], c["w"])


@pytest.mark.parametrize("name", ["grid64", "rmat10_0", "grid16x16_5"])
def test_degree_rank(name):
    c = gg.make_config(name)
    order = c["order"]
    assert np.array_equal(np.sort(order), np.arange(c["n"]))
    deg = np.diff(c["row_ptr"])[order]
    assert (np.diff(deg) <= 0).all()


def test_mix64_known_values():
    # splitmix64 output for state 0 and 1 (first output of the generator)
    assert int(gg.mix64(np.array([0], np.uint64))[0]) == 0xE220A8397B1DCDAF
    assert int(gg.mix64(np.array([1], np.uint64))[0]) == 0x910A2DEC89025CC1


def test_directed_rmat():
    """Directed R-MAT: the samples of the undirected generator read as arcs,
    no self-loops, no duplicate arcs, not symmetric, rows sorted; the
    reversed CSR holds the same arcs; the rank orders by total degree."""
    c = gg.make_config("rmat12d9")
    n, row, col, w = c["n"], c["row_ptr"], c["col"], c["w"]
    assert c["directed"] and row[0] == 0 and row[-1] == len(col) == len(w) == c["m"]
    src = np.repeat(np.arange(n), np.diff(row))
    assert (col != src).all()
    key = src.astype(np.int64) * n + col
    assert (np.diff(key) > 0).all()                              # sorted, no duplicates
    rev = col.astype(np.int64) * n + src
    assert not np.array_equal(np.sort(key), np.sort(rev))       # genuinely directed
    assert w.min() >= 1 and w.max() <= 1000
    trow, tcol, tw = gg.transpose_csr(row, col, w)
    tsrc = np.repeat(np.arange(n), np.diff(trow))
    fwd = sorted(zip(src.tolist(), col.tolist(), w.tolist()))
    back = sorted(zip(tcol.tolist(), tsrc.tolist(), tw.tolist()))
    assert fwd == back
    deg = np.diff(row) + np.bincount(col, minlength=n)
    assert (np.diff(deg[c["order"]]) <= 0).all()
    # same samples as the undirected generator of the same seed
    n2, u2, v2, _ = gg.rmat_edges(12, 8, *gg.RMAT_ABC, 9, 1, 1000)
    und = set(zip(u2.tolist(), v2.tolist()))
    assert all((min(a, b), max(a, b)) in und for a, b in zip(src.tolist()[:2000], col.tolist()[:2000]))
    d2 = gg.make_config("rmat12d9")
    assert np.array_equal(d2["col"], col) and np.array_equal(d2["w"], w)
