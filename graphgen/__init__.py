"""Seeded synthetic inputs for the CHL build: graphs, rankings and query pairs.

This module only synthesises inputs. It holds none of the labeling
arithmetic, so both the CPU oracle (tests) and the HIP library (tests, bench)
can take their inputs from it without sharing any of the method's code.

Every generator is deterministic in its seed. Random numbers come from
numpy's PCG64 bit generator (``numpy.random.Generator(PCG64(seed))``); the
exact sequence of draws is documented on each function so the recipe can be
re-implemented elsewhere.

Graph representation: an undirected simple graph is returned as a canonical
edge list ``(u, v, w)`` with ``u < v``, sorted by ``(u, v)``, no duplicates,
no self-loops, int32 weights ``>= 1``. ``to_csr`` turns it into a symmetric
CSR (int64 ``row_ptr``, int32 ``col``, int32 ``w``, each row sorted by col).

Ranking: ``order[i]`` is the vertex of rank position ``i``; ``order[0]`` is the
most important vertex (the root of the first shortest-path tree). This is the
network hierarchy R of the paper (Section 1, notation table; a higher R is
more important and the tree of v is built n - R(v)-th).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "mix64", "canonical_edges", "grid_edges", "rmat_edges", "random_edges",
    "to_csr", "degree_rank", "random_rank", "query_pairs", "make_config",
    "CONFIGS",
]

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_G = np.uint64(0x9E3779B97F4A7C15)


def mix64(x):
    """splitmix64 finaliser (Steele, Lea, Flood 2014), vectorised, uint64 in/out."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = z + _G
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def canonical_edges(u, v, n):
    """Undirected edge set from endpoint arrays: drop self-loops, orient u<v,
    deduplicate, sort by (u, v). Returns (u, v) int64 arrays."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * np.int64(n) + hi)
    return key // n, key % n


def _weights(m, wlo, whi, seed):
    """One weight per canonical edge, uniform on the inclusive range, drawn in
    canonical edge order from PCG64(seed) via Generator.integers."""
    return _rng(seed).integers(wlo, whi + 1, size=m, dtype=np.int64).astype(np.int32)


def grid_edges(rows, cols, wlo, whi, seed, diag_prob=0.0):
    """rows x cols 4-neighbour grid, vertex id r*cols + c.

    With ``diag_prob > 0`` each cell (r, c) with r < rows-1 independently gets,
    with that probability, one diagonal shortcut to (r+1, c-1) or (r+1, c+1)
    (a fair coin picks the side; out-of-range sides are skipped). The two
    draws per cell come from PCG64(seed + 1): first ``random(rows*cols)`` for
    the Bernoulli trial, then ``integers(0, 2, rows*cols)`` for the side.
    Weights: one per canonical edge from PCG64(seed), see ``_weights``.
    """
    n = rows * cols
    r, c = np.divmod(np.arange(n, dtype=np.int64), cols)
    us, vs = [], []
    right = c < cols - 1
    us.append(np.nonzero(right)[0]); vs.append(us[-1] + 1)
    down = r < rows - 1
    us.append(np.nonzero(down)[0]); vs.append(us[-1] + cols)
    if diag_prob > 0:
        g = _rng(seed + 1)
        trial = g.random(n) < diag_prob
        side = g.integers(0, 2, size=n)
        dc = np.where(side == 0, -1, 1)
        tc = c + dc
        ok = trial & down & (tc >= 0) & (tc < cols)
        src = np.nonzero(ok)[0]
        us.append(src); vs.append((r[src] + 1) * cols + tc[src])
    u, v = canonical_edges(np.concatenate(us), np.concatenate(vs), n)
    return n, u, v, _weights(len(u), wlo, whi, seed)


def rmat_edges(scale, edge_factor, a, b, c, seed, wlo, whi):
    """R-MAT graph (Chakrabarti, Zhan, Faloutsos 2004) without noise or id
    scrambling: ``edge_factor * 2**scale`` samples; for each of the ``scale``
    bit levels (most significant first) one ``random(samples)`` draw from
    PCG64(seed) picks the quadrant a | b | c | d. Self-loops and duplicate
    edges are removed. Weights: PCG64(seed + 7919), see ``_weights``.
    """
    n = 1 << scale
    s = edge_factor * n
    g = _rng(seed)
    u = np.zeros(s, dtype=np.int64)
    v = np.zeros(s, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for lvl in range(scale):
        x = g.random(s)
        bit = np.int64(1 << (scale - 1 - lvl))
        right = ((x >= a) & (x < ab)) | (x >= abc)
        down = x >= ab
        v += np.where(right, bit, 0)
        u += np.where(down, bit, 0)
    u, v = canonical_edges(u, v, n)
    return n, u, v, _weights(len(u), wlo, whi, seed + 7919)


def rmat_arcs(scale, edge_factor, a, b, c, seed, wlo, whi):
    """Directed R-MAT graph: the samples of ``rmat_edges`` read as arcs u -> v
    (row quadrant = source), self-loops and duplicate arcs removed, sorted by
    (u, v). Weights, one per arc in that order: PCG64(seed + 7919)."""
    n = 1 << scale
    s = edge_factor * n
    g = _rng(seed)
    u = np.zeros(s, dtype=np.int64)
    v = np.zeros(s, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for lvl in range(scale):
        x = g.random(s)
        bit = np.int64(1 << (scale - 1 - lvl))
        right = ((x >= a) & (x < ab)) | (x >= abc)
        down = x >= ab
        v += np.where(right, bit, 0)
        u += np.where(down, bit, 0)
    keep = u != v
    key = np.unique(u[keep] * np.int64(n) + v[keep])
    u, v = key // n, key % n
    return n, u, v, _weights(len(u), wlo, whi, seed + 7919)


def to_csr_directed(n, u, v, w):
    """Out-arc CSR of a directed arc list (row u holds u -> v), rows sorted by col."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.int32)
    perm = np.lexsort((v, u))
    u, v, w = u[perm], v[perm], w[perm]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(u, minlength=n), out=row_ptr[1:])
    return row_ptr, v.astype(np.int32), w.astype(np.int32)


def transpose_csr(row_ptr, col, w):
    """CSR of the reversed graph (row v holds the arcs u -> v as v <- u),
    rows sorted by col."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = len(row_ptr) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    return to_csr_directed(n, np.asarray(col, dtype=np.int64), src, w)


def random_edges(n, m, wlo, whi, seed):
    """Uniform random graph: m endpoint pairs from PCG64(seed), then
    canonicalised (so fewer than m edges may remain). Weights from
    PCG64(seed + 1)."""
    g = _rng(seed)
    u = g.integers(0, n, size=m)
    v = g.integers(0, n, size=m)
    u, v = canonical_edges(u, v, n)
    return n, u, v, _weights(len(u), wlo, whi, seed + 1)


def to_csr(n, u, v, w):
    """Symmetric CSR from a canonical undirected edge list. Rows sorted by col."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.int32)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    ww = np.concatenate([w, w])
    perm = np.lexsort((dst, src))
    src, dst, ww = src[perm], dst[perm], ww[perm]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return row_ptr, dst.astype(np.int32), ww.astype(np.int32)


def degree_rank(row_ptr, seed):
    """Degree-descending ranking; ties by mix64(seed xor id) ascending, then id.
    Degree = number of CSR entries in the row (distinct neighbours for the
    simple graphs produced here). Returns ``order`` (int32)."""
    n = len(row_ptr) - 1
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    ids = np.arange(n, dtype=np.uint64)
    h = mix64(ids ^ np.uint64(seed))
    order = np.lexsort((ids, h, -deg))
    return order.astype(np.int32)


def degree_rank_directed(row_ptr, col, seed):
    """Ranking of a directed graph by total degree (out + in) descending;
    ties as in ``degree_rank``."""
    n = len(row_ptr) - 1
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64)) + np.bincount(np.asarray(col, dtype=np.int64), minlength=n)
    ids = np.arange(n, dtype=np.uint64)
    h = mix64(ids ^ np.uint64(seed))
    return np.lexsort((ids, h, -deg)).astype(np.int32)


def random_rank(n, seed):
    """Uniformly random ranking: a PCG64(seed) permutation."""
    return _rng(seed).permutation(n).astype(np.int32)


def query_pairs(n, q, seed):
    """q uniform (u, v) pairs in [0, n)^2 from PCG64(seed): int32 array [q, 2]."""
    return _rng(seed).integers(0, n, size=(q, 2), dtype=np.int64).astype(np.int32)


RMAT_ABC = (0.57, 0.19, 0.19)


def make_config(name):
    """Named workloads. Returns a dict with n, row_ptr, col, w, order and,
    where the workload has one, a query pair array.

    grid64      : 64x64 4-neighbour grid, weights [1,100] seed 1, degree rank
                  (tie seed 1), 10^4 query pairs seed 101.
    rmat16      : R-MAT scale 16, 8n samples, a,b,c = .57,.19,.19, seed 2,
                  weights [1,1000], degree rank (tie seed 2), 10^6 pairs seed 102.
    grid1024d   : 1024x1024 grid + 5% diagonal shortcuts, weights [1,10^4]
                  seed 3, degree rank (tie seed 3).
    rmat20      : R-MAT scale 20, 8n samples, seed 4, weights [1,65536],
                  degree rank (tie seed 4).
    rmat16dir   : directed R-MAT scale 16 (the samples read as arcs), seed 5,
                  weights [1,1000], total-degree rank (tie seed 5), 10^6 pairs
                  seed 105; out-arc CSR, "directed": True.
    rmat<s>_<i> : serving build requests, R-MAT scale s, seed 500+i,
                  weights [1,1000], degree rank.
    Smaller stand-ins used by tests: grid<r>x<c>_<seed>, rmat<s>s<seed>,
    rmat<s>d<seed> (directed), rmat<s>s<seed>w<b> (weights [1, 2^b]).
    """
    if name == "rmat16dir" or (name.startswith("rmat") and name[4:].replace("d", "", 1).isdigit() and "d" in name[4:]):
        if name == "rmat16dir":
            sc, sd, qseed, q = 16, 5, 105, 1_000_000
        else:
            sc, sd = (int(t) for t in name[4:].split("d"))
            qseed, q = sd + 100, 10_000
        n, u, v, w = rmat_arcs(sc, 8, *RMAT_ABC, sd, 1, 1000)
        row_ptr, col, ww = to_csr_directed(n, u, v, w)
        order = degree_rank_directed(row_ptr, col, sd)
        return {"name": name, "n": n, "m": len(u), "row_ptr": row_ptr, "col": col, "w": ww, "order": order,
                "pairs": query_pairs(n, q, qseed), "directed": True}
    if name == "grid64":
        n, u, v, w = grid_edges(64, 64, 1, 100, 1)
        seed, qseed, q = 1, 101, 10_000
    elif name == "rmat16":
        n, u, v, w = rmat_edges(16, 8, *RMAT_ABC, 2, 1, 1000)
        seed, qseed, q = 2, 102, 1_000_000
    elif name == "grid1024d":
        n, u, v, w = grid_edges(1024, 1024, 1, 10_000, 3, diag_prob=0.05)
        seed, qseed, q = 3, 103, 1_000_000
    elif name == "rmat20":
        n, u, v, w = rmat_edges(20, 8, *RMAT_ABC, 4, 1, 65536)
        seed, qseed, q = 4, 104, 1_000_000
    elif name.startswith("rmat") and "_" in name:
        s, i = name[4:].split("_")
        s, i = int(s), int(i)
        n, u, v, w = rmat_edges(s, 8, *RMAT_ABC, 500 + i, 1, 1000)
        seed, qseed, q = 500 + i, 600 + i, 10_000
    elif name.startswith("rmat") and "s" in name[4:] and "w" in name[4:]:
        s, rest = name[4:].split("s")
        sd, wb = rest.split("w")
        s, sd, wb = int(s), int(sd), int(wb)
        n, u, v, w = rmat_edges(s, 8, *RMAT_ABC, sd, 1, 1 << wb)
        seed, qseed, q = sd, sd + 100, 10_000
    elif name.startswith("rmat") and "s" in name[4:]:
        s, sd = name[4:].split("s")
        s, sd = int(s), int(sd)
        n, u, v, w = rmat_edges(s, 8, *RMAT_ABC, sd, 1, 1000)
        seed, qseed, q = sd, sd + 100, 10_000
    elif name.startswith("grid") and "x" in name:
        dims, sd = name[4:].split("_")
        r, c = (int(t) for t in dims.split("x"))
        diag = 0.05 if r >= 128 else 0.0
        n, u, v, w = grid_edges(r, c, 1, 10_000 if diag else 100, int(sd), diag)
        seed, qseed, q = int(sd), int(sd) + 100, 10_000
    else:
        raise KeyError(name)
    row_ptr, col, ww = to_csr(n, u, v, w)
    order = degree_rank(row_ptr, seed)
    return {"name": name, "n": n, "m": len(u), "row_ptr": row_ptr, "col": col,
            "w": ww, "order": order, "pairs": query_pairs(n, q, qseed)}


CONFIGS = ("grid64", "rmat16", "grid1024d", "rmat20")


def poisson_arrivals(q, rate, seed, t0=0.0):
    """Arrival times (seconds, non-decreasing) of an open-loop Poisson stream
    of q requests at `rate` per second: cumulative sums of exponential gaps
    drawn from PCG64(seed)."""
    gaps = _rng(seed).exponential(1.0 / rate, size=q)
    return t0 + np.cumsum(gaps)
