"""Commutative digests of a labeling, for parity at sizes where two full
label sets do not fit side by side (test infrastructure, no part of the
method's arithmetic).

Every label (v, h, d) -- vertex v (input id), hub h (rank position), distance
d -- gets the 64-bit tag

    t = mix64(((h << 32) | d) XOR mix64(v))

(mix64 = the splitmix64 finaliser of graphgen). Sums of tags modulo 2^64 do
not depend on the order in which the labels are visited, so the same numbers
come out of the oracle's labels and of an exported GPU labeling:

    C[v] = |L_v|, D[v] = sum of the tags of L_v           (vertex side)
    F[h] = labels with hub h, E[h] = sum of their tags     (hub side: the
                                                            labels of root h)

Golden files keep block sums of these (blocks of BLOCK consecutive vertex ids
or hub positions) and the hub-side pair of selected roots; a mismatch names the
block or the root.
"""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

import graphgen as gg

BLOCK = 1024
U64 = np.uint64


def _range_digest(offsets, hub, dist, va, vb, n):
    a, b = int(offsets[va]), int(offsets[vb])
    cnt = np.diff(offsets[va:vb + 1]).astype(np.int64)
    mv = np.repeat(gg.mix64(np.arange(va, vb, dtype=np.uint64)), cnt)
    h = np.asarray(hub[a:b]).astype(np.uint64)
    d = np.asarray(dist[a:b]).astype(np.int64)
    if d.size and (d.min() < 0 or d.max() > 0xFFFFFFFF):
        raise ValueError("distance outside [0, 2^32)")
    t = gg.mix64(((h << U64(32)) | d.astype(np.uint64)) ^ mv)
    del mv, d
    cs = np.zeros(t.size + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        np.cumsum(t, dtype=np.uint64, out=cs[1:])
        rel = (offsets[va:vb + 1] - a).astype(np.int64)
        D = cs[rel[1:]] - cs[rel[:-1]]
    E = np.zeros(n, dtype=np.uint64)
    hi = h.astype(np.int64)
    if hi.size and (hi.min() < 0 or hi.max() >= n):
        raise ValueError("hub position outside [0, n)")
    np.add.at(E, hi, t)
    F = np.bincount(hi, minlength=n).astype(np.int64)
    return va, vb, cnt, D, F, E


def label_digests(offsets, hub, dist, threads=None, chunk=1 << 23):
    """(C, D, F, E) of a labeling given as offsets[n+1], hub[L], dist[L]
    (host arrays; any integer dtypes). Work is split into vertex ranges of
    about `chunk` labels, run on a thread pool (numpy releases the GIL)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    total = int(offsets[-1])
    cuts = np.searchsorted(offsets, np.arange(0, total, chunk, dtype=np.int64), side="right") - 1
    cuts = np.unique(np.concatenate([[0], np.clip(cuts, 0, n), [n]]))
    ranges = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    C = np.zeros(n, dtype=np.int64)
    D = np.zeros(n, dtype=np.uint64)
    F = np.zeros(n, dtype=np.int64)
    E = np.zeros(n, dtype=np.uint64)
    threads = threads or min(16, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(_range_digest, offsets, hub, dist, a, b, n) for a, b in ranges]
        for f in cf.as_completed(futs):
            va, vb, cnt, Dv, Fh, Eh = f.result()
            C[va:vb] = cnt
            D[va:vb] = Dv
            F += Fh
            with np.errstate(over="ignore"):
                E += Eh
    return C, D, F, E


def root_tag(r, v, d):
    """Hub-side tag sum E[r] of the labels (v[i], r, d[i]) of one root."""
    mv = gg.mix64(np.asarray(v, dtype=np.int64).astype(np.uint64))
    t = gg.mix64(((np.uint64(r) << U64(32)) | np.asarray(d, dtype=np.int64).astype(np.uint64)) ^ mv)
    with np.errstate(over="ignore"):
        return int(t.sum(dtype=np.uint64))


def block_sums(cnt, tag, block=BLOCK):
    """[(count sum, tag sum mod 2^64)] per block of `block` consecutive entries."""
    n = len(cnt)
    nb = (n + block - 1) // block
    pad = nb * block - n
    c = np.concatenate([np.asarray(cnt, dtype=np.int64), np.zeros(pad, np.int64)]).reshape(nb, block)
    t = np.concatenate([np.asarray(tag, dtype=np.uint64), np.zeros(pad, np.uint64)]).reshape(nb, block)
    with np.errstate(over="ignore"):
        ts = t.sum(axis=1, dtype=np.uint64)
    return [[int(a), int(b)] for a, b in zip(c.sum(axis=1), ts)]


def root_sample(n, top=1000, strat=1000):
    """Rank positions checked one by one: the top `top` roots (the largest
    trees, grown in the first levels) and `strat` rank-stratified ones."""
    top = min(top, n)
    rest = n - top
    s = [top + (rest * j) // strat for j in range(strat)] if rest > 0 else []
    return sorted(set(range(top)) | set(s))


def summary(offsets, hub, dist, threads=None, block=BLOCK, roots=None):
    """The dict stored in a golden digest file (and recomputed by the tests)."""
    C, D, F, E = label_digests(offsets, hub, dist, threads=threads)
    n = len(C)
    roots = root_sample(n) if roots is None else roots
    sizes = C
    hist = np.bincount(np.floor(np.log2(np.maximum(sizes, 1))).astype(np.int64))
    return {
        "n": int(n), "total": int(C.sum()), "block": block,
        "vertex_blocks": block_sums(C, D, block),
        "hub_blocks": block_sums(F, E, block),
        "roots": [int(r) for r in roots],
        "root_labels": [int(F[r]) for r in roots],
        "root_tags": [int(E[r]) for r in roots],
        "label_size_hist_log2": {"[%d,%d)" % (1 << k, 2 << k): int(v) for k, v in enumerate(hist) if v},
        "max_label_size": int(sizes.max()) if n else 0,
    }


def compare(got, want):
    """List of mismatch descriptions between two summaries (empty = equal)."""
    bad = []
    for k in ("n", "total", "block"):
        if got[k] != want[k]:
            bad.append("%s: %r != %r" % (k, got[k], want[k]))
    for side in ("vertex_blocks", "hub_blocks"):
        for i, (x, y) in enumerate(zip(got[side], want[side])):
            if x != y:
                bad.append("%s[%d] (ids %d..%d): %r != %r" % (side, i, i * want["block"],
                                                              (i + 1) * want["block"] - 1, x, y))
    if got["roots"] != want["roots"]:
        bad.append("root samples differ")
    else:
        for r, a, b, x, y in zip(want["roots"], got["root_labels"], want["root_labels"], got["root_tags"],
                                 want["root_tags"]):
            if a != b or x != y:
                bad.append("root %d: %d labels / tag %d, expected %d / %d" % (r, a, x, b, y))
    return bad
