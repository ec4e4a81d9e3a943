"""Independent pins for the CHL oracle: brute force, closed forms and worked
examples. Nothing here calls a shortest-path routine of the oracle; the
distances come from Floyd-Warshall (numpy) or from the closed form of the
graph family, and the labels from the definition of the CHL: (h, d(v,h)) is
in L_v exactly when h is the highest ranked vertex of SP_{v,h}, the set of
vertices on all shortest v-h paths, inclusive (Section 1 of the paper).

Each ``check_*`` function takes an oracle library handle so the same pins can
be run against deliberately broken copies of the oracle (tests that plant a
mistake must see some pin fail).
"""
from __future__ import annotations

import os

import numpy as np

import graphgen as gg
import oracle

INF = np.iinfo(np.int64).max // 4
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------- helpers
def csr_from_edges(n, edges):
    """edges: iterable of (u, v, w) undirected; may hold parallel edges."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 3)
    src = np.concatenate([e[:, 0], e[:, 1]])
    dst = np.concatenate([e[:, 1], e[:, 0]])
    w = np.concatenate([e[:, 2], e[:, 2]])
    p = np.lexsort((dst, src))
    src, dst, w = src[p], dst[p], w[p]
    row = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row[1:])
    return row, dst.astype(np.int32), w.astype(np.int32)


def floyd_warshall(n, row, col, w):
    D = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(D, 0)
    for v in range(n):
        for e in range(row[v], row[v + 1]):
            u = col[e]
            if u != v:
                D[v, u] = min(D[v, u], w[e])
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    D[D >= INF] = INF
    return D


def brute_labels(D, order):
    """The CHL by definition from an all-pairs distance matrix."""
    n = len(order)
    pos = np.empty(n, dtype=np.int64)
    pos[np.asarray(order)] = np.arange(n)
    labels = {v: [] for v in range(n)}
    for h in range(n):
        dh = D[:, h]                                      # d(w, h)
        reach = dh < INF
        # on[v, w]: w lies on some shortest v-h path
        on = (D + dh[None, :] == dh[:, None]) & reach[None, :] & reach[:, None] & (D < INF)
        minpos = np.where(on, pos[None, :], n).min(axis=1)
        for v in np.nonzero(reach & (minpos == pos[h]))[0]:
            labels[int(v)].append((int(pos[h]), int(D[v, h])))
    for v in labels:
        labels[v].sort()
    return labels


def oracle_labels(lab):
    return {v: lab.of(v) for v in range(lab.n)}


def pos_of(order):
    pos = np.empty(len(order), dtype=np.int64)
    pos[np.asarray(order)] = np.arange(len(order))
    return pos


def load_golden(name):
    n, order, edges, labels = None, None, [], {}
    pos = None
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].split()
        if not line:
            continue
        if line[0] == "n":
            n = int(line[1])
            labels = {v: [] for v in range(n)}
        elif line[0] == "order":
            order = np.array([int(t) for t in line[1:]], dtype=np.int32)
            pos = pos_of(order)
        elif line[0] == "edge":
            edges.append(tuple(int(t) for t in line[1:]))
        elif line[0] == "label":
            v, h, d = (int(t) for t in line[1:])
            labels[v].append((int(pos[h]), d))
    for v in labels:
        labels[v].sort()
    return n, order, edges, labels


def all_modes(row, col, w, order, lib):
    return [oracle.chl(row, col, w, order, mode=m, threads=2, lib=lib)
            for m in (oracle.MODE_DEFINITION, oracle.MODE_PLANT, oracle.MODE_PLANT_FULL)]


# ---------------------------------------------------------------- pins
def check_golden(lib, name):
    n, order, edges, want = load_golden(name)
    row, col, w = csr_from_edges(n, edges)
    for lab in all_modes(row, col, w, order, lib):
        got = oracle_labels(lab)
        assert got == want, (name, got, want)


def check_bruteforce(lib, n, m, wmax, seed, rank="random"):
    """Random multigraph with small weights (many ties): every oracle mode
    equals the definition evaluated on Floyd-Warshall distances; queries
    equal the distances (cover property); every label is needed (minimality,
    by deleting it and finding a pair that breaks)."""
    g = np.random.default_rng(seed)
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, wmax + 1, m))]
    row, col, w = csr_from_edges(n, e)
    order = (gg.random_rank(n, seed) if rank == "random" else gg.degree_rank(row, seed))
    D = floyd_warshall(n, row, col, w)
    want = brute_labels(D, order)
    labs = all_modes(row, col, w, order, lib)
    for lab in labs:
        assert oracle_labels(lab) == want
    lab = labs[1]
    uu, vv = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([uu.ravel(), vv.ravel()], 1).astype(np.int32)
    q = oracle.query(lab, pairs, lib=lib).reshape(n, n)
    Dq = np.where(D >= INF, -1, D)
    assert np.array_equal(q, Dq)
    return lab, D, order


def expected_plant_stats(row, col, w, order, D):
    """Work of the early-terminating tree of every root, from the definition.

    Pops follow the global (distance, rank position) order of the root's
    component. Before each pop the queue holds the unpopped vertices adjacent
    to popped ones; such a vertex u is clean (its best ancestor is the root)
    when u does not outrank the root and every popped neighbour p that attains
    u's tentative distance is clean, i.e. has the root as the highest ranked
    vertex of SP_{root,p}. The tree stops before the first pop at which no
    queued vertex is clean. Returns [n, 3] = (settled, arcs, labels) indexed
    by root rank position."""
    n = len(order)
    pos = pos_of(order)
    out = np.zeros((n, 3), dtype=np.int64)
    deg = np.diff(row)
    for hp in range(n):
        h = int(order[hp])
        d = D[h]
        comp = np.nonzero(d < INF)[0]
        seq = comp[np.lexsort((pos[comp], d[comp]))]
        # clean[x]: no vertex of SP_{h,x} outranks h
        on = (D[:, comp] + d[None, comp] == d[:, None]) & (D[:, comp] < INF)
        clean = {int(x): bool(pos[comp][on[x]].min() == hp) for x in comp}
        popped = set()
        k = 0
        for k, x in enumerate(seq):
            tent = {}
            for p in popped:
                for e in range(row[p], row[p + 1]):
                    u = int(col[e])
                    if u in popped:
                        continue
                    t = d[p] + w[e]
                    if u not in tent or t < tent[u][0]:
                        tent[u] = [t, clean[p]]
                    elif t == tent[u][0]:
                        tent[u][1] = tent[u][1] and clean[p]
            if k > 0 and not any(c and pos[u] > hp for u, (t, c) in tent.items()):
                break
            popped.add(int(x))
        else:
            k = len(seq)
        out[hp, 0] = k
        out[hp, 1] = sum(int(deg[x]) for x in popped)
        out[hp, 2] = sum(1 for x in popped if clean[x])
    return out


def check_stats(lib, n, m, wmax, seed):
    """Per-root settled / arcs / labels counts of both PLaNT modes."""
    g = np.random.default_rng(seed)
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, wmax + 1, m))]
    row, col, w = csr_from_edges(n, e)
    order = gg.random_rank(n, seed)
    D = floyd_warshall(n, row, col, w)
    want = expected_plant_stats(row, col, w, order, D)
    lab = oracle.chl(row, col, w, order, mode=oracle.MODE_PLANT, threads=1, lib=lib)
    assert np.array_equal(lab.stats[:, :3], want)
    full = oracle.chl(row, col, w, order, mode=oracle.MODE_PLANT_FULL, threads=1, lib=lib)
    deg = np.diff(row)
    comp = [(D[int(order[hp])] < INF) for hp in range(n)]
    assert np.array_equal(full.stats[:, 0], [c.sum() for c in comp])
    assert np.array_equal(full.stats[:, 1], [deg[c].sum() for c in comp])


def check_minimal(lib, lab, D, rng_seed=0, samples=40):
    """Removing a label breaks the cover of some pair (Definition 2)."""
    n = lab.n
    g = np.random.default_rng(rng_seed)
    idx = g.choice(lab.total, size=min(samples, lab.total), replace=False)
    Dq = np.where(D >= INF, -1, D)
    for k in idx:
        keep = np.ones(lab.total, dtype=bool)
        keep[k] = False
        v = int(np.searchsorted(lab.offsets, k, side="right") - 1)
        counts = np.diff(lab.offsets)
        counts[v] -= 1
        off = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(counts, out=off[1:])
        red = oracle.Labels(off, lab.hub_pos[keep], lab.dist[keep])
        pairs = np.stack([np.full(n, v), np.arange(n)], 1).astype(np.int32)
        q = oracle.query(red, pairs, lib=lib)
        assert not np.array_equal(q, Dq[v]), "label %d of vertex %d is redundant" % (k, v)


def check_path(lib, n, seed):
    """Path 0-1-...-(n-1) with positive weights: SP_{v,h} is the segment, so
    (h, .) in L_v iff h has the smallest rank position on the segment."""
    g = np.random.default_rng(seed)
    ws = g.integers(1, 10, n - 1)
    row, col, w = csr_from_edges(n, [(i, i + 1, int(ws[i])) for i in range(n - 1)])
    order = gg.random_rank(n, seed)
    pos = pos_of(order)
    pre = np.concatenate([[0], np.cumsum(ws)])
    want = {v: sorted((int(pos[h]), int(abs(pre[v] - pre[h]))) for h in range(n)
                      if pos[h] == pos[min(v, h):max(v, h) + 1].min()) for v in range(n)}
    for lab in all_modes(row, col, w, order, lib):
        assert oracle_labels(lab) == want


def check_star(lib, leaves, seed):
    """Star, centre 0: a leaf l gets the centre iff the centre outranks it,
    and another leaf l' iff l' outranks both l and the centre."""
    n = leaves + 1
    g = np.random.default_rng(seed)
    ws = g.integers(1, 20, leaves)
    row, col, w = csr_from_edges(n, [(0, i + 1, int(ws[i])) for i in range(leaves)])
    order = gg.random_rank(n, seed)
    pos = pos_of(order)
    want = {v: [] for v in range(n)}
    want[0].append((int(pos[0]), 0))
    for l in range(1, n):
        want[l].append((int(pos[l]), 0))
        if pos[0] < pos[l]:
            want[l].append((int(pos[0]), int(ws[l - 1])))
        else:
            want[0].append((int(pos[l]), int(ws[l - 1])))
        for l2 in range(1, n):
            if l2 != l and pos[l2] < min(pos[l], pos[0]):
                want[l].append((int(pos[l2]), int(ws[l - 1] + ws[l2 - 1])))
    for v in want:
        want[v].sort()
    for lab in all_modes(row, col, w, order, lib):
        assert oracle_labels(lab) == want


def check_complete(lib, n, seed):
    """K_n with unit weights: L_v = {(v,0)} + {(u,1) : u outranks v};
    n(n+1)/2 labels in total."""
    row, col, w = csr_from_edges(n, [(a, b, 1) for a in range(n) for b in range(a + 1, n)])
    order = gg.random_rank(n, seed)
    pos = pos_of(order)
    want = {v: sorted([(int(pos[v]), 0)] + [(int(pos[u]), 1) for u in range(n) if pos[u] < pos[v]])
            for v in range(n)}
    for lab in all_modes(row, col, w, order, lib):
        assert lab.total == n * (n + 1) // 2
        assert oracle_labels(lab) == want


def check_unit_grid(lib, a, b, seed):
    """a x b grid, unit weights: SP_{v,h} is the whole axis-aligned rectangle
    spanned by v and h, so (h, Manhattan distance) is in L_v iff h has the
    smallest rank position in that rectangle."""
    n = a * b
    edges = [(r * b + c, r * b + c + 1, 1) for r in range(a) for c in range(b - 1)]
    edges += [(r * b + c, (r + 1) * b + c, 1) for r in range(a - 1) for c in range(b)]
    row, col, w = csr_from_edges(n, edges)
    order = gg.random_rank(n, seed)
    P = pos_of(order).reshape(a, b)
    want = {v: [] for v in range(n)}
    for v in range(n):
        rv, cv = divmod(v, b)
        for h in range(n):
            rh, ch = divmod(h, b)
            rect = P[min(rv, rh):max(rv, rh) + 1, min(cv, ch):max(cv, ch) + 1]
            if P[rh, ch] == rect.min():
                want[v].append((int(P[rh, ch]), abs(rv - rh) + abs(cv - ch)))
        want[v].sort()
    for lab in all_modes(row, col, w, order, lib):
        assert oracle_labels(lab) == want


def check_even_cycle(lib, k, seed):
    """C_{2k}, unit weights: the shortest path between vertices at cyclic
    distance d < k is the unique arc; antipodal pairs (d = k) have the whole
    cycle as SP, so their label exists only for the cycle's top vertex."""
    n = 2 * k
    row, col, w = csr_from_edges(n, [(i, (i + 1) % n, 1) for i in range(n)])
    order = gg.random_rank(n, seed)
    pos = pos_of(order)
    want = {v: [] for v in range(n)}
    for v in range(n):
        for h in range(n):
            d = (h - v) % n
            if d == 0:
                sp = [v]
            elif d < k:
                sp = [(v + i) % n for i in range(d + 1)]
            elif d > k:
                sp = [(v - i) % n for i in range(n - d + 1)]
            else:
                sp = list(range(n))
            if pos[h] == min(pos[x] for x in sp):
                want[v].append((int(pos[h]), min(d, n - d)))
        want[v].sort()
    for lab in all_modes(row, col, w, order, lib):
        assert oracle_labels(lab) == want


def check_tree(lib, n, seed):
    """Random weighted tree: SP is the unique tree path; (h, .) in L_v iff h
    has the smallest rank position on it."""
    g = np.random.default_rng(seed)
    par = [int(g.integers(0, i)) for i in range(1, n)]
    ws = g.integers(1, 50, n - 1)
    edges = [(i + 1, par[i], int(ws[i])) for i in range(n - 1)]
    row, col, w = csr_from_edges(n, edges)
    order = gg.random_rank(n, seed)
    pos = pos_of(order)
    parent = [-1] + par
    pw = [0] + [int(x) for x in ws]

    def to_root(x):
        p = [x]
        while parent[p[-1]] >= 0:
            p.append(parent[p[-1]])
        return p

    want = {v: [] for v in range(n)}
    for v in range(n):
        pv = to_root(v)
        for h in range(n):
            ph = to_root(h)
            common = set(pv) & set(ph)
            lca = next(x for x in pv if x in common)
            path = pv[:pv.index(lca) + 1] + ph[:ph.index(lca)]
            dist = sum(pw[x] for x in pv[:pv.index(lca)]) + sum(pw[x] for x in ph[:ph.index(lca)])
            if pos[h] == min(pos[x] for x in path):
                want[v].append((int(pos[h]), dist))
        want[v].sort()
    for lab in all_modes(row, col, w, order, lib):
        assert oracle_labels(lab) == want


def check_sssp(lib, seed):
    g = np.random.default_rng(seed)
    n, m = 40, 90
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, 7, m))]
    row, col, w = csr_from_edges(n, e)
    D = floyd_warshall(n, row, col, w)
    for s in range(0, n, 7):
        got = oracle.sssp(row, col, w, s, lib=lib)
        assert np.array_equal(got, np.where(D[s] >= INF, -1, D[s]))


def check_pruned(lib, n, m, wmax, seed):
    """Pruned trees (Section 4.3) give the definition's labels."""
    g = np.random.default_rng(seed)
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, wmax + 1, m))]
    row, col, w = csr_from_edges(n, e)
    order = gg.random_rank(n, seed)
    want = brute_labels(floyd_warshall(n, row, col, w), order)
    for eta, grown in ((2, 2), (4, 6), (8, 8)):
        lab = oracle.chl_pruned(row, col, w, order, eta, grown, threads=2, lib=lib)
        assert oracle_labels(lab) == want, (eta, grown)
    lab = oracle.chl_pruned(row, col, w, order, levels=[2, 6, 18], pmain=18, threads=2, lib=lib)
    assert oracle_labels(lab) == want


# ---------------------------------------------------------------- shortest paths
def sp_parent(D, row, col, w, h, v):
    """Smallest-id neighbour p of v that is the next vertex of a shortest v-h
    path (D[h][p] + w(p,v) = D[h][v]), from Floyd-Warshall distances; -1 if
    none (v = h)."""
    best = -1
    for e in range(row[v], row[v + 1]):
        p = int(col[e])
        if D[h, p] < INF and D[h, p] + int(w[e]) == D[h, v] and (best < 0 or p < best):
            best = p
    return best


def check_parent_labels(lab, par, slot, D, row, col, w, order):
    """Every label's parent is the smallest-id shortest-path neighbour
    towards its hub (Floyd-Warshall), and slot points at the parent's label
    of the same hub, whose distance is D[h][parent]."""
    off, hub, dist = lab.offsets, lab.hub_pos, lab.dist
    for v in range(lab.n):
        for i in range(off[v], off[v + 1]):
            h = int(order[hub[i]])
            want = sp_parent(D, row, col, w, h, v)
            assert par[i] == want, (v, h, par[i], want)
            if want < 0:
                assert v == h and slot[i] == -1
                continue
            j = off[want] + slot[i]
            assert off[want] <= j < off[want + 1]
            assert hub[j] == hub[i] and dist[j] == D[h, want]


def check_path_walks(paths, D, row, col, w, order):
    """paths = (hops, path_off, path) for all n*n pairs in row-major order.
    Connected pairs: the path starts at u, ends at v, follows arcs whose
    weights sum to D[u][v], passes through h_m, the highest ranked vertex of
    SP_{u,v}, and both halves step to the smallest-id shortest-path
    neighbour towards h_m. Disconnected pairs: hops -1, no vertices."""
    hops, poff, path = paths
    n = len(D)
    pos = pos_of(order)
    wmin = {}
    for v in range(n):
        for e in range(row[v], row[v + 1]):
            key = (v, int(col[e]))
            wmin[key] = min(wmin.get(key, INF), int(w[e]))
    for u in range(n):
        for v in range(n):
            k = u * n + v
            P = path[poff[k]:poff[k + 1]].tolist()
            if D[u, v] >= INF:
                assert hops[k] == -1 and not P
                continue
            assert len(P) == hops[k] + 1 and P[0] == u and P[-1] == v
            assert sum(wmin[(P[t], P[t + 1])] for t in range(len(P) - 1)) == D[u, v]
            on = [x for x in range(n) if D[u, x] + D[x, v] == D[u, v]]
            hm = min(on, key=lambda x: pos[x])
            assert hm in P, (u, v, hm, P)
            a = P.index(hm)
            for half in (P[:a + 1], P[a:][::-1]):
                for t in range(len(half) - 1):
                    assert half[t + 1] == sp_parent(D, row, col, w, hm, half[t]), (u, v, half)


def check_paths_bruteforce(lib, n, m, wmax, seed):
    """Parents and all-pairs paths of a random multigraph with ties."""
    g = np.random.default_rng(seed)
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, wmax + 1, m))]
    row, col, w = csr_from_edges(n, e)
    order = gg.random_rank(n, seed)
    D = floyd_warshall(n, row, col, w)
    lab = oracle.chl(row, col, w, order, threads=2, lib=lib)
    par, slot = oracle.parents(lab, row, col, w, lib=lib)
    check_parent_labels(lab, par, slot, D, row, col, w, order)
    uu, vv = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([uu.ravel(), vv.ravel()], 1).astype(np.int32)
    check_path_walks(oracle.paths(lab, par, slot, pairs, lib=lib), D, row, col, w, order)


def check_path_graph_walks(lib, n, seed):
    """Path 0-1-...-(n-1): the shortest u-v path is the segment between them."""
    g = np.random.default_rng(seed)
    ws = g.integers(1, 10, n - 1)
    row, col, w = csr_from_edges(n, [(i, i + 1, int(ws[i])) for i in range(n - 1)])
    order = gg.random_rank(n, seed)
    lab = oracle.chl(row, col, w, order, threads=2, lib=lib)
    par, slot = oracle.parents(lab, row, col, w, lib=lib)
    uu, vv = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([uu.ravel(), vv.ravel()], 1).astype(np.int32)
    hops, poff, path = oracle.paths(lab, par, slot, pairs, lib=lib)
    for k, (u, v) in enumerate(pairs.tolist()):
        step = 1 if v >= u else -1
        assert path[poff[k]:poff[k + 1]].tolist() == list(range(u, v + step, step))
        assert hops[k] == abs(u - v)


# ---------------------------------------------------------------- directed graphs
def csr_from_arcs(n, arcs):
    """Out-arc CSR of directed arcs (u, v, w); may hold parallel arcs and loops."""
    a = np.asarray(list(arcs), dtype=np.int64).reshape(-1, 3)
    p = np.lexsort((a[:, 1], a[:, 0]))
    a = a[p]
    row = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(a[:, 0], minlength=n), out=row[1:])
    return row, a[:, 1].astype(np.int32), a[:, 2].astype(np.int32)


def check_directed_bruteforce(lib, n, m, wmax, seed):
    """Random directed multigraph: L_out(v) holds (h, d(v,h)) exactly when h
    tops every shortest v->h path, L_in(v) holds (h, d(h,v)) exactly when h
    tops every shortest h->v path (the definition on Floyd-Warshall
    distances of the arcs, and of the reversed arcs), and the merge of
    L_out(u) with L_in(v) gives d(u, v) for all pairs."""
    g = np.random.default_rng(seed)
    a = [(int(x), int(y), int(z)) for x, y, z in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, wmax + 1, m))]
    row, col, w = csr_from_arcs(n, a)
    order = gg.random_rank(n, seed)
    D = floyd_warshall(n, row, col, w)
    want_out, want_in = brute_labels(D, order), brute_labels(np.ascontiguousarray(D.T), order)
    for mode in (oracle.MODE_PLANT, oracle.MODE_PLANT_FULL):
        lo, li = oracle.chl_directed(row, col, w, order, mode=mode, threads=2, lib=lib)
        assert oracle_labels(lo) == want_out and oracle_labels(li) == want_in, mode
    uu, vv = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([uu.ravel(), vv.ravel()], 1).astype(np.int32)
    q = oracle.query_directed(lo, li, pairs, lib=lib).reshape(n, n)
    assert np.array_equal(q, np.where(D >= INF, -1, D))


def check_directed_cycle(lib, n, seed):
    """Directed cycle 0 -> 1 -> ... -> n-1 -> 0: the only v->h path runs
    forward around the cycle, so (h, .) is in L_out(v) iff h has the
    smallest rank position on the arc v..h, and in L_in(v) iff on h..v."""
    g = np.random.default_rng(seed)
    ws = g.integers(1, 9, n)
    row, col, w = csr_from_arcs(n, [(i, (i + 1) % n, int(ws[i])) for i in range(n)])
    order = gg.random_rank(n, seed)
    pos = pos_of(order)

    def seg(a, b):                    # vertices a, a+1, ..., b (mod n) and the length a -> b
        k = (b - a) % n
        vs = [(a + t) % n for t in range(k + 1)]
        return vs, int(sum(ws[(a + t) % n] for t in range(k)))

    want_out = {v: [] for v in range(n)}
    want_in = {v: [] for v in range(n)}
    for v in range(n):
        for h in range(n):
            vs, d = seg(v, h)
            if min(pos[x] for x in vs) == pos[h]:
                want_out[v].append((int(pos[h]), d))
            vs, d = seg(h, v)
            if min(pos[x] for x in vs) == pos[h]:
                want_in[v].append((int(pos[h]), d))
    for v in range(n):
        want_out[v].sort()
        want_in[v].sort()
    lo, li = oracle.chl_directed(row, col, w, order, threads=2, lib=lib)
    assert oracle_labels(lo) == want_out and oracle_labels(li) == want_in


def check_symmetric_as_directed(lib, n, m, seed):
    """An undirected graph given as its two arcs per edge: both label sets
    equal the undirected labeling."""
    g = np.random.default_rng(seed)
    e = [(int(a), int(b), int(c)) for a, b, c in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, 4, m))]
    row, col, w = csr_from_edges(n, e)
    order = gg.random_rank(n, seed)
    lab = oracle.chl(row, col, w, order, mode=oracle.MODE_DEFINITION, threads=2, lib=lib)
    lo, li = oracle.chl_directed(row, col, w, order, threads=2, lib=lib)
    assert oracle_labels(lo) == oracle_labels(lab) == oracle_labels(li)


def check_directed_pruned(lib, n, m, wmax, seed):
    """Rank-prefix pruning on the combined graph of a directed graph (the
    graph and its reversal, ranks interleaved; d(h, x) from the out-labels,
    d(x, u) from the in-labels of the prefix): both label sets equal the
    definition on Floyd-Warshall distances, for several level schedules,
    odd prefix sizes included."""
    g = np.random.default_rng(seed)
    a = [(int(x), int(y), int(z)) for x, y, z in
         zip(g.integers(0, n, m), g.integers(0, n, m), g.integers(1, wmax + 1, m))]
    row, col, w = csr_from_arcs(n, a)
    order = gg.random_rank(n, seed)
    D = floyd_warshall(n, row, col, w)
    want_out, want_in = brute_labels(D, order), brute_labels(np.ascontiguousarray(D.T), order)
    r2, c2, w2, o2 = oracle.combined_directed(row, col, w, order)
    for lv, pm in (([2, 6, 18], 18), ([3, 7, 21], 21), ([4], 4)):
        lab = oracle.chl_pruned(r2, c2, w2, o2, levels=lv, pmain=pm, half=n, threads=2, lib=lib)
        lo, li = oracle.split_combined(lab, n)
        assert oracle_labels(lo) == want_out and oracle_labels(li) == want_in, (lv, pm)


def run_all(lib):
    """Every pin, smallish; used against planted mistakes."""
    check_golden(lib, "fig1_example.txt")
    check_golden(lib, "reading1_counterexample.txt")
    for s in range(6):
        check_bruteforce(lib, 24, 40, 3, s)
        check_bruteforce(lib, 30, 45, 2, 100 + s, rank="degree")
    check_path(lib, 12, 1)
    check_star(lib, 7, 2)
    check_complete(lib, 7, 3)
    check_unit_grid(lib, 4, 5, 4)
    check_even_cycle(lib, 5, 5)
    check_tree(lib, 15, 6)
    check_sssp(lib, 7)
    for s in range(4):
        check_stats(lib, 20, 34, 2, 200 + s)
    for s in range(4):
        check_pruned(lib, 26, 44, 3, 300 + s)
    for s in range(4):
        check_paths_bruteforce(lib, 22, 40, 2 + s % 2, 400 + s)
    check_path_graph_walks(lib, 14, 8)
    for s in range(4):
        check_directed_bruteforce(lib, 20, 50, 1 + s % 3, 600 + s)
    check_directed_cycle(lib, 9, 3)
    check_symmetric_as_directed(lib, 25, 40, 7)
    for s in range(3):
        check_directed_pruned(lib, 24, 70, 1 + s, 800 + s)
