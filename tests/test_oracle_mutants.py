"""Plant plausible mistakes in a copy of the oracle source (CPU only) and
check that the pins of tests/pins.py catch every one of them."""
import os

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "chl_oracle.c")

MUTANTS = {
    # Algorithm 3: drop the equal-distance ancestor update (tie rule)
    "no_tie_rule": ("else if (nd == delta[u]) a[u] = top_of(pos, nA, pA);", ";"),
    # Algorithm 3 read literally: an outranked vertex is not relaxed
    "prune_tree": ("out_v[nl] = v; out_d[nl] = delta[v]; nl++;\n        }",
                   "out_v[nl] = v; out_d[nl] = delta[v]; nl++;\n        } else continue;"),
    # rank direction flipped in argmax R
    "rank_flip": ("return pos[x] < pos[y] ? x : y;", "return pos[x] > pos[y] ? x : y;"),
    # cnt never grows: early termination fires too soon
    "cnt_no_inc": ("if (a[u] == h && pA != h) cnt++;", "if (a[u] == h && pA != h) {}"),
    # cnt never shrinks on ancestor change
    "cnt_no_dec": ("else if (a[u] != h && pA == h) cnt--;", ";"),
    # definition: a vertex of equal rank counted as outranking (drops self label)
    "def_self": ("uint8_t o = pos[v] < pos[h];", "uint8_t o = pos[v] <= pos[h];"),
    # definition: any closer neighbour treated as a shortest-path predecessor
    "def_pred": ("w->dist[p] + wt[e] == w->dist[v]", "w->dist[p] < w->dist[v]"),
    # edge weight dropped in the relaxation
    "unit_weight": ("int64_t nd = delta[v] + wt[e];", "int64_t nd = delta[v] + 1;"),
    # heap ordered by rank instead of distance
    "heap_order": ("return x->d < y->d || (x->d == y->d && x->p < y->p);",
                   "return x->p < y->p || (x->p == y->p && x->d < y->d);"),
    # query keeps the largest common-hub sum
    "query_max": ("if (best < 0 || s < best) best = s;", "if (best < 0 || s > best) best = s;"),
    # query merge advances the wrong list
    "query_skip": ("if (hub[i] < hub[j]) i++;", "if (hub[i] < hub[j]) j++;"),
    # sparse reset forgets the ancestor array
    "reset_anc": ("w->dist[v] = INF64; w->anc[v] = v;", "w->dist[v] = INF64;"),
    # pruning threshold one too high: drops shortest clean candidates
    "prune_threshold": ("prefix_query(P, h, u) <= nd) continue;", "prefix_query(P, h, u) <= nd + 1) continue;"),
    # prefix label distances one too small: over-pruning
    "prefix_dist": ("P->dist[k] = ld[t][i];", "P->dist[k] = ld[t][i] - 1;"),
    # sssp: wrong weight index
    # parent: largest-id shortest-path neighbour instead of the smallest
    "parent_max": ("if (best < 0 || p < best) { best = p;", "if (best < 0 || p > best) { best = p;"),
    # parent: any closer neighbour holding the hub taken as the next vertex
    "parent_dist": ("if (j < 0 || dist[j] + wt[e] != dist[i]) continue;",
                    "if (j < 0 || dist[j] >= dist[i]) continue;"),
    # path: the least important hub among equal sums
    "path_tie": ("if (best < 0 || s < best) { best = s; bi = i; bj = j; }",
                 "if (best < 0 || s <= best) { best = s; bi = i; bj = j; }"),
    # path: v's half not reversed
    "path_reverse": ("o[hu + 1 + t] = tmp[hv - 1 - t];", "o[hu + 1 + t] = tmp[t];"),
    # directed query keeps the largest common-hub sum
    "query2_max": ("int64_t s = dist_out[i] + dist_in[j];\n                if (best < 0 || s < best) best = s;",
                   "int64_t s = dist_out[i] + dist_in[j];\n                if (best < 0 || s > best) best = s;"),
    # directed query merge advances the wrong list
    "query2_skip": ("if (hub_out[i] < hub_in[j]) i++;", "if (hub_out[i] < hub_in[j]) j++;"),
    # directed pruning: the root's own in-labels taken for d(h, x)
    "dir_prune_side": ("const int32_t flip = P->half ? 1 : 0;", "const int32_t flip = 0;"),
    "sssp_w": ("int64_t nd = it.d + wt[e];\n            if (nd < out[col[e]])",
               "int64_t nd = it.d + wt[row_ptr[it.v]];\n            if (nd < out[col[e]])"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation site not found: " + name
    mut = tmp_path / ("m_%s.c" % name)
    mut.write_text(src.replace(old, new))
    so = str(tmp_path / ("m_%s.so" % name))
    oracle.build(src=str(mut), out=so)
    lib = oracle.load(so)
    with pytest.raises(AssertionError):
        pins.run_all(lib)
