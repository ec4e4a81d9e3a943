/*
 * Drives every entry point of the CPU oracle (oracle/chl_oracle.c) on small
 * random multigraphs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitize.py). It also checks that
 * the definition and the PLaNT trees (with and without early termination,
 * and with rank-prefix pruning) give the same labels, so a run exercises
 * the same code as the pinned tests.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oracle_run oracle_run;
oracle_run* oracle_run_roots(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* wt,
                             const int32_t* order, const int32_t* roots, int64_t nroots, int mode, int nthreads);
oracle_run* oracle_run_roots_levels(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* wt,
                                    const int32_t* order, const int32_t* roots, int64_t nroots,
                                    const int32_t* bounds, int32_t nb, int32_t pmain, int32_t half, int nthreads);
int64_t oracle_run_total(const oracle_run* R);
int64_t oracle_run_count(const oracle_run* R, int64_t t);
void oracle_run_labels(const oracle_run* R, int64_t t, int32_t* v, int64_t* d);
void oracle_run_stats(const oracle_run* R, int64_t* out);
void oracle_run_assemble(const oracle_run* R, int64_t* offsets, int32_t* hub_pos, int64_t* dist);
void oracle_run_free(oracle_run* R);
void oracle_query(const int64_t* offsets, const int32_t* hub_pos, const int64_t* dist, const int32_t* pairs,
                  int64_t q, int64_t* out);
void oracle_query2(const int64_t* off_out, const int32_t* hub_out, const int64_t* dist_out, const int64_t* off_in,
                   const int32_t* hub_in, const int64_t* dist_in, const int32_t* pairs, int64_t q, int64_t* out);
void oracle_sssp(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* wt, int32_t src, int64_t* out);
void oracle_parents(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* wt, const int64_t* off,
                    const int32_t* hub, const int64_t* dist, int32_t* parent, int32_t* slot);
void oracle_paths(const int64_t* off, const int32_t* hub, const int64_t* dist, const int32_t* parent,
                  const int32_t* slot, const int32_t* pairs, int64_t q, int64_t* hops, const int64_t* path_off,
                  int32_t* path);

static uint64_t rs = 88172645463325252ull;
static uint32_t rnd(uint32_t k) {   /* xorshift64 (Marsaglia 2003), uniform-ish in [0, k) */
    rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;
    return (uint32_t)(rs % k);
}

typedef struct { int64_t* off; int32_t* hub; int64_t* dist; int64_t total; } labeling;

static labeling run_all(int32_t n, const int64_t* row, const int32_t* col, const int32_t* w, const int32_t* order,
                    int mode, const int32_t* bounds, int nb) {
    oracle_run* R = nb ? oracle_run_roots_levels(n, row, col, w, order, NULL, 0, bounds, nb, bounds[nb - 1], 0, 3)
                       : oracle_run_roots(n, row, col, w, order, NULL, 0, mode, 3);
    labeling L;
    L.total = oracle_run_total(R);
    L.off = malloc(sizeof(int64_t) * (size_t)(n + 1));
    L.hub = malloc(sizeof(int32_t) * (size_t)(L.total + 1));
    L.dist = malloc(sizeof(int64_t) * (size_t)(L.total + 1));
    oracle_run_assemble(R, L.off, L.hub, L.dist);
    int64_t* st = malloc(sizeof(int64_t) * 4 * (size_t)n);
    oracle_run_stats(R, st);
    for (int64_t t = 0; t < n; t++) {
        int64_t c = oracle_run_count(R, t);
        int32_t* v = malloc(sizeof(int32_t) * (size_t)(c + 1));
        int64_t* d = malloc(sizeof(int64_t) * (size_t)(c + 1));
        oracle_run_labels(R, t, v, d);
        free(v); free(d);
    }
    free(st);
    oracle_run_free(R);
    return L;
}

static int same(const labeling* a, const labeling* b, int32_t n) {
    if (a->total != b->total) return 0;
    return !memcmp(a->off, b->off, sizeof(int64_t) * (size_t)(n + 1)) &&
           !memcmp(a->hub, b->hub, sizeof(int32_t) * (size_t)a->total) &&
           !memcmp(a->dist, b->dist, sizeof(int64_t) * (size_t)a->total);
}

static void drop(labeling* L) { free(L->off); free(L->hub); free(L->dist); }

int main(int argc, char** argv) {
    int iters = argc > 1 ? atoi(argv[1]) : 300;
    for (int it = 0; it < iters; it++) {
        int32_t n = 2 + (int32_t)rnd(90);
        int32_t m = n / 2 + (int32_t)rnd(3 * (uint32_t)n);
        int32_t wmax = 1 + (int32_t)rnd(5);
        /* symmetric CSR of m random edges (self-loops and parallel edges kept) */
        int32_t* eu = malloc(sizeof(int32_t) * (size_t)m);
        int32_t* ev = malloc(sizeof(int32_t) * (size_t)m);
        int32_t* ew = malloc(sizeof(int32_t) * (size_t)m);
        int64_t* row = calloc((size_t)n + 1, sizeof(int64_t));
        for (int32_t e = 0; e < m; e++) {
            eu[e] = (int32_t)rnd((uint32_t)n); ev[e] = (int32_t)rnd((uint32_t)n); ew[e] = 1 + (int32_t)rnd((uint32_t)wmax);
            row[eu[e] + 1]++; row[ev[e] + 1]++;
        }
        for (int32_t v = 0; v < n; v++) row[v + 1] += row[v];
        int32_t* col = malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
        int32_t* w = malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
        int64_t* fill = calloc((size_t)n, sizeof(int64_t));
        for (int32_t e = 0; e < m; e++) {
            int64_t a = row[eu[e]] + fill[eu[e]]++, b = row[ev[e]] + fill[ev[e]]++;
            col[a] = ev[e]; w[a] = ew[e]; col[b] = eu[e]; w[b] = ew[e];
        }
        int32_t* order = malloc(sizeof(int32_t) * (size_t)n);
        for (int32_t i = 0; i < n; i++) order[i] = i;
        for (int32_t i = n - 1; i > 0; i--) { int32_t j = (int32_t)rnd((uint32_t)i + 1); int32_t t = order[i]; order[i] = order[j]; order[j] = t; }

        labeling D = run_all(n, row, col, w, order, 0, NULL, 0);
        labeling P = run_all(n, row, col, w, order, 1, NULL, 0);
        labeling F = run_all(n, row, col, w, order, 2, NULL, 0);
        int32_t bounds[3] = {1 + n / 8, 1 + n / 4, 1 + n / 2};
        labeling Q = run_all(n, row, col, w, order, 1, bounds, 3);
        if (!same(&D, &P, n) || !same(&D, &F, n) || !same(&D, &Q, n)) {
            fprintf(stderr, "iteration %d: labelings differ\n", it);
            return 1;
        }
        /* queries against Dijkstra, parents and paths */
        int32_t q = 64;
        int32_t* pairs = malloc(sizeof(int32_t) * 2 * (size_t)q);
        for (int32_t k = 0; k < 2 * q; k++) pairs[k] = (int32_t)rnd((uint32_t)n);
        int64_t* out = malloc(sizeof(int64_t) * (size_t)q);
        int64_t* sp = malloc(sizeof(int64_t) * (size_t)n);
        oracle_query(D.off, D.hub, D.dist, pairs, q, out);
        for (int32_t k = 0; k < q; k++) {
            oracle_sssp(n, row, col, w, pairs[2 * k], sp);
            if (sp[pairs[2 * k + 1]] != out[k]) { fprintf(stderr, "iteration %d: query %d wrong\n", it, k); return 1; }
        }
        oracle_query2(D.off, D.hub, D.dist, D.off, D.hub, D.dist, pairs, q, out);
        int32_t* par = malloc(sizeof(int32_t) * (size_t)(D.total + 1));
        int32_t* slot = malloc(sizeof(int32_t) * (size_t)(D.total + 1));
        oracle_parents(n, row, col, w, D.off, D.hub, D.dist, par, slot);
        int64_t* hops = malloc(sizeof(int64_t) * (size_t)q);
        oracle_paths(D.off, D.hub, D.dist, par, slot, pairs, q, hops, NULL, NULL);
        int64_t* poff = malloc(sizeof(int64_t) * (size_t)(q + 1));
        poff[0] = 0;
        for (int32_t k = 0; k < q; k++) poff[k + 1] = poff[k] + (hops[k] >= 0 ? hops[k] + 1 : 0);
        int32_t* path = malloc(sizeof(int32_t) * (size_t)(poff[q] + 1));
        oracle_paths(D.off, D.hub, D.dist, par, slot, pairs, q, hops, poff, path);
        free(path); free(poff); free(hops); free(par); free(slot); free(sp); free(out); free(pairs);
        drop(&D); drop(&P); drop(&F); drop(&Q);
        free(eu); free(ev); free(ew); free(row); free(col); free(w); free(fill); free(order);
    }
    printf("oracle driver: %d graphs ok\n", iters);
    return 0;
}
