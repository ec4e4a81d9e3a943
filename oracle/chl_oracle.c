/*
 * CPU oracle for the Canonical Hub Labeling (CHL) -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this file's library. It shares no code, header or table with the
 * HIP library and must never be reached from the product path.
 *
 * Everything here is plain, sequential per root, and int64 in distances.
 * Vertices keep their input ids; the ranking enters only through
 * pos[v] = rank position (pos[order[i]] = i, 0 = most important), so that
 * "x outranks y" (R(x) > R(y) in the paper's notation) is pos[x] < pos[y].
 *
 * Two independent computations of the labels with hub h (root h):
 *
 *  (1) oracle_def_tree -- the definition. A label (h, d(v,h)) belongs to L_v
 *      exactly when h is the highest ranked vertex of SP_{v,h}, the set of
 *      vertices on all shortest v-h paths, inclusive (Section 1, CHL of
 *      Abraham et al. and the notation table; Lemma 1 of Section 3.1 states
 *      the converse, that any other label is redundant). It runs a complete
 *      Dijkstra from h, then walks the vertices in order of distance and marks
 *      v "outranked" when v itself outranks h or some shortest-path
 *      predecessor p (d(h,p) + w(p,v) = d(h,v)) is outranked; this is the
 *      recursion SP_{h,v} = {v} U (union over those p of SP_{h,p}).
 *
 *  (2) oracle_plant_tree -- the PLaNTDijkstra procedure (Section 4.2,
 *      Algorithm 3) in the paper's order and notation: distances delta[],
 *      most-important-ancestor a[], the equal-distance ancestor update, and
 *      the counter cnt of queued vertices whose ancestor is the root, used
 *      for early termination. Two readings are taken where the printed
 *      algorithm is ambiguous:
 *        - the "skip if an ancestor outranks the root" test skips only the
 *          label, never the relaxation of the vertex's edges (PLaNT prunes
 *          labels, not trees: Section 1 and the footnote on early
 *          termination in Section 4.2);
 *        - cnt counts queued, not yet popped, vertices whose ancestor is the
 *          root, and is tested before every pop.
 *      The heap pops by (distance, rank position); this tie order fixes the
 *      counted work (vertices settled, arcs scanned) but not the labels.
 *
 * oracle_chl() runs one of them for every root (roots handed out to
 * threads by an atomic counter in rank order, the paper's task queue of
 * Section 3.1) and assembles L_v sorted by hub rank position, most important
 * hub first (Algorithm 2's sort step; the query merge of Section 5 relies on
 * it). oracle_query() answers distance queries by the sorted-list merge of
 * Section 5 (QLSN): the minimum of d_u + d_v over common hubs, -1 when the
 * lists share no hub. The definition form scans a vertex's own row for its
 * shortest-path predecessors, so it needs a symmetric graph; for a directed
 * graph the PLaNT form run on the graph gives the in-labels (trees grown
 * along the arcs) and run on the reversed graph the out-labels, and
 * oracle_query2() merges L_out(u) with L_in(v). oracle_parents() and
 * oracle_paths() add the shortest-path extension of Section 4.4: per label
 * the next vertex towards its hub, and paths as two chains of parents joined
 * at the common hub.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define INF64 INT64_MAX

/* ---------------- binary heap of (dist, pos, v) ---------------- */
typedef struct { int64_t d; int32_t p; int32_t v; } hitem;
typedef struct { hitem* a; int64_t size, cap; } heap_t;

static int hless(const hitem* x, const hitem* y) {
    return x->d < y->d || (x->d == y->d && x->p < y->p);
}
static void hpush(heap_t* h, hitem it) {
    if (h->size == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->a = (hitem*)realloc(h->a, (size_t)h->cap * sizeof(hitem));
    }
    int64_t i = h->size++;
    while (i > 0) {
        int64_t par = (i - 1) / 2;
        if (!hless(&it, &h->a[par])) break;
        h->a[i] = h->a[par];
        i = par;
    }
    h->a[i] = it;
}
static hitem hpop(heap_t* h) {
    hitem top = h->a[0];
    hitem last = h->a[--h->size];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= h->size) break;
        if (c + 1 < h->size && hless(&h->a[c + 1], &h->a[c])) c++;
        if (!hless(&h->a[c], &last)) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->size > 0) h->a[i] = last;
    return top;
}

/* ---------------- per-thread workspace ---------------- */
typedef struct {
    int32_t n;
    int64_t* dist;      /* delta[] */
    int32_t* anc;       /* a[] (PLaNT) */
    uint8_t* settled;
    uint8_t* outr;      /* outranked flag (definition) */
    int32_t* touched;   /* vertices whose state left its initial value */
    int64_t ntouched;
    int32_t* popped;    /* pop order (definition) */
    heap_t heap;
} ws_t;

static ws_t* ws_new(int32_t n) {
    ws_t* w = (ws_t*)calloc(1, sizeof(ws_t));
    w->n = n;
    w->dist = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    w->anc = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    w->settled = (uint8_t*)calloc((size_t)n, 1);
    w->outr = (uint8_t*)calloc((size_t)n, 1);
    w->touched = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    w->popped = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    for (int32_t v = 0; v < n; v++) { w->dist[v] = INF64; w->anc[v] = v; }
    return w;
}
static void ws_free(ws_t* w) {
    free(w->dist); free(w->anc); free(w->settled); free(w->outr);
    free(w->touched); free(w->popped); free(w->heap.a); free(w);
}
/* restore every touched entry to its initial value (sparse re-initialisation) */
static void ws_reset(ws_t* w) {
    for (int64_t i = 0; i < w->ntouched; i++) {
        int32_t v = w->touched[i];
        w->dist[v] = INF64; w->anc[v] = v; w->settled[v] = 0; w->outr[v] = 0;
    }
    w->ntouched = 0;
    w->heap.size = 0;
}

typedef struct { int64_t settled, arcs, labels; int32_t early; } tree_stats;

/* (1) definition: labels with hub h. out_v/out_d receive the labelled
 * vertices and distances (capacity n). Returns the label count. */
int64_t oracle_def_tree(ws_t* w, const int64_t* row_ptr, const int32_t* col,
                        const int32_t* wt, const int32_t* pos, int32_t h,
                        int32_t* out_v, int64_t* out_d, tree_stats* st) {
    int64_t npop = 0, arcs = 0;
    w->dist[h] = 0; w->touched[w->ntouched++] = h;
    hpush(&w->heap, (hitem){0, pos[h], h});
    while (w->heap.size) {                       /* plain Dijkstra, no pruning */
        hitem it = hpop(&w->heap);
        int32_t v = it.v;
        if (w->settled[v] || it.d != w->dist[v]) continue;
        w->settled[v] = 1;
        w->popped[npop++] = v;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int32_t u = col[e];
            int64_t nd = it.d + wt[e];
            arcs++;
            if (nd < w->dist[u]) {
                if (w->dist[u] == INF64) w->touched[w->ntouched++] = u;
                w->dist[u] = nd;
                hpush(&w->heap, (hitem){nd, pos[u], u});
            }
        }
    }
    int64_t nl = 0;
    for (int64_t i = 0; i < npop; i++) {         /* non-decreasing distance */
        int32_t v = w->popped[i];
        uint8_t o = pos[v] < pos[h];
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1] && !o; e++) {
            int32_t p = col[e];
            if (w->dist[p] != INF64 && w->dist[p] + wt[e] == w->dist[v]) o |= w->outr[p];
        }
        w->outr[v] = o;
        if (!o) { out_v[nl] = v; out_d[nl] = w->dist[v]; nl++; }
    }
    if (st) { st->settled = npop; st->arcs = arcs; st->labels = nl; st->early = 0; }
    ws_reset(w);
    return nl;
}

/* argmax of R over {x, y}: the one with the smaller rank position */
static inline int32_t top_of(const int32_t* pos, int32_t x, int32_t y) {
    return pos[x] < pos[y] ? x : y;
}

/* Prefix labels used for pruning (Section 4.3): for every vertex, its labels
 * whose hub has rank position < e, sorted by hub; all of them are final once
 * the trees of the roots at rank positions < e are done. */
typedef struct {
    int32_t e;
    int64_t* off;      /* [n+1] */
    int32_t* hub;      /* rank positions */
    int64_t* dist;
    int32_t half;      /* combined graph of a directed graph: n/2, else 0 */
} prefix_t;

/* Length of the shortest root-u walk through a hub of the prefix: the
 * minimum of d(h,x) + d(x,u) over prefix hubs x in both label sets
 * (INF64 if none). On the combined graph of a directed graph (the graph on
 * ids [0, half), its reversal on [half, 2 half), rank positions interleaved:
 * v at 2 pos(v), its reversed copy at 2 pos(v) + 1), d(x,u) is u's label
 * from x, and d(h,x) is the label of h's copy in the other half from x's
 * copy, at rank position x ^ 1 (the footnote of Section 1 gives a directed
 * graph forward and backward labels; the test itself is Section 4.3's). */
static int64_t prefix_query(const prefix_t* P, int32_t h, int32_t u) {
    const int32_t flip = P->half ? 1 : 0;
    const int32_t hg = flip ? (h < P->half ? h + P->half : h - P->half) : h;
    int64_t i = P->off[hg], ie = P->off[hg + 1], j = P->off[u], je = P->off[u + 1];
    int64_t best = INF64;
    while (i < ie && j < je) {
        const int32_t xh = P->hub[i] ^ flip;
        if (xh < P->hub[j]) i++;
        else if (xh > P->hub[j]) j++;
        else {
            int64_t s = P->dist[i] + P->dist[j];
            if (s < best) best = s;
            i++; j++;
        }
    }
    return best;
}

/* (2) PLaNTDijkstra (Algorithm 3) with the readings stated above. With a
 * prefix P (roots below P->e done, h not among them), a relaxation whose
 * tentative distance is not below the prefix query of (h, u) is skipped:
 * such a candidate is either not shortest or runs through a prefix hub,
 * which outranks h, so it cannot produce a label (Section 4.3). */
static int64_t plant_tree_p(ws_t* w, const int64_t* row_ptr, const int32_t* col,
                            const int32_t* wt, const int32_t* pos, int32_t h,
                            int early_term, const prefix_t* P, int32_t* out_v, int64_t* out_d,
                            tree_stats* st);

int64_t oracle_plant_tree(ws_t* w, const int64_t* row_ptr, const int32_t* col,
                          const int32_t* wt, const int32_t* pos, int32_t h,
                          int early_term, int32_t* out_v, int64_t* out_d,
                          tree_stats* st) {
    return plant_tree_p(w, row_ptr, col, wt, pos, h, early_term, NULL, out_v, out_d, st);
}

static int64_t plant_tree_p(ws_t* w, const int64_t* row_ptr, const int32_t* col,
                            const int32_t* wt, const int32_t* pos, int32_t h,
                            int early_term, const prefix_t* P, int32_t* out_v, int64_t* out_d,
                            tree_stats* st) {
    int64_t* delta = w->dist;
    int32_t* a = w->anc;
    int64_t nl = 0, npop = 0, arcs = 0, cnt;
    int32_t stopped = 0;
    delta[h] = 0; a[h] = h; w->touched[w->ntouched++] = h;
    hpush(&w->heap, (hitem){0, pos[h], h});
    cnt = 1;
    while (w->heap.size) {
        if (early_term && cnt == 0) { stopped = 1; break; }   /* early termination */
        hitem it = hpop(&w->heap);
        int32_t v = it.v;
        if (w->settled[v] || it.d != delta[v]) continue;     /* stale queue entry */
        w->settled[v] = 1;
        npop++;
        int32_t nA = top_of(pos, v, a[v]);
        if (a[v] == h) cnt--;
        if (!(pos[nA] < pos[h])) {                           /* R[nA] > R[h] skips the label only */
            out_v[nl] = v; out_d[nl] = delta[v]; nl++;
        }
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int32_t u = col[e];
            int64_t nd = delta[v] + wt[e];
            int32_t pA = a[u];
            arcs++;
            if (P && nd <= delta[u] && prefix_query(P, h, u) <= nd) continue;   /* pruned */
            if (nd < delta[u]) a[u] = top_of(pos, nA, u);
            else if (nd == delta[u]) a[u] = top_of(pos, nA, pA);
            if (a[u] == h && pA != h) cnt++;
            else if (a[u] != h && pA == h) cnt--;
            if (nd < delta[u]) {
                if (delta[u] == INF64) w->touched[w->ntouched++] = u;
                delta[u] = nd;
                hpush(&w->heap, (hitem){nd, pos[u], u});
            }
        }
    }
    if (st) { st->settled = npop; st->arcs = arcs; st->labels = nl; st->early = stopped && w->heap.size > 0; }
    ws_reset(w);
    return nl;
}

/* ---------------- whole-labeling driver ---------------- */
typedef struct {
    int32_t n;
    const int64_t* row_ptr; const int32_t* col; const int32_t* wt;
    int32_t* pos; const int32_t* order;
    int mode;                       /* 0 definition, 1 PLaNT + early term, 2 PLaNT without */
    const prefix_t* prefix;         /* pruning labels, or NULL */
    const int32_t* roots; int64_t nroots;   /* root rank positions to run */
    _Atomic int64_t next;
    int32_t** lv; int64_t** ld; int64_t* cnt;  /* per task (index into roots) */
    tree_stats* stats;
} job_t;

static void* worker(void* arg) {
    job_t* J = (job_t*)arg;
    ws_t* w = ws_new(J->n);
    int32_t* bv = (int32_t*)malloc((size_t)J->n * sizeof(int32_t));
    int64_t* bd = (int64_t*)malloc((size_t)J->n * sizeof(int64_t));
    for (;;) {
        int64_t t = atomic_fetch_add(&J->next, 1);
        if (t >= J->nroots) break;
        int32_t h = J->order[J->roots[t]];
        tree_stats st;
        int64_t nl = J->mode == 0
            ? oracle_def_tree(w, J->row_ptr, J->col, J->wt, J->pos, h, bv, bd, &st)
            : plant_tree_p(w, J->row_ptr, J->col, J->wt, J->pos, h, J->mode == 1,
                           J->prefix && J->pos[h] >= J->prefix->e ? J->prefix : NULL, bv, bd, &st);
        J->lv[t] = (int32_t*)malloc((size_t)(nl ? nl : 1) * sizeof(int32_t));
        J->ld[t] = (int64_t*)malloc((size_t)(nl ? nl : 1) * sizeof(int64_t));
        memcpy(J->lv[t], bv, (size_t)nl * sizeof(int32_t));
        memcpy(J->ld[t], bd, (size_t)nl * sizeof(int64_t));
        J->cnt[t] = nl;
        J->stats[t] = st;
    }
    free(bv); free(bd); ws_free(w);
    return NULL;
}

typedef struct {
    int32_t n; int64_t nroots;
    int32_t* roots;                  /* root rank positions, in task order */
    int32_t** lv; int64_t** ld; int64_t* cnt;
    tree_stats* stats;
} oracle_run;

static int32_t* make_pos(int32_t n, const int32_t* order) {
    int32_t* pos = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    for (int32_t i = 0; i < n; i++) pos[order[i]] = i;
    return pos;
}

/* Run the trees of the given root rank positions (roots == NULL: all, in
 * rank order). Returns a handle holding per-root labels and statistics. */
static oracle_run* run_roots_p(int32_t n, const int64_t* row_ptr, const int32_t* col,
                               const int32_t* wt, const int32_t* order,
                               const int32_t* roots, int64_t nroots, int mode,
                               int nthreads, const prefix_t* prefix) {
    oracle_run* R = (oracle_run*)calloc(1, sizeof(oracle_run));
    R->n = n;
    if (!roots) nroots = n;
    R->nroots = nroots;
    R->roots = (int32_t*)malloc((size_t)(nroots ? nroots : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < nroots; i++) R->roots[i] = roots ? roots[i] : (int32_t)i;
    R->lv = (int32_t**)calloc((size_t)(nroots ? nroots : 1), sizeof(int32_t*));
    R->ld = (int64_t**)calloc((size_t)(nroots ? nroots : 1), sizeof(int64_t*));
    R->cnt = (int64_t*)calloc((size_t)(nroots ? nroots : 1), sizeof(int64_t));
    R->stats = (tree_stats*)calloc((size_t)(nroots ? nroots : 1), sizeof(tree_stats));
    job_t J = {0};
    J.n = n; J.row_ptr = row_ptr; J.col = col; J.wt = wt; J.order = order;
    J.pos = make_pos(n, order); J.mode = mode; J.roots = R->roots; J.nroots = nroots;
    J.prefix = prefix;
    atomic_init(&J.next, 0);
    J.lv = R->lv; J.ld = R->ld; J.cnt = R->cnt; J.stats = R->stats;
    if (nthreads < 1) nthreads = 1;
    pthread_t* th = (pthread_t*)malloc((size_t)nthreads * sizeof(pthread_t));
    for (int i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, worker, &J);
    for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    free(th); free(J.pos);
    return R;
}

oracle_run* oracle_run_roots(int32_t n, const int64_t* row_ptr, const int32_t* col,
                             const int32_t* wt, const int32_t* order,
                             const int32_t* roots, int64_t nroots, int mode,
                             int nthreads) {
    return run_roots_p(n, row_ptr, col, wt, order, roots, nroots, mode, nthreads, NULL);
}

int64_t oracle_run_count(const oracle_run* R, int64_t t) { return R->cnt[t]; }

int64_t oracle_run_total(const oracle_run* R) {
    int64_t s = 0;
    for (int64_t t = 0; t < R->nroots; t++) s += R->cnt[t];
    return s;
}

/* labels of task t: vertices and distances, in the order the tree emitted them */
void oracle_run_labels(const oracle_run* R, int64_t t, int32_t* v, int64_t* d) {
    memcpy(v, R->lv[t], (size_t)R->cnt[t] * sizeof(int32_t));
    memcpy(d, R->ld[t], (size_t)R->cnt[t] * sizeof(int64_t));
}

/* per task: settled, arcs, labels, early-terminated flag (4 int64 each) */
void oracle_run_stats(const oracle_run* R, int64_t* out) {
    for (int64_t t = 0; t < R->nroots; t++) {
        out[4 * t + 0] = R->stats[t].settled;
        out[4 * t + 1] = R->stats[t].arcs;
        out[4 * t + 2] = R->stats[t].labels;
        out[4 * t + 3] = R->stats[t].early;
    }
}

/* Assemble L_v for every vertex v (input ids): offsets[n+1], hub rank
 * positions and distances, each L_v sorted by hub rank position. Tasks are
 * visited in increasing root rank position, so appending keeps every L_v
 * sorted. Only meaningful for a run over all roots. */
void oracle_run_assemble(const oracle_run* R, int64_t* offsets, int32_t* hub_pos,
                         int64_t* dist) {
    int32_t n = R->n;
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* byroot = (int64_t*)malloc((size_t)(R->nroots ? R->nroots : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < R->nroots; i++) byroot[i] = -1;
    for (int64_t t = 0; t < R->nroots; t++) byroot[R->roots[t]] = t;
    memset(offsets, 0, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t t = 0; t < R->nroots; t++)
        for (int64_t i = 0; i < R->cnt[t]; i++) offsets[R->lv[t][i] + 1]++;
    for (int32_t v = 0; v < n; v++) offsets[v + 1] += offsets[v];
    for (int64_t p = 0; p < R->nroots; p++) {
        int64_t t = byroot[p];
        if (t < 0) continue;
        for (int64_t i = 0; i < R->cnt[t]; i++) {
            int32_t v = R->lv[t][i];
            int64_t k = offsets[v] + fill[v]++;
            hub_pos[k] = (int32_t)p;
            dist[k] = R->ld[t][i];
        }
    }
    free(fill); free(byroot);
}

void oracle_run_free(oracle_run* R) {
    if (!R) return;
    for (int64_t t = 0; t < R->nroots; t++) { free(R->lv[t]); free(R->ld[t]); }
    free(R->lv); free(R->ld); free(R->cnt); free(R->stats); free(R->roots); free(R);
}

/* Prefix labels of hubs [0, e) from a run whose task t is the root of rank
 * position t (t < e): appended in hub order, so every list is sorted. */
static void prefix_build(prefix_t* P, int32_t n, int32_t e, int32_t** lv, int64_t** ld,
                         const int64_t* cnt) {
    P->e = e;
    P->off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int32_t t = 0; t < e; t++)
        for (int64_t i = 0; i < cnt[t]; i++) P->off[lv[t][i] + 1]++;
    for (int32_t v = 0; v < n; v++) P->off[v + 1] += P->off[v];
    int64_t tot = P->off[n];
    P->hub = (int32_t*)malloc((size_t)(tot ? tot : 1) * sizeof(int32_t));
    P->dist = (int64_t*)malloc((size_t)(tot ? tot : 1) * sizeof(int64_t));
    int64_t* fill = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    for (int32_t t = 0; t < e; t++)
        for (int64_t i = 0; i < cnt[t]; i++) {
            int32_t v = lv[t][i];          /* input id, as the query indexes it */
            int64_t k = P->off[v] + fill[v]++;
            P->hub[k] = t;
            P->dist[k] = ld[t][i];
        }
    free(fill);
}

static void prefix_free(prefix_t* P) { free(P->off); free(P->hub); free(P->dist); }

/* Trees with rank-prefix pruning (Section 4.3), grown in levels. bounds =
 * g_0 < g_1 < ... < g_L: the roots at rank positions [0, g_0) grow without
 * pruning; the roots of level [g_{j-1}, g_j) are pruned by the labels of the
 * hubs [0, g_{j-1}), complete by then; every root at rank position >= g_L is
 * pruned by the hubs [0, pmain) (pmain <= g_L; 0 = no pruning). Returns a run
 * over the requested roots (NULL = all roots in rank order). PLaNT with early
 * termination throughout. */
oracle_run* oracle_run_roots_levels(int32_t n, const int64_t* row_ptr, const int32_t* col,
                                    const int32_t* wt, const int32_t* order,
                                    const int32_t* roots, int64_t nroots,
                                    const int32_t* bounds, int32_t nb, int32_t pmain, int32_t half,
                                    int nthreads) {
    int32_t gl = nb > 0 ? bounds[nb - 1] : 0;
    if (gl > n) gl = n;
    if (gl < 0) gl = 0;
    if (pmain > gl) pmain = gl;
    /* rank positions [0, gl), level by level */
    int32_t** lv = (int32_t**)calloc((size_t)(gl ? gl : 1), sizeof(int32_t*));
    int64_t** ld = (int64_t**)calloc((size_t)(gl ? gl : 1), sizeof(int64_t*));
    int64_t* cnt = (int64_t*)calloc((size_t)(gl ? gl : 1), sizeof(int64_t));
    tree_stats* hst = (tree_stats*)calloc((size_t)(gl ? gl : 1), sizeof(tree_stats));
    int32_t lo = 0;
    for (int32_t j = 0; j < nb && lo < gl; j++) {
        int32_t hi = bounds[j] < gl ? bounds[j] : gl;
        if (hi <= lo) continue;
        int32_t* lvl = (int32_t*)malloc((size_t)(hi - lo) * sizeof(int32_t));
        for (int32_t r = lo; r < hi; r++) lvl[r - lo] = r;
        prefix_t P;
        int pr = j > 0;
        if (pr) prefix_build(&P, n, lo, lv, ld, cnt);
        P.half = half;
        oracle_run* R = run_roots_p(n, row_ptr, col, wt, order, lvl, hi - lo, 1, nthreads, pr ? &P : NULL);
        for (int32_t r = lo; r < hi; r++) {
            lv[r] = R->lv[r - lo]; ld[r] = R->ld[r - lo]; cnt[r] = R->cnt[r - lo]; hst[r] = R->stats[r - lo];
            R->lv[r - lo] = NULL; R->ld[r - lo] = NULL;
        }
        oracle_run_free(R);
        if (pr) prefix_free(&P);
        free(lvl);
        lo = hi;
    }
    /* requested roots: those below gl come from the levels, the rest grow now */
    if (!roots) nroots = n;
    int32_t* req = (int32_t*)malloc((size_t)(nroots ? nroots : 1) * sizeof(int32_t));
    int32_t* late = (int32_t*)malloc((size_t)(nroots ? nroots : 1) * sizeof(int32_t));
    int64_t nlate = 0;
    for (int64_t i = 0; i < nroots; i++) {
        req[i] = roots ? roots[i] : (int32_t)i;
        if (req[i] >= gl) late[nlate++] = req[i];
    }
    prefix_t P;
    if (pmain > 0) prefix_build(&P, n, pmain, lv, ld, cnt);
    P.half = half;
    oracle_run* L = run_roots_p(n, row_ptr, col, wt, order, late, nlate, 1, nthreads, pmain > 0 ? &P : NULL);
    oracle_run* R = (oracle_run*)calloc(1, sizeof(oracle_run));
    R->n = n; R->nroots = nroots;
    R->roots = req;
    R->lv = (int32_t**)calloc((size_t)(nroots ? nroots : 1), sizeof(int32_t*));
    R->ld = (int64_t**)calloc((size_t)(nroots ? nroots : 1), sizeof(int64_t*));
    R->cnt = (int64_t*)calloc((size_t)(nroots ? nroots : 1), sizeof(int64_t));
    R->stats = (tree_stats*)calloc((size_t)(nroots ? nroots : 1), sizeof(tree_stats));
    int64_t li = 0;
    for (int64_t i = 0; i < nroots; i++) {
        int32_t r = req[i];
        if (r >= gl) {
            R->lv[i] = L->lv[li]; R->ld[i] = L->ld[li]; R->cnt[i] = L->cnt[li]; R->stats[i] = L->stats[li];
            L->lv[li] = NULL; L->ld[li] = NULL;
            li++;
        } else {
            /* a copy, since a root may be requested twice */
            R->cnt[i] = cnt[r]; R->stats[i] = hst[r];
            R->lv[i] = (int32_t*)malloc((size_t)(cnt[r] ? cnt[r] : 1) * sizeof(int32_t));
            R->ld[i] = (int64_t*)malloc((size_t)(cnt[r] ? cnt[r] : 1) * sizeof(int64_t));
            memcpy(R->lv[i], lv[r], (size_t)cnt[r] * sizeof(int32_t));
            memcpy(R->ld[i], ld[r], (size_t)cnt[r] * sizeof(int64_t));
        }
    }
    oracle_run_free(L);
    if (pmain > 0) prefix_free(&P);
    for (int32_t r = 0; r < gl; r++) { free(lv[r]); free(ld[r]); }
    free(lv); free(ld); free(cnt); free(hst); free(late);
    return R;
}

/* ---------------- queries ---------------- */
/* Sorted-list merge over the two label lists (Section 5, QLSN). */
static int64_t merge_query(const int64_t* off, const int32_t* hub, const int64_t* dist,
                           int32_t u, int32_t v) {
    int64_t i = off[u], ie = off[u + 1], j = off[v], je = off[v + 1];
    int64_t best = -1;
    while (i < ie && j < je) {
        if (hub[i] < hub[j]) i++;
        else if (hub[i] > hub[j]) j++;
        else {
            int64_t s = dist[i] + dist[j];
            if (best < 0 || s < best) best = s;
            i++; j++;
        }
    }
    return best;
}

void oracle_query(const int64_t* offsets, const int32_t* hub_pos, const int64_t* dist,
                  const int32_t* pairs, int64_t q, int64_t* out) {
    for (int64_t k = 0; k < q; k++)
        out[k] = merge_query(offsets, hub_pos, dist, pairs[2 * k], pairs[2 * k + 1]);
}

/* Directed graphs (footnote of Section 1): two label sets, L_out(u) with
 * hubs reached from u and L_in(v) with hubs that reach v; d(u, v) is the
 * minimum of d(u, h) + d(h, v) over hubs common to L_out(u) and L_in(v). */
void oracle_query2(const int64_t* off_out, const int32_t* hub_out, const int64_t* dist_out,
                   const int64_t* off_in, const int32_t* hub_in, const int64_t* dist_in,
                   const int32_t* pairs, int64_t q, int64_t* out) {
    for (int64_t k = 0; k < q; k++) {
        int32_t u = pairs[2 * k], v = pairs[2 * k + 1];
        int64_t i = off_out[u], ie = off_out[u + 1], j = off_in[v], je = off_in[v + 1];
        int64_t best = -1;
        while (i < ie && j < je) {
            if (hub_out[i] < hub_in[j]) i++;
            else if (hub_out[i] > hub_in[j]) j++;
            else {
                int64_t s = dist_out[i] + dist_in[j];
                if (best < 0 || s < best) best = s;
                i++; j++;
            }
        }
        out[k] = best;
    }
}

/* Plain Dijkstra distances from src; -1 for unreachable vertices. */
void oracle_sssp(int32_t n, const int64_t* row_ptr, const int32_t* col,
                 const int32_t* wt, int32_t src, int64_t* out) {
    heap_t hp = {0};
    uint8_t* done = (uint8_t*)calloc((size_t)n, 1);
    for (int32_t v = 0; v < n; v++) out[v] = INF64;
    out[src] = 0;
    hpush(&hp, (hitem){0, 0, src});
    while (hp.size) {
        hitem it = hpop(&hp);
        if (done[it.v] || it.d != out[it.v]) continue;
        done[it.v] = 1;
        for (int64_t e = row_ptr[it.v]; e < row_ptr[it.v + 1]; e++) {
            int64_t nd = it.d + wt[e];
            if (nd < out[col[e]]) { out[col[e]] = nd; hpush(&hp, (hitem){nd, 0, col[e]}); }
        }
    }
    for (int32_t v = 0; v < n; v++) if (out[v] == INF64) out[v] = -1;
    free(done); free(hp.a);
}

/* ---------------- shortest paths from the labels ----------------
 * Keeping with each label (h, d(v,h)) of L_v the next vertex from v towards
 * h turns the labeling into a shortest-path oracle (Section 4.4, last
 * paragraph): the path u -> v through the common hub h is u's chain of
 * parents down to h followed by the reverse of v's chain.
 *
 * Parent of (h, d) in L_v: a neighbour p of v with d(p,h) + w(p,v) = d(v,h),
 * i.e. the next vertex of some shortest v-h path. Every such p holds the
 * label (h, d(p,h)) itself: a shortest p-h path followed by the arc (p,v)
 * is a shortest v-h path, so SP_{p,h} lies inside SP_{v,h}, whose highest
 * ranked vertex is h. The paper leaves the choice among several such p
 * open; the neighbour with the smallest input id is taken. slot = position
 * of p's label (h, .) within L_p, so a walk takes one step per edge. The
 * hub's own label (v = h, d = 0) has parent -1 (positive weights: no
 * neighbour can reach h in 0 - w). */
static int64_t find_hub(const int64_t* off, const int32_t* hub, int32_t x, int32_t h) {
    int64_t lo = off[x], hi = off[x + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (hub[mid] < h) lo = mid + 1; else hi = mid;
    }
    return (lo < off[x + 1] && hub[lo] == h) ? lo : -1;
}

void oracle_parents(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* wt,
                    const int64_t* off, const int32_t* hub, const int64_t* dist,
                    int32_t* parent, int32_t* slot) {
    for (int32_t v = 0; v < n; v++)
        for (int64_t i = off[v]; i < off[v + 1]; i++) {
            int32_t best = -1, bslot = -1;
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
                int32_t p = col[e];
                int64_t j = find_hub(off, hub, p, hub[i]);
                if (j < 0 || dist[j] + wt[e] != dist[i]) continue;
                if (best < 0 || p < best) { best = p; bslot = (int32_t)(j - off[p]); }
            }
            parent[i] = best;
            slot[i] = bslot;
        }
}

/* Follow the parents from label index i of vertex x down to the hub; writes
 * the vertices (x first) to out when out != NULL; returns the edge count. */
static int64_t walk(const int64_t* off, const int32_t* parent, const int32_t* slot,
                    int32_t x, int64_t i, int32_t* out) {
    int64_t k = 0;
    if (out) out[0] = x;
    while (parent[i] >= 0) {
        int32_t p = parent[i];
        i = off[p] + slot[i];
        x = p;
        k++;
        if (out) out[k] = x;
    }
    return k;
}

/* Path queries. The hub is the common hub with the smallest d_u + d_v and,
 * among equal sums, the most important one (smallest rank position): the
 * highest ranked vertex of SP_{u,v}. hops[k] = number of edges, -1 when the
 * two lists share no hub. With path != NULL, the hops[k] + 1 vertices of
 * pair k, u first and v last, go to path[path_off[k] ...]. */
void oracle_paths(const int64_t* off, const int32_t* hub, const int64_t* dist,
                  const int32_t* parent, const int32_t* slot, const int32_t* pairs, int64_t q,
                  int64_t* hops, const int64_t* path_off, int32_t* path) {
    for (int64_t k = 0; k < q; k++) {
        int32_t u = pairs[2 * k], v = pairs[2 * k + 1];
        int64_t i = off[u], ie = off[u + 1], j = off[v], je = off[v + 1];
        int64_t best = -1, bi = -1, bj = -1;
        while (i < ie && j < je) {
            if (hub[i] < hub[j]) i++;
            else if (hub[i] > hub[j]) j++;
            else {
                int64_t s = dist[i] + dist[j];
                if (best < 0 || s < best) { best = s; bi = i; bj = j; }
                i++; j++;
            }
        }
        if (best < 0) { hops[k] = -1; continue; }
        int64_t hu = walk(off, parent, slot, u, bi, NULL);
        int64_t hv = walk(off, parent, slot, v, bj, NULL);
        hops[k] = hu + hv;
        if (!path) continue;
        int32_t* o = path + path_off[k];
        walk(off, parent, slot, u, bi, o);
        int32_t* tmp = (int32_t*)malloc((size_t)(hv + 1) * sizeof(int32_t));
        walk(off, parent, slot, v, bj, tmp);
        for (int64_t t = 0; t < hv; t++) o[hu + 1 + t] = tmp[hv - 1 - t];
        free(tmp);
    }
}
