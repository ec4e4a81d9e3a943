/*
 * chl.h -- C-ABI of the MI355X (gfx950) library that builds and queries the
 * Canonical Hub Labeling (CHL) with PLaNT trees.
 *
 * Paper: "Planting Trees for scalable and efficient Canonical Hub Labeling"
 * (arXiv 1907.00140). Definitions used throughout:
 *   - hub label (h, d(v,h)) of vertex v, label set L_v, cover property and
 *     distance query by common hubs: Section 1;
 *   - ranking R, the canonical labeling (only the highest ranked vertex of a
 *     shortest path becomes the hub of its two ends): Section 1;
 *   - PLaNT trees (one shortest-path tree per root, labels emitted only where
 *     no vertex of any shortest root-v path outranks the root, early
 *     termination once every queued vertex is outranked): Section 4.2,
 *     Algorithm 3;
 *   - label sets sorted by hub rank and the sorted-list merge query (QLSN):
 *     Algorithm 2's sort step and Section 5.
 *
 * Conventions shared by every call:
 *   - The graph is undirected with positive int32 edge weights, given as a
 *     symmetric CSR; ids are 0..n-1 ("input ids"). chl_build_directed takes
 *     the out-arc CSR of a directed graph instead.
 *   - The ranking is a permutation order[0..n-1]; order[0] is the most
 *     important vertex. The rank position of v is pos(v), with order[pos(v)]
 *     = v. Hubs are reported by rank position ("hub_pos"), so L_v is sorted
 *     by hub_pos ascending = most important hub first. chl_labels_hub_vertex
 *     maps hub_pos back to input ids.
 *   - Every L_v contains its own label (pos(v), 0).
 *   - Pointers are device pointers unless a parameter says otherwise; all
 *     device work is queued on `stream` (a hipStream_t; NULL = the null
 *     stream). Calls that return a value computed on the device synchronise
 *     that stream before returning.
 *   - Return value: CHL_OK (0) or a negative CHL_ERR_* code. No exception
 *     crosses this boundary. Output parameters are written only on success.
 *   - Calls on distinct handles may run concurrently from different host
 *     threads. A handle must not be freed while another call uses it.
 */
#ifndef CHL_H
#define CHL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define CHL_OK 0
#define CHL_ERR_INVALID_ARG (-1)    /* bad sizes, CSR, ranking, weights, ids or options */
#define CHL_ERR_OOM (-2)            /* the allocator returned NULL */
#define CHL_ERR_HIP (-3)            /* a HIP runtime call failed */
#define CHL_ERR_DIST_OVERFLOW (-4)  /* a label distance does not fit in int32 */
#define CHL_ERR_NO_DEVICE (-5)      /* no usable gfx950 device */
#define CHL_ERR_BUSY (-6)           /* server: request rejected (budget or queue full) */

/* Text for an error code; never NULL, static storage. */
const char* chl_error_string(int code);

/* ---- graph view ----
 * Symmetric CSR of an undirected graph (Section 1: G(V, E, W), positive
 * weights). All arrays are device memory, borrowed for the duration of the
 * call (they must stay valid until the call returns).
 *   row_ptr[n+1]: int64, row_ptr[0] = 0, non-decreasing, row_ptr[n] = n_arcs
 *   col[n_arcs] : int32 neighbour ids in [0, n)
 *   w[n_arcs]   : int32 weights >= 1
 * The arc multiset must be symmetric: every arc (v, u, w) has a matching
 * (u, v, w). Parallel arcs are allowed (the smallest weight decides the
 * distance); self-loops are allowed and have no effect.
 * Requirements checked by chl_build (CHL_ERR_INVALID_ARG otherwise):
 * 1 <= n <= 2^31 - 2, 0 <= n_arcs <= 2^32 - 1, and all of the above. */
typedef struct chl_graph {
    int32_t n;
    int64_t n_arcs;
    const int64_t* row_ptr;
    const int32_t* col;
    const int32_t* w;
} chl_graph;

/* ---- device memory allocator ----
 * Every device buffer the library keeps or uses as scratch is obtained from
 * alloc(bytes, ctx) and returned with free(ptr, ctx). alloc returns NULL on
 * failure (the call then fails with CHL_ERR_OOM and frees what it took).
 * Passing NULL for the allocator selects hipMalloc / hipFree. The allocator
 * must stay valid until every handle created with it has been freed. */
typedef struct chl_allocator {
    void* (*alloc)(size_t bytes, void* ctx);
    void (*free)(void* ptr, void* ctx);
    void* ctx;
} chl_allocator;

/* ---- build options ---- */
#define CHL_MODE_BATCHED 0  /* persistent kernel: one workgroup per tree,
                               roots_in_flight trees at once, roots taken from
                               a rank-ordered work queue */
#define CHL_MODE_PLAIN 1    /* one root per launch; the whole device grows that
                               single tree (rank order, one tree at a time) */

typedef struct chl_build_opts {
    int32_t mode;            /* CHL_MODE_BATCHED or CHL_MODE_PLAIN */
    int32_t roots_in_flight; /* batched: trees in flight (= workgroups) of the
                                main phase, and at most that many (<= 512) in
                                the pruning levels; 0 = tuned (levels: 512) */
    int32_t wg_size;         /* 64, 128, 256, 512 or 1024 threads (plain form:
                                256 or 512), also for the pruning levels;
                                0 = tuned (levels: 1024) */
    int64_t delta;           /* bucket width of the delta-stepping frontier; 0 = tuned */
    int32_t early_term;      /* 1: stop a tree once no queued vertex is clean
                                (Section 4.2, early termination); 0: grow every
                                tree over its whole component. Same labels. */
    int32_t stats;           /* 1: keep per-root statistics (chl_build_stats) */
    int32_t autotune;        /* 1: parameters left at 0 are chosen by timing a
                                probe set of roots (cached per graph signature);
                                0: they take fixed defaults */
    int32_t root_count;      /* 0: every root (the complete labeling). > 0: only
                                the roots at rank positions root_begin +
                                i * root_stride, i < root_count; the result then
                                holds exactly the labels whose hub is one of
                                them (trees are independent, Section 4.2) */
    int32_t root_begin;
    int32_t root_stride;     /* >= 1 when root_count > 0 */
    int32_t prune_hubs;      /* batched form: rank-prefix pruning (Section 4.3).
                                The trees of roots [0, 16) grow first; each
                                later level of roots [g, 8g) -- [g, 2g) and
                                [g, 4g) in turn after levels whose roots
                                emitted >= 2^21 labels -- is pruned by the
                                labels of the hubs [0, g)
                                (complete by then), up to a prefix of
                                prune_hubs hubs (<= 8192); every other tree is
                                pruned by that prefix. A relaxation is dropped
                                when a walk through a prefix hub is no longer.
                                Same labels either way. > 0: that prefix size;
                                0: min(8192, max(64, n/64)), kept only if the
                                16-hub level halves the work of a probe of
                                later trees (decided once per graph and
                                ranking, cached; always kept when autotune is
                                0); < 0: off. Ignored by the plain form. */
    int32_t team_wgs;        /* batched form: workgroups per tree for the levels
                                of rank-prefix pruning that hold fewer trees than
                                the device holds workgroups (the first, largest
                                trees). 0: chosen from the device size; 1: one
                                workgroup per tree; 2..16: that many, capped so
                                that every team of a launch is resident (a
                                cooperative launch). Same labels either way. */
    int32_t group_levels;    /* batched form: 0: levels of 16 to 512 trees grow
                                in groups of 16 trees of consecutive roots, one
                                group per team of workgroups, their per-vertex
                                keys side by side (one cache line holds a
                                vertex's keys of all 16 trees); -1: each tree
                                alone (teams or one workgroup). Ignored when
                                team_wgs is 1. Same labels either way. */
    int32_t small_trees;     /* batched form, main phase: 1: one 64-thread
                                workgroup per tree with the tree's state in
                                LDS (at most 128 vertices reached and 256
                                prefix labels of the root; the trees that
                                need more are grown by the batched kernel
                                afterwards); -1: the batched kernel alone;
                                0: chosen by the autotuner (off when autotune
                                is 0). Same labels either way. */
    int32_t hybrid_psi;      /* batched form, undirected, complete builds: the
                                Hybrid construction (Section 4.2.1) with
                                switching threshold Psi_th = hybrid_psi (the
                                paper uses 100 for scale-free graphs, 500 for
                                road networks); 0: off (PLaNT trees for every
                                root). The main phase grows PLaNT trees in
                                windows of consecutive roots, the first of
                                r = max(64, n / 64) roots, each next one twice
                                as large up to max(r, 8 * roots_in_flight);
                                once the vertex relaxations per label (Psi,
                                Section 4.2.1) of a window's last r trees
                                exceed Psi_th, the remaining roots grow as
                                pruned Dijkstra trees with rank queries
                                (Algorithm 1), in supersteps of
                                max(64, 2 * roots_in_flight) roots doubling
                                each time, pruned by the distance query over
                                every label of the roots before the superstep;
                                after each superstep its redundant labels are
                                removed by the cleaning query DQ_Clean
                                (Algorithm 2). Same labels as without it. */
} chl_build_opts;

/* Defaults: batched, everything tuned, early termination on, stats on. */
void chl_build_opts_default(chl_build_opts* opts);

/* Opaque labeling handle (device resident). */
typedef struct chl_labels chl_labels;

/* Build the canonical labeling of graph g under ranking order[] (device
 * int32[n], order[0] most important, must be a permutation of 0..n-1).
 * opts may be NULL (defaults). On success *out receives a handle that the
 * caller owns and releases with chl_labels_free. Synchronises `stream`.
 * Errors: CHL_ERR_INVALID_ARG (see chl_graph; also order not a permutation,
 * bad options), CHL_ERR_OOM, CHL_ERR_HIP, CHL_ERR_DIST_OVERFLOW (some label
 * distance is >= 2^31 - 1), CHL_ERR_NO_DEVICE. */
int chl_build(const chl_graph* g, const int32_t* order, const chl_build_opts* opts,
              const chl_allocator* alloc, void* stream, chl_labels** out);

/* ---- directed graphs (footnote of Section 1: every vertex gets forward and
 * backward labels, and a query merges the source's with the target's) ----
 * g holds the out-arcs of a directed graph (row v lists the arcs v -> col[e];
 * no symmetry is required; the other conditions of chl_graph apply). The
 * handle holds two labelings under the same ranking: L_out(v) = the labels
 * (h, d(v, h)) such that h is the highest ranked vertex on every shortest
 * v -> h path (trees grown on the reversed graph), and L_in(v) = the labels
 * (h, d(h, v)) such that h tops every shortest h -> v path (trees grown along
 * the arcs). chl_query answers d(u, v) = min over hubs common to L_out(u) and
 * L_in(v) of d(u, h) + d(h, v); chl_labels_info and chl_labels_export give
 * L_out, chl_labels_export_in gives L_in. Both sets come from one build over
 * a combined graph of 2n vertices, the graph and its reversal, with the
 * ranking interleaved (v at rank position 2 pos(v), its reversed copy at
 * 2 pos(v) + 1); the options apply to that build, so roots_in_flight,
 * prune_hubs, root_begin/count/stride and the statistics' prune_hubs and
 * prefix_roots count in its rank positions (two per vertex), and the
 * rank-prefix pruning (Section 4.3) takes d(h, x) from the out-labels and
 * d(x, u) from the in-labels of the prefix. Per-root statistics are not
 * kept (chl_build_stats with per_root != NULL returns CHL_ERR_INVALID_ARG).
 * chl_labels_parents and the path queries return CHL_ERR_INVALID_ARG on a
 * directed handle. Requires n <= 2^30 - 2 and n_arcs <= 2^31 - 1.
 * Synchronises `stream`. Errors as for chl_build. */
int chl_build_directed(const chl_graph* g, const int32_t* order, const chl_build_opts* opts,
                       const chl_allocator* alloc, void* stream, chl_labels** out);

/* 1 for a directed labeling (then *in_total = number of in-labels), 0 for an
 * undirected one (*in_total = total), CHL_ERR_INVALID_ARG for NULL. in_total
 * may be NULL. */
int chl_labels_directed(const chl_labels* h, int64_t* in_total);

/* Copy the in-labels of a directed labeling out, in the layout of
 * chl_labels_export (offsets[n+1], hub_pos[in_total], dist[in_total]).
 * CHL_ERR_INVALID_ARG for an undirected handle. */
int chl_labels_export_in(const chl_labels* h, int64_t* offsets, int32_t* hub_pos,
                         int32_t* dist, int to_host, void* stream);

/* Number of vertices and total number of labels (host outputs). */
int chl_labels_info(const chl_labels* h, int32_t* n, int64_t* total);

/* Copy the labeling out: offsets[n+1] (int64; L_v is entries
 * offsets[v]..offsets[v+1]-1, v an input id), hub_pos[total] (int32 rank
 * positions, strictly increasing within each L_v) and dist[total] (int32).
 * Any output pointer may be NULL to skip it. to_host = 1: outputs are host
 * memory (the call synchronises `stream`); 0: device memory (asynchronous). */
int chl_labels_export(const chl_labels* h, int64_t* offsets, int32_t* hub_pos,
                      int32_t* dist, int to_host, void* stream);

/* hub_vertex[p] = input id of the vertex at rank position p (= order[p]),
 * int32[n]; host or device output as for chl_labels_export. */
int chl_labels_hub_vertex(const chl_labels* h, int32_t* hub_vertex, int to_host, void* stream);

/* Point-to-point shortest distance queries by sorted-list merge of the two
 * label sets (Section 5, single-copy mode): pairs[2q] = (u0, v0, u1, v1, ...)
 * int32 input ids on the device; out[q] int64 on the device receives
 * d(u,v), 0 when u == v, -1 when u and v are in different components (for a
 * directed labeling: when no path leads from u to v).
 * q = 0 is a no-op. Synchronises `stream` (ids are validated on the device);
 * an id outside [0, n) gives CHL_ERR_INVALID_ARG (out is then unspecified). */
int chl_query(const chl_labels* h, const int32_t* pairs, int64_t q, int64_t* out, void* stream);

/* ---- shortest paths (Section 4.4, last paragraph: a label that also keeps
 * the tree parent of its vertex answers path queries in time linear in the
 * path's edge count) ----
 * Parent of the label (h, d) of L_v: the neighbour p of v with the smallest
 * input id such that d(p, h) + w(p, v) = d, i.e. the next vertex of a
 * shortest v-h path (every such p holds a label of hub h); -1 for a hub's
 * own label (v = h). slot: the position of p's label of hub h within L_p
 * (-1 with parent -1).
 *
 * Compute the parents of every label of h: parent[total] and slot[total]
 * (int32, device, caller-owned, in the label order of chl_labels_export).
 * g must be the graph the labeling was built from (device CSR, input ids);
 * g->n must equal the labeling's n. Takes 256 bytes of scratch (a work
 * queue counter) from the labeling's allocator. Synchronises `stream`.
 * Errors: CHL_ERR_INVALID_ARG (NULL or mismatched arguments, a directed
 * labeling; an arc with a neighbour outside [0, n) or a weight < 1, or a
 * malformed row: such arcs are skipped and the parents are then
 * unspecified), CHL_ERR_OOM, CHL_ERR_HIP. */
int chl_labels_parents(const chl_labels* h, const chl_graph* g, int32_t* parent, int32_t* slot,
                       void* stream);

/* Path lengths for pairs[2q] (device int32 input ids, as for chl_query),
 * with the parent and slot arrays of chl_labels_parents (device): hops[q]
 * (device int64) = number of edges of the path from u to v, 0 when u == v,
 * -1 when u and v are disconnected, -2 for an invalid pair. path_off
 * (device int64[q+1], may be NULL) receives the exclusive prefix sum of the
 * per-pair vertex counts (hops + 1, or 0 when disconnected), so path_off[q]
 * is the size of the path array chl_query_paths fills. The path of a pair
 * runs through the common hub h that gives d(u, v) (the most important one
 * among equal sums, i.e. the highest ranked vertex of SP_{u,v}): u's chain
 * of parents down to h, then the reverse of v's chain. Allocates q * 8 bytes
 * plus scan scratch through the labeling's allocator when path_off is given.
 * Synchronises `stream`. Errors: CHL_ERR_INVALID_ARG (an id outside
 * [0, n), or parent/slot arrays that do not fit the labeling),
 * CHL_ERR_OOM, CHL_ERR_HIP. */
int chl_query_path_hops(const chl_labels* h, const int32_t* parent, const int32_t* slot,
                        const int32_t* pairs, int64_t q, int64_t* hops, int64_t* path_off,
                        void* stream);

/* The variant of chl_query_path_hops for callers that cannot allocate device
 * memory during the call (code under stream capture, tight serving loops,
 * hosts that forbid allocation): the same arguments, results and errors, but
 * the per-pair vertex counts and the prefix sum's temporaries live in a
 * fixed device array of the library (8 * CHL_NOALLOC_MAX_PAIRS + 64 KiB
 * bytes, one copy per GPU, held until the process ends) instead of memory
 * taken from the labeling's allocator. q > CHL_NOALLOC_MAX_PAIRS gives
 * CHL_ERR_INVALID_ARG. Calls on one GPU share that array: the library
 * serialises them (each synchronises `stream` before it returns), so calls
 * from several host threads take turns. */
#define CHL_NOALLOC_MAX_PAIRS (1 << 20)
int chl_query_path_hops_noalloc(const chl_labels* h, const int32_t* parent, const int32_t* slot,
                                const int32_t* pairs, int64_t q, int64_t* hops, int64_t* path_off,
                                void* stream);

/* Write the paths: the vertices (input ids, u first, v last) of pair k go
 * to path[path_off[k] .. path_off[k+1]-1] (device int32, caller-owned,
 * path_off[q] entries) for path_off as returned by chl_query_path_hops for
 * the same pairs. A pair whose range does not hold exactly its hops + 1
 * vertices gets CHL_ERR_INVALID_ARG; nothing is written outside a pair's
 * range. Synchronises `stream`. */
int chl_query_paths(const chl_labels* h, const int32_t* parent, const int32_t* slot,
                    const int32_t* pairs, int64_t q, const int64_t* path_off, int32_t* path,
                    void* stream);

/* ---- statistics ---- */
#define CHL_MAX_LEVELS 16
typedef struct chl_stats {
    int64_t n;               /* vertices (= roots) */
    int64_t labels;          /* total labels */
    int64_t settled;         /* vertex relaxations performed (a vertex relaxed
                                again after its key dropped counts again) */
    int64_t arcs;            /* arcs relaxed */
    int64_t early_trees;     /* trees that stopped with vertices still queued */
    int64_t key_bits;        /* 32 or 64: width of the packed (distance, clean) key */
    int64_t roots_in_flight; /* parameters actually used */
    int64_t wg_size;
    int64_t delta;
    int64_t prune_hubs;      /* size of the pruning prefix of the main phase (0: none) */
    int64_t prefix_roots;    /* roots grown before the main phase (0: none) */
    int64_t launches;        /* kernel launches of the main tree phase */
    int64_t clock_khz;       /* device wall clock of the per-root tick counts */
    double tree_ms;          /* device time of the main tree phase (every root
                                not grown for the common label table) */
    double prefix_ms;        /* trees of the prefix levels and their regrouping */
    double kernel_ms;        /* device time of every tree-kernel launch of the
                                build (prefix levels and main phase; excludes
                                the autotuner's and the pruning decision's
                                probes) */
    int64_t kernel_launches; /* number of those launches */
    double assemble_ms;      /* device time of label assembly */
    double prep_ms;          /* validation + rank renumbering */
    double tune_ms;          /* autotuner probe time (0 when cached or off) */
    /* rank-prefix levels grown before the main phase (Section 4.3): level i
       holds the roots [level_end[i-1], level_end[i]) (level_end[-1] = 0) and
       is pruned by the labels of the hubs [0, level_end[i-1]) (level 0 is
       unpruned); the main phase grows the roots [level_end[levels-1], n)
       pruned by the hubs [0, prune_hubs). levels = 0: no level ran. */
    int64_t levels;
    int64_t level_end[CHL_MAX_LEVELS];
    double level_ms[CHL_MAX_LEVELS];   /* device time of each level's tree launches */
    int64_t level_teams[CHL_MAX_LEVELS];  /* workgroups per tree of the level (1: batched
                                             kernel); -w: groups of 16 trees, w
                                             workgroups per group */
    int64_t small_trees;     /* workgroups of the small-tree kernel in the main
                                phase (0: not used) */
    /* Hybrid construction (chl_build_opts::hybrid_psi): the rank position
       from which the pruned construction grew the roots (n: PLaNT trees
       throughout; 0 when off), the Psi of the window that triggered it, the
       supersteps, the labels the pruned trees emitted and those the
       cleaning removed, and the device time of the cleaning (table
       regrouping, DQ_Clean, compaction) */
    int64_t hybrid_switch;
    double hybrid_psi;
    int64_t hybrid_supersteps;
    int64_t hybrid_emitted;
    int64_t hybrid_removed;
    double hybrid_clean_ms;
} chl_stats;

/* Totals into *totals (host, may be NULL). per_root (may be NULL) receives
 * int64[n][6] indexed by root rank position: vertex relaxations, arcs
 * relaxed, labels, stopped early (0/1), relaxation rounds, and the tree's
 * duration in device wall-clock ticks (batched form; 0 in the plain form
 * and for a main-phase root whose tree is the root alone -- no arcs, or
 * every neighbour outranks it -- whose single label is written without
 * growing a tree, and whose arcs and stopped-early entries are then 0);
 * host or device as for chl_labels_export. Per-root data needs opts.stats=1,
 * otherwise CHL_ERR_INVALID_ARG is returned when per_root is not NULL. */
int chl_build_stats(const chl_labels* h, chl_stats* totals, int64_t* per_root,
                    int to_host, void* stream);

/* Release a handle and its device memory (NULL is a no-op). */
void chl_labels_free(chl_labels* h);

/* ---- measurement ----
 * Ceiling of the tree kernels' relaxation step (the atomic minimum on a
 * packed key that realises Algorithm 3's distance and ancestor update):
 * about `ops` random atomic minima (32- or 64-bit, key_bits) on the device
 * array buf of `words` keys, which the call first sets to all ones. *done
 * receives the number performed, *ms the device time (events on `stream`).
 * buf is caller-owned device memory of words * key_bits / 8 bytes.
 * Synchronises `stream`. */
int chl_microbench_atomic_min(void* buf, int64_t words, int key_bits, int64_t ops, int64_t* done,
                              double* ms, void* stream);

/* ---- continuous-batching server ----
 * A host thread that owns device streams, keeps labelings resident, batches
 * distance queries that have arrived and admits build requests by their
 * device-memory footprint, so that queries and builds overlap on the device.
 * Times are seconds on the server's clock, which starts at chl_server_start.
 * Latency of a request = completion time - scheduled arrival time. */
typedef struct chl_server chl_server;

typedef struct chl_server_opts {
    size_t mem_budget;          /* bytes of device memory builds may hold at once */
    int32_t max_batch;          /* max queries per device batch */
    int32_t build_streams;      /* concurrent builds (streams) */
    int32_t build_wg;           /* workgroups a build may occupy (caps its share) */
    int32_t reserved;
} chl_server_opts;

void chl_server_opts_default(chl_server_opts* o);
/* Create a server. alloc == NULL: builds allocate from the device's default
 * stream-ordered memory pool on their build streams (nothing is reserved
 * up front; the pool reuses memory that earlier builds freed). alloc != NULL: builds (and
 * the labelings they produce, released by chl_server_destroy) take device
 * memory from that allocator instead; it must be callable from the server's
 * threads and stay valid until chl_server_destroy returns (the server
 * synchronises a build's stream before it returns memory to it, since such
 * an allocator is not ordered with the build streams).
 * Budget: a build is admitted when its footprint estimate
 * (chl_server_build_footprint) fits what other builds hold; memory it needs
 * beyond the estimate is charged while it runs, and an allocation that would
 * take the builds past mem_budget fails, after which the request is queued
 * again with a larger estimate (at most four attempts; then its status is
 * CHL_ERR_OOM). Builds in flight never hold more than mem_budget bytes
 * together; a finished build's labeling stays resident outside the budget,
 * like the labelings added with chl_server_add_labels. */
int chl_server_create(const chl_server_opts* o, const chl_allocator* alloc, chl_server** out);

/* Register a resident labeling for queries; returns its graph id (>= 0) in
 * *graph_id. The server does not take ownership. */
int chl_server_add_labels(chl_server* s, const chl_labels* h, int32_t* graph_id);

/* Requests are submitted before chl_server_start (or after chl_server_wait
 * has returned); a submit while the server runs returns CHL_ERR_BUSY.
 *
 * Schedule q queries against graph_id: host arrays pairs[2q] (input ids) and
 * t_arrival[q] (non-decreasing seconds). Results go to host out[q] (int64)
 * and per-query latency to host lat[q] (seconds); both must stay valid until
 * chl_server_wait returns. */
int chl_server_submit_queries(chl_server* s, int32_t graph_id, const int32_t* pairs,
                              const double* t_arrival, int64_t q, int64_t* out, double* lat);

/* Schedule a build of a host-side graph (host CSR arrays, copied at submit)
 * arriving at t_arrival. On completion the labeling is registered (its graph
 * id written to *graph_id) and its latency to *lat. *status receives the
 * build's return code (CHL_ERR_BUSY when its footprint exceeds the whole
 * budget). */
int chl_server_submit_build(chl_server* s, int32_t n, int64_t n_arcs, const int64_t* row_ptr,
                            const int32_t* col, const int32_t* w, const int32_t* order,
                            double t_arrival, int32_t* graph_id, double* lat, int32_t* status);

/* Device-memory footprint (bytes) that admission charges for a build of a
 * graph with n vertices and n_arcs arcs on this server (an estimate; see
 * chl_server_create for what happens when a build needs more). */
size_t chl_server_build_footprint(const chl_server* s, int32_t n, int64_t n_arcs);

/* Trace of the last run (since chl_server_start), for latency analysis: up
 * to cap rows of 5 doubles (host memory) in completion order; *count
 * receives the number of rows recorded (which may exceed cap).
 *   query batch: (0, earliest scheduled arrival of its queries, time it was
 *                 queued on the device, time its completion was observed,
 *                 number of queries)
 *   build:       (1, scheduled arrival, time it was admitted, time it
 *                 completed, vertices)
 * Times are seconds on the server's clock. */
int chl_server_trace(chl_server* s, double* rows, int64_t cap, int64_t* count);

/* Largest number of device-memory bytes charged to builds at one time since
 * the server was created (never more than mem_budget). */
size_t chl_server_budget_peak(const chl_server* s);

/* Start the clock and the dispatch thread; returns immediately. */
int chl_server_start(chl_server* s);

/* Block until every submitted request has completed. */
int chl_server_wait(chl_server* s);

/* Labeling produced by a completed build (owned by the server). */
const chl_labels* chl_server_labels(chl_server* s, int32_t graph_id);

/* Stop the thread and free everything the server owns. */
void chl_server_destroy(chl_server* s);

#ifdef __cplusplus
}
#endif
#endif /* CHL_H */
