// Internal declarations of the CHL library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/chl.h"

namespace chl {

// ---------------------------------------------------------------- keys
// A tree's per-vertex state is one packed key: (distance << 1) | clean, where
// clean = 1 means that no vertex of any shortest root-v path found so far
// outranks the root. An atomic minimum on the key keeps the shorter distance,
// and on equal distance prefers clean = 0, which is the OR of "outranked"
// over all equal-distance predecessors (the equal-distance ancestor update of
// Algorithm 3, Section 4.2). All ones = not reached.
template <typename K> struct KeyTraits;
template <> struct KeyTraits<uint32_t> { static constexpr uint32_t INF = 0xFFFFFFFFu; };
template <> struct KeyTraits<uint64_t> { static constexpr uint64_t INF = ~0ull; };

// per-root statistics columns: vertex relaxations, arcs relaxed, labels,
// stopped early, relaxation rounds, device wall-clock ticks of the tree
constexpr int STAT_COLS = 6;

// error bits written by kernels
enum : int32_t {
    ERR_BIT_OVERFLOW = 1,     // a label distance >= 2^31 - 1
    ERR_BIT_INVALID = 2,      // invalid input detected on the device
    ERR_BIT_POOL = 4,         // label pool full (host grows it and resumes)
    ERR_BIT_TEAM = 8,         // a team barrier wait exceeded its bound (team aborted)
};

// Graph after rank renumbering: vertex id = rank position, so "u outranks
// the root h" is u < h. arcs[e] = (neighbour << 32) | weight, each row sorted.
struct RGraph {
    int32_t n;
    int64_t m;
    const int64_t* row;
    const uint64_t* arc;
};

// Label pool written by the tree phase: one entry per label, in the order
// trees finish (structure of arrays).
struct Pool {
    int32_t* v;       // labelled vertex (rank position)
    int32_t* hub;     // hub (rank position = root)
    int32_t* dist;    // distance
    unsigned long long cap;
    unsigned long long* cursor;     // device counter of used entries
    unsigned long long* fail_base;  // smallest reservation that did not fit
};

// Per-slot state of the trees in flight.
struct Slots {
    int32_t k;            // number of slots
    int64_t stride;       // elements per slot in key / touched / list arrays
    int64_t fstride;      // flag words per slot
    void* key;            // K[k][stride], all INF between trees
    uint32_t* flags;      // [k][fstride], 4 bits per vertex, all 0 between trees
    int32_t* touched;     // [k][stride]
    int32_t* lists;       // [k][3][stride]: two near lists, one far list
};

struct TreeParams {
    RGraph g;
    Slots s;
    Pool pool;
    int64_t delta;
    int32_t early_term;
    // root work queue (batched form)
    int32_t* next_root;     // device counter into roots[] (or into [0, n))
    int32_t nroots;
    const int32_t* roots;   // NULL: root index = counter value
    int32_t* stop;          // set when the pool is full
    int32_t* failed;        // roots that could not emit (pool full)
    int32_t* nfailed;
    int32_t* far2;          // plain form: filtered far list, n entries
    int32_t root_base;      // batched form without a root list: root = root_base + counter
    int32_t pop_batch;      // batched form: queue positions taken per atomic (>= 1)
    // rank-prefix pruning: the labels found so far, grouped by vertex (rank
    // position), plab[poff[v] .. poff[v+1]) = (hub << 32) | dist;
    // trees of roots >= pbound prune with the hubs [0, pbound) (their labels
    // are complete); poff == NULL or pbound == 0 disables pruning
    const int64_t* poff;
    const uint64_t* plab;
    int32_t pbound;
    // pmin[v] <= every distance in v's group (NULL: none): a walk through a
    // prefix hub from root h to v is at least (h's smallest prefix distance)
    // + pmin[v], so a candidate below that bound skips reading v's group
    const uint32_t* pmin;
    // 1: plab entries are (dist << 32) | hub and each group is sorted by
    // distance (the batched kernel's main phase); 0: (hub << 32) | dist
    int32_t dmaj;
    // batched form, main phase and its probes: 1 = the root's prefix
    // distances in a small LDS hash instead of a dense LDS array (more
    // workgroups resident); a root with more than HASH_MAX_LABELS prefix
    // labels is not grown but appended to ovf (count *novf), for a dense run
    int32_t hashdh;
    int32_t* ovf;
    int32_t* novf;
    // 1 for the combined graph of a directed build (the graph's vertices at
    // even rank positions 2i, their reversed copies at 2i + 1): a root's
    // distances to the prefix hubs are those of its partner h ^ 1 from the
    // hubs x ^ 1, d(h, x) being d'(x ^ 1, h ^ 1) on the reversed copy; 0 else
    int32_t partner;
    // pruned construction of the Hybrid (batched form, phase 3): the root's
    // distances to the hubs [0, pbound) in dhg, n words per slot, all ones
    // between trees (pbound may exceed what LDS holds); every tree's pool
    // range in rlab[2 * root] = first entry, rlab[2 * root + 1] = count
    uint32_t* dhg;
    int64_t* rlab;
    // team and group launches: 1 = a team's workgroups are taken from one
    // XCD (workgroup b of a launch runs on XCD b % 8), 0 = consecutive ids
    int32_t xcd_map;
    // outputs
    int64_t* stats;         // [n][STAT_COLS] by root or NULL
    int32_t* err;
};

// ---------------------------------------------------------------- launchers
// prep.hip
int launch_validate(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                    const int32_t* w, const int32_t* order, int32_t* pos, int32_t* cnt,
                    int32_t* err, int32_t* maxw, hipStream_t st);
int launch_renumber(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                    const int32_t* w, const int32_t* order, const int32_t* pos,
                    int64_t* rrow, uint64_t* rarc, hipStream_t st);
int launch_rank_degrees(int32_t n, const int64_t* row_ptr, const int32_t* order, int64_t* rdeg,
                        hipStream_t st);
int launch_check_symmetric(int32_t n, int64_t m, const int64_t* rrow, const uint64_t* rarc,
                           int32_t* err, hipStream_t st);
// prep.hip: the reversed graph of a validated CSR (input ids): trow[n+1],
// tcol/tw[m], each row sorted by (neighbour, weight); cnt[n], cursor[n],
// tkey[m] and scan_temp (scan_temp_bytes(n)) are scratch
int launch_transpose(int32_t n, int64_t m, const int64_t* row, const int32_t* col, const int32_t* w,
                     int32_t* cnt, int64_t* trow, unsigned long long* cursor, uint64_t* tkey,
                     int32_t* tcol, int32_t* tw, void* scan_temp, hipStream_t st);
// prep.hip: the combined graph of a directed build (2n vertices: the graph
// and its reversal, ranks interleaved), and the split of its labeling into
// in-labels (in place in hub2/dist2, hub positions halved) and out-labels
// (out_off[n+1], out_hub / out_dist[total - off2[n]])
int launch_directed_union(int32_t n, int64_t m, const int64_t* row, const int32_t* col, const int32_t* w,
                          const int32_t* order, const int64_t* trow, const int32_t* tcol, const int32_t* tw,
                          int64_t* row2, int32_t* col2, int32_t* w2, int32_t* order2, hipStream_t st);
int launch_directed_split(int32_t n, int64_t total, const int64_t* off2, int32_t* hub2, const int32_t* dist2,
                          int64_t* out_off, int32_t* out_hub, int32_t* out_dist, hipStream_t st);
// out[64]: 16 samples x (row offset, ranking entry, neighbour, weight)
int launch_sample_input(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                        const int32_t* order, int64_t* out, hipStream_t st);

// scan.hip: exclusive prefix sum of int64 in[n] into out[n+1] (out[n] = total)
size_t scan_temp_bytes(int64_t n);
int launch_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* temp, hipStream_t st);
int launch_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* temp, hipStream_t st);

// segsort.hip: sort every segment [off[i], off[i+1]) of keys ascending
size_t segsort_temp_bytes(int64_t nseg);
int launch_segsort_u64(uint64_t* keys, const int64_t* off, int64_t nseg, int64_t total,
                       void* temp, hipStream_t st);

// tree.hip
// phase: 0 main phase of a build, 1 autotuner probe, 2 common-label roots
int launch_tree_batched(const TreeParams& p, int key_bits, int wg, int phase, hipStream_t st);
int launch_tree_plain(const TreeParams& p, int key_bits, int wg, int grid, int32_t root,
                      int32_t* gstate, hipStream_t st);
int plain_grid_size(int key_bits, int wg);
size_t plain_gstate_words();
// Teams: nteams teams of team_size workgroups each grow the trees of the
// root queue, one tree per team at a time (cooperative launch). Team slot i
// is s.key/flags/touched/lists slot i plus far2[i * n]; tstate holds
// TEAM_WORDS int64 words per team, zeroed before the launch.
constexpr int TEAM_WORDS = 32;
int launch_tree_team(const TreeParams& p, int key_bits, int wg, int team_size, int nteams,
                     long long* tstate, int32_t* far2, hipStream_t st);
int team_capacity(int key_bits, int wg);   // co-resident workgroups of the team kernel
// Groups: ngroups teams of team_size 1024-thread workgroups; each team grows
// GROUP_TREES trees of consecutive queue entries at a time, their keys vertex-
// major (group slot i: s.key holds n * GROUP_TREES keys at i * s.stride *
// GROUP_TREES; touched / lists as for teams; far2 [i * n]; gmask 4n words at
// i * 2n: two mask words per vertex, zero between groups; gstate GROUP_WORDS
// words per team, zeroed before the launch). Cooperative launch; pbound <=
// GROUP_MAX_PREFIX.
// Small trees: one 64-thread workgroup per tree, its state in LDS (at most
// 128 vertices, at most 256 prefix labels of its root); roots of trees that
// do not fit are appended to ovf (count *novf, zeroed by the caller) without
// emitting anything. Same root queue, pool and statistics as the batched form.
int launch_tree_small(const TreeParams& p, int key_bits, int nwg, int32_t* ovf, int32_t* novf, hipStream_t st);
int small_capacity(int key_bits);   // co-resident workgroups of the small kernel
constexpr int GROUP_TREES = 16;
constexpr int GROUP_WORDS = 256;
constexpr int GROUP_MAX_PREFIX = 1024;
int launch_tree_group(const TreeParams& p, int key_bits, int wg, int team_size, int ngroups, long long* gstate,
                      int32_t* far2, uint32_t* gmask, hipStream_t st);
int group_capacity(int key_bits, int pbound);   // co-resident workgroups of the group kernel

// assemble.hip
int launch_assemble(int32_t n, const int32_t* order, const Pool& pool, uint64_t total,
                    int32_t* count, int64_t* offsets, int32_t* fill, uint64_t* tmp,
                    int32_t* hub_pos, int32_t* dist, void* scan_temp, void* sort_temp,
                    hipStream_t st);

// assemble.hip: the labels of the pool entries [0, used) grouped by vertex
// (rank position), as (hub << 32) | dist words, from the groups of the
// entries [0, from) (off_old / lab_old; NULL when from == 0) and the entries
// [from, used); count holds the running group sizes (cleared when from == 0).
// The pruning test takes a minimum over a vertex's entries, so their order
// within a group is free.
int launch_prefix_extend(int32_t n, const Pool& pool, uint64_t from, uint64_t used, int32_t* count,
                         const int64_t* off_old, const uint64_t* lab_old, int64_t* off_new, uint64_t* lab_new,
                         int32_t* fill, void* scan_temp, hipStream_t st);
// assemble.hip: pmin[v] = min(pmin[v], distance) over the pool entries
// [from, to) of v (pmin starts all ones and only decreases, so it stays a
// lower bound of v's group when entries leave it)
int launch_group_min(const Pool& pool, uint64_t from, uint64_t to, uint32_t* pmin, hipStream_t st);
// assemble.hip: out[i] = in[i] with its two 32-bit halves exchanged
int launch_swap_halves(const uint64_t* in, uint64_t* out, uint64_t total, hipStream_t st);
// assemble.hip: count[v] = size of v's group in off (0 for every v when
// off is NULL): the running sizes that launch_prefix_extend continues from
int launch_group_sizes(int32_t n, const int64_t* off, int32_t* count, hipStream_t st);
// roots among the rank positions [lo, lo + cnt) whose tree is the root alone
// (no arcs: flag[i] = 1; every neighbour outranks it: 2; else 0), one[i] =
// flag[i] != 0, pos = exclusive prefix sums of one (pos[cnt] = their
// number); then their single labels (r, r, 0) go to the pool entries
// [base, base + pos[cnt]), their statistics rows to stats (if not NULL), and
// the other roots, in rank order, to roots[0, cnt - pos[cnt])
int launch_trivial_count(int32_t lo, int32_t cnt, const int64_t* row, const uint64_t* arc, int32_t* flag,
                         int32_t* one, int64_t* pos, void* scan_temp, hipStream_t st);
int launch_trivial_split(int32_t lo, int32_t cnt, const int32_t* flag, const int64_t* pos, const Pool& pool,
                         uint64_t base, int32_t* roots, int64_t* stats, hipStream_t st);
// hybrid.hip: the cleaning query DQ_Clean (Algorithm 2) over the labels of
// the roots [lo, hi), whose pool ranges rlab holds (first entry, count per
// root) inside [from, ...); (poff, plab) groups every label so far by vertex,
// those of [lo, hi) included. keep[i - from] = 0 for a redundant label, 1
// else; stats (may be NULL) gets each root's kept label count in column 2.
// dcbuf: clean_workgroups(hi - lo, n) * n words, all ones (left so).
int clean_workgroups(int32_t nroots, int32_t n);
int launch_clean(int32_t lo, int32_t hi, int32_t n, const int64_t* rlab, const Pool& pool, uint64_t from,
                 const int64_t* poff, const uint64_t* plab, uint32_t* dcbuf, int32_t* keep, int64_t* stats,
                 hipStream_t st);
// hybrid.hip: the pool entries [from, from + cnt) whose keep flag is 1, in
// order, into (tv, th, td); pos receives cnt + 1 exclusive sums (pos[cnt] =
// entries kept); scan_temp holds scan_temp_bytes(cnt)
int launch_compact(const Pool& pool, uint64_t from, uint64_t cnt, const int32_t* keep, int64_t* pos, void* scan_temp,
                   int32_t* tv, int32_t* th, int32_t* td, hipStream_t st);
// assemble.hip: the roots [g, g2) of a pruning level into roots[0, g2 - g),
// most prefix labels first (poff: the prefix groups; a directed build counts
// the group of the partner h ^ 1 when it lies in [g, g2)), ties by rank; keys
// holds g2 - g words and off2 two. Everything stays on the stream.
int launch_level_order(const int64_t* poff, int32_t g, int32_t g2, int32_t partner, uint64_t* keys,
                       int64_t* off2, int32_t* roots, hipStream_t st);
// assemble.hip: totals of the per-root statistics (settled, arcs, stopped
// early) into sums[0..2] (zeroed by the caller)
int launch_stat_sums(int32_t n, const int64_t* stats, int64_t* sums, hipStream_t st);
constexpr int HASH_MIN_PREFIX = 4096;   // prefixes from this size hash the root's distances
constexpr int HASH_MAX_LABELS = 512;    // prefix labels of a root that the hash holds
constexpr int MAX_PREFIX = 8192;   // largest pruning prefix (root distances live in LDS, 32 KB)

// query.hip: d(u, v) from the lists of u in (off_u, hub_u, dist_u) and of v
// in (off_v, hub_v, dist_v) (the same arrays for an undirected labeling;
// out- and in-labels for a directed one)
int launch_query(int32_t n, const int64_t* off_u, const int32_t* hub_u, const int32_t* dist_u,
                 const int64_t* off_v, const int32_t* hub_v, const int32_t* dist_v,
                 const int32_t* pairs, int64_t q, int64_t* out, int32_t* err, double avg_len,
                 hipStream_t st);

}  // namespace chl

// Device-resident labeling behind the opaque handle of the C-ABI. For a
// directed graph offsets/hub_pos/dist hold the out-labels and in_* the
// in-labels.
struct chl_labels {
    int32_t n = 0;
    int64_t total = 0;
    int64_t* offsets = nullptr;   // [n+1], by input id
    int32_t* hub_pos = nullptr;   // [total]
    int32_t* dist = nullptr;      // [total]
    int directed = 0;
    int64_t in_total = 0;
    int64_t* in_offsets = nullptr;
    int32_t* in_hub_pos = nullptr;
    int32_t* in_dist = nullptr;
    int32_t* order = nullptr;     // [n] = hub_vertex
    int64_t* per_root = nullptr;  // [n][4] or null
    int32_t* qerr = nullptr;      // query error word
    chl_stats st{};
    chl_allocator alloc{};
    std::mutex qmu;
};
