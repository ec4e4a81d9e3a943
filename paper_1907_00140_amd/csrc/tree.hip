// PLaNT trees on gfx950 (Section 4.2, Algorithm 3).
//
// One tree per root h computes exact distances d(h, v) and whether some
// vertex of some shortest h-v path outranks h. v receives the label
// (h, d(h, v)) exactly when no such vertex exists. Vertices are renumbered by
// rank position, so "u outranks h" is u < h.
//
// Frontier: Dijkstra's priority queue is replaced by delta-stepping with a
// near list (tentative distance below the current bucket bound T) and a far
// list (everything else). Near vertices are relaxed in rounds until the
// bucket is a fixpoint; then the far list is filtered, the bound moves to the
// bucket of the smallest pending distance, and the next bucket starts.
// Relaxation is an atomic minimum on the packed key (distance << 1 | clean):
// the candidate of arc (v, u, w) is ((d_v + w) << 1) | (clean_v & (u > h)),
// so a key that drops only in the clean bit is also an improvement, and on
// equal distance the outranked flag wins (OR over equal-distance
// predecessors: the equal-distance ancestor update of Algorithm 3).
//
// Early termination (Section 4.2): at a bucket boundary every vertex with a
// distance below the bound is final. If no pending vertex (far list) is
// clean, no clean vertex remains to be found: along any shortest path to a
// clean vertex, the first vertex that is not final would be pending with its
// final, clean key. The tree stops there; every clean key is then final.
//
// Dedup of the lists uses 4 bits per vertex in a flag word array: bit 0/1 =
// "in near list 0/1" (the two near lists alternate between rounds), bit 2 =
// "in far list". A vertex improved during a round is pushed to the next near
// list unless its bit for that list is set, so every improvement made during
// a round is relaxed in the next round, with no ordering needed between the
// key update and the flag update. Lists therefore never hold a vertex twice
// and fit in n entries.
//
// Batched form: a persistent kernel, one workgroup per tree; each workgroup
// owns a slot of per-tree state and pops roots from a rank-ordered work queue
// (the paper's atomic task counter, Section 3.1). Team form: the same queue,
// one tree per team of workgroups, for launches with fewer trees than the
// device holds workgroups. Plain form: the whole grid grows one tree per
// cooperative launch.
#include <hip/hip_cooperative_groups.h>

#include "internal.h"

namespace cg = cooperative_groups;

namespace chl {

namespace {

constexpr uint32_t FAR_BIT = 4u;

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Append for every lane with pred set: one atomic per wave on *counter.
// Returns the slot index for lanes with pred, undefined otherwise.
template <typename C>
__device__ __forceinline__ int64_t wave_append(bool pred, C* counter) {
    uint64_t m = __ballot(pred);
    if (m == 0) return -1;
    int leader = __ffsll((unsigned long long)m) - 1;
    int64_t base = 0;
    if ((int)__lane_id() == leader) base = (int64_t)atomicAdd(counter, (C)__popcll(m));
    base = __shfl(base, leader);
    return base + lanes_below(m);
}

template <int SCOPE, typename T>
__device__ __forceinline__ T ld(T* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, SCOPE); }
template <int SCOPE, typename T>
__device__ __forceinline__ void st(T* p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, SCOPE); }
template <int SCOPE, typename T>
__device__ __forceinline__ T amin(T* p, T v) { return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, SCOPE); }
template <int SCOPE>
__device__ __forceinline__ uint32_t aor(uint32_t* p, uint32_t v) { return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, SCOPE); }
template <int SCOPE>
__device__ __forceinline__ uint32_t aand(uint32_t* p, uint32_t v) { return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, SCOPE); }

__device__ __forceinline__ uint32_t fshift(int32_t v) { return (uint32_t)(v & 7) * 4u; }

// Entries of the vertex lists (near, far, touched) are read and written with
// relaxed atomics at the scope of the workgroups that share the tree: plain
// accesses in the batched form (workgroup scope), device-coherent ones when a
// team of workgroups shares it, so that a team barrier needs no cache
// write-back. A vertex id read from a list is clamped into [0, n): it always
// is in range; the clamp only guarantees that no access can leave the arrays.
template <int SCOPE>
__device__ __forceinline__ int32_t lget(const int32_t* p, int32_t n) {
    const uint32_t v = (uint32_t)__hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, SCOPE);
    return (int32_t)(v < (uint32_t)n ? v : (uint32_t)(n - 1));
}
template <int SCOPE>
__device__ __forceinline__ void lput(int32_t* p, int32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, SCOPE); }

// Block-wide exclusive scan of uint32 (WG threads). wsum: WG/64 entries of LDS.
template <int WG>
__device__ __forceinline__ uint32_t block_scan(uint32_t x, uint32_t* wsum, uint32_t& total) {
    constexpr int NW = WG / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(v, d);
        if (lane >= d) v += y;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        uint32_t s = lane < NW ? wsum[lane] : 0u;
#pragma unroll
        for (int d = 1; d < NW; d <<= 1) {
            uint32_t y = __shfl_up(s, d);
            if (lane >= d) s += y;
        }
        if (lane < NW) wsum[lane] = s;
    }
    __syncthreads();
    total = wsum[NW - 1];
    uint32_t ex = (w ? wsum[w - 1] : 0u) + v - x;
    return ex;
}

template <int WG, typename T, typename F>
__device__ __forceinline__ T block_reduce(T x, T* red, T ident, F op) {
    constexpr int NW = WG / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x = op(x, __shfl_xor(x, d));
    if (lane == 0) red[w] = x;
    __syncthreads();
    T r = ident;
#pragma unroll
    for (int i = 0; i < NW; i++) r = op(r, red[i]);
    __syncthreads();
    return r;
}

template <typename K>
__device__ __forceinline__ K pack(uint64_t d, uint32_t clean) { return (K)((d << 1) | clean); }

// LDS of the block-level frontier expansion.
template <typename K, int WG>
struct Expand {
    int64_t beg[WG];
    K key[WG];
    uint32_t off[WG];
    uint32_t wsum[WG / 64];
};

// Relax every arc of the vertices cur[base .. base+nv) (nv <= WG), balanced
// over the block by arc index: thread t handles arcs t, t+WG, ... of the
// chunk, RELAX_ILP of them at a time so that their loads are in flight
// together. Improved vertices go to the touched list (the first time they
// are reached), to the next near list (new distance below T) or to the far
// list, through wave-aggregated appends on the counters. Every clean key
// set here raises *umax (largest clean distance so far); clean far pushes
// are counted in *cnt_far_clean.
constexpr int RELAX_ILP = 4;

// The root's distances to its prefix hubs as an open-addressing LDS hash
// (keys -1 when free, at most half full): the main phase's roots have a few
// dozen prefix labels, and a dense array of prefix-size words limits how
// many workgroups a compute unit holds.
constexpr int HCAP = 2 * HASH_MAX_LABELS;

__device__ __forceinline__ uint32_t hash_slot(uint32_t x) {
    return (x * 2654435761u) >> (32 - __builtin_ctz((uint32_t)HCAP));
}

__device__ __forceinline__ uint32_t hash_lookup(const int32_t* hk, const uint32_t* hv, uint32_t x) {
    uint32_t s = hash_slot(x);
    for (int i = 0; i < HCAP; i++, s = (s + 1) & (HCAP - 1)) {
        const int32_t k = hk[s];
        if (k == (int32_t)x) return hv[s];
        if (k < 0) return 0xFFFFFFFFu;
    }
    return 0xFFFFFFFFu;
}

template <int C>
struct HashLds {
    int32_t k[C];
    uint32_t v[C];
};

template <typename K, int WG, int SCOPE, typename C>
__device__ __forceinline__ void relax_block(const RGraph& g, K* key, uint32_t* flags,
                                            const int32_t* cur, int32_t base, int32_t nv,
                                            uint32_t curbit, uint32_t nextbit, int32_t h,
                                            int64_t T, int32_t* touched, int32_t* next,
                                            int32_t* far, C* cnt_touched, C* cnt_next,
                                            C* cnt_far, C* cnt_far_clean, unsigned long long* umax,
                                            const int64_t* poff, const uint64_t* plab, uint32_t pbound,
                                            const uint32_t* dh, Expand<K, WG>& X, uint64_t& arcs,
                                            bool rank_query = false, const uint32_t* pmin = nullptr,
                                            uint32_t dhmin = 0, bool dmaj = false,
                                            const int32_t* hk = nullptr) {
    const int tid = threadIdx.x;
    uint32_t deg = 0;
    if (tid < nv) {
        int32_t v = lget<SCOPE>(&cur[base + tid], g.n);
        aand<SCOPE>(&flags[v >> 3], ~(curbit << fshift(v)));
        K kv = ld<SCOPE>(&key[v]);
        int64_t b = g.row[v];
        deg = (uint32_t)(g.row[v + 1] - b);
        X.beg[tid] = b;
        X.key[tid] = kv;
    }
    uint32_t total;
    uint32_t ex = block_scan<WG>(deg, X.wsum, total);
    X.off[tid] = ex;
    __syncthreads();
    arcs += total;
    unsigned long long my_umax = 0;
    bool my_umax_set = false;
    for (uint32_t e0 = tid; e0 < total; e0 += WG * RELAX_ILP) {
        int own[RELAX_ILP];
        uint64_t a[RELAX_ILP];
        K seen[RELAX_ILP];
#pragma unroll
        for (int j = 0; j < RELAX_ILP; j++) {
            const uint32_t e = e0 + j * WG;
            int lo = 0, hi = nv - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (X.off[mid] <= e) lo = mid; else hi = mid - 1;
            }
            own[j] = lo;
        }
#pragma unroll
        for (int j = 0; j < RELAX_ILP; j++) {
            const uint32_t e = e0 + j * WG;
            a[j] = e < total ? g.arc[X.beg[own[j]] + (e - X.off[own[j]])] : 0;
        }
#pragma unroll
        for (int j = 0; j < RELAX_ILP; j++) {
            const uint32_t e = e0 + j * WG;
            seen[j] = e < total ? ld<SCOPE>(&key[(int32_t)(a[j] >> 32)]) : (K)0;
        }
#pragma unroll
        for (int j = 0; j < RELAX_ILP; j++) {
            const uint32_t e = e0 + j * WG;
            const bool valid = e < total;
            const int32_t u = (int32_t)(a[j] >> 32);
            const K kv = X.key[own[j]];
            const uint64_t nd = (uint64_t)(kv >> 1) + (uint32_t)a[j];
            const K nk = pack<K>(nd, (uint32_t)(kv & 1) & (uint32_t)(u > h));
            // Keys only decrease, so a value read earlier is never below the
            // current one: when the candidate is not below it, the atomic
            // would fail and is skipped.
            bool cand = valid && nk < seen[j];
            // rank query of the pruned construction (Algorithm 1): a vertex
            // that outranks the root is neither labelled nor expanded
            if (rank_query && u < h) cand = false;
            // no walk through a prefix hub is shorter than the root's nearest
            // prefix hub plus u's: below that bound u's group is not read
            if (cand && dh && (!pmin || (uint64_t)dhmin + pmin[u] <= nd)) {
                // Rank-prefix pruning (Section 4.3): the labels of the hubs
                // [0, pbound), complete because their trees are done, give the
                // length of the shortest root-u walk through each of them
                // (dh holds the root's side). If one is no longer than the
                // candidate, the candidate is either not a shortest path or a
                // shortest path through a hub that outranks the root; either
                // way it cannot lead to a label, and a vertex whose true key
                // is clean never has such a hub on its shortest paths, so
                // dropping the candidate changes no label. u's entries are read
                // 8 at a time until one prunes.
                const int64_t lb = poff[u], le = poff[u + 1];
                for (int64_t i = lb; i < le && cand; i += 8) {
                    uint64_t lx[8];
#pragma unroll
                    for (int z = 0; z < 8; z++) lx[z] = i + z < le ? plab[i + z] : ~0ull;
#pragma unroll
                    for (int z = 0; z < 8; z++) {
                        const uint32_t x = dmaj ? (uint32_t)lx[z] : (uint32_t)(lx[z] >> 32);
                        const uint32_t dd = dmaj ? (uint32_t)(lx[z] >> 32) : (uint32_t)lx[z];
                        if (x >= pbound) continue;
                        const uint32_t a = hk ? hash_lookup(hk, dh, x) : dh[x];
                        if (a != 0xFFFFFFFFu && (uint64_t)a + dd <= nd) cand = false;
                    }
                    // groups ordered by distance: no later entry is closer
                    if (dmaj && (uint64_t)(uint32_t)(lx[7] >> 32) + dhmin > nd) break;
                }
            }
            K old = seen[j];
            if (cand) old = amin<SCOPE>(&key[u], nk);
            const bool imp = cand && nk < old;
            const bool first = imp && old == KeyTraits<K>::INF;
            const bool tonear = imp && (int64_t)nd < T;
            bool pnear = false, pfar = false;
            if (imp) {
                if (nk & 1) { my_umax = my_umax > nd ? my_umax : nd; my_umax_set = true; }
                uint32_t bit = (tonear ? nextbit : FAR_BIT) << fshift(u);
                uint32_t o = aor<SCOPE>(&flags[u >> 3], bit);
                bool fresh = (o & bit) == 0;
                pnear = fresh && tonear;
                pfar = fresh && !tonear;
            }
            int64_t q = wave_append(first, cnt_touched);
            if (first && q < g.n) lput<SCOPE>(&touched[q], u);
            q = wave_append(pnear, cnt_next);
            if (pnear && q < g.n) lput<SCOPE>(&next[q], u);
            q = wave_append(pfar, cnt_far);
            if (pfar && q < g.n) lput<SCOPE>(&far[q], u);
            const bool pfc = pfar && (nk & 1);
            (void)wave_append(pfc, cnt_far_clean);
        }
    }
    if (my_umax_set) atomicMax(umax, my_umax);
    __syncthreads();
}

// ---------------------------------------------------------------- batched
template <typename K, int WG>
struct BatchedLds {
    Expand<K, WG> X;
    unsigned long long red64[WG / 64];
    int32_t red32[WG / 64];
    int32_t ncur, cnt_next, cnt_far, cnt_touched, nkeep, far_clean;
    int32_t root;
    int32_t bnext, bend;      // root queue positions taken by this workgroup, not yet grown
    uint32_t dhmin;           // smallest distance of the root to a prefix hub
    unsigned long long umax;
    long long pool_base;
};

// Early termination between rounds. Pending vertices are the current near
// list and the far list. If none of them is clean, and no pending distance
// can be at or below the largest clean distance ever set (umax), no later
// relaxation can create or change a clean key: every vertex whose true key
// is clean already has it (the first unfinished vertex on a shortest path to
// it would be pending and clean), and every clean key is final. The pending
// distances are bounded below by the smallest near key and by T (far
// entries hold distances >= T; a far vertex whose key dropped below T has
// been pushed to the near list as well). far_clean counts clean pushes to
// the far list since the last filter, an upper bound of its clean entries.
template <typename K, int WG, int SC>
__device__ __forceinline__ bool may_stop(BatchedLds<K, WG>& S, const K* key, const int32_t* cur,
                                         int32_t ncur, int64_t T) {
    constexpr int NW = WG / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // one reduction of (smallest pending distance, any pending vertex clean):
    // the distance in the high bits, the clean flag in bit 0 of the OR half
    unsigned long long mn = ~0ull;
    int32_t cl = 0;
    for (int32_t i = tid; i < ncur; i += WG) {
        K kv = ld<SC>(const_cast<K*>(&key[cur[i]]));
        unsigned long long d = (unsigned long long)(kv >> 1);
        mn = d < mn ? d : mn;
        cl |= (int32_t)(kv & 1);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(mn, d);
        mn = o < mn ? o : mn;
        cl |= __shfl_xor(cl, d);
    }
    if (lane == 0) { S.red64[w] = mn; S.red32[w] = cl; }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NW; i++) {
        mn = S.red64[i] < mn ? S.red64[i] : mn;
        cl |= S.red32[i];
    }
    __syncthreads();
    unsigned long long lb = mn < (unsigned long long)T ? mn : (unsigned long long)T;
    return cl == 0 && lb > S.umax;
}

// PHASE names the launch (0: main phase of a build, 1: autotuner probe,
// 2: the common-label roots grown before the main phase), so that profiles
// separate them; PHASE 3 is the pruned construction of the Hybrid
// (Section 4.2.1): pruned Dijkstra with rank queries (Algorithm 1), every
// vertex it reaches labelled, the distance queries answered by all labels
// of the hubs [0, p.pbound), the root's side in the global p.dhg, and each
// tree's pool range recorded in p.rlab for the cleaning that follows.
// PRUNE: rank-prefix pruning with p.poff / p.plab; the root's distances to
// the prefix hubs live in dynamic LDS (p.pbound words) below phase 3.
template <typename K, int WG, int PHASE, bool PRUNE, bool HS>
__global__ __launch_bounds__(WG) void k_tree_batched(TreeParams p) {
    constexpr int SC = __HIP_MEMORY_SCOPE_WORKGROUP;
    constexpr bool HYB = PHASE == 3;
    __shared__ BatchedLds<K, WG> S;
    __shared__ HashLds<HS ? HCAP : 1> H;
    extern __shared__ uint32_t dh_lds[];
    const int tid = threadIdx.x;
    const int64_t slot = blockIdx.x;
    uint32_t* dh = HYB ? p.dhg + slot * p.s.stride : HS ? H.v : dh_lds;
    K* key = (K*)p.s.key + slot * p.s.stride;
    uint32_t* flags = p.s.flags + slot * p.s.fstride;
    int32_t* touched = p.s.touched + slot * p.s.stride;
    int32_t* lists = p.s.lists + slot * 3 * p.s.stride;
    int32_t* far = lists + 2 * p.s.stride;
    const int64_t delta = p.delta;
    // dh is all ones between trees: a tree sets its root's entries and
    // clears them when it is done (the global array of phase 3 is set to
    // all ones when it is allocated)
    if (PRUNE && !HYB && !HS)
        for (int x = tid; x < p.pbound; x += WG) dh[x] = 0xFFFFFFFFu;
    if (HS)
        for (int x = tid; x < HCAP; x += WG) H.k[x] = -1;
    if (tid == 0) { S.bnext = 0; S.bend = 0; }

    for (;;) {
        if (tid == 0) {
            // roots are taken from the queue pop_batch at a time (one atomic
            // on the shared counter per batch); once the pool is full, the
            // roots taken but not grown are handed back as failed
            int32_t r = -1;
            const bool stopped = __hip_atomic_load(p.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            if (stopped) {
                for (int32_t c = S.bnext; c < S.bend; c++)
                    p.failed[atomicAdd(p.nfailed, 1)] = p.roots ? p.roots[c] : p.root_base + c;
                S.bnext = S.bend;
            } else if (S.bnext >= S.bend) {
                const int32_t c = atomicAdd(p.next_root, p.pop_batch);
                S.bnext = c;
                S.bend = c < p.nroots ? min(p.nroots, c + p.pop_batch) : c;
            }
            if (S.bnext < S.bend) {
                r = p.roots ? p.roots[S.bnext] : p.root_base + S.bnext;
                S.bnext++;
            }
            S.root = r;
            S.dhmin = 0xFFFFFFFFu;
        }
        __syncthreads();
        const int32_t h = S.root;
        if (h < 0) break;
        const bool prune = PRUNE && h >= p.pbound;
        const uint32_t px = (uint32_t)p.partner;
        const int32_t hg = h ^ (int32_t)px;          // whose prefix labels give d(h, x)
        if (HS && prune && p.poff[hg + 1] - p.poff[hg] > HASH_MAX_LABELS) {
            // more prefix labels than the hash holds: grown afterwards with
            // the dense array (no emission, no statistics here)
            if (tid == 0) p.ovf[atomicAdd(p.novf, 1)] = h;
            __syncthreads();
            continue;
        }
        if (prune)
            for (int64_t i = p.poff[hg] + tid; i < p.poff[hg + 1]; i += WG) {
                const uint64_t lx = p.plab[i];
                const uint32_t x = p.dmaj ? (uint32_t)lx : (uint32_t)(lx >> 32), y = x ^ px;
                const uint32_t dd = p.dmaj ? (uint32_t)(lx >> 32) : (uint32_t)lx;
                if (x < (uint32_t)p.pbound && y < (uint32_t)p.pbound) {
                    if (HS) {
                        uint32_t s = hash_slot(y);
                        while (atomicCAS(&H.k[s], -1, (int32_t)y) != -1) s = (s + 1) & (HCAP - 1);
                        H.v[s] = dd;
                    } else {
                        dh[y] = dd;
                    }
                    atomicMin(&S.dhmin, dd);
                }
            }

        // ---- init: root key (0, clean) in near list 0
        if (tid == 0) {
            st<SC>(&key[h], pack<K>(0, 1));
            touched[0] = h;
            lists[0] = h;
            aor<SC>(&flags[h >> 3], 1u << fshift(h));
            S.ncur = 1; S.cnt_next = 0; S.cnt_far = 0; S.cnt_touched = 1;
            S.far_clean = 0; S.umax = 0;
        }
        __syncthreads();
        int64_t T = delta;
        int it = 0;
        uint64_t arcs = 0, settled = 0;
        const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
        bool early = false;
        for (;;) {
            // ---- rounds inside the bucket until no near vertex is left
            bool stopped = false;
            for (;;) {
                const int32_t ncur = S.ncur;
                const uint32_t curbit = 1u << (it & 1), nextbit = 1u << ((it + 1) & 1);
                int32_t* cur = lists + (int64_t)(it & 1) * p.s.stride;
                int32_t* next = lists + (int64_t)((it + 1) & 1) * p.s.stride;
                // (the first round holds only the root, which is clean)
                if (p.early_term && it > 0 && S.far_clean == 0 && may_stop<K, WG, SC>(S, key, cur, ncur, T)) {
                    // drop the pending entries: clear their list bits
                    for (int32_t i = tid; i < ncur; i += WG) aand<SC>(&flags[cur[i] >> 3], ~(curbit << fshift(cur[i])));
                    for (int32_t i = tid; i < S.cnt_far; i += WG) aand<SC>(&flags[far[i] >> 3], ~(FAR_BIT << fshift(far[i])));
                    early = ncur > 0 || S.cnt_far > 0;
                    stopped = true;
                    __syncthreads();
                    break;
                }
                settled += ncur;
                for (int32_t base = 0; base < ncur; base += WG)
                    relax_block<K, WG, SC>(p.g, key, flags, cur, base, min(WG, ncur - base), curbit,
                                           nextbit, h, T, touched, next, far, &S.cnt_touched,
                                           &S.cnt_next, &S.cnt_far, &S.far_clean, &S.umax, p.poff,
                                           p.plab, (uint32_t)p.pbound, prune ? dh : nullptr, S.X, arcs, HYB,
                                           p.pmin, S.dhmin, p.dmaj != 0, HS ? H.k : nullptr);
                __syncthreads();
                it++;
                if (tid == 0) { S.ncur = S.cnt_next; S.cnt_next = 0; }
                __syncthreads();
                if (S.ncur == 0) break;
            }
            if (stopped) break;
            // ---- bucket done: drop settled far entries, find the smallest
            //      pending distance and whether any pending vertex is clean
            int32_t nfar = S.cnt_far;
            // nothing pending at all (most trees of the main phase end so):
            // the tree is complete without the filter's reductions
            if (nfar == 0) break;
            if (tid == 0) { S.nkeep = 0; }
            __syncthreads();
            unsigned long long mymin = ~0ull;
            int32_t myclean = 0;
            for (int32_t base = 0; base < nfar; base += WG) {
                const int32_t i = base + tid;
                bool keep = false;
                int32_t v = 0;
                K kv = 0;
                if (i < nfar) {
                    v = far[i];
                    aand<SC>(&flags[v >> 3], ~(FAR_BIT << fshift(v)));
                    kv = ld<SC>(&key[v]);
                    keep = (int64_t)(kv >> 1) >= T;
                }
                __syncthreads();                         // chunk read before compaction writes
                int64_t q = wave_append(keep, &S.nkeep);
                if (keep) {
                    far[q] = v;
                    mymin = min(mymin, (unsigned long long)(kv >> 1));
                    myclean += (int32_t)(kv & 1);
                }
                __syncthreads();
            }
            unsigned long long mn = block_reduce<WG>(mymin, S.red64, ~0ull,
                [](unsigned long long a, unsigned long long b) { return a < b ? a : b; });
            int32_t ncl = block_reduce<WG>(myclean, S.red32, 0, [](int32_t a, int32_t b) { return a + b; });
            nfar = S.nkeep;
            if (nfar == 0 || (p.early_term && ncl == 0)) { early = nfar > 0; break; }
            // ---- next bucket: the one holding the smallest pending distance
            T = ((int64_t)mn / delta + 1) * delta;
            int32_t* cur = lists + (int64_t)(it & 1) * p.s.stride;
            const uint32_t curbit = 1u << (it & 1);
            if (tid == 0) { S.ncur = 0; S.cnt_far = 0; S.far_clean = 0; }
            __syncthreads();
            for (int32_t base = 0; base < nfar; base += WG) {
                const int32_t i = base + tid;
                int32_t v = 0;
                bool tonear = false, tofar = false, fclean = false;
                if (i < nfar) {
                    v = far[i];
                    K kv = ld<SC>(&key[v]);
                    tonear = (int64_t)(kv >> 1) < T;
                    tofar = !tonear;
                    fclean = tofar && (kv & 1);
                }
                __syncthreads();
                int64_t q = wave_append(tonear, &S.ncur);
                if (tonear) { cur[q] = v; aor<SC>(&flags[v >> 3], curbit << fshift(v)); }
                q = wave_append(tofar, &S.cnt_far);
                if (tofar) { far[q] = v; aor<SC>(&flags[v >> 3], FAR_BIT << fshift(v)); }
                (void)wave_append(fclean, &S.far_clean);
                __syncthreads();
            }
        }
        // far entries left behind have had their far bit cleared

        // ---- emit labels of clean vertices, reset the slot
        const int32_t nt = S.cnt_touched;
        int32_t mycnt = 0;
        for (int32_t i = tid; i < nt; i += WG) mycnt += (int32_t)(ld<SC>(&key[touched[i]]) & 1);
        const int32_t nl = block_reduce<WG>(mycnt, S.red32, 0, [](int32_t a, int32_t b) { return a + b; });
        if (tid == 0) {
            unsigned long long b = atomicAdd(p.pool.cursor, (unsigned long long)nl);
            if (b + (unsigned long long)nl > p.pool.cap) {
                S.pool_base = -1;
                atomicOr(p.err, ERR_BIT_POOL);
                atomicExch(p.stop, 1);
                atomicMin(p.pool.fail_base, b);
                p.failed[atomicAdd(p.nfailed, 1)] = h;
            } else {
                S.pool_base = (long long)b;
            }
            S.nkeep = 0;
        }
        __syncthreads();
        const long long pb = S.pool_base;
        bool ovf = false;
        for (int32_t base = 0; base < nt; base += WG) {
            const int32_t i = base + tid;
            bool lab = false;
            int32_t v = 0;
            uint64_t d = 0;
            if (i < nt) {
                v = touched[i];
                K kv = ld<SC>(&key[v]);
                lab = (kv & 1) != 0;
                d = (uint64_t)(kv >> 1);
                st<SC>(&key[v], KeyTraits<K>::INF);
            }
            int64_t q = wave_append(lab, &S.nkeep);
            if (lab && pb >= 0) {
                ovf |= d > 0x7FFFFFFEull;
                p.pool.v[pb + q] = v;
                p.pool.hub[pb + q] = h;
                p.pool.dist[pb + q] = (int32_t)d;
            }
        }
        if (ovf) atomicOr(p.err, ERR_BIT_OVERFLOW);
        if (HYB && tid == 0 && pb >= 0) {
            p.rlab[2 * (int64_t)h] = pb;
            p.rlab[2 * (int64_t)h + 1] = nl;
        }
        if (p.stats && tid == 0) {
            // every thread of the block accumulated the same settled / arc counts
            int64_t* s = p.stats + (int64_t)h * STAT_COLS;
            s[0] = (int64_t)settled; s[1] = (int64_t)arcs; s[2] = nl; s[3] = early ? 1 : 0;
            s[4] = it; s[5] = (int64_t)(__builtin_amdgcn_s_memrealtime() - t_start);
        }
        // every read of dh is behind the emission's barriers
        if (HS && prune)
            for (int x = tid; x < HCAP; x += WG) H.k[x] = -1;
        if (prune && !HS)
            for (int64_t i = p.poff[hg] + tid; i < p.poff[hg + 1]; i += WG) {
                const uint32_t x = p.dmaj ? (uint32_t)p.plab[i] : (uint32_t)(p.plab[i] >> 32), y = x ^ px;
                if (x < (uint32_t)p.pbound && y < (uint32_t)p.pbound) dh[y] = 0xFFFFFFFFu;
            }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- plain
// Device-wide tree: every workgroup of a cooperative grid works on the same
// root. Global state words (int64):
enum {
    G_CNT0 = 0, G_CNT1, G_CNT2,   // near list counts, rotating by round % 3
    G_FAR, G_FAR2, G_TOUCHED,     // far list, filtered far list, touched list
    G_MIN, G_CLEAN, G_T, G_DONE, G_EARLY,
    G_SETTLED, G_ARCS, G_NLAB, G_BASE, G_FILL, G_FARCLEAN, G_UMAX,
    G_WORDS
};

template <typename K, int WG>
struct PlainLds {
    Expand<K, WG> X;
    unsigned long long red64[WG / 64];
};

template <typename K, int WG>
__global__ __launch_bounds__(WG) void k_tree_plain(TreeParams p, int32_t h, long long* gs) {
    constexpr int SC = __HIP_MEMORY_SCOPE_AGENT;
    __shared__ PlainLds<K, WG> S;
    cg::grid_group grid = cg::this_grid();
    const int tid = threadIdx.x;
    const int64_t gtid = (int64_t)blockIdx.x * WG + tid;
    const int64_t gthreads = (int64_t)gridDim.x * WG;
    K* key = (K*)p.s.key;
    uint32_t* flags = p.s.flags;
    int32_t* touched = p.s.touched;
    int32_t* lists = p.s.lists;            // near0, near1, far
    int32_t* far = lists + 2 * p.s.stride;
    int32_t* far2 = p.far2;                // filtered far list (n entries)
    const int64_t delta = p.delta;

    if (gtid == 0) {
        for (int i = 0; i < G_WORDS; i++) gs[i] = 0;
        gs[G_MIN] = 0x7FFFFFFFFFFFFFFFll;
        st<SC>(&key[h], pack<K>(0, 1));
        touched[0] = h;
        lists[0] = h;
        aor<SC>(&flags[h >> 3], 1u << fshift(h));
        gs[G_CNT0] = 1;
        gs[G_TOUCHED] = 1;
        gs[G_T] = delta;
        __threadfence();
    }
    grid.sync();
    int it = 0;
    uint64_t arcs = 0;
    for (;;) {
        // ---- one round over the near list
        const int64_t T = gs[G_T];
        const int32_t ncur = (int32_t)gs[G_CNT0 + it % 3];
        const uint32_t curbit = 1u << (it & 1), nextbit = 1u << ((it + 1) & 1);
        int32_t* cur = lists + (int64_t)(it & 1) * p.s.stride;
        int32_t* next = lists + (int64_t)((it + 1) & 1) * p.s.stride;
        if (ncur > 0) {
            for (int32_t base = blockIdx.x * WG; base < ncur; base += gridDim.x * WG)
                relax_block<K, WG, SC>(p.g, key, flags, cur, base, min(WG, ncur - base), curbit,
                                       nextbit, h, T, touched, next, far,
                                       (unsigned long long*)&gs[G_TOUCHED],
                                       (unsigned long long*)&gs[G_CNT0 + (it + 1) % 3],
                                       (unsigned long long*)&gs[G_FAR],
                                       (unsigned long long*)&gs[G_FARCLEAN],
                                       (unsigned long long*)&gs[G_UMAX], nullptr, nullptr, 0u, nullptr, S.X,
                                       arcs);
            if (gtid == 0) { gs[G_CNT0 + (it + 2) % 3] = 0; gs[G_SETTLED] += ncur; }
            __threadfence();
            grid.sync();
            it++;
            continue;
        }
        // ---- bucket done: filter far into far2 (drop settled entries)
        const int32_t nfar = (int32_t)gs[G_FAR];
        unsigned long long mymin = ~0ull, myclean = 0;
        for (int64_t i = gtid; i < nfar; i += gthreads) {
            int32_t v = far[i];
            aand<SC>(&flags[v >> 3], ~(FAR_BIT << fshift(v)));
            K kv = ld<SC>(&key[v]);
            bool keep = (int64_t)(kv >> 1) >= T;
            if (keep) {
                mymin = min(mymin, (unsigned long long)(kv >> 1));
                myclean += (unsigned long long)(kv & 1);
            }
            int64_t q = wave_append(keep, (unsigned long long*)&gs[G_FAR2]);
            if (keep) far2[q] = v;
        }
        mymin = block_reduce<WG>(mymin, S.red64, ~0ull,
            [](unsigned long long a, unsigned long long b) { return a < b ? a : b; });
        myclean = block_reduce<WG>(myclean, S.red64, 0ull,
            [](unsigned long long a, unsigned long long b) { return a + b; });
        if (tid == 0) {
            if (mymin != ~0ull) atomicMin((unsigned long long*)&gs[G_MIN], mymin);
            atomicAdd((unsigned long long*)&gs[G_CLEAN], myclean);
        }
        __threadfence();
        grid.sync();
        const int32_t nkeep = (int32_t)gs[G_FAR2];
        const bool done = nkeep == 0 || (p.early_term && gs[G_CLEAN] == 0);
        const int64_t Tn = ((int64_t)gs[G_MIN] / delta + 1) * delta;
        grid.sync();                              // everyone has read the filter results
        if (done) {
            if (gtid == 0) gs[G_EARLY] = nkeep > 0;
            break;
        }
        if (gtid == 0) {
            gs[G_FAR] = 0; gs[G_FAR2] = 0; gs[G_CLEAN] = 0; gs[G_MIN] = 0x7FFFFFFFFFFFFFFFll;
            gs[G_T] = Tn;
        }
        // far2 -> near (current list of the next round) or back to far
        int32_t* ncurl = lists + (int64_t)(it & 1) * p.s.stride;
        const uint32_t nb = 1u << (it & 1);
        grid.sync();
        for (int64_t i = gtid; i < nkeep; i += gthreads) {
            int32_t v = far2[i];
            K kv = ld<SC>(&key[v]);
            bool tonear = (int64_t)(kv >> 1) < Tn;
            int64_t q = wave_append(tonear, (unsigned long long*)&gs[G_CNT0 + it % 3]);
            if (tonear) { ncurl[q] = v; aor<SC>(&flags[v >> 3], nb << fshift(v)); }
            q = wave_append(!tonear, (unsigned long long*)&gs[G_FAR]);
            if (!tonear) { far[q] = v; aor<SC>(&flags[v >> 3], FAR_BIT << fshift(v)); }
        }
        __threadfence();
        grid.sync();
    }
    // ---- emit
    const int64_t nt = gs[G_TOUCHED];
    unsigned long long mycnt = 0;
    for (int64_t i = gtid; i < nt; i += gthreads) mycnt += (unsigned long long)(ld<SC>(&key[touched[i]]) & 1);
    mycnt = block_reduce<WG>(mycnt, S.red64, 0ull, [](unsigned long long a, unsigned long long b) { return a + b; });
    if (tid == 0) atomicAdd((unsigned long long*)&gs[G_NLAB], mycnt);
    if (tid == 0) atomicAdd((unsigned long long*)&gs[G_ARCS], (unsigned long long)arcs);
    __threadfence();
    grid.sync();
    if (gtid == 0) {
        unsigned long long nl = (unsigned long long)gs[G_NLAB];
        unsigned long long b = atomicAdd(p.pool.cursor, nl);
        if (b + nl > p.pool.cap) {
            gs[G_BASE] = -1;
            atomicOr(p.err, ERR_BIT_POOL);
            atomicMin(p.pool.fail_base, b);
            p.failed[atomicAdd(p.nfailed, 1)] = h;
        } else {
            gs[G_BASE] = (long long)b;
        }
        __threadfence();
    }
    grid.sync();
    const long long pb = gs[G_BASE];
    bool ovf = false;
    for (int64_t i = gtid; i < nt; i += gthreads) {
        int32_t v = touched[i];
        K kv = ld<SC>(&key[v]);
        bool lab = (kv & 1) != 0;
        uint64_t d = (uint64_t)(kv >> 1);
        st<SC>(&key[v], KeyTraits<K>::INF);
        int64_t q = wave_append(lab, (unsigned long long*)&gs[G_FILL]);
        if (lab && pb >= 0) {
            ovf |= d > 0x7FFFFFFEull;
            p.pool.v[pb + q] = v;
            p.pool.hub[pb + q] = h;
            p.pool.dist[pb + q] = (int32_t)d;
        }
    }
    if (ovf) atomicOr(p.err, ERR_BIT_OVERFLOW);
    if (p.stats && gtid == 0) {
        // counters of this tree are complete after the last grid barrier
        int64_t* s = p.stats + (int64_t)h * STAT_COLS;
        s[0] = gs[G_SETTLED]; s[1] = gs[G_ARCS]; s[2] = gs[G_NLAB]; s[3] = gs[G_EARLY];
        s[4] = it; s[5] = 0;
    }
}

// ---------------------------------------------------------------- teams
// A team of W workgroups grows one tree at a time: the rounds of the plain
// form confined to W workgroups, with the rank-ordered root queue of the
// batched form over the teams. It serves the first trees of a build, which
// span most of the graph and are too few to fill the device with one
// workgroup each. The team's words (int64, zero at launch):
enum {
    T_CNT0 = 0, T_CNT1, T_CNT2,   // near list counts, rotating by round % 3
    T_FAR, T_FAR2, T_TOUCHED,     // far list, filtered far list, touched list
    T_MIN, T_CLEAN, T_T,          // bucket-end filter results, bucket bound
    T_SETTLED, T_ARCS, T_NLAB, T_BASE, T_FILL, T_FARCLEAN, T_UMAX,
    T_ROOT,
    T_SMIN0, T_SMIN1, T_SCL0, T_SCL1,   // round-level stop test, by round parity
    T_BAR, T_ABORT,
    T_WORDS_USED
};
static_assert(T_WORDS_USED <= TEAM_WORDS, "team words");

// Polls of a barrier counter before the team gives up (seconds; a barrier
// normally completes within microseconds).
constexpr int TEAM_SPIN_LIMIT = 1 << 22;

template <typename K, int WG>
struct TeamLds {
    Expand<K, WG> X;
    unsigned long long red64[WG / 64];
    int ok;
    uint32_t dhmin;           // smallest distance of the root to a prefix hub
};

template <typename T>
__device__ __forceinline__ T twl(long long* tw, int i) {
    return (T)__hip_atomic_load(&tw[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void tws(long long* tw, int i, long long v) {
    __hip_atomic_store(&tw[i], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier of the W workgroups of a team. Everything the workgroups of a team
// share (keys, flags, list entries, team words) is accessed with
// device-coherent atomics, so a barrier needs no cache write-back or
// invalidation: every wave waits until its own memory operations have
// completed, then the first thread of the workgroup adds one arrival to the
// team counter and waits until it reaches nb * W, nb being the number of team
// barriers so far (the same in every workgroup of the team, which all run the
// same sequence of barriers). Returns false when the team is aborted: a wait
// that exceeded TEAM_SPIN_LIMIT polls, here or in another workgroup of the
// team.
template <typename L>
__device__ __forceinline__ bool team_sync(long long* tw, int W, unsigned long long& nb, L& S, int32_t* err) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    nb++;
    if (threadIdx.x == 0) {
        unsigned long long* bar = (unsigned long long*)&tw[T_BAR];
        int ok = 1;
        atomicAdd(bar, 1ull);
        const unsigned long long target = nb * (unsigned long long)W;
        for (int spins = 0;
             __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; spins++) {
            if (spins > TEAM_SPIN_LIMIT || twl<long long>(tw, T_ABORT) != 0) {
                ok = 0;
                tws(tw, T_ABORT, 1);
                atomicOr(err, ERR_BIT_TEAM);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        S.ok = ok;
    }
    __syncthreads();
    return S.ok != 0;
}

// The dispatcher hands the workgroups of a launch to the eight XCDs in turn
// (workgroup b to XCD b % 8), each XCD with its own L2. With xcd_map set, a
// launch of G workgroups (G a multiple of 8) numbers them XCD by XCD, so
// that a team of consecutive numbers shares one L2 (W dividing G / 8) or
// two.
__device__ __forceinline__ int team_index(int b, int G, int xcd_map) {
    return xcd_map && G % 8 == 0 ? (b % 8) * (G / 8) + b / 8 : b;
}

template <typename K, int WG, bool PRUNE>
__global__ __launch_bounds__(WG) void k_tree_team(TreeParams p, int W, long long* tstate, int32_t* far2_all) {
    constexpr int SC = __HIP_MEMORY_SCOPE_AGENT;
    typedef unsigned long long ull;
    __shared__ TeamLds<K, WG> S;
    extern __shared__ uint32_t dh[];
    const int tid = threadIdx.x;
    const int lb = team_index(blockIdx.x, gridDim.x, p.xcd_map);
    const int team = lb / W, trank = lb % W;
    const int64_t tgtid = (int64_t)trank * WG + tid, tthreads = (int64_t)W * WG;
    const bool leader = trank == 0 && tid == 0;
    long long* tw = tstate + (int64_t)team * TEAM_WORDS;
    K* key = (K*)p.s.key + team * p.s.stride;
    uint32_t* flags = p.s.flags + team * p.s.fstride;
    int32_t* touched = p.s.touched + team * p.s.stride;
    int32_t* lists = p.s.lists + team * 3 * p.s.stride;
    int32_t* far = lists + 2 * p.s.stride;
    int32_t* far2 = far2_all + team * p.s.stride;
    const int32_t n = p.g.n;
    const int64_t delta = p.delta;
    const long long INF = 0x7FFFFFFFFFFFFFFFll;
    ull nb = 0;
    uint64_t t_start = 0;

    for (;;) {
        // ---- the team leader takes the next root and sets up its tree
        if (leader) {
            int32_t r = -1;
            if (ld<SC>(p.stop) == 0) {
                int32_t c = atomicAdd(p.next_root, 1);
                if (c < p.nroots) r = p.roots ? p.roots[c] : p.root_base + c;
            }
            if (r >= 0) {
                for (int i = 0; i < T_ROOT; i++) tws(tw, i, 0);
                tws(tw, T_CNT0, 1);
                tws(tw, T_TOUCHED, 1);
                tws(tw, T_MIN, INF);
                tws(tw, T_T, delta);
                tws(tw, T_SMIN0, INF); tws(tw, T_SMIN1, INF);
                tws(tw, T_SCL0, 0); tws(tw, T_SCL1, 0);
                st<SC>(&key[r], pack<K>(0, 1));
                lput<SC>(&touched[0], r);
                lput<SC>(&lists[0], r);
                aor<SC>(&flags[r >> 3], 1u << fshift(r));
                t_start = __builtin_amdgcn_s_memrealtime();
            }
            tws(tw, T_ROOT, r);
        }
        if (!team_sync(tw, W, nb, S, p.err)) return;
        const int32_t h = twl<int32_t>(tw, T_ROOT);
        if (h < 0) return;
        const bool prune = PRUNE && h >= p.pbound;
        if (prune) {
            for (int x = tid; x < p.pbound; x += WG) dh[x] = 0xFFFFFFFFu;
            if (tid == 0) S.dhmin = 0xFFFFFFFFu;
            __syncthreads();
            const uint32_t px = (uint32_t)p.partner;
            const int32_t hg = h ^ (int32_t)px;      // whose prefix labels give d(h, x)
            for (int64_t i = p.poff[hg] + tid; i < p.poff[hg + 1]; i += WG) {
                const uint64_t lx = p.plab[i];
                const uint32_t x = p.dmaj ? (uint32_t)lx : (uint32_t)(lx >> 32), y = x ^ px;
                const uint32_t dd = p.dmaj ? (uint32_t)(lx >> 32) : (uint32_t)lx;
                if (x < (uint32_t)p.pbound && y < (uint32_t)p.pbound) {
                    dh[y] = dd;
                    atomicMin(&S.dhmin, dd);
                }
            }
            __syncthreads();
        }
        int it = 0;
        bool early = false;
        uint64_t arcs = 0;
        for (;;) {
            // words of the next round's stop test start clean
            if (leader) { tws(tw, T_SMIN0 + ((it + 1) & 1), INF); tws(tw, T_SCL0 + ((it + 1) & 1), 0); }
            const int64_t T = twl<int64_t>(tw, T_T);
            const int32_t ncur = min(twl<int32_t>(tw, T_CNT0 + it % 3), n);
            const uint32_t curbit = 1u << (it & 1), nextbit = 1u << ((it + 1) & 1);
            int32_t* cur = lists + (int64_t)(it & 1) * p.s.stride;
            int32_t* next = lists + (int64_t)((it + 1) & 1) * p.s.stride;
            if (ncur > 0) {
                // ---- early termination between rounds (the test of the
                //      batched form, over the whole team)
                if (p.early_term && twl<long long>(tw, T_FARCLEAN) == 0) {
                    ull mn = ~0ull, cl = 0;
                    for (int64_t i = tgtid; i < ncur; i += tthreads) {
                        const K kv = ld<SC>(&key[lget<SC>(&cur[i], n)]);
                        const ull d = (ull)(kv >> 1);
                        mn = d < mn ? d : mn;
                        cl |= (ull)(kv & 1);
                    }
                    mn = block_reduce<WG>(mn, S.red64, ~0ull, [](ull a, ull b) { return a < b ? a : b; });
                    cl = block_reduce<WG>(cl, S.red64, 0ull, [](ull a, ull b) { return a | b; });
                    if (tid == 0) {
                        if (mn != ~0ull) atomicMin((ull*)&tw[T_SMIN0 + (it & 1)], mn);
                        if (cl) atomicOr((ull*)&tw[T_SCL0 + (it & 1)], cl);
                    }
                    if (!team_sync(tw, W, nb, S, p.err)) return;
                    const ull smin = twl<ull>(tw, T_SMIN0 + (it & 1));
                    const ull lb = smin < (ull)T ? smin : (ull)T;
                    if (twl<ull>(tw, T_SCL0 + (it & 1)) == 0 && lb > twl<ull>(tw, T_UMAX)) {
                        const int32_t nfar = min(twl<int32_t>(tw, T_FAR), n);
                        for (int64_t i = tgtid; i < ncur; i += tthreads) {
                            const int32_t v = lget<SC>(&cur[i], n);
                            aand<SC>(&flags[v >> 3], ~(curbit << fshift(v)));
                        }
                        for (int64_t i = tgtid; i < nfar; i += tthreads) {
                            const int32_t v = lget<SC>(&far[i], n);
                            aand<SC>(&flags[v >> 3], ~(FAR_BIT << fshift(v)));
                        }
                        early = true;
                        break;
                    }
                }
                // the near list split evenly over the team's workgroups (a
                // small frontier would otherwise leave most of them idle)
                const int32_t chunk = min(WG, (ncur + W - 1) / W);
                for (int32_t base = trank * chunk; base < ncur; base += W * chunk)
                    relax_block<K, WG, SC>(p.g, key, flags, cur, base, min(chunk, ncur - base), curbit,
                                           nextbit, h, T, touched, next, far, (ull*)&tw[T_TOUCHED],
                                           (ull*)&tw[T_CNT0 + (it + 1) % 3], (ull*)&tw[T_FAR],
                                           (ull*)&tw[T_FARCLEAN], (ull*)&tw[T_UMAX], p.poff, p.plab,
                                           (uint32_t)p.pbound, prune ? dh : nullptr, S.X, arcs, false,
                                           p.pmin, S.dhmin, p.dmaj != 0);
                if (leader) {
                    tws(tw, T_CNT0 + (it + 2) % 3, 0);
                    tws(tw, T_SETTLED, twl<long long>(tw, T_SETTLED) + ncur);
                }
                if (!team_sync(tw, W, nb, S, p.err)) return;
                it++;
                continue;
            }
            // ---- bucket done: filter far into far2 (drop settled entries)
            const int32_t nfar = min(twl<int32_t>(tw, T_FAR), n);
            ull mymin = ~0ull, myclean = 0;
            for (int64_t i = tgtid; i < nfar; i += tthreads) {
                const int32_t v = lget<SC>(&far[i], n);
                aand<SC>(&flags[v >> 3], ~(FAR_BIT << fshift(v)));
                const K kv = ld<SC>(&key[v]);
                const bool keep = (int64_t)(kv >> 1) >= T;
                if (keep) {
                    mymin = min(mymin, (ull)(kv >> 1));
                    myclean += (ull)(kv & 1);
                }
                const int64_t q = wave_append(keep, (ull*)&tw[T_FAR2]);
                if (keep && q < n) lput<SC>(&far2[q], v);
            }
            mymin = block_reduce<WG>(mymin, S.red64, ~0ull, [](ull a, ull b) { return a < b ? a : b; });
            myclean = block_reduce<WG>(myclean, S.red64, 0ull, [](ull a, ull b) { return a + b; });
            if (tid == 0) {
                if (mymin != ~0ull) atomicMin((ull*)&tw[T_MIN], mymin);
                if (myclean) atomicAdd((ull*)&tw[T_CLEAN], myclean);
            }
            if (!team_sync(tw, W, nb, S, p.err)) return;
            const int32_t nkeep = min(twl<int32_t>(tw, T_FAR2), n);
            const bool done = nkeep == 0 || (p.early_term && twl<long long>(tw, T_CLEAN) == 0);
            const int64_t Tn = done ? 0 : (twl<int64_t>(tw, T_MIN) / delta + 1) * delta;
            if (!team_sync(tw, W, nb, S, p.err)) return;   // everyone has read the results
            if (done) { early = nkeep > 0; break; }
            if (leader) {
                tws(tw, T_FAR, 0); tws(tw, T_FAR2, 0); tws(tw, T_CLEAN, 0); tws(tw, T_MIN, INF);
                tws(tw, T_T, Tn); tws(tw, T_FARCLEAN, 0);
            }
            if (!team_sync(tw, W, nb, S, p.err)) return;
            // ---- next bucket: far2 -> near list of this round, or back to far
            int32_t* ncurl = lists + (int64_t)(it & 1) * p.s.stride;
            for (int64_t i = tgtid; i < nkeep; i += tthreads) {
                const int32_t v = lget<SC>(&far2[i], n);
                const K kv = ld<SC>(&key[v]);
                const bool tonear = (int64_t)(kv >> 1) < Tn;
                int64_t q = wave_append(tonear, (ull*)&tw[T_CNT0 + it % 3]);
                if (tonear && q < n) { lput<SC>(&ncurl[q], v); aor<SC>(&flags[v >> 3], curbit << fshift(v)); }
                q = wave_append(!tonear, (ull*)&tw[T_FAR]);
                if (!tonear && q < n) { lput<SC>(&far[q], v); aor<SC>(&flags[v >> 3], FAR_BIT << fshift(v)); }
                (void)wave_append(!tonear && (kv & 1), (ull*)&tw[T_FARCLEAN]);
            }
            if (!team_sync(tw, W, nb, S, p.err)) return;
        }
        // ---- emit the labels of clean vertices, reset the slot
        const int64_t nt = min(twl<int64_t>(tw, T_TOUCHED), (int64_t)n);
        ull mycnt = 0;
        for (int64_t i = tgtid; i < nt; i += tthreads) mycnt += (ull)(ld<SC>(&key[lget<SC>(&touched[i], n)]) & 1);
        mycnt = block_reduce<WG>(mycnt, S.red64, 0ull, [](ull a, ull b) { return a + b; });
        if (tid == 0) {
            atomicAdd((ull*)&tw[T_NLAB], mycnt);
            atomicAdd((ull*)&tw[T_ARCS], (ull)arcs);
        }
        if (!team_sync(tw, W, nb, S, p.err)) return;
        if (leader) {
            const ull nl = twl<ull>(tw, T_NLAB);
            const ull b = atomicAdd(p.pool.cursor, nl);
            if (b + nl > p.pool.cap) {
                tws(tw, T_BASE, -1);
                atomicOr(p.err, ERR_BIT_POOL);
                atomicExch(p.stop, 1);
                atomicMin(p.pool.fail_base, b);
                p.failed[atomicAdd(p.nfailed, 1)] = h;
            } else {
                tws(tw, T_BASE, (long long)b);
            }
        }
        if (!team_sync(tw, W, nb, S, p.err)) return;
        const long long pb = twl<long long>(tw, T_BASE);
        const long long nl = twl<long long>(tw, T_NLAB);
        bool ovf = false;
        for (int64_t i = tgtid; i < nt; i += tthreads) {
            const int32_t v = lget<SC>(&touched[i], n);
            const K kv = ld<SC>(&key[v]);
            const bool lab = (kv & 1) != 0;
            const uint64_t d = (uint64_t)(kv >> 1);
            st<SC>(&key[v], KeyTraits<K>::INF);
            const int64_t q = wave_append(lab, (ull*)&tw[T_FILL]);
            if (lab && pb >= 0 && q < nl) {
                ovf |= d > 0x7FFFFFFEull;
                p.pool.v[pb + q] = v;
                p.pool.hub[pb + q] = h;
                p.pool.dist[pb + q] = (int32_t)d;
            }
        }
        if (ovf) atomicOr(p.err, ERR_BIT_OVERFLOW);
        if (p.stats && leader) {
            int64_t* s = p.stats + (int64_t)h * STAT_COLS;
            s[0] = twl<long long>(tw, T_SETTLED); s[1] = twl<long long>(tw, T_ARCS);
            s[2] = twl<long long>(tw, T_NLAB); s[3] = early ? 1 : 0;
            s[4] = it; s[5] = (int64_t)(__builtin_amdgcn_s_memrealtime() - t_start);
        }
        // the tree is done in every workgroup before the leader resets the words
        if (!team_sync(tw, W, nb, S, p.err)) return;
    }
}

// ---------------------------------------------------------------- small
// One wave per tree, its whole state in LDS: a hash table of at most SCAP
// vertices (vertex id, packed key, list flags) and the near and far lists as
// table slots. Most trees of the main phase settle a few vertices, and a tree
// then needs a few kilobytes instead of an n-sized slot, so that 32 trees fit
// on a compute unit and their key accesses stay on chip. The root's
// distances to the prefix hubs (rank-prefix pruning) sit in a second small
// hash table. A tree that needs more room than either table holds is given
// up without emitting anything and its root appended to an overflow list,
// which the host runs with the batched kernel afterwards (trees are
// independent, Section 4.2). Rounds, buckets, early termination and label
// emission follow the batched form step for step, with table slots in place
// of vertex ids.
constexpr int SCAP = 128;            // vertices a tree may reach in LDS
constexpr int SPH = 512;             // prefix-label table of a root (at most SPH / 2 labels)
constexpr int32_t S_EMPTY = -1;

template <typename K>
struct SmallLds {
    int32_t ids[SCAP];
    K keys[SCAP];
    uint32_t flg[SCAP];              // bit 0/1: in near list 0/1, bit 2: in far list
    uint16_t lst[3][SCAP];           // near list 0, near list 1, far list (slots)
    int32_t phub[SPH];               // root's prefix labels: hub (S_EMPTY: free)
    uint32_t pdist[SPH];             //                       distance
    int64_t beg[64];                 // relaxation of up to 64 list entries
    uint32_t off[64];
    K ekey[64];
    int32_t esl[64];
    uint32_t wsum[1];
    unsigned long long red64[1];
    int32_t red32[1];
    int32_t ncur, cnt_next, cnt_far, nkeep, far_clean, nused, bad, fill;
    int32_t root, bnext, bend;
    uint32_t dhmin;                  // smallest distance of the root to a prefix hub
    unsigned long long umax;
    long long pool_base;
};

__device__ __forceinline__ uint32_t shash(uint32_t x, uint32_t cap) {
    return (x * 2654435761u) >> (32 - __builtin_ctz(cap));
}

// slot of u in the table, or -1
template <typename K>
__device__ __forceinline__ int slookup(SmallLds<K>& S, int32_t u) {
    uint32_t s = shash((uint32_t)u, SCAP);
    for (int i = 0; i < SCAP; i++, s = (s + 1) & (SCAP - 1)) {
        const int32_t x = __hip_atomic_load(&S.ids[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (x == u) return (int)s;
        if (x == S_EMPTY) return -1;
    }
    return -1;
}

// slot of u, inserted if absent (its key is then INF); -1 when the table is full
template <typename K>
__device__ __forceinline__ int sinsert(SmallLds<K>& S, int32_t u) {
    uint32_t s = shash((uint32_t)u, SCAP);
    for (int i = 0; i < SCAP; i++, s = (s + 1) & (SCAP - 1)) {
        const int32_t x = atomicCAS(&S.ids[s], S_EMPTY, u);
        if (x == S_EMPTY) { atomicAdd(&S.nused, 1); return (int)s; }
        if (x == u) return (int)s;
    }
    return -1;
}

// the root's distance to prefix hub x (0xFFFFFFFF: none)
template <typename K>
__device__ __forceinline__ uint32_t sprefix(const SmallLds<K>& S, uint32_t x) {
    uint32_t s = shash(x, SPH);
    for (int i = 0; i < SPH; i++, s = (s + 1) & (SPH - 1)) {
        const int32_t y = S.phub[s];
        if (y == (int32_t)x) return S.pdist[s];
        if (y == S_EMPTY) return 0xFFFFFFFFu;
    }
    return 0xFFFFFFFFu;
}

// One round over the list entries cur[base .. base + nv), nv <= 64: the
// batched form's relaxation with table slots. An arc to a vertex that is not
// in the table (and not pruned) inserts it; a full table marks the tree bad.
template <typename K, bool PRUNE>
__device__ __forceinline__ void srelax(const TreeParams& p, SmallLds<K>& S, const uint16_t* cur, int32_t base,
                                       int32_t nv, uint32_t curbit, uint32_t nextbit, int32_t h, int64_t T,
                                       uint16_t* next, uint16_t* far, uint64_t& arcs) {
    constexpr int SCW = __HIP_MEMORY_SCOPE_WORKGROUP;
    const int lane = threadIdx.x;
    uint32_t deg = 0;
    if (lane < nv) {
        const int32_t s = cur[base + lane];
        atomicAnd(&S.flg[s], ~curbit);
        const int32_t v = S.ids[s];
        const int64_t b = p.g.row[v];
        deg = (uint32_t)(p.g.row[v + 1] - b);
        S.beg[lane] = b;
        S.ekey[lane] = S.keys[s];
        S.esl[lane] = s;
    }
    uint32_t inc = deg;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    const uint32_t total = __shfl(inc, 63);
    S.off[lane] = inc - deg;
    __syncthreads();
    arcs += total;
    unsigned long long my_umax = 0;
    for (uint32_t e0 = lane; e0 < total; e0 += 64 * RELAX_ILP) {
        int own[RELAX_ILP];
        uint64_t a[RELAX_ILP];
#pragma unroll
        for (int j = 0; j < RELAX_ILP; j++) {
            const uint32_t e = e0 + j * 64;
            int lo = 0, hi = nv - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (S.off[mid] <= e) lo = mid; else hi = mid - 1;
            }
            own[j] = lo;
            a[j] = e < total ? p.g.arc[S.beg[lo] + (e - S.off[lo])] : 0;
        }
#pragma unroll
        for (int j = 0; j < RELAX_ILP; j++) {
            const uint32_t e = e0 + j * 64;
            const bool valid = e < total;
            const int32_t u = (int32_t)(a[j] >> 32);
            const K kv = S.ekey[own[j]];
            const uint64_t nd = (uint64_t)(kv >> 1) + (uint32_t)a[j];
            const K nk = pack<K>(nd, (uint32_t)(kv & 1) & (uint32_t)(u > h));
            int su = valid ? slookup(S, u) : -1;
            const K seen = su >= 0 ? __hip_atomic_load(&S.keys[su], __ATOMIC_RELAXED, SCW) : KeyTraits<K>::INF;
            bool cand = valid && nk < seen;
            if (PRUNE && cand && (!p.pmin || (uint64_t)S.dhmin + p.pmin[u] <= nd)) {
                // rank-prefix pruning (Section 4.3), as in the other forms,
                // with the root's prefix distances from the LDS table (and
                // the same bound)
                const int64_t lb = p.poff[u], le = p.poff[u + 1];
                for (int64_t i = lb; i < le && cand; i += 4) {
                    uint64_t lx[4];
#pragma unroll
                    for (int z = 0; z < 4; z++) lx[z] = i + z < le ? p.plab[i + z] : ~0ull;
#pragma unroll
                    for (int z = 0; z < 4; z++) {
                        const uint32_t x = (uint32_t)(lx[z] >> 32);
                        if (x >= (uint32_t)p.pbound) continue;
                        const uint32_t ax = sprefix(S, x);
                        if (ax != 0xFFFFFFFFu && (uint64_t)ax + (uint32_t)lx[z] <= nd) cand = false;
                    }
                }
            }
            if (cand && su < 0) {
                su = sinsert(S, u);
                if (su < 0) { S.bad = 1; cand = false; }
            }
            K old = seen;
            if (cand) old = atomicMin(&S.keys[su], nk);
            const bool imp = cand && nk < old;
            const bool tonear = imp && (int64_t)nd < T;
            bool pnear = false, pfar = false;
            if (imp) {
                if (nk & 1) my_umax = my_umax > nd ? my_umax : nd;
                const uint32_t bit = tonear ? nextbit : FAR_BIT;
                const uint32_t o = atomicOr(&S.flg[su], bit);
                const bool fresh = (o & bit) == 0;
                pnear = fresh && tonear;
                pfar = fresh && !tonear;
            }
            int64_t q = wave_append(pnear, &S.cnt_next);
            if (pnear && q < SCAP) next[q] = (uint16_t)su;
            q = wave_append(pfar, &S.cnt_far);
            if (pfar && q < SCAP) far[q] = (uint16_t)su;
            (void)wave_append(pfar && (nk & 1), &S.far_clean);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(my_umax, d);
        my_umax = o > my_umax ? o : my_umax;
    }
    if (lane == 0 && my_umax > S.umax) S.umax = my_umax;
    __syncthreads();
}

template <typename K, bool PRUNE>
__global__ __launch_bounds__(64) void k_tree_small(TreeParams p, int32_t* ovf, int32_t* novf) {
    __shared__ SmallLds<K> S;
    const int lane = threadIdx.x;
    const int64_t delta = p.delta;
    for (int i = lane; i < SCAP; i += 64) {
        S.ids[i] = S_EMPTY;
        S.keys[i] = KeyTraits<K>::INF;
        S.flg[i] = 0;
    }
    for (int i = lane; i < SPH; i += 64) S.phub[i] = S_EMPTY;
    if (lane == 0) { S.bnext = 0; S.bend = 0; }
    __syncthreads();
    for (;;) {
        if (lane == 0) {
            // roots are taken pop_batch at a time, as in the batched form
            int32_t r = -1;
            const bool stopped = __hip_atomic_load(p.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            if (stopped) {
                for (int32_t c = S.bnext; c < S.bend; c++)
                    p.failed[atomicAdd(p.nfailed, 1)] = p.roots ? p.roots[c] : p.root_base + c;
                S.bnext = S.bend;
            } else if (S.bnext >= S.bend) {
                const int32_t c = atomicAdd(p.next_root, p.pop_batch);
                S.bnext = c;
                S.bend = c < p.nroots ? min(p.nroots, c + p.pop_batch) : c;
            }
            if (S.bnext < S.bend) {
                r = p.roots ? p.roots[S.bnext] : p.root_base + S.bnext;
                S.bnext++;
            }
            S.root = r;
            S.ncur = 1; S.cnt_next = 0; S.cnt_far = 0; S.far_clean = 0; S.umax = 0; S.bad = 0; S.nused = 0;
            S.fill = 0;
            S.dhmin = 0xFFFFFFFFu;
        }
        __syncthreads();
        const int32_t h = S.root;
        if (h < 0) break;
        const bool prune = PRUNE && h >= p.pbound;
        if (prune) {
            // the root's prefix labels (a directed build reads the partner's)
            const uint32_t px = (uint32_t)p.partner;
            const int32_t hg = h ^ (int32_t)px;
            const int64_t lb = p.poff[hg], le = p.poff[hg + 1];
            if (le - lb > SPH / 2) {
                if (lane == 0) S.bad = 1;       // (the table stays at most half full)
            } else {
                for (int64_t i = lb + lane; i < le; i += 64) {
                    const uint64_t lx = p.plab[i];
                    const uint32_t x = (uint32_t)(lx >> 32), y = x ^ px;
                    if (x < (uint32_t)p.pbound && y < (uint32_t)p.pbound) {
                        uint32_t s = shash(y, SPH);
                        while (atomicCAS(&S.phub[s], S_EMPTY, (int32_t)y) != S_EMPTY) s = (s + 1) & (SPH - 1);
                        atomicMin(&S.dhmin, (uint32_t)lx);
                        S.pdist[s] = (uint32_t)lx;
                    }
                }
            }
        }
        if (lane == 0) {
            const int s = sinsert(S, h);
            S.keys[s] = pack<K>(0, 1);
            S.flg[s] = 1u;
            S.lst[0][0] = (uint16_t)s;
        }
        __syncthreads();
        int64_t T = delta;
        int it = 0;
        uint64_t arcs = 0, settled = 0;
        const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
        bool early = false;
        for (;;) {
            if (S.bad) break;
            bool stopped = false;
            for (;;) {
                const int32_t ncur = S.ncur;
                const uint32_t curbit = 1u << (it & 1), nextbit = 1u << ((it + 1) & 1);
                const uint16_t* cur = S.lst[it & 1];
                uint16_t* next = S.lst[(it + 1) & 1];
                if (p.early_term && it > 0 && S.far_clean == 0) {
                    // the batched form's stop test over the current list
                    unsigned long long mn = ~0ull;
                    int32_t cl = 0;
                    for (int32_t i = lane; i < ncur; i += 64) {
                        const K kv = S.keys[cur[i]];
                        mn = min(mn, (unsigned long long)(kv >> 1));
                        cl |= (int32_t)(kv & 1);
                    }
#pragma unroll
                    for (int d = 32; d >= 1; d >>= 1) {
                        const unsigned long long o = __shfl_xor(mn, d);
                        mn = o < mn ? o : mn;
                        cl |= __shfl_xor(cl, d);
                    }
                    const unsigned long long lbd = mn < (unsigned long long)T ? mn : (unsigned long long)T;
                    if (cl == 0 && lbd > S.umax) {
                        for (int32_t i = lane; i < ncur; i += 64) atomicAnd(&S.flg[cur[i]], ~curbit);
                        for (int32_t i = lane; i < S.cnt_far; i += 64) atomicAnd(&S.flg[S.lst[2][i]], ~FAR_BIT);
                        early = ncur > 0 || S.cnt_far > 0;
                        stopped = true;
                        __syncthreads();
                        break;
                    }
                }
                settled += ncur;
                for (int32_t base = 0; base < ncur; base += 64)
                    srelax<K, PRUNE>(p, S, cur, base, min(64, ncur - base), curbit, nextbit, h, T, next, S.lst[2],
                                     arcs);
                it++;
                if (lane == 0) { S.ncur = min(S.cnt_next, SCAP); S.cnt_next = 0; }
                __syncthreads();
                if (S.ncur == 0 || S.bad) break;
            }
            if (stopped || S.bad) break;
            // bucket done: drop settled far entries, then move the next bucket in
            const int32_t nfar = min(S.cnt_far, SCAP);
            if (lane == 0) S.nkeep = 0;
            __syncthreads();
            unsigned long long mymin = ~0ull;
            int32_t myclean = 0;
            for (int32_t base = 0; base < nfar; base += 64) {
                const int32_t i = base + lane;
                bool keep = false;
                int32_t s = 0;
                K kv = 0;
                if (i < nfar) {
                    s = S.lst[2][i];
                    atomicAnd(&S.flg[s], ~FAR_BIT);
                    kv = S.keys[s];
                    keep = (int64_t)(kv >> 1) >= T;
                }
                __syncthreads();
                const int64_t q = wave_append(keep, &S.nkeep);
                if (keep) {
                    S.lst[2][q] = (uint16_t)s;
                    mymin = min(mymin, (unsigned long long)(kv >> 1));
                    myclean += (int32_t)(kv & 1);
                }
                __syncthreads();
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                const unsigned long long o = __shfl_xor(mymin, d);
                mymin = o < mymin ? o : mymin;
                myclean += __shfl_xor(myclean, d);
            }
            const int32_t nk2 = S.nkeep;
            if (nk2 == 0 || (p.early_term && myclean == 0)) { early = nk2 > 0; break; }
            T = ((int64_t)mymin / delta + 1) * delta;
            uint16_t* curl = S.lst[it & 1];
            const uint32_t curbit = 1u << (it & 1);
            if (lane == 0) { S.ncur = 0; S.cnt_far = 0; S.far_clean = 0; }
            __syncthreads();
            for (int32_t base = 0; base < nk2; base += 64) {
                const int32_t i = base + lane;
                int32_t s = 0;
                bool tonear = false, tofar = false, fclean = false;
                if (i < nk2) {
                    s = S.lst[2][i];
                    const K kv = S.keys[s];
                    tonear = (int64_t)(kv >> 1) < T;
                    tofar = !tonear;
                    fclean = tofar && (kv & 1);
                }
                __syncthreads();
                int64_t q = wave_append(tonear, &S.ncur);
                if (tonear) { curl[q] = (uint16_t)s; atomicOr(&S.flg[s], curbit); }
                q = wave_append(tofar, &S.cnt_far);
                if (tofar) { S.lst[2][q] = (uint16_t)s; atomicOr(&S.flg[s], FAR_BIT); }
                (void)wave_append(fclean, &S.far_clean);
                __syncthreads();
            }
        }
        if (S.bad) {
            // the tree outgrew LDS: the batched kernel grows it later
            if (lane == 0) ovf[atomicAdd(novf, 1)] = h;
        } else {
            // emit the labels of clean slots
            int32_t mycnt = 0;
            for (int i = lane; i < SCAP; i += 64)
                mycnt += (S.ids[i] != S_EMPTY && (S.keys[i] & 1)) ? 1 : 0;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) mycnt += __shfl_xor(mycnt, d);
            const int32_t nl = mycnt;
            if (lane == 0) {
                const unsigned long long b = atomicAdd(p.pool.cursor, (unsigned long long)nl);
                if (b + (unsigned long long)nl > p.pool.cap) {
                    S.pool_base = -1;
                    atomicOr(p.err, ERR_BIT_POOL);
                    atomicExch(p.stop, 1);
                    atomicMin(p.pool.fail_base, b);
                    p.failed[atomicAdd(p.nfailed, 1)] = h;
                } else {
                    S.pool_base = (long long)b;
                }
            }
            __syncthreads();
            const long long pb = S.pool_base;
            bool ovfd = false;
            for (int i = lane; i < SCAP; i += 64) {
                const bool lab = S.ids[i] != S_EMPTY && (S.keys[i] & 1);
                const uint64_t d = (uint64_t)(S.keys[i] >> 1);
                const int64_t q = wave_append(lab, &S.fill);
                if (lab && pb >= 0) {
                    ovfd |= d > 0x7FFFFFFEull;
                    p.pool.v[pb + q] = S.ids[i];
                    p.pool.hub[pb + q] = h;
                    p.pool.dist[pb + q] = (int32_t)d;
                }
            }
            if (ovfd) atomicOr(p.err, ERR_BIT_OVERFLOW);
            if (p.stats && lane == 0) {
                int64_t* s = p.stats + (int64_t)h * STAT_COLS;
                s[0] = (int64_t)settled; s[1] = (int64_t)arcs; s[2] = nl; s[3] = early ? 1 : 0;
                s[4] = it; s[5] = (int64_t)(__builtin_amdgcn_s_memrealtime() - t_start);
            }
        }
        __syncthreads();
        // clear the tables for the next tree
        for (int i = lane; i < SCAP; i += 64) {
            S.ids[i] = S_EMPTY;
            S.keys[i] = KeyTraits<K>::INF;
            S.flg[i] = 0;
        }
        if (prune) for (int i = lane; i < SPH; i += 64) S.phub[i] = S_EMPTY;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- groups
// A team of W workgroups grows GT trees of consecutive roots together: the
// trees of a pruning level whose roots are close in rank reach largely the
// same vertices, at about the same distances. Their per-vertex state is kept
// vertex-major, key[v * GT + b] being tree b's key of v, so the GT keys of a
// vertex share one cache line (64-bit keys: 128 B), and one pass over a
// frontier vertex's arcs relaxes them for every tree that has the vertex
// pending. A random access to the key array then serves up to GT trees
// instead of one, and u's prefix labels, read by the pruning test, are read
// once for the trees that reach u in the same round.
//
// Per vertex v, besides the keys: mask[v] holds, per near list (bits 0-15
// list 0, 16-31 list 1, alternating by round as in the other forms), the
// trees that have v pending in it; fmask[v] holds the trees with v pending
// in the far list (bits 0-15), FAR_IN (v is in the far list) and TOUCHED (v
// is in the touched list). A vertex is listed once per list whatever the
// number of trees that have it pending. The bucket bound T is shared by the
// group (the next bucket is the one of the smallest pending distance of any
// tree); each tree keeps its own early-termination test and stops on its
// own. Labels and statistics are those of each tree alone.
constexpr int GT = GROUP_TREES;
static_assert(GT == 16, "the masks hold 16 trees per half word");
constexpr uint32_t GBITS = (1u << GT) - 1;
constexpr uint32_t GF_FAR_IN = 1u << 16, GF_TOUCHED = 1u << 17;
enum {
    GW_CNT0 = 0, GW_CNT1x, GW_CNT2x,      // near list counts, rotating by round % 3
    GW_FARL = 3, GW_FAR2L, GW_TOUCHEDL,   // far list, filtered far list, touched list
    GW_MINP = 6, GW_TB = 8,              // smallest kept far distance, bucket bound
    GW_NLABT = 10, GW_BASEP, GW_FILLP,    // labels of the group, pool base, fill
    GW_BAR = T_BAR, GW_ABORT = T_ABORT,  // barrier words (shared with team_sync)
    GW_ROOT = 32,                       // per-tree words from here, GT each:
    GW_UMAX = GW_ROOT + GT, GW_FCLEAN = GW_UMAX + GT, GW_SMIN = GW_FCLEAN + GT,  // SMIN: 2 parities
    GW_SCL = GW_SMIN + 2 * GT, GW_CLEAN = GW_SCL + 2 * GT, GW_SETTLEDB = GW_CLEAN + GT, GW_ARCSB = GW_SETTLEDB + GT,
    GW_NLABB = GW_ARCSB + GT, GW_KEPTM = GW_NLABB + GT,   // trees with far entries kept at the last filter
    GW_WORDS_USED = GW_KEPTM + 1
};
static_assert(GW_WORDS_USED <= GROUP_WORDS, "group words");
static_assert(T_BAR < GW_ROOT && T_ABORT < GW_ROOT && T_BAR > GW_FILLP, "group word layout");

template <typename K, int WG>
struct GroupLds {
    int64_t beg[WG];          // row start of the chunk's vertices
    int32_t vtx[WG];          // the vertices
    uint32_t msk[WG];         // trees to expand at each of them
    uint32_t off[WG];         // exclusive scan of deg * popcount(msk)
    uint32_t wsum[WG / 64];
    unsigned long long red64[WG / 64];
    int32_t hroot[GT];
    unsigned long long lmin[GT], lumax[GT];
    uint32_t lcl[GT], lfcl[GT];
    unsigned long long lset[GT], larc[GT], lnl[GT];
    uint32_t dhmin[GT];       // each tree's smallest distance to a prefix hub
    int ok;
};

// work items in flight per thread
constexpr int GROUP_ILP = 4;

// What the relaxation of a group's work items needs besides the launch
// parameters.
template <typename K>
struct GroupCtx {
    K* key;
    uint32_t* mask;
    uint32_t* fmask;
    int32_t* touched;
    int32_t* next;
    int32_t* far;
    long long* tw;
    int64_t T;
    uint32_t nsh;     // bit offset of the next round's half of mask
    uint32_t pb;      // pruning prefix (0: none)
    int32_t n;
    int it;
};

// Relax the work items [e_lo, e_hi) of a round, GROUP_ILP per thread at a
// time; decode(e, arc, tree, key of the expanded vertex) gives item e.
// Improved (vertex, tree) pairs go to the next near list or the far list,
// vertices reached for the first time by any tree to the touched list; the
// per-tree largest clean distance, clean far pushes and counts accumulate
// in LDS.
template <typename K, int WG, bool PRUNE, typename D>
__device__ __forceinline__ void group_relax(const TreeParams& p, const GroupCtx<K>& cx, GroupLds<K, WG>& S,
                                            const uint32_t* dh, uint32_t e_lo, uint32_t e_hi, D decode) {
    constexpr int SC = __HIP_MEMORY_SCOPE_AGENT;
    typedef unsigned long long ull;
    for (uint32_t e0 = e_lo + threadIdx.x; e0 < e_hi; e0 += WG * GROUP_ILP) {
        int tb[GROUP_ILP];
        uint64_t a[GROUP_ILP];
        K kv[GROUP_ILP], seen[GROUP_ILP];
#pragma unroll
        for (int j = 0; j < GROUP_ILP; j++) {
            const uint32_t e = e0 + j * WG;
            a[j] = 0; tb[j] = 0; kv[j] = 0;
            if (e < e_hi) decode(e, a[j], tb[j], kv[j]);
        }
        // (lanes of one arc read the key line of its target once)
#pragma unroll
        for (int j = 0; j < GROUP_ILP; j++) {
            const uint32_t e = e0 + j * WG;
            seen[j] = e < e_hi ? ld<SC>(&cx.key[(int64_t)(a[j] >> 32) * GT + tb[j]]) : (K)0;
        }
#pragma unroll
        for (int j = 0; j < GROUP_ILP; j++) {
            const uint32_t e = e0 + j * WG;
            const bool valid = e < e_hi;
            const int b = tb[j];
            const int32_t u = (int32_t)(a[j] >> 32);
            const int32_t h = S.hroot[b];
            const uint64_t nd = (uint64_t)(kv[j] >> 1) + (uint32_t)a[j];
            const K nk = pack<K>(nd, (uint32_t)(kv[j] & 1) & (uint32_t)(u > h));
            bool cand = valid && nk < seen[j];
            if (PRUNE && cand && cx.pb && (!p.pmin || (uint64_t)S.dhmin[b] + p.pmin[u] <= nd)) {
                // rank-prefix pruning (Section 4.3), as in the other forms,
                // with this tree's root distances (and the same bound)
                const uint32_t* dhb = dh + (int64_t)b * cx.pb;
                const int64_t lb = p.poff[u], le = p.poff[u + 1];
                for (int64_t i = lb; i < le && cand; i += 4) {
                    uint64_t lx[4];
#pragma unroll
                    for (int z = 0; z < 4; z++) lx[z] = i + z < le ? p.plab[i + z] : ~0ull;
#pragma unroll
                    for (int z = 0; z < 4; z++) {
                        const uint32_t x = p.dmaj ? (uint32_t)lx[z] : (uint32_t)(lx[z] >> 32);
                        const uint32_t dd = p.dmaj ? (uint32_t)(lx[z] >> 32) : (uint32_t)lx[z];
                        if (x >= cx.pb) continue;
                        const uint32_t ax = dhb[x];
                        if (ax != 0xFFFFFFFFu && (uint64_t)ax + dd <= nd) cand = false;
                    }
                    // groups ordered by distance: no later entry is closer
                    if (p.dmaj && (uint64_t)(uint32_t)(lx[3] >> 32) + S.dhmin[b] > nd) break;
                }
            }
            K old = seen[j];
            if (cand) old = amin<SC>(&cx.key[(int64_t)u * GT + b], nk);
            const bool imp = cand && nk < old;
            const bool tonear = imp && (int64_t)nd < cx.T;
            bool pnear = false, pfar = false, ptouch = false;
            if (imp) {
                if (nk & 1) {
                    atomicMax(&S.lumax[b], (ull)nd);
                    if (!tonear) atomicAdd(&S.lfcl[b], 1u);
                }
                if (tonear) {
                    const uint32_t bit = 1u << (cx.nsh + (uint32_t)b);
                    const uint32_t o = __hip_atomic_fetch_or(&cx.mask[u], bit, __ATOMIC_RELAXED, SC);
                    pnear = ((o >> cx.nsh) & GBITS) == 0;
                } else {
                    const uint32_t o = aor<SC>(&cx.fmask[u], (1u << b) | GF_FAR_IN);
                    pfar = (o & GF_FAR_IN) == 0;
                }
                if (old == KeyTraits<K>::INF) {
                    const uint32_t o = aor<SC>(&cx.fmask[u], GF_TOUCHED);
                    ptouch = (o & GF_TOUCHED) == 0;
                }
            }
            int64_t q = wave_append(ptouch, (ull*)&cx.tw[GW_TOUCHEDL]);
            if (ptouch && q < cx.n) lput<SC>(&cx.touched[q], u);
            q = wave_append(pnear, (ull*)&cx.tw[GW_CNT0 + (cx.it + 1) % 3]);
            if (pnear && q < cx.n) lput<SC>(&cx.next[q], u);
            q = wave_append(pfar, (ull*)&cx.tw[GW_FARL]);
            if (pfar && q < cx.n) lput<SC>(&cx.far[q], u);
        }
    }
}

__device__ __forceinline__ int nth_bit(uint32_t m, int j) {
    for (int k = 0; k < j; k++) m &= m - 1;
    return __ffs(m) - 1;
}

template <typename K, int WG, bool PRUNE>
__global__ __launch_bounds__(WG) void k_tree_group(TreeParams p, int W, long long* gstate, int32_t* far2_all,
                                                   uint32_t* gmask_all) {
    constexpr int SC = __HIP_MEMORY_SCOPE_AGENT;
    typedef unsigned long long ull;
    __shared__ GroupLds<K, WG> S;
    extern __shared__ uint32_t dh[];     // [GT][pbound]: each tree's root distances to the prefix hubs
    const int tid = threadIdx.x;
    const int lb = team_index(blockIdx.x, gridDim.x, p.xcd_map);
    const int team = lb / W, trank = lb % W;
    const int64_t tgtid = (int64_t)trank * WG + tid, tthreads = (int64_t)W * WG;
    const bool leader = trank == 0 && tid == 0;
    const int32_t n = p.g.n;
    long long* tw = gstate + (int64_t)team * GROUP_WORDS;
    K* key = (K*)p.s.key + (int64_t)team * p.s.stride * GT;
    uint32_t* mask = gmask_all + (int64_t)team * 2 * p.s.stride;
    uint32_t* fmask = mask + p.s.stride;
    int32_t* touched = p.s.touched + (int64_t)team * p.s.stride;
    int32_t* lists = p.s.lists + (int64_t)team * 3 * p.s.stride;
    int32_t* far = lists + 2 * p.s.stride;
    int32_t* far2 = far2_all + (int64_t)team * p.s.stride;
    const int64_t delta = p.delta;
    const long long INF = 0x7FFFFFFFFFFFFFFFll;
    const uint32_t pb = PRUNE ? (uint32_t)p.pbound : 0u;
    ull nb = 0;
    uint64_t t_start = 0;

    for (;;) {
        // ---- the leader takes the next GT roots and sets up their trees
        if (leader) {
            int32_t c = 0x7FFFFFFF;
            if (ld<SC>(p.stop) == 0) c = atomicAdd(p.next_root, GT);
            for (int i = 0; i < GW_ROOT; i++)
                if (i != GW_BAR && i != GW_ABORT) tws(tw, i, 0);
            for (int i = GW_ROOT; i < GW_WORDS_USED; i++) tws(tw, i, 0);
            tws(tw, GW_MINP, INF);
            tws(tw, GW_TB, delta);
            int32_t nr = 0;
            for (int b = 0; b < GT; b++) {
                tws(tw, GW_SMIN + b, INF);
                tws(tw, GW_SMIN + GT + b, INF);
                const int32_t q = c + b;
                const int32_t r = c < p.nroots && q < p.nroots ? (p.roots ? p.roots[q] : p.root_base + q) : -1;
                tws(tw, GW_ROOT + b, r);
                if (r >= 0 && r < n) {
                    st<SC>(&key[(int64_t)r * GT + b], pack<K>(0, 1));
                    __hip_atomic_fetch_or(&mask[r], 1u << b, __ATOMIC_RELAXED, SC);
                    aor<SC>(&fmask[r], GF_TOUCHED);
                    lput<SC>(&lists[nr], r);
                    lput<SC>(&touched[nr], r);
                    nr++;
                }
            }
            tws(tw, GW_CNT0, nr);
            tws(tw, GW_TOUCHEDL, nr);
            t_start = __builtin_amdgcn_s_memrealtime();
        }
        if (!team_sync(tw, W, nb, S, p.err)) return;
        uint32_t alive = 0;
        if (tid < GT) S.hroot[tid] = twl<int32_t>(tw, GW_ROOT + tid);
        __syncthreads();
        for (int b = 0; b < GT; b++)
            if (S.hroot[b] >= 0) alive |= 1u << b;
        if (!alive) return;
        const uint32_t valid = alive;
        if (PRUNE) {
            // each tree's distances to the prefix hubs, from its root's
            // prefix labels (a directed build reads the partner's)
            for (int64_t x = tid; x < (int64_t)GT * pb; x += WG) dh[x] = 0xFFFFFFFFu;
            if (tid < GT) S.dhmin[tid] = 0xFFFFFFFFu;
            __syncthreads();
            const uint32_t px = (uint32_t)p.partner;
            for (int b = 0; b < GT; b++) {
                const int32_t h = S.hroot[b];
                if (h < 0 || (uint32_t)h < pb) continue;
                const int32_t hg = h ^ (int32_t)px;
                for (int64_t i = p.poff[hg] + tid; i < p.poff[hg + 1]; i += WG) {
                    const uint64_t lx = p.plab[i];
                    const uint32_t x = p.dmaj ? (uint32_t)lx : (uint32_t)(lx >> 32), y = x ^ px;
                    const uint32_t dd = p.dmaj ? (uint32_t)(lx >> 32) : (uint32_t)lx;
                    if (x < pb && y < pb) {
                        dh[b * pb + y] = dd;
                        atomicMin(&S.dhmin[b], dd);
                    }
                }
            }
            __syncthreads();
        }
        uint32_t early_m = 0;
        int it = 0;
        for (;;) {
            const int par = it & 1;
            if (leader)
                for (int b = 0; b < GT; b++) {
                    tws(tw, GW_SMIN + (par ^ 1) * GT + b, INF);
                    tws(tw, GW_SCL + (par ^ 1) * GT + b, 0);
                }
            const int64_t T = twl<int64_t>(tw, GW_TB);
            const int32_t ncur = min(twl<int32_t>(tw, GW_CNT0 + it % 3), n);
            const uint32_t sh = 16u * (uint32_t)par, nsh = 16u * (uint32_t)(par ^ 1);
            int32_t* cur = lists + (int64_t)par * p.s.stride;
            int32_t* next = lists + (int64_t)(par ^ 1) * p.s.stride;
            if (ncur > 0) {
                // ---- per-tree early termination between rounds (the test of
                //      the other forms, for every tree with no clean far push)
                uint32_t cand_stop = 0;
                for (int b = 0; b < GT; b++)
                    if ((alive >> b & 1) && twl<long long>(tw, GW_FCLEAN + b) == 0) cand_stop |= 1u << b;
                if (p.early_term && cand_stop) {
                    if (tid < GT) { S.lmin[tid] = ~0ull; S.lcl[tid] = 0; }
                    __syncthreads();
                    for (int64_t i = tgtid; i < ncur; i += tthreads) {
                        const int32_t v = lget<SC>(&cur[i], n);
                        uint32_t m = (ld<SC>(&mask[v]) >> sh) & cand_stop;
                        while (m) {
                            const int b = __ffs(m) - 1;
                            m &= m - 1;
                            const K kv = ld<SC>(&key[(int64_t)v * GT + b]);
                            atomicMin(&S.lmin[b], (ull)(kv >> 1));
                            if (kv & 1) atomicOr(&S.lcl[b], 1u);
                        }
                    }
                    __syncthreads();
                    if (tid < GT && (cand_stop >> tid & 1)) {
                        if (S.lmin[tid] != ~0ull) atomicMin((ull*)&tw[GW_SMIN + par * GT + tid], S.lmin[tid]);
                        if (S.lcl[tid]) atomicOr((ull*)&tw[GW_SCL + par * GT + tid], 1ull);
                    }
                    if (!team_sync(tw, W, nb, S, p.err)) return;
                    uint32_t stopm = 0;
                    for (int b = 0; b < GT; b++) {
                        if (!(cand_stop >> b & 1)) continue;
                        const ull smin = twl<ull>(tw, GW_SMIN + par * GT + b);
                        const ull lb = smin < (ull)T ? smin : (ull)T;
                        if (twl<ull>(tw, GW_SCL + par * GT + b) == 0 && lb > twl<ull>(tw, GW_UMAX + b)) stopm |= 1u << b;
                    }
                    // a stopped tree keeps its pending bits; every later read of
                    // a mask is restricted to the trees still growing
                    // (a tree that stops here still had near entries, or far ones)
                    for (int b = 0; b < GT; b++)
                        if ((stopm >> b & 1) && twl<ull>(tw, GW_SMIN + par * GT + b) != (ull)INF) early_m |= 1u << b;
                    alive &= ~stopm;
                    if (!alive) break;
                }
                // ---- relax: the near list split evenly over the team's
                //      workgroups; each chunk's work items are (vertex, arc,
                //      tree) triples, trees fastest, so that consecutive lanes
                //      read the same arc and the same key line
                const GroupCtx<K> cx{key, mask, fmask, touched, next, far, tw, T, nsh, pb, n, it};
                const int32_t chunk = min(WG, (ncur + W - 1) / W);
                if (tid < GT) { S.lumax[tid] = 0; S.lfcl[tid] = 0; S.lset[tid] = 0; S.larc[tid] = 0; }
                __syncthreads();
                for (int32_t base = trank * chunk; base < ncur; base += W * chunk) {
                    const int32_t nv = min(chunk, ncur - base);
                    uint32_t items = 0;
                    if (tid < nv) {
                        const int32_t v = lget<SC>(&cur[base + tid], n);
                        const uint32_t old = __hip_atomic_fetch_and(&mask[v], ~(GBITS << sh), __ATOMIC_RELAXED, SC);
                        const uint32_t m = (old >> sh) & alive;
                        const int64_t b0 = p.g.row[v];
                        const uint32_t deg = (uint32_t)(p.g.row[v + 1] - b0);
                        for (uint32_t mm = m; mm;) {
                            const int b = __ffs(mm) - 1;
                            mm &= mm - 1;
                            atomicAdd(&S.lset[b], 1ull);
                            atomicAdd(&S.larc[b], (ull)deg);
                        }
                        S.beg[tid] = b0;
                        S.vtx[tid] = v;
                        S.msk[tid] = m;
                        items = deg * (uint32_t)__popc(m);
                    }
                    uint32_t total;
                    const uint32_t ex = block_scan<WG>(items, S.wsum, total);   // (synchronises the block)
                    S.off[tid] = ex;
                    __syncthreads();
                    group_relax<K, WG, PRUNE>(p, cx, S, dh, 0, total, [&](uint32_t e, uint64_t& a, int& b, K& kv) {
                        int lo = 0, hi = nv - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (S.off[mid] <= e) lo = mid; else hi = mid - 1;
                        }
                        const uint32_t m = S.msk[lo];
                        const uint32_t pc = (uint32_t)max(1, __popc(m));
                        const uint32_t r = e - S.off[lo];
                        b = nth_bit(m, (int)(r % pc));
                        a = p.g.arc[S.beg[lo] + r / pc];
                        kv = ld<SC>(&key[(int64_t)S.vtx[lo] * GT + b]);
                    });
                    __syncthreads();
                }
                if (tid < GT) {
                    if (S.lumax[tid]) atomicMax((ull*)&tw[GW_UMAX + tid], S.lumax[tid]);
                    if (S.lfcl[tid]) atomicAdd((ull*)&tw[GW_FCLEAN + tid], (ull)S.lfcl[tid]);
                    if (S.lset[tid]) atomicAdd((ull*)&tw[GW_SETTLEDB + tid], S.lset[tid]);
                    if (S.larc[tid]) atomicAdd((ull*)&tw[GW_ARCSB + tid], S.larc[tid]);
                }
                if (leader) tws(tw, GW_CNT0 + (it + 2) % 3, 0);
                if (!team_sync(tw, W, nb, S, p.err)) return;
                it++;
                continue;
            }
            // ---- bucket done: filter the far list into far2, keeping for each
            //      vertex the trees whose key is still at or beyond T
            const int32_t nfar = min(twl<int32_t>(tw, GW_FARL), n);
            if (tid < GT) S.lcl[tid] = 0;
            __syncthreads();
            ull mymin = ~0ull;
            for (int64_t i = tgtid; i < nfar; i += tthreads) {
                const int32_t v = lget<SC>(&far[i], n);
                const uint32_t fm = ld<SC>(&fmask[v]);
                uint32_t m = fm & GBITS & alive, keep = 0;
                while (m) {
                    const int b = __ffs(m) - 1;
                    m &= m - 1;
                    const K kv = ld<SC>(&key[(int64_t)v * GT + b]);
                    if ((int64_t)(kv >> 1) >= T) {
                        keep |= 1u << b;
                        mymin = min(mymin, (ull)(kv >> 1));
                        if (kv & 1) atomicAdd(&S.lcl[b], 1u);
                    }
                }
                // the far bits of trees no longer growing are dropped too
                aand<SC>(&fmask[v], ~((GBITS & ~keep) | GF_FAR_IN));
                if (keep) atomicOr((ull*)&tw[GW_KEPTM], (ull)keep);
                const int64_t q = wave_append(keep != 0, (ull*)&tw[GW_FAR2L]);
                if (keep && q < n) lput<SC>(&far2[q], v);
            }
            mymin = block_reduce<WG>(mymin, S.red64, ~0ull, [](ull x, ull y) { return x < y ? x : y; });
            __syncthreads();
            if (tid == 0 && mymin != ~0ull) atomicMin((ull*)&tw[GW_MINP], mymin);
            if (tid < GT && S.lcl[tid]) atomicAdd((ull*)&tw[GW_CLEAN + tid], (ull)S.lcl[tid]);
            if (!team_sync(tw, W, nb, S, p.err)) return;
            const int32_t nkeep = min(twl<int32_t>(tw, GW_FAR2L), n);
            // a tree with no clean vertex left in the far list stops (the
            // bucket-end test of the other forms)
            if (p.early_term) {
                uint32_t stopm = 0;
                for (int b = 0; b < GT; b++)
                    if ((alive >> b & 1) && twl<long long>(tw, GW_CLEAN + b) == 0) stopm |= 1u << b;
                alive &= ~stopm;
                early_m |= stopm & (uint32_t)twl<ull>(tw, GW_KEPTM);   // stopped with far entries left
            }
            const bool done = nkeep == 0 || alive == 0;
            const int64_t Tn = done ? 0 : (twl<int64_t>(tw, GW_MINP) / delta + 1) * delta;
            if (!team_sync(tw, W, nb, S, p.err)) return;   // everyone has read the results
            if (done) break;
            if (leader) {
                tws(tw, GW_FARL, 0); tws(tw, GW_FAR2L, 0); tws(tw, GW_MINP, INF); tws(tw, GW_TB, Tn); tws(tw, GW_KEPTM, 0);
                for (int b = 0; b < GT; b++) { tws(tw, GW_CLEAN + b, 0); tws(tw, GW_FCLEAN + b, 0); }
            }
            if (!team_sync(tw, W, nb, S, p.err)) return;
            // ---- next bucket: each kept (vertex, tree) goes to the near list of
            //      this round when its distance is below the new bound, else
            //      back to the far list
            if (tid < GT) S.lfcl[tid] = 0;
            __syncthreads();
            for (int64_t i = tgtid; i < nkeep; i += tthreads) {
                const int32_t v = lget<SC>(&far2[i], n);
                const uint32_t fm = ld<SC>(&fmask[v]);
                uint32_t m = fm & GBITS & alive, tonear = 0, tofar = 0;
                while (m) {
                    const int b = __ffs(m) - 1;
                    m &= m - 1;
                    const K kv = ld<SC>(&key[(int64_t)v * GT + b]);
                    if ((int64_t)(kv >> 1) < Tn) {
                        tonear |= 1u << b;
                    } else {
                        tofar |= 1u << b;
                        if (kv & 1) atomicAdd(&S.lfcl[b], 1u);
                    }
                }
                bool pn = false, pf = false;
                if (tonear) {
                    aand<SC>(&fmask[v], ~tonear);
                    const uint32_t o = __hip_atomic_fetch_or(&mask[v], tonear << sh, __ATOMIC_RELAXED, SC);
                    pn = ((o >> sh) & GBITS) == 0;
                }
                if (tofar) {
                    const uint32_t o = aor<SC>(&fmask[v], GF_FAR_IN);
                    pf = (o & GF_FAR_IN) == 0;
                }
                int64_t q = wave_append(pn, (ull*)&tw[GW_CNT0 + it % 3]);
                if (pn && q < n) lput<SC>(&cur[q], v);
                q = wave_append(pf, (ull*)&tw[GW_FARL]);
                if (pf && q < n) lput<SC>(&far[q], v);
            }
            __syncthreads();
            if (tid < GT && S.lfcl[tid]) atomicAdd((ull*)&tw[GW_FCLEAN + tid], (ull)S.lfcl[tid]);
            if (!team_sync(tw, W, nb, S, p.err)) return;
        }
        // ---- labels: a touched vertex v gets (v, h_b, d) for every tree b of
        //      the group whose key of v is reached and clean
        const int64_t nt = min(twl<int64_t>(tw, GW_TOUCHEDL), (int64_t)n);
        if (tid < GT) S.lnl[tid] = 0;
        __syncthreads();
        for (int64_t i = tgtid; i < nt; i += tthreads) {
            const int32_t v = lget<SC>(&touched[i], n);
            for (int b = 0; b < GT; b++) {
                if (!(valid >> b & 1)) continue;
                const K kv = ld<SC>(&key[(int64_t)v * GT + b]);
                if (kv != KeyTraits<K>::INF && (kv & 1)) atomicAdd(&S.lnl[b], 1ull);
            }
        }
        __syncthreads();
        if (tid < GT && S.lnl[tid]) {
            atomicAdd((ull*)&tw[GW_NLABB + tid], S.lnl[tid]);
            atomicAdd((ull*)&tw[GW_NLABT], S.lnl[tid]);
        }
        if (!team_sync(tw, W, nb, S, p.err)) return;
        if (leader) {
            const ull nl = twl<ull>(tw, GW_NLABT);
            const ull b0 = atomicAdd(p.pool.cursor, nl);
            if (b0 + nl > p.pool.cap) {
                tws(tw, GW_BASEP, -1);
                atomicOr(p.err, ERR_BIT_POOL);
                atomicExch(p.stop, 1);
                atomicMin(p.pool.fail_base, b0);
                for (int b = 0; b < GT; b++)
                    if (valid >> b & 1) p.failed[atomicAdd(p.nfailed, 1)] = twl<int32_t>(tw, GW_ROOT + b);
            } else {
                tws(tw, GW_BASEP, (long long)b0);
            }
        }
        if (!team_sync(tw, W, nb, S, p.err)) return;
        const long long pbase = twl<long long>(tw, GW_BASEP);
        const long long nl = twl<long long>(tw, GW_NLABT);
        bool ovf = false;
        for (int64_t i = tgtid; i < nt; i += tthreads) {
            const int32_t v = lget<SC>(&touched[i], n);
            for (int b = 0; b < GT; b++) {
                K kv = KeyTraits<K>::INF;
                if (valid >> b & 1) {
                    kv = ld<SC>(&key[(int64_t)v * GT + b]);
                    st<SC>(&key[(int64_t)v * GT + b], KeyTraits<K>::INF);
                }
                const bool lab = kv != KeyTraits<K>::INF && (kv & 1);
                const uint64_t d = (uint64_t)(kv >> 1);
                const int64_t q = wave_append(lab, (ull*)&tw[GW_FILLP]);
                if (lab && pbase >= 0 && q < nl) {
                    ovf |= d > 0x7FFFFFFEull;
                    p.pool.v[pbase + q] = v;
                    p.pool.hub[pbase + q] = S.hroot[b];
                    p.pool.dist[pbase + q] = (int32_t)d;
                }
            }
            st<SC>(&mask[v], 0u);
            st<SC>(&fmask[v], 0u);
        }
        if (ovf) atomicOr(p.err, ERR_BIT_OVERFLOW);
        if (p.stats && leader) {
            const int64_t ticks = (int64_t)(__builtin_amdgcn_s_memrealtime() - t_start);
            for (int b = 0; b < GT; b++) {
                if (!(valid >> b & 1)) continue;
                int64_t* s = p.stats + (int64_t)S.hroot[b] * STAT_COLS;
                s[0] = twl<long long>(tw, GW_SETTLEDB + b); s[1] = twl<long long>(tw, GW_ARCSB + b);
                s[2] = twl<long long>(tw, GW_NLABB + b); s[3] = (early_m >> b) & 1;
                s[4] = it; s[5] = ticks;
            }
        }
        // the group is done in every workgroup before the leader resets the words
        if (!team_sync(tw, W, nb, S, p.err)) return;
    }
}

template <typename K, int WG>
int launch_batched_t(const TreeParams& p, int phase, hipStream_t st) {
    const bool pr = p.poff != nullptr && p.pbound > 0;
    const size_t dl = pr ? (size_t)p.pbound * 4 : 0;
    const dim3 g(p.s.k), b(WG);
    const bool hs = pr && p.hashdh && p.ovf && p.novf;
    if (phase == 3) {
        if (!pr || !p.dhg || !p.rlab) return -1;
        hipLaunchKernelGGL((k_tree_batched<K, WG, 3, true, false>), g, b, 0, st, p);
    } else if (phase == 1 && hs) hipLaunchKernelGGL((k_tree_batched<K, WG, 1, true, true>), g, b, 0, st, p);
    else if (phase == 1 && pr) hipLaunchKernelGGL((k_tree_batched<K, WG, 1, true, false>), g, b, dl, st, p);
    else if (phase == 1) hipLaunchKernelGGL((k_tree_batched<K, WG, 1, false, false>), g, b, 0, st, p);
    else if (phase == 2 && pr) hipLaunchKernelGGL((k_tree_batched<K, WG, 2, true, false>), g, b, dl, st, p);
    else if (phase == 2) hipLaunchKernelGGL((k_tree_batched<K, WG, 2, false, false>), g, b, 0, st, p);
    else if (hs) hipLaunchKernelGGL((k_tree_batched<K, WG, 0, true, true>), g, b, 0, st, p);
    else if (pr) hipLaunchKernelGGL((k_tree_batched<K, WG, 0, true, false>), g, b, dl, st, p);
    else hipLaunchKernelGGL((k_tree_batched<K, WG, 0, false, false>), g, b, 0, st, p);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename K, int WG>
int launch_plain_t(const TreeParams& p, int grid, int32_t root, int32_t* gstate, hipStream_t st) {
    TreeParams pp = p;
    long long* gs = (long long*)gstate;
    void* args[] = {(void*)&pp, (void*)&root, (void*)&gs};
    hipError_t e = hipLaunchCooperativeKernel((const void*)k_tree_plain<K, WG>, dim3(grid), dim3(WG),
                                              args, 0, st);
    return e == hipSuccess ? 0 : -1;
}

template <typename K, int WG>
int launch_team_t(const TreeParams& p, int W, int nteams, long long* tstate, int32_t* far2, hipStream_t st) {
    TreeParams pp = p;
    const bool pr = p.poff != nullptr && p.pbound > 0;
    const size_t dl = pr ? (size_t)p.pbound * 4 : 0;
    void* args[] = {(void*)&pp, (void*)&W, (void*)&tstate, (void*)&far2};
    const void* f = pr ? (const void*)k_tree_team<K, WG, true> : (const void*)k_tree_team<K, WG, false>;
    hipError_t e = hipLaunchCooperativeKernel(f, dim3(nteams * W), dim3(WG), args, dl, st);
    return e == hipSuccess ? 0 : -1;
}

template <typename K>
int launch_small_t(const TreeParams& p, int nwg, int32_t* ovf, int32_t* novf, hipStream_t st) {
    const bool pr = p.poff != nullptr && p.pbound > 0;
    if (pr) hipLaunchKernelGGL((k_tree_small<K, true>), dim3(nwg), dim3(64), 0, st, p, ovf, novf);
    else hipLaunchKernelGGL((k_tree_small<K, false>), dim3(nwg), dim3(64), 0, st, p, ovf, novf);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename K>
int small_capacity_t() {
    int dev = 0, per = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tree_small<K, true>, 64, 0) != hipSuccess) return 0;
    return per * cus;
}

template <typename K, int WG>
int launch_group_t(const TreeParams& p, int W, int ngroups, long long* gstate, int32_t* far2, uint32_t* gmask,
                   hipStream_t st) {
    TreeParams pp = p;
    const bool pr = p.poff != nullptr && p.pbound > 0;
    const size_t dl = pr ? (size_t)GT * p.pbound * 4 : 0;
    void* args[] = {(void*)&pp, (void*)&W, (void*)&gstate, (void*)&far2, (void*)&gmask};
    const void* f = pr ? (const void*)k_tree_group<K, WG, true> : (const void*)k_tree_group<K, WG, false>;
    hipError_t e = hipLaunchCooperativeKernel(f, dim3(ngroups * W), dim3(WG), args, dl, st);
    return e == hipSuccess ? 0 : -1;
}

template <typename K, int WG>
int group_capacity_t(int pbound) {
    int dev = 0, per = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tree_group<K, WG, true>, WG, (size_t)GT * pbound * 4) !=
        hipSuccess)
        return 0;
    return per * cus;
}

template <typename K, int WG>
int team_capacity_t() {
    int dev = 0, per = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    // the pruned kernel with the largest prefix of a team launch bounds both
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tree_team<K, WG, true>, WG, MAX_PREFIX * 4) !=
        hipSuccess)
        return 0;
    return per * cus;
}

template <typename K, int WG>
int plain_grid_t() {
    int dev = 0, per = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tree_plain<K, WG>, WG, 0) != hipSuccess) return 0;
    return per * cus;
}

}  // namespace

int launch_tree_batched(const TreeParams& p, int key_bits, int wg, int phase, hipStream_t st) {
    if (key_bits == 32) {
        if (wg == 64) return launch_batched_t<uint32_t, 64>(p, phase, st);
        if (wg == 128) return launch_batched_t<uint32_t, 128>(p, phase, st);
        if (wg == 256) return launch_batched_t<uint32_t, 256>(p, phase, st);
        if (wg == 512) return launch_batched_t<uint32_t, 512>(p, phase, st);
        if (wg == 1024) return launch_batched_t<uint32_t, 1024>(p, phase, st);
    } else {
        if (wg == 64) return launch_batched_t<uint64_t, 64>(p, phase, st);
        if (wg == 128) return launch_batched_t<uint64_t, 128>(p, phase, st);
        if (wg == 256) return launch_batched_t<uint64_t, 256>(p, phase, st);
        if (wg == 512) return launch_batched_t<uint64_t, 512>(p, phase, st);
        if (wg == 1024) return launch_batched_t<uint64_t, 1024>(p, phase, st);
    }
    return -1;
}

int launch_tree_plain(const TreeParams& p, int key_bits, int wg, int grid, int32_t root,
                      int32_t* gstate, hipStream_t st) {
    if (key_bits == 32) {
        if (wg == 256) return launch_plain_t<uint32_t, 256>(p, grid, root, gstate, st);
        if (wg == 512) return launch_plain_t<uint32_t, 512>(p, grid, root, gstate, st);
    } else {
        if (wg == 256) return launch_plain_t<uint64_t, 256>(p, grid, root, gstate, st);
        if (wg == 512) return launch_plain_t<uint64_t, 512>(p, grid, root, gstate, st);
    }
    return -1;
}

int plain_grid_size(int key_bits, int wg) {
    if (key_bits == 32) return wg == 256 ? plain_grid_t<uint32_t, 256>() : plain_grid_t<uint32_t, 512>();
    return wg == 256 ? plain_grid_t<uint64_t, 256>() : plain_grid_t<uint64_t, 512>();
}

size_t plain_gstate_words() { return G_WORDS; }

int launch_tree_team(const TreeParams& p, int key_bits, int wg, int team_size, int nteams,
                     long long* tstate, int32_t* far2, hipStream_t st) {
    if (team_size < 1 || nteams < 1) return -1;
    if (key_bits == 32) {
        if (wg == 512) return launch_team_t<uint32_t, 512>(p, team_size, nteams, tstate, far2, st);
        if (wg == 1024) return launch_team_t<uint32_t, 1024>(p, team_size, nteams, tstate, far2, st);
    } else {
        if (wg == 512) return launch_team_t<uint64_t, 512>(p, team_size, nteams, tstate, far2, st);
        if (wg == 1024) return launch_team_t<uint64_t, 1024>(p, team_size, nteams, tstate, far2, st);
    }
    return -1;
}

int launch_tree_group(const TreeParams& p, int key_bits, int wg, int team_size, int ngroups, long long* gstate,
                      int32_t* far2, uint32_t* gmask, hipStream_t st) {
    if (team_size < 1 || ngroups < 1 || wg != 1024) return -1;
    if (key_bits == 32) return launch_group_t<uint32_t, 1024>(p, team_size, ngroups, gstate, far2, gmask, st);
    return launch_group_t<uint64_t, 1024>(p, team_size, ngroups, gstate, far2, gmask, st);
}

int launch_tree_small(const TreeParams& p, int key_bits, int nwg, int32_t* ovf, int32_t* novf, hipStream_t st) {
    if (nwg < 1) return -1;
    return key_bits == 32 ? launch_small_t<uint32_t>(p, nwg, ovf, novf, st) : launch_small_t<uint64_t>(p, nwg, ovf, novf, st);
}

int small_capacity(int key_bits) {
    return key_bits == 32 ? small_capacity_t<uint32_t>() : small_capacity_t<uint64_t>();
}

int group_capacity(int key_bits, int pbound) {
    return key_bits == 32 ? group_capacity_t<uint32_t, 1024>(pbound) : group_capacity_t<uint64_t, 1024>(pbound);
}

int team_capacity(int key_bits, int wg) {
    if (key_bits == 32) return wg == 512 ? team_capacity_t<uint32_t, 512>() : team_capacity_t<uint32_t, 1024>();
    return wg == 512 ? team_capacity_t<uint64_t, 512>() : team_capacity_t<uint64_t, 1024>();
}

}  // namespace chl
