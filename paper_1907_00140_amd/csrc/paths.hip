// Shortest paths from the labeling (Section 4.4, last paragraph): with each
// label (h, d(v,h)) of L_v the next vertex from v towards h is kept, and a
// shortest u-v path is u's chain of these parents down to the common hub h
// that gives d(u,v), followed by the reverse of v's chain.
//
// Parent of (h, d) in L_v: the smallest-id neighbour p of v with
// d(p,h) + w(p,v) = d. Every such p carries the label (h, d(p,h)) (a
// shortest p-h path extended by the arc (p,v) is a shortest v-h path, so h
// tops SP_{p,h} as well), so the parents are found from the finished labels
// and the graph alone, after the build: for each arc (v,p), the entries of
// L_p are looked up in L_v. slot = the position of p's label of the same hub
// within L_p, so that a walk takes one step per edge.
//
// k_parents: one wave per vertex v, vertices taken from a queue in rank
// order (an atomic counter over hub_vertex[]: under a degree ranking the
// heaviest rows go first, and no wave is left with a run of them, as a fixed
// stride over input ids would leave one on an R-MAT graph, whose
// high-degree ids are those with few bits set). A pass whose labels are all
// v's own (distance 0, no parent) skips the arcs. L_v (up to PCH labels per
// pass) sits in LDS as sorted hubs, distances and a 64-bit candidate
// (p << 32 | slot) per label. The arcs of v are taken 64 at a time; each lane owns one arc and
// the wave splits the flattened (arc, entry of L_p) index space evenly over
// its lanes (inclusive scan of the list lengths, a 6-step search for the
// arc of an index), so a hub vertex with thousands of neighbours is spread
// over the lanes as well as a grid vertex with four. A neighbour list is cut
// to the hub range of the labels in LDS by binary search: above, when its
// last hub lies beyond the range (every hub of L_v ranks at most as low as
// v itself, so for the important, high-degree vertices of a degree ranking
// this drops nearly all of each neighbour's list), and below when L_v takes
// several passes.
// A matching entry (same hub, d(p,h) + w = d) takes an LDS atomic minimum.
//
// k_path: a group of G lanes per pair finds the hub by the merge of the two
// sorted lists (smallest d_u + d_v, and the most important hub among equal
// sums: the highest ranked vertex of SP_{u,v}); then lane 0 walks u's chain
// and lane 1 walks v's chain. The first pass counts edges; the second writes
// u's chain from the front of the pair's output range and v's chain from its
// back.
#include "internal.h"

#include <algorithm>
#include <climits>
#include <mutex>

namespace chl {

namespace {

constexpr int PW = 4;       // waves per workgroup of k_parents
constexpr int PCH = 256;    // labels of L_v per LDS pass

struct ParentLds {
    unsigned long long cand[PCH];
    int32_t hub[PCH];
    int32_t dist[PCH];
    int64_t inc[64];        // inclusive scan of the (cut) list lengths of the 64 arcs
    int64_t beg[64];        // first entry of each arc's (cut) list
    int64_t base[64];       // off[p] of each arc (slot = entry - base)
    int32_t p[64];
    int32_t w[64];
};

// LDS written by some lanes of a wave and read by others: order the wave's
// accesses (a wave executes in lockstep; this keeps the compiler from moving
// LDS accesses across the point)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t lower_hub(const int32_t* __restrict__ hub, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (hub[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(64 * PW) void k_parents(int32_t n, int64_t m, const int64_t* __restrict__ row,
                                                     const int32_t* __restrict__ col, const int32_t* __restrict__ wt,
                                                     const int64_t* __restrict__ off, const int32_t* __restrict__ hub,
                                                     const int32_t* __restrict__ dist, int32_t* __restrict__ parent,
                                                     int32_t* __restrict__ slot, const int32_t* __restrict__ vorder,
                                                     unsigned long long* next, int32_t* err) {
    __shared__ ParentLds lds[PW];
    const int lane = threadIdx.x & 63;
    ParentLds& S = lds[threadIdx.x >> 6];
    for (;;) {
        unsigned long long idx = 0;
        if (lane == 0) idx = atomicAdd(next, 1ull);
        idx = __shfl(idx, 0);
        if (idx >= (unsigned long long)n) break;
        const int32_t v = vorder[idx];
        if (v < 0 || v >= n) {
            if (lane == 0) atomicOr(err, ERR_BIT_INVALID);
            continue;
        }
        const int64_t lb = off[v], le = off[v + 1];
        int64_t eb = row[v], ee = row[v + 1];
        if (eb < 0 || ee < eb || ee > m) {          // malformed row: no arcs, flagged
            if (lane == 0) atomicOr(err, ERR_BIT_INVALID);
            eb = ee = 0;
        }
        for (int64_t c0 = lb; c0 < le; c0 += PCH) {
            const int cn = (int)std::min<int64_t>(PCH, le - c0);
            for (int i = lane; i < cn; i += 64) {
                S.hub[i] = hub[c0 + i];
                S.dist[i] = dist[c0 + i];
                S.cand[i] = ~0ull;
            }
            const bool whole = c0 == lb && c0 + cn == le;
            const int32_t hlo = hub[c0], hhi = hub[c0 + cn - 1];
            bool far = false;                          // some label of the pass is not v's own
            for (int i = lane; i < cn; i += 64) far |= dist[c0 + i] != 0;
            const bool any_far = __ballot(far) != 0;
            wave_sync();
            for (int64_t e0 = any_far ? eb : ee; e0 < ee; e0 += 64) {
                const int64_t e = e0 + lane;
                int64_t len = 0, beg = 0, base = 0;
                int32_t p = 0, w = 0;
                if (e < ee) {
                    p = col[e];
                    w = wt[e];
                    if (p >= 0 && p < n && w >= 1) {
                        base = off[p];
                        int64_t end = off[p + 1];
                        beg = !whole ? lower_hub(hub, base, end, hlo) : base;
                        if (end > beg && hub[end - 1] > hhi) end = lower_hub(hub, beg, end, hhi + 1);
                        len = end - beg;
                    } else {
                        atomicOr(err, ERR_BIT_INVALID);
                    }
                }
                int64_t inc = len;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int64_t t = __shfl_up(inc, d);
                    if (lane >= d) inc += t;
                }
                S.inc[lane] = inc;
                S.beg[lane] = beg;
                S.base[lane] = base;
                S.p[lane] = p;
                S.w[lane] = w;
                const int64_t total = __shfl(inc, 63);
                wave_sync();
                for (int64_t t = lane; t < total; t += 64) {
                    int a = 0, z = 63;                     // first arc with inc > t
                    while (a < z) {
                        const int mid = (a + z) >> 1;
                        if (S.inc[mid] > t) z = mid; else a = mid + 1;
                    }
                    const int64_t j = S.beg[a] + (t - (a ? S.inc[a - 1] : 0));
                    const int32_t hj = hub[j];
                    int lo = 0, hi = cn;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (S.hub[mid] < hj) lo = mid + 1; else hi = mid;
                    }
                    if (lo < cn && S.hub[lo] == hj && (int64_t)dist[j] + S.w[a] == (int64_t)S.dist[lo])
                        atomicMin(&S.cand[lo], ((unsigned long long)(uint32_t)S.p[a] << 32) |
                                                   (uint32_t)(j - S.base[a]));
                }
                wave_sync();
            }
            for (int i = lane; i < cn; i += 64) {
                const unsigned long long c = S.cand[i];
                parent[c0 + i] = c == ~0ull ? -1 : (int32_t)(c >> 32);
                slot[c0 + i] = c == ~0ull ? -1 : (int32_t)(uint32_t)c;
            }
            wave_sync();
        }
    }
}

// One step of a chain towards hub h: label index i of some vertex -> label
// index of its parent, or -1 at the hub; -2 when the parent arrays do not
// fit the labeling (parent or slot out of range, or a label of another hub).
__device__ __forceinline__ int64_t step(int32_t n, const int64_t* __restrict__ off,
                                        const int32_t* __restrict__ hub, const int32_t* __restrict__ parent,
                                        const int32_t* __restrict__ slot, int32_t h, int64_t i, int32_t* x) {
    const int32_t p = parent[i];
    if (p < 0) return -1;
    if (p >= n) return -2;
    const int64_t b = off[p];
    const int32_t s = slot[i];
    if (s < 0 || s >= off[p + 1] - b || hub[b + s] != h) return -2;
    *x = p;
    return b + s;
}

// WRITE = false: hops[k] = edges of pair k's path (-1 disconnected, -2
// invalid pair or inconsistent parents) and len[k] = hops + 1 or 0.
// WRITE = true: the vertices of pair k go to path[path_off[k], path_off[k+1]).
template <int G, bool WRITE>
__global__ __launch_bounds__(256) void k_path(int32_t n, const int64_t* __restrict__ off,
                                              const int32_t* __restrict__ hub, const int32_t* __restrict__ dist,
                                              const int32_t* __restrict__ parent, const int32_t* __restrict__ slot,
                                              const int32_t* __restrict__ pairs, int64_t q,
                                              int64_t* __restrict__ hops, int64_t* __restrict__ len,
                                              const int64_t* __restrict__ path_off, int32_t* __restrict__ path,
                                              int32_t* err) {
    const int gl = threadIdx.x & (G - 1);
    const int64_t grp = ((int64_t)blockIdx.x * 256 + threadIdx.x) / G;
    const int64_t ngrp = ((int64_t)gridDim.x * 256) / G;
    for (int64_t k = grp; k < q; k += ngrp) {
        const int32_t u = pairs[2 * k], v = pairs[2 * k + 1];
        const bool ok = u >= 0 && u < n && v >= 0 && v < n;
        // best = (d_u + d_v) << 31 | hub: the smallest sum, then the smallest hub
        unsigned long long best = ~0ull;
        if (ok) {
            int64_t ab = off[u], ae = off[u + 1], bb = off[v], be = off[v + 1];
            if (ae - ab > be - bb) {
                int64_t t = ab; ab = bb; bb = t;
                t = ae; ae = be; be = t;
            }
            for (int64_t i = ab + gl; i < ae; i += G) {
                const int32_t x = hub[i];
                const int64_t lo = lower_hub(hub, bb, be, x);
                if (lo < be && hub[lo] == x) {
                    const unsigned long long s = (unsigned long long)((int64_t)dist[i] + (int64_t)dist[lo]);
                    const unsigned long long key = (s << 31) | (uint32_t)x;
                    best = key < best ? key : best;
                }
            }
        }
#pragma unroll
        for (int d = G / 2; d >= 1; d >>= 1) {
            const unsigned long long o = __shfl_xor(best, d, G);
            best = o < best ? o : best;
        }
        if (!ok || best == ~0ull) {
            if (!WRITE && gl == 0) {
                hops[k] = ok ? -1 : -2;
                if (len) len[k] = 0;
                if (!ok) atomicOr(err, ERR_BIT_INVALID);
            }
            continue;
        }
        const int32_t h = (int32_t)(best & 0x7FFFFFFFull);
        // lane 0 walks u's chain, lane 1 v's chain
        int64_t chain = 0;
        bool bad = false;
        if (gl < 2) {
            int32_t x = gl == 0 ? u : v;
            int64_t i = lower_hub(hub, off[x], off[x + 1], h);
            if (i == off[x + 1] || hub[i] != h) {
                bad = true;
            } else if (WRITE) {
                const int64_t pb = path_off[k], pe = path_off[k + 1];
                int64_t at = gl == 0 ? pb : pe - 1;
                if (at >= pb && at < pe) path[at] = x;
                for (;;) {
                    const int64_t nx = step(n, off, hub, parent, slot, h, i, &x);
                    if (nx < 0) { bad = nx == -2; break; }
                    i = nx;
                    if (++chain > n) { bad = true; break; }
                    at = gl == 0 ? pb + chain : pe - 1 - chain;
                    if (at < pb || at >= pe) { bad = true; break; }
                    path[at] = x;
                }
            } else {
                for (;;) {
                    const int64_t nx = step(n, off, hub, parent, slot, h, i, &x);
                    if (nx < 0) { bad = nx == -2; break; }
                    i = nx;
                    if (++chain > n) { bad = true; break; }
                }
            }
        }
        const int64_t other = __shfl_xor(chain, 1, G);
        const int bad_any = __shfl_xor((int)bad, 1, G) | (int)bad;
        if (gl == 0) {
            if (WRITE) {
                if (bad_any || path_off[k + 1] - path_off[k] != chain + other + 1) atomicOr(err, ERR_BIT_INVALID);
            } else {
                hops[k] = bad_any ? -2 : chain + other;
                if (len) len[k] = bad_any ? 0 : chain + other + 1;
                if (bad_any) atomicOr(err, ERR_BIT_INVALID);
            }
        }
    }
}

int group_for(const chl_labels* h) {
    const double avg = h->n ? (double)h->total / h->n : 1.0;
    return avg <= 24 ? 8 : avg <= 96 ? 16 : avg <= 256 ? 32 : 64;
}

template <bool WRITE>
int launch_path(const chl_labels* h, const int32_t* parent, const int32_t* slot, const int32_t* pairs, int64_t q,
                int64_t* hops, int64_t* len, const int64_t* path_off, int32_t* path, hipStream_t st) {
    const int G = group_for(h);
    int64_t blocks = (q * G + 255) / 256;
    blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, 1 << 16));
#define CHL_PATH_LAUNCH(GG)                                                                              \
    hipLaunchKernelGGL((k_path<GG, WRITE>), dim3(blocks), dim3(256), 0, st, h->n, h->offsets, h->hub_pos, \
                       h->dist, parent, slot, pairs, q, hops, len, path_off, path, h->qerr)
    switch (G) {
        case 8: CHL_PATH_LAUNCH(8); break;
        case 16: CHL_PATH_LAUNCH(16); break;
        case 32: CHL_PATH_LAUNCH(32); break;
        default: CHL_PATH_LAUNCH(64); break;
    }
#undef CHL_PATH_LAUNCH
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// clear the handle's error word, run f, read the word back (the word is per
// handle: calls on one handle serialise here)
template <typename F>
int with_err(const chl_labels* hc, hipStream_t st, F f) {
    chl_labels* h = const_cast<chl_labels*>(hc);
    std::lock_guard<std::mutex> lk(h->qmu);
    if (hipMemsetAsync(h->qerr, 0, 4, st) != hipSuccess) return CHL_ERR_HIP;
    const int rc = f();
    if (rc) return rc;
    int32_t e = 0;
    if (hipMemcpyAsync(&e, h->qerr, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return CHL_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return CHL_ERR_HIP;
    return e ? CHL_ERR_INVALID_ARG : CHL_OK;
}

}  // namespace

}  // namespace chl

using namespace chl;

extern "C" int chl_labels_parents(const chl_labels* h, const chl_graph* g, int32_t* parent, int32_t* slot,
                                  void* stream) {
    (void)hipGetLastError();   // launches are checked with hipGetLastError
    if (!h || !g || h->directed || g->n != h->n || g->n_arcs < 0 || !g->row_ptr) return CHL_ERR_INVALID_ARG;
    if (g->n_arcs > 0 && (!g->col || !g->w)) return CHL_ERR_INVALID_ARG;
    if (h->total > 0 && (!parent || !slot)) return CHL_ERR_INVALID_ARG;
    if (h->total == 0 || h->n == 0) return CHL_OK;
    hipStream_t st = (hipStream_t)stream;
    // the vertex queue's counter
    auto* next = (unsigned long long*)h->alloc.alloc(256, h->alloc.ctx);
    if (!next) return CHL_ERR_OOM;
    const int rc = with_err(h, st, [&]() {
        if (hipMemsetAsync(next, 0, 8, st) != hipSuccess) return CHL_ERR_HIP;
        const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(((int64_t)h->n + PW - 1) / PW, 2048));
        hipLaunchKernelGGL(k_parents, dim3(blocks), dim3(64 * PW), 0, st, h->n, g->n_arcs, g->row_ptr, g->col,
                           g->w, h->offsets, h->hub_pos, h->dist, parent, slot, h->order, next, h->qerr);
        return hipGetLastError() == hipSuccess ? CHL_OK : CHL_ERR_HIP;
    });
    (void)hipStreamSynchronize(st);
    h->alloc.free(next, h->alloc.ctx);
    return rc;
}

extern "C" int chl_query_path_hops(const chl_labels* h, const int32_t* parent, const int32_t* slot,
                                   const int32_t* pairs, int64_t q, int64_t* hops, int64_t* path_off,
                                   void* stream) {
    (void)hipGetLastError();   // launches are checked with hipGetLastError
    if (!h || h->directed || q < 0 || (q > 0 && (!pairs || !hops || !parent || !slot))) return CHL_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (q == 0) {
        if (path_off && hipMemsetAsync(path_off, 0, 8, st) != hipSuccess) return CHL_ERR_HIP;
        return CHL_OK;
    }
    int64_t* len = nullptr;
    void* temp = nullptr;
    if (path_off) {
        len = (int64_t*)h->alloc.alloc((size_t)q * 8, h->alloc.ctx);
        temp = h->alloc.alloc(scan_temp_bytes(q), h->alloc.ctx);
        if (!len || !temp) {
            if (len) h->alloc.free(len, h->alloc.ctx);
            if (temp) h->alloc.free(temp, h->alloc.ctx);
            return CHL_ERR_OOM;
        }
    }
    int rc = with_err(h, st, [&]() {
        if (launch_path<false>(h, parent, slot, pairs, q, hops, len, nullptr, nullptr, st))
            return CHL_ERR_HIP;
        if (len && launch_scan_i64(len, path_off, q, temp, st)) return CHL_ERR_HIP;
        return CHL_OK;
    });
    if (len) {
        // the stream has been synchronised by with_err (or the launch failed)
        (void)hipStreamSynchronize(st);
        h->alloc.free(len, h->alloc.ctx);
        h->alloc.free(temp, h->alloc.ctx);
    }
    return rc;
}

// ---- the variant of chl_query_path_hops that allocates nothing: its
// scratch (per-pair vertex counts and the scan's temporaries) is a
// file-scope device array, one copy per GPU, whose address each device
// reports once through hipGetSymbolAddress.
namespace {
constexpr size_t NOALLOC_BYTES = (size_t)CHL_NOALLOC_MAX_PAIRS * 8 + (64u << 10);
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;                       // one call at a time (the calls share the array)
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of this device's copy of the array (nullptr on failure)
void* noalloc_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_noalloc_ptr[dev] = p;
    }
    return g_noalloc_ptr[dev];
}
}  // namespace

extern "C" int chl_query_path_hops_noalloc(const chl_labels* h, const int32_t* parent, const int32_t* slot,
                                           const int32_t* pairs, int64_t q, int64_t* hops, int64_t* path_off,
                                           void* stream) {
    (void)hipGetLastError();   // launches are checked with hipGetLastError
    if (!h || h->directed || q < 0 || (q > 0 && (!pairs || !hops || !parent || !slot))) return CHL_ERR_INVALID_ARG;
    if (q > CHL_NOALLOC_MAX_PAIRS) return CHL_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (q == 0) {
        if (path_off && hipMemsetAsync(path_off, 0, 8, st) != hipSuccess) return CHL_ERR_HIP;
        return CHL_OK;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    unsigned char* base = (unsigned char*)noalloc_scratch();
    if (!base) return CHL_ERR_HIP;
    int64_t* len = nullptr;
    void* temp = nullptr;
    if (path_off) {
        len = (int64_t*)base;                           // q entries, all written by the kernel
        temp = base + (size_t)CHL_NOALLOC_MAX_PAIRS * 8;  // the scan's temporaries
        if (scan_temp_bytes(q) > NOALLOC_BYTES - (size_t)CHL_NOALLOC_MAX_PAIRS * 8) return CHL_ERR_INVALID_ARG;
    }
    // with_err synchronises the stream before it returns, so the next call
    // (serialised by the lock) never finds this call's work in flight
    return with_err(h, st, [&]() {
        if (launch_path<false>(h, parent, slot, pairs, q, hops, len, nullptr, nullptr, st)) return CHL_ERR_HIP;
        if (len && launch_scan_i64(len, path_off, q, temp, st)) return CHL_ERR_HIP;
        return CHL_OK;
    });
}

extern "C" int chl_query_paths(const chl_labels* h, const int32_t* parent, const int32_t* slot,
                               const int32_t* pairs, int64_t q, const int64_t* path_off, int32_t* path,
                               void* stream) {
    (void)hipGetLastError();   // launches are checked with hipGetLastError
    if (!h || h->directed || q < 0 || (q > 0 && (!pairs || !parent || !slot || !path_off))) return CHL_ERR_INVALID_ARG;
    if (q == 0) return CHL_OK;
    hipStream_t st = (hipStream_t)stream;
    return with_err(h, st, [&]() {
        return launch_path<true>(h, parent, slot, pairs, q, nullptr, nullptr, path_off, path, st) ? CHL_ERR_HIP
                                                                                                  : CHL_OK;
    });
}
