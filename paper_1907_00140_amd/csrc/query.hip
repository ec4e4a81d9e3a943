// Distance queries by merge of two sorted label lists (Section 5, labels of
// every vertex held by one device): d(u, v) = min over hubs common to L_u
// and L_v of d_u + d_v, -1 when they share none (for a directed graph L_u is
// u's out-list and L_v v's in-list, footnote of Section 1). A group of G
// lanes answers one query: each lane takes every G-th hub of the shorter
// list and looks it up by binary search in the longer one (both lists are
// sorted by hub rank position), then the group reduces the minimum. Large
// batches over short lists first give each query one lane (k_query_tier);
// long lists are staged in LDS (k_query_lds).
#include "internal.h"

namespace chl {

namespace {

// Lower bound of hub x in hub[lo, hi).
__device__ __forceinline__ int64_t lower_hub(const int32_t* __restrict__ hub, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (hub[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Two tiers in one pass. Every lane first takes one query of its wave's 64:
// when the shorter list has at most SMALL entries (a vertex with only its
// own label, frequent in scale-free graphs, or very few), the lane answers
// it alone. The other queries of the 64 are then answered by groups of G
// lanes of the same wave, a few at a time, their list bounds passed between
// lanes by shuffles: every lane of a group takes every G-th hub of the
// shorter list, searches it in the longer one, and the group reduces.
constexpr int SMALL = 2;

template <int G>
__global__ __launch_bounds__(256) void k_query_tier(int32_t n, const int64_t* __restrict__ off_u,
                                               const int32_t* __restrict__ hub_u,
                                               const int32_t* __restrict__ dist_u,
                                               const int64_t* __restrict__ off_v,
                                               const int32_t* __restrict__ hub_v,
                                               const int32_t* __restrict__ dist_v,
                                               const int32_t* __restrict__ pairs, int64_t q,
                                               int64_t* __restrict__ out, int32_t* err) {
    constexpr int NSUB = 64 / G;
    const int lane = threadIdx.x & 63, sub = lane / G, gl = lane & (G - 1);
    const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
    for (int64_t base = wave * 64; base < q; base += nwaves * 64) {
        const int64_t k = base + lane;
        bool big = false;
        int64_t ab = 0, ae = 0, bb = 0, be = 0;
        int swapped = 0;
        if (k < q) {
            const int32_t u = pairs[2 * k], v = pairs[2 * k + 1];
            if (u >= 0 && u < n && v >= 0 && v < n) {
                ab = off_u[u]; ae = off_u[u + 1]; bb = off_v[v]; be = off_v[v + 1];
                if (ae - ab > be - bb) {
                    int64_t t = ab; ab = bb; bb = t;
                    t = ae; ae = be; be = t;
                    swapped = 1;
                }
                if (ae - ab <= SMALL) {
                    const int32_t *ha = swapped ? hub_v : hub_u, *da = swapped ? dist_v : dist_u;
                    const int32_t *hb = swapped ? hub_u : hub_v, *db = swapped ? dist_u : dist_v;
                    int64_t best = INT64_MAX;
                    for (int64_t i = ab; i < ae; i++) {
                        const int32_t x = ha[i];
                        const int64_t lo = lower_hub(hb, bb, be, x);
                        if (lo < be && hb[lo] == x) {
                            const int64_t sum = (int64_t)da[i] + (int64_t)db[lo];
                            best = sum < best ? sum : best;
                        }
                    }
                    out[k] = best == INT64_MAX ? -1 : best;
                } else {
                    big = true;
                }
            } else {
                atomicOr(err, ERR_BIT_INVALID);
                out[k] = -2;
            }
        }
        // the remaining queries of the wave, NSUB at a time, one per group
        unsigned long long mask = __ballot(big);
        while (mask) {
            unsigned long long m = mask;
            for (int j = 0; j < sub && m; j++) m &= m - 1;
            const int src = m ? __ffsll((long long)m) - 1 : 0;
            const bool has = m != 0;
            const int64_t gab = __shfl(ab, src), gae = __shfl(ae, src);
            const int64_t gbb = __shfl(bb, src), gbe = __shfl(be, src);
            const int gsw = __shfl(swapped, src);
            int64_t best = INT64_MAX;
            if (has) {
                const int32_t *ha = gsw ? hub_v : hub_u, *da = gsw ? dist_v : dist_u;
                const int32_t *hb = gsw ? hub_u : hub_v, *db = gsw ? dist_u : dist_v;
                for (int64_t i = gab + gl; i < gae; i += G) {
                    const int32_t x = ha[i];
                    const int64_t lo = lower_hub(hb, gbb, gbe, x);
                    if (lo < gbe && hb[lo] == x) {
                        const int64_t sum = (int64_t)da[i] + (int64_t)db[lo];
                        best = sum < best ? sum : best;
                    }
                }
            }
#pragma unroll
            for (int d = G / 2; d >= 1; d >>= 1) {
                const int64_t o = __shfl_xor(best, d, G);
                best = o < best ? o : best;
            }
            if (has && gl == 0) out[base + src] = best == INT64_MAX ? -1 : best;
            for (int j = 0; j < NSUB && mask; j++) mask &= mask - 1;
        }
    }
}

// Long lists (hundreds to thousands of labels, road-like graphs): one wave
// per query. The shorter list's hubs are copied into the wave's LDS with
// coalesced loads; the lanes then read the longer list 64 hubs at a time,
// also coalesced, and look each up by binary search in LDS, so that global
// memory sees each list once, in order, instead of a chain of dependent
// loads per hub. A shorter list beyond QCAP hubs is searched in global
// memory instead.
constexpr int QCAP = 2560;   // 10 KB of LDS per wave: 16 waves per compute unit
constexpr int QW = 4;        // waves per workgroup
constexpr int QILP = 4;      // loads in flight per lane

__global__ __launch_bounds__(64 * QW) void k_query_lds(int32_t n, const int64_t* __restrict__ off_u,
                                                       const int32_t* __restrict__ hub_u,
                                                       const int32_t* __restrict__ dist_u,
                                                       const int64_t* __restrict__ off_v,
                                                       const int32_t* __restrict__ hub_v,
                                                       const int32_t* __restrict__ dist_v,
                                                       const int32_t* __restrict__ pairs, int64_t q,
                                                       int64_t* __restrict__ out, int32_t* err) {
    __shared__ int32_t sh_all[QW][QCAP];
    const int lane = threadIdx.x & 63;
    int32_t* sh = sh_all[threadIdx.x >> 6];
    const int64_t wave = ((int64_t)blockIdx.x * 64 * QW + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * 64 * QW) >> 6;
    for (int64_t k = wave; k < q; k += nwaves) {
        const int32_t u = pairs[2 * k], v = pairs[2 * k + 1];
        const bool ok = u >= 0 && u < n && v >= 0 && v < n;
        int64_t best = INT64_MAX;
        if (ok) {
            int64_t ab = off_u[u], ae = off_u[u + 1], bb = off_v[v], be = off_v[v + 1];
            const int32_t *ha = hub_u, *da = dist_u, *hb = hub_v, *db = dist_v;
            if (ae - ab > be - bb) {
                int64_t t = ab; ab = bb; bb = t;
                t = ae; ae = be; be = t;
                ha = hub_v; da = dist_v; hb = hub_u; db = dist_u;
            }
            const int64_t la = ae - ab;
            if (la <= QCAP) {
                for (int64_t t0 = lane; t0 < la; t0 += 64 * QILP) {
                    int32_t x[QILP];
#pragma unroll
                    for (int r = 0; r < QILP; r++) x[r] = t0 + r * 64 < la ? ha[ab + t0 + r * 64] : 0;
#pragma unroll
                    for (int r = 0; r < QILP; r++)
                        if (t0 + r * 64 < la) sh[t0 + r * 64] = x[r];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int64_t t0 = bb + lane; t0 < be; t0 += 64 * QILP) {
                    int32_t x[QILP];
#pragma unroll
                    for (int r = 0; r < QILP; r++) x[r] = t0 + r * 64 < be ? hb[t0 + r * 64] : INT32_MAX;
#pragma unroll
                    for (int r = 0; r < QILP; r++) {
                        int lo = 0, hi = (int)la;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (sh[mid] < x[r]) lo = mid + 1; else hi = mid;
                        }
                        if (t0 + r * 64 < be && lo < la && sh[lo] == x[r]) {
                            const int64_t sum = (int64_t)da[ab + lo] + (int64_t)db[t0 + r * 64];
                            best = sum < best ? sum : best;
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else {
                for (int64_t i = ab + lane; i < ae; i += 64) {
                    const int32_t x = ha[i];
                    const int64_t lo = lower_hub(hb, bb, be, x);
                    if (lo < be && hb[lo] == x) {
                        const int64_t sum = (int64_t)da[i] + (int64_t)db[lo];
                        best = sum < best ? sum : best;
                    }
                }
            }
        } else if (lane == 0) {
            atomicOr(err, ERR_BIT_INVALID);
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const int64_t o = __shfl_xor(best, d);
            best = o < best ? o : best;
        }
        if (lane == 0) out[k] = ok ? (best == INT64_MAX ? -1 : best) : -2;
    }
}

// One group of G lanes per query (lists long on average, or few queries).
template <int G>
__global__ __launch_bounds__(256) void k_query_group(int32_t n, const int64_t* __restrict__ off_u,
                                               const int32_t* __restrict__ hub_u,
                                               const int32_t* __restrict__ dist_u,
                                               const int64_t* __restrict__ off_v,
                                               const int32_t* __restrict__ hub_v,
                                               const int32_t* __restrict__ dist_v,
                                               const int32_t* __restrict__ pairs, int64_t q,
                                               int64_t* __restrict__ out, int32_t* err) {
    const int gl = threadIdx.x & (G - 1);
    const int64_t grp = ((int64_t)blockIdx.x * 256 + threadIdx.x) / G;
    const int64_t ngrp = ((int64_t)gridDim.x * 256) / G;
    for (int64_t k = grp; k < q; k += ngrp) {
        const int32_t u = pairs[2 * k], v = pairs[2 * k + 1];
        const bool ok = u >= 0 && u < n && v >= 0 && v < n;
        int64_t best = INT64_MAX;
        if (ok) {
            int64_t ab = off_u[u], ae = off_u[u + 1], bb = off_v[v], be = off_v[v + 1];
            const int32_t *ha = hub_u, *da = dist_u, *hb = hub_v, *db = dist_v;
            if (ae - ab > be - bb) {
                int64_t t = ab; ab = bb; bb = t;
                t = ae; ae = be; be = t;
                ha = hub_v; da = dist_v; hb = hub_u; db = dist_u;
            }
            for (int64_t i = ab + gl; i < ae; i += G) {
                const int32_t x = ha[i];
                int64_t lo = bb, hi = be;
                while (lo < hi) {
                    int64_t mid = (lo + hi) >> 1;
                    if (hb[mid] < x) lo = mid + 1; else hi = mid;
                }
                if (lo < be && hb[lo] == x) {
                    int64_t s = (int64_t)da[i] + (int64_t)db[lo];
                    best = s < best ? s : best;
                }
            }
        } else if (gl == 0) {
            atomicOr(err, ERR_BIT_INVALID);
        }
#pragma unroll
        for (int d = G / 2; d >= 1; d >>= 1) {
            int64_t o = __shfl_xor(best, d, G);
            best = o < best ? o : best;
        }
        if (gl == 0) out[k] = ok ? (best == INT64_MAX ? -1 : best) : -2;
    }
}

}  // namespace

int launch_query(int32_t n, const int64_t* off_u, const int32_t* hub_u, const int32_t* dist_u,
                 const int64_t* off_v, const int32_t* hub_v, const int32_t* dist_v,
                 const int32_t* pairs, int64_t q, int64_t* out, int32_t* err, double avg_len,
                 hipStream_t st) {
    if (q <= 0) return 0;
    const int G = avg_len <= 24 ? 8 : avg_len <= 96 ? 16 : avg_len <= 256 ? 32 : 64;
    // the two-tier kernel for short lists and batches that fill the device
    // with one wave per 64 queries (its groups then only take the longer
    // lists: 16 lanes up to an average of 32 labels, else 32, measured on
    // R-MAT 16, directed R-MAT 16 and R-MAT 20); else one group per query
    const bool tier = G <= 16 && q >= (1 << 16);
    const int GT = avg_len <= 32 ? 16 : 32;
    int64_t blocks = tier ? (q + 255) / 256 : (q * G + 255) / 256;
    if (blocks > 1 << 20) blocks = 1 << 20;
    if (blocks < 1) blocks = 1;
#define CHL_QUERY(KER, GG)                                                                                  \
    hipLaunchKernelGGL(KER<GG>, dim3(blocks), dim3(256), 0, st, n, off_u, hub_u, dist_u, off_v, hub_v, dist_v, \
                       pairs, q, out, err)
    if (G >= 32) {
        // one wave per query, the shorter list in LDS
        int64_t wb = (q + QW - 1) / QW;
        if (wb > 1 << 20) wb = 1 << 20;
        hipLaunchKernelGGL(k_query_lds, dim3(wb), dim3(64 * QW), 0, st, n, off_u, hub_u, dist_u, off_v, hub_v,
                           dist_v, pairs, q, out, err);
    } else if (tier) {
        if (GT == 16) CHL_QUERY(k_query_tier, 16);
        else CHL_QUERY(k_query_tier, 32);
    } else {
        if (G == 8) CHL_QUERY(k_query_group, 8);
        else CHL_QUERY(k_query_group, 16);
    }
#undef CHL_QUERY
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace chl
