// Distance queries by merge of two sorted label lists (Section 5, labels of
// every vertex held by one device): d(u, v) = min over hubs common to L_u
// and L_v of d_u + d_v, -1 when they share none (for a directed graph L_u is
// u's out-list and L_v v's in-list, footnote of Section 1). A group of G
// lanes answers one query: each lane takes every G-th hub of the shorter
// list and looks it up by binary search in the longer one (both lists are
// sorted by hub rank position), then the group reduces the minimum.
#include "internal.h"

namespace chl {

namespace {

template <int G>
__global__ __launch_bounds__(256) void k_query(int32_t n, const int64_t* __restrict__ off_u,
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
    int G = avg_len <= 24 ? 8 : avg_len <= 96 ? 16 : avg_len <= 256 ? 32 : 64;
    int64_t blocks = (q * G + 255) / 256;
    if (blocks > 1 << 20) blocks = 1 << 20;
    if (blocks < 1) blocks = 1;
    switch (G) {
        case 8: hipLaunchKernelGGL(k_query<8>, dim3(blocks), dim3(256), 0, st, n, off_u, hub_u, dist_u, off_v, hub_v, dist_v, pairs, q, out, err); break;
        case 16: hipLaunchKernelGGL(k_query<16>, dim3(blocks), dim3(256), 0, st, n, off_u, hub_u, dist_u, off_v, hub_v, dist_v, pairs, q, out, err); break;
        case 32: hipLaunchKernelGGL(k_query<32>, dim3(blocks), dim3(256), 0, st, n, off_u, hub_u, dist_u, off_v, hub_v, dist_v, pairs, q, out, err); break;
        default: hipLaunchKernelGGL(k_query<64>, dim3(blocks), dim3(256), 0, st, n, off_u, hub_u, dist_u, off_v, hub_v, dist_v, pairs, q, out, err); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace chl
