// Label cleaning of the Hybrid construction (Section 4.2.1; the cleaning
// query DQ_Clean of Algorithm 2). The trees of one superstep of the pruned
// construction run concurrently and cannot see each other's labels, so a
// tree may label a vertex that a higher-ranked root of the same superstep
// covers. Such a label (h, d) of v is redundant: some hub w outranking h
// (w < h in rank position) is common to L_v and L_h with
// d(v, w) + d(h, w) <= d. The labels of every hub outranking h are in the
// grouped table by then (the superstep's own labels included), so the test
// finds every redundant label, and it never removes a label of the CHL: a
// stored distance is the length of a real walk, so a hit means a hub that
// outranks h lies on a shortest v-h path (or d is not the distance at all).
#include <algorithm>

#include "internal.h"

namespace chl {

namespace {

constexpr int CW = 256;   // threads per cleaning workgroup, one wave per label

// One workgroup per root h at a time: h's labels of the hubs that outrank it
// scattered into a dense array (dc, n words per workgroup, all ones between
// roots), then one wave per label (v, h, d) of h's tree scans v's group.
// keep[i - from] = 1 for a label that stays, 0 for a redundant one.
__global__ __launch_bounds__(CW) void k_clean(int32_t lo, int32_t hi, int64_t n, const int64_t* __restrict__ rlab,
                                              const int32_t* __restrict__ pv, const int32_t* __restrict__ pd,
                                              const int64_t* __restrict__ poff, const uint64_t* __restrict__ plab,
                                              uint32_t* __restrict__ dcbuf, uint64_t from,
                                              int32_t* __restrict__ keep, int64_t* __restrict__ stats) {
    __shared__ int32_t kept;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t* dc = dcbuf + (int64_t)blockIdx.x * n;
    for (int32_t h = lo + (int32_t)blockIdx.x; h < hi; h += (int32_t)gridDim.x) {
        if (tid == 0) kept = 0;
        const int64_t hb = poff[h], he = poff[h + 1];
        for (int64_t i = hb + tid; i < he; i += CW) {
            const uint64_t e = plab[i];
            const uint32_t w = (uint32_t)(e >> 32);
            if (w < (uint32_t)h) dc[w] = (uint32_t)e;
        }
        __syncthreads();
        const int64_t base = rlab[2 * (int64_t)h], cnt = rlab[2 * (int64_t)h + 1];
        for (int64_t j = wave; j < cnt; j += CW / 64) {
            const int32_t v = pv[base + j];
            const uint64_t d = (uint32_t)pd[base + j];
            const int64_t vb = poff[v], ve = poff[v + 1];
            bool red = false;
            for (int64_t i0 = vb; i0 < ve; i0 += 64) {
                const int64_t i = i0 + lane;
                if (i < ve) {
                    const uint64_t e = plab[i];
                    const uint32_t w = (uint32_t)(e >> 32);
                    if (w < (uint32_t)h) {
                        const uint32_t a = dc[w];
                        red = a != 0xFFFFFFFFu && (uint64_t)a + (uint32_t)e <= d;
                    }
                }
                if (__ballot(red)) { red = true; break; }
            }
            if (lane == 0) {
                keep[base + j - (int64_t)from] = red ? 0 : 1;
                if (!red) atomicAdd(&kept, 1);
            }
        }
        __syncthreads();
        if (stats && tid == 0) stats[(int64_t)h * STAT_COLS + 2] = kept;
        for (int64_t i = hb + tid; i < he; i += CW) {
            const uint32_t w = (uint32_t)(plab[i] >> 32);
            if (w < (uint32_t)h) dc[w] = 0xFFFFFFFFu;
        }
        __syncthreads();
    }
}

// the kept entries of the pool range, in order, to out (pos: exclusive
// prefix sums of keep)
__global__ void k_compact(uint64_t cnt, const int32_t* __restrict__ keep, const int64_t* __restrict__ pos,
                          const int32_t* __restrict__ pv, const int32_t* __restrict__ ph,
                          const int32_t* __restrict__ pd, int32_t* __restrict__ ov, int32_t* __restrict__ oh,
                          int32_t* __restrict__ od) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (keep[i]) {
            const int64_t q = pos[i];
            ov[q] = pv[i];
            oh[q] = ph[i];
            od[q] = pd[i];
        }
    }
}

int blocks(uint64_t work) {
    uint64_t b = (work + 255) / 256;
    return (int)(b < 1 ? 1 : b > 4096 ? 4096 : b);
}

}  // namespace

// at most 2048 workgroups (8 per CU) and 1 GiB of dense arrays
int clean_workgroups(int32_t nroots, int32_t n) {
    int64_t w = std::min<int64_t>(2048, std::max<int64_t>(1, ((int64_t)1 << 28) / std::max<int32_t>(1, n)));
    return (int)std::max<int64_t>(1, std::min<int64_t>(w, nroots));
}

int launch_clean(int32_t lo, int32_t hi, int32_t n, const int64_t* rlab, const Pool& pool, uint64_t from,
                 const int64_t* poff, const uint64_t* plab, uint32_t* dcbuf, int32_t* keep, int64_t* stats,
                 hipStream_t st) {
    if (hi <= lo) return 0;
    hipLaunchKernelGGL(k_clean, dim3(clean_workgroups(hi - lo, n)), dim3(CW), 0, st, lo, hi, (int64_t)n, rlab,
                       pool.v, pool.dist, poff, plab, dcbuf, from, keep, stats);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_compact(const Pool& pool, uint64_t from, uint64_t cnt, const int32_t* keep, int64_t* pos, void* scan_temp,
                   int32_t* tv, int32_t* th, int32_t* td, hipStream_t st) {
    if (cnt == 0) return 0;
    if (launch_scan_i32_to_i64(keep, pos, (int64_t)cnt, scan_temp, st)) return -1;
    hipLaunchKernelGGL(k_compact, dim3(blocks(cnt)), dim3(256), 0, st, cnt, keep, pos, pool.v + from,
                       pool.hub + from, pool.dist + from, tv, th, td);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace chl
