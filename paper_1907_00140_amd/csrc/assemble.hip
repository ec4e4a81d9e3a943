// Label assembly: from the pool written by the trees (one entry per label,
// in the order the trees finished) to one list per vertex, sorted by hub
// rank position, most important hub first (the sort step of Algorithm 2;
// the merge query of Section 5 needs it). Count labels per vertex (input
// id), exclusive scan into offsets, scatter (hub << 32 | dist) words into
// their vertex's segment, sort every segment, split into hub_pos / dist.
// Hubs inside one L_v are distinct, so the sorted order is unique whatever
// order the trees finished in.
#include "internal.h"

namespace chl {

namespace {

__global__ void k_zero32(int32_t* a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

__global__ void k_count(const int32_t* __restrict__ pv, uint64_t total, const int32_t* __restrict__ order,
                        int32_t* __restrict__ count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&count[order ? order[pv[i]] : pv[i]], 1);
}

__global__ void k_scatter(const int32_t* __restrict__ pv, const int32_t* __restrict__ ph,
                          const int32_t* __restrict__ pd, uint64_t total, const int32_t* __restrict__ order,
                          const int64_t* __restrict__ offsets, int32_t* __restrict__ fill,
                          uint64_t* __restrict__ tmp) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        int32_t v = order ? order[pv[i]] : pv[i];
        int64_t p = offsets[v] + atomicAdd(&fill[v], 1);
        tmp[p] = ((uint64_t)(uint32_t)ph[i] << 32) | (uint32_t)pd[i];
    }
}

__global__ void k_split(const uint64_t* __restrict__ tmp, uint64_t total, int32_t* __restrict__ hub,
                        int32_t* __restrict__ dist) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t x = tmp[i];
        hub[i] = (int32_t)(x >> 32);
        dist[i] = (int32_t)(uint32_t)x;
    }
}

int g(uint64_t work) {
    uint64_t b = (work + 255) / 256;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;   // grid-stride: 16 blocks per CU saturate HBM and leave room for other streams
    return (int)b;
}

}  // namespace

int launch_assemble(int32_t n, const int32_t* order, const Pool& pool, uint64_t total,
                    int32_t* count, int64_t* offsets, int32_t* fill, uint64_t* tmp,
                    int32_t* hub_pos, int32_t* dist, void* scan_temp, void* sort_temp,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_zero32, dim3(g(n)), dim3(256), 0, st, count, (int64_t)n);
    hipLaunchKernelGGL(k_zero32, dim3(g(n)), dim3(256), 0, st, fill, (int64_t)n);
    if (total > 0)
        hipLaunchKernelGGL(k_count, dim3(g(total)), dim3(256), 0, st, pool.v, total, order, count);
    if (launch_scan_i32_to_i64(count, offsets, n, scan_temp, st)) return -1;
    if (total > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(g(total)), dim3(256), 0, st, pool.v, pool.hub, pool.dist, total,
                           order, offsets, fill, tmp);
        if (launch_segsort_u64(tmp, offsets, n, (int64_t)total, sort_temp, st)) return -1;
        hipLaunchKernelGGL(k_split, dim3(g(total)), dim3(256), 0, st, tmp, total, hub_pos, dist);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Totals of the per-root statistics columns 0 (settled), 1 (arcs) and 3
// (stopped early) into sums[0..2]; 256 threads per block, one atomic per
// block and column.
__global__ void k_stat_sums(int32_t n, const int64_t* __restrict__ st, unsigned long long* __restrict__ sums) {
    __shared__ unsigned long long red[3][4];
    unsigned long long a = 0, b = 0, c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a += (unsigned long long)st[i * STAT_COLS];
        b += (unsigned long long)st[i * STAT_COLS + 1];
        c += (unsigned long long)st[i * STAT_COLS + 3];
    }
    for (int d = 32; d >= 1; d >>= 1) {
        a += __shfl_xor(a, d);
        b += __shfl_xor(b, d);
        c += __shfl_xor(c, d);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][w] = a; red[1][w] = b; red[2][w] = c; }
    __syncthreads();
    if (threadIdx.x < 3) {
        const unsigned long long t = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        if (t) atomicAdd(&sums[threadIdx.x], t);
    }
}

int launch_stat_sums(int32_t n, const int64_t* stats, int64_t* sums, hipStream_t st) {
    int grid = (int)std::min<int64_t>(1024, ((int64_t)n + 255) / 256);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_stat_sums, dim3(grid), dim3(256), 0, st, n, stats, (unsigned long long*)sums);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Roots among the rank positions [lo, lo + cnt) whose tree is the root
// alone. A root r without arcs settles only itself; a root all of whose
// neighbours outrank it (rank positions below r: the last arc of r's row,
// sorted by target, has a smaller target) reaches every other vertex
// through a neighbour that outranks it, so Algorithm 3 flags every vertex
// but r and the tree stops at once. Either way r's only label is (r, r, 0):
// flag[i] = 1 (no arcs) or 2 (neighbours all outrank r) marks them, and
// after the scan k_trivial_split writes their labels to the pool (from entry
// base on, in rank order) and their statistics rows, and lists the other
// roots, in rank order, for the tree kernels.
__global__ void k_trivial_flags(int32_t lo, int32_t cnt, const int64_t* __restrict__ row,
                                const uint64_t* __restrict__ arc, int32_t* __restrict__ flag) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const int32_t r = lo + i;
        const int64_t b = row[r], e = row[(int64_t)r + 1];
        flag[i] = b == e ? 1 : (int32_t)(arc[e - 1] >> 32) < r ? 2 : 0;
    }
}

__global__ void k_trivial_mark(int32_t cnt, const int32_t* __restrict__ flag, int32_t* __restrict__ one) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
        one[i] = flag[i] != 0 ? 1 : 0;
}

__global__ void k_trivial_split(int32_t lo, int32_t cnt, const int32_t* __restrict__ flag,
                                const int64_t* __restrict__ pos, int32_t* __restrict__ pv, int32_t* __restrict__ ph,
                                int32_t* __restrict__ pd, uint64_t base, int32_t* __restrict__ roots,
                                int64_t* __restrict__ stats) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const int32_t r = lo + i;
        const int64_t q = pos[i];
        if (flag[i]) {
            pv[base + q] = r;
            ph[base + q] = r;
            pd[base + q] = 0;
            if (stats) {
                // settled, arcs relaxed, labels, stopped early (no tree was
                // grown, so none), rounds, ticks
                int64_t* sr = stats + (int64_t)r * STAT_COLS;
                sr[0] = 1;
                sr[1] = 0;
                sr[2] = 1;
                sr[3] = 0;
                sr[4] = 1;
                sr[5] = 0;
            }
        } else {
            roots[i - q] = r;
        }
    }
}

int launch_trivial_count(int32_t lo, int32_t cnt, const int64_t* row, const uint64_t* arc, int32_t* flag,
                         int32_t* one, int64_t* pos, void* scan_temp, hipStream_t st) {
    if (cnt <= 0) return 0;
    const int blocks = (int)std::min<int64_t>(4096, ((int64_t)cnt + 255) / 256);
    hipLaunchKernelGGL(k_trivial_flags, dim3(blocks), dim3(256), 0, st, lo, cnt, row, arc, flag);
    hipLaunchKernelGGL(k_trivial_mark, dim3(blocks), dim3(256), 0, st, cnt, flag, one);
    if (hipGetLastError() != hipSuccess) return -1;
    return launch_scan_i32_to_i64(one, pos, cnt, scan_temp, st);
}

int launch_trivial_split(int32_t lo, int32_t cnt, const int32_t* flag, const int64_t* pos, const Pool& pool,
                         uint64_t base, int32_t* roots, int64_t* stats, hipStream_t st) {
    if (cnt <= 0) return 0;
    const int blocks = (int)std::min<int64_t>(4096, ((int64_t)cnt + 255) / 256);
    hipLaunchKernelGGL(k_trivial_split, dim3(blocks), dim3(256), 0, st, lo, cnt, flag, pos, pool.v, pool.hub,
                       pool.dist, base, roots, stats);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// fill[v] = size of v's old group (0 without old groups)
__global__ void k_old_sizes(int32_t n, const int64_t* __restrict__ off_old, int32_t* __restrict__ fill) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        fill[v] = off_old ? (int32_t)(off_old[v + 1] - off_old[v]) : 0;
}

// one wave per vertex: its old group to the front of its new group
__global__ void k_move_groups(int32_t n, const int64_t* __restrict__ off_old, const uint64_t* __restrict__ lab_old,
                              const int64_t* __restrict__ off_new, uint64_t* __restrict__ lab_new) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += nwaves) {
        const int64_t b = off_old[v], e = off_old[v + 1], o = off_new[v];
        for (int64_t i = b + lane; i < e; i += 64) lab_new[o + (i - b)] = lab_old[i];
    }
}

// sort key of root h of a level: (2^32 - 1 - its prefix-label count) << 32 | h
__global__ void k_level_keys(const int64_t* __restrict__ poff, int32_t g, int32_t g2, int32_t partner,
                             uint64_t* __restrict__ keys, int64_t* __restrict__ off2) {
    const int32_t nr = g2 - g;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += gridDim.x * blockDim.x) {
        const int32_t h = g + i;
        int32_t hp = h ^ partner;
        if (hp < g || hp >= g2) hp = h;
        const uint32_t size = (uint32_t)(poff[hp + 1] - poff[hp]);
        keys[i] = ((uint64_t)(0xFFFFFFFFu - size) << 32) | (uint32_t)h;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        off2[0] = 0;
        off2[1] = nr;
    }
}

__global__ void k_level_roots(const uint64_t* __restrict__ keys, int32_t nr, int32_t* __restrict__ roots) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += gridDim.x * blockDim.x)
        roots[i] = (int32_t)(uint32_t)keys[i];
}

int launch_level_order(const int64_t* poff, int32_t g, int32_t g2, int32_t partner, uint64_t* keys,
                       int64_t* off2, int32_t* roots, hipStream_t st) {
    const int32_t nr = g2 - g;
    if (nr <= 0) return 0;
    const int blocks = (nr + 255) / 256 < 1024 ? (nr + 255) / 256 : 1024;
    hipLaunchKernelGGL(k_level_keys, dim3(blocks), dim3(256), 0, st, poff, g, g2, partner, keys, off2);
    if (launch_segsort_u64(keys, off2, 1, nr, nullptr, st)) return -1;
    hipLaunchKernelGGL(k_level_roots, dim3(blocks), dim3(256), 0, st, keys, nr, roots);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void k_group_min(const int32_t* __restrict__ pv, const int32_t* __restrict__ pd, uint64_t cnt,
                            uint32_t* __restrict__ pmin) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
         i += (uint64_t)gridDim.x * blockDim.x)
        atomicMin(&pmin[pv[i]], (uint32_t)pd[i]);
}

int launch_group_min(const Pool& pool, uint64_t from, uint64_t to, uint32_t* pmin, hipStream_t st) {
    if (to <= from) return 0;
    hipLaunchKernelGGL(k_group_min, dim3(g(to - from)), dim3(256), 0, st, pool.v + from, pool.dist + from, to - from,
                       pmin);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void k_swap_halves(const uint64_t* __restrict__ in, uint64_t* __restrict__ out, uint64_t total) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = in[i];
        out[i] = (x << 32) | (x >> 32);
    }
}

int launch_swap_halves(const uint64_t* in, uint64_t* out, uint64_t total, hipStream_t st) {
    if (!total) return 0;
    hipLaunchKernelGGL(k_swap_halves, dim3(g(total)), dim3(256), 0, st, in, out, total);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_group_sizes(int32_t n, const int64_t* off, int32_t* count, hipStream_t st) {
    hipLaunchKernelGGL(k_old_sizes, dim3(g(n)), dim3(256), 0, st, n, off, count);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prefix_extend(int32_t n, const Pool& pool, uint64_t from, uint64_t used, int32_t* count,
                         const int64_t* off_old, const uint64_t* lab_old, int64_t* off_new, uint64_t* lab_new,
                         int32_t* fill, void* scan_temp, hipStream_t st) {
    if (!off_old) hipLaunchKernelGGL(k_zero32, dim3(g(n)), dim3(256), 0, st, count, (int64_t)n);
    const uint64_t add = used - from;
    if (add > 0)
        hipLaunchKernelGGL(k_count, dim3(g(add)), dim3(256), 0, st, pool.v + from, add, (const int32_t*)nullptr,
                           count);
    if (launch_scan_i32_to_i64(count, off_new, n, scan_temp, st)) return -1;
    hipLaunchKernelGGL(k_old_sizes, dim3(g(n)), dim3(256), 0, st, n, off_old, fill);
    if (off_old)
        hipLaunchKernelGGL(k_move_groups, dim3(g((uint64_t)n * 64)), dim3(256), 0, st, n, off_old, lab_old, off_new,
                           lab_new);
    if (add > 0)
        hipLaunchKernelGGL(k_scatter, dim3(g(add)), dim3(256), 0, st, pool.v + from, pool.hub + from,
                           pool.dist + from, add, (const int32_t*)nullptr, off_new, fill, lab_new);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace chl
