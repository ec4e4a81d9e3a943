// Input validation and rank renumbering of the CSR.
//
// After renumbering, vertex id = rank position (order[0] -> 0, the most
// important vertex; the paper's tree of v is built n - R(v)-th, Section 4.1),
// so "u outranks h" is the integer comparison u < h, a root's hub id is its
// index, and high-rank hubs are contiguous. Each renumbered row is sorted by
// (neighbour, weight) and stored as one 64-bit word per arc,
// (neighbour << 32) | weight, so the tree kernels read an arc with a single
// 8-byte load.
#include "internal.h"

#include <algorithm>

namespace chl {

namespace {

__global__ void k_order(int32_t n, const int32_t* __restrict__ order, int32_t* __restrict__ pos,
                        int32_t* __restrict__ cnt, int32_t* err) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t o = order[i];
        if (o < 0 || o >= n) { atomicOr(err, ERR_BIT_INVALID); continue; }
        atomicAdd(&cnt[o], 1);
        pos[o] = (int32_t)i;
    }
}

__global__ void k_rows(int32_t n, int64_t m, const int64_t* __restrict__ row,
                       const int32_t* __restrict__ cnt, int32_t* err) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n;
         v += (int64_t)gridDim.x * blockDim.x) {
        bool bad = false;
        if (v == 0) bad |= row[0] != 0;
        if (v == n) bad |= row[n] != m;
        if (v < n) bad |= row[v + 1] < row[v] || cnt[v] != 1;
        if (bad) atomicOr(err, ERR_BIT_INVALID);
    }
}

// 256 threads per block; one atomic per block on the shared maximum
__global__ void k_arcs(int32_t n, int64_t m, const int32_t* __restrict__ col,
                       const int32_t* __restrict__ w, int32_t* err, int32_t* maxw) {
    __shared__ int32_t red[4];
    int32_t mx = 0;
    bool bad = false;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t c = col[e], x = w[e];
        bad |= c < 0 || c >= n || x < 1;
        mx = max(mx, x);
    }
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(maxw, max(max(red[0], red[1]), max(red[2], red[3])));
    if (bad) atomicOr(err, ERR_BIT_INVALID);
}

__global__ void k_rdeg(int32_t n, const int64_t* __restrict__ row, const int32_t* __restrict__ order,
                       int64_t* __restrict__ rdeg) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = order[p];
        rdeg[p] = row[v + 1] - row[v];
    }
}

// one wave per renumbered row
__global__ void k_copy(int32_t n, const int64_t* __restrict__ row, const int32_t* __restrict__ col,
                       const int32_t* __restrict__ w, const int32_t* __restrict__ order,
                       const int32_t* __restrict__ pos, const int64_t* __restrict__ rrow,
                       uint64_t* __restrict__ rarc) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p = wave; p < n; p += nwaves) {
        int32_t v = order[p];
        int64_t b = row[v], e = row[v + 1], o = rrow[p];
        for (int64_t i = b + lane; i < e; i += 64)
            rarc[o + (i - b)] = ((uint64_t)(uint32_t)pos[col[i]] << 32) | (uint32_t)w[i];
    }
}

__device__ __forceinline__ int64_t lower(const uint64_t* a, int64_t lo, int64_t hi, uint64_t k) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// every arc (p, u, w) must be matched by as many (u, p, w) as there are
// (p, u, w): rows are sorted, so both counts are run lengths found by binary
// search. One thread per arc (the first of its run does the check), so that
// long rows spread over many threads; its row is found by binary search in
// the row offsets.
__global__ void k_sym(int32_t n, int64_t m, const int64_t* __restrict__ rrow, const uint64_t* __restrict__ rarc,
                      int32_t* err) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        // row p of arc i: the last p with rrow[p] <= i
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (rrow[mid] <= i) lo = mid; else hi = mid - 1;
        }
        const int64_t p = lo, b = rrow[p], e = rrow[p + 1];
        const uint64_t k = rarc[i];
        if (i > b && rarc[i - 1] == k) continue;          // first of its run only
        int64_t c1 = 1;
        while (i + c1 < e && rarc[i + c1] == k) c1++;
        const uint32_t u = (uint32_t)(k >> 32);
        const uint64_t kr = ((uint64_t)(uint32_t)p << 32) | (uint32_t)k;
        int64_t l = lower(rarc, rrow[u], rrow[u + 1], kr);
        int64_t c2 = 0;
        while (l + c2 < rrow[u + 1] && rarc[l + c2] == kr) c2++;
        bad |= c1 != c2;
    }
    if (bad) atomicOr(err, ERR_BIT_INVALID);
}

// reversed graph: in-degree counts, then one wave per row scatters its
// arcs v -> u as (v << 32) | w into row u (positions from a per-row cursor),
// a segmented sort orders each row, and k_tsplit unpacks the words
__global__ void k_indeg(int64_t m, const int32_t* __restrict__ col, int32_t* __restrict__ cnt) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[col[e]], 1);
}

__global__ void k_tscatter(int32_t n, const int64_t* __restrict__ row, const int32_t* __restrict__ col,
                           const int32_t* __restrict__ w, unsigned long long* __restrict__ cursor,
                           uint64_t* __restrict__ tkey) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += nwaves)
        for (int64_t e = row[v] + lane; e < row[v + 1]; e += 64) {
            const unsigned long long p = atomicAdd(&cursor[col[e]], 1ull);
            tkey[p] = ((uint64_t)(uint32_t)v << 32) | (uint32_t)w[e];
        }
}

__global__ void k_tsplit(int64_t m, const uint64_t* __restrict__ tkey, int32_t* __restrict__ tcol,
                         int32_t* __restrict__ tw) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = tkey[e];
        tcol[e] = (int32_t)(k >> 32);
        tw[e] = (int32_t)(uint32_t)k;
    }
}

// combined graph of a directed build: vertices [0, n) are the graph's,
// [n, 2n) their reversed copies (row n + v = the reversed row v, its
// neighbours shifted by n); ranking interleaved, order2[2i] = order[i],
// order2[2i + 1] = order[i] + n
__global__ void k_dunion(int32_t n, int64_t m, const int64_t* __restrict__ row, const int32_t* __restrict__ col,
                         const int32_t* __restrict__ w, const int32_t* __restrict__ order,
                         const int64_t* __restrict__ trow, const int32_t* __restrict__ tcol,
                         const int32_t* __restrict__ tw, int64_t* __restrict__ row2, int32_t* __restrict__ col2,
                         int32_t* __restrict__ w2, int32_t* __restrict__ order2) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t v = t0; v <= n; v += stride) {
        row2[v] = row[v];
        row2[n + v] = m + trow[v];
    }
    for (int64_t v = t0; v < n; v += stride) {
        order2[2 * v] = order[v];
        order2[2 * v + 1] = order[v] + n;
    }
    for (int64_t e = t0; e < m; e += stride) {
        col2[e] = col[e];
        w2[e] = w[e];
        col2[m + e] = tcol[e] + n;
        w2[m + e] = tw[e];
    }
}

// labels of the combined graph back to the two sets: in-labels are those of
// vertices [0, n) (kept in place, hub positions halved), out-labels those of
// [n, 2n) (copied out, hub positions halved)
__global__ void k_dsplit(int32_t n, const int64_t* __restrict__ off2, int32_t* __restrict__ hub2,
                         const int32_t* __restrict__ dist2, int64_t* __restrict__ out_off,
                         int32_t* __restrict__ out_hub, int32_t* __restrict__ out_dist) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tin = off2[n], tall = off2[2 * (int64_t)n];
    for (int64_t v = t0; v <= n; v += stride) out_off[v] = off2[n + v] - tin;
    for (int64_t i = t0; i < tall; i += stride) {
        const int32_t hp = hub2[i] >> 1;
        if (i < tin) {
            hub2[i] = hp;
        } else {
            out_hub[i - tin] = hp;
            out_dist[i - tin] = dist2[i];
        }
    }
}

int grid_for(int64_t work, int block) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;   // grid-stride kernels: 16 blocks per CU
    return (int)g;
}

}  // namespace

int launch_validate(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                    const int32_t* w, const int32_t* order, int32_t* pos, int32_t* cnt,
                    int32_t* err, int32_t* maxw, hipStream_t st) {
    hipLaunchKernelGGL(k_order, dim3(grid_for(n, 256)), dim3(256), 0, st, n, order, pos, cnt, err);
    hipLaunchKernelGGL(k_rows, dim3(grid_for((int64_t)n + 1, 256)), dim3(256), 0, st, n, m, row_ptr, cnt, err);
    if (m > 0)
        hipLaunchKernelGGL(k_arcs, dim3(grid_for(m, 256) < 2048 ? grid_for(m, 256) : 2048), dim3(256), 0, st, n, m,
                           col, w, err, maxw);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_renumber(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                    const int32_t* w, const int32_t* order, const int32_t* pos,
                    int64_t* rrow, uint64_t* rarc, hipStream_t st) {
    // rrow is first filled with degrees (in rank order) by the caller's scan
    (void)m;
    hipLaunchKernelGGL(k_copy, dim3(grid_for((int64_t)n * 64, 256)), dim3(256), 0, st, n, row_ptr, col,
                       w, order, pos, rrow, rarc);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_rank_degrees(int32_t n, const int64_t* row_ptr, const int32_t* order, int64_t* rdeg,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_rdeg, dim3(grid_for(n, 256)), dim3(256), 0, st, n, row_ptr, order, rdeg);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// 16 row offsets, ranking entries, neighbours and weights at fixed positions
// of the input (the signature that keys the tuning caches).
__global__ void k_sample(int32_t n, int64_t m, const int64_t* __restrict__ row, const int32_t* __restrict__ col,
                         const int32_t* __restrict__ w, const int32_t* __restrict__ order, int64_t* __restrict__ out) {
    const int i = threadIdx.x;
    if (i < 16) {
        const int64_t v = (int64_t)n * i / 16;
        const int64_t e = m ? m * i / 16 : 0;
        out[4 * i] = row[v];
        out[4 * i + 1] = order[v];
        out[4 * i + 2] = m ? col[e] : 0;
        out[4 * i + 3] = m ? w[e] : 0;
    }
}

int launch_sample_input(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                        const int32_t* order, int64_t* out, hipStream_t st) {
    if (n <= 0) return -1;
    hipLaunchKernelGGL(k_sample, dim3(1), dim3(64), 0, st, n, m, row_ptr, col, w, order, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_transpose(int32_t n, int64_t m, const int64_t* row, const int32_t* col, const int32_t* w,
                     int32_t* cnt, int64_t* trow, unsigned long long* cursor, uint64_t* tkey,
                     int32_t* tcol, int32_t* tw, void* scan_temp, hipStream_t st) {
    if (hipMemsetAsync(cnt, 0, (size_t)n * 4, st) != hipSuccess) return -1;
    if (m > 0) hipLaunchKernelGGL(k_indeg, dim3(grid_for(m, 256)), dim3(256), 0, st, m, col, cnt);
    if (launch_scan_i32_to_i64(cnt, trow, n, scan_temp, st)) return -1;
    if (hipMemcpyAsync(cursor, trow, (size_t)n * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) return -1;
    if (m > 0) {
        hipLaunchKernelGGL(k_tscatter, dim3(grid_for((int64_t)n * 64, 256)), dim3(256), 0, st, n, row, col, w,
                           cursor, tkey);
        if (launch_segsort_u64(tkey, trow, n, m, nullptr, st)) return -1;
        hipLaunchKernelGGL(k_tsplit, dim3(grid_for(m, 256)), dim3(256), 0, st, m, tkey, tcol, tw);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_directed_union(int32_t n, int64_t m, const int64_t* row, const int32_t* col, const int32_t* w,
                          const int32_t* order, const int64_t* trow, const int32_t* tcol, const int32_t* tw,
                          int64_t* row2, int32_t* col2, int32_t* w2, int32_t* order2, hipStream_t st) {
    hipLaunchKernelGGL(k_dunion, dim3(grid_for(std::max<int64_t>(m, (int64_t)n + 1), 256)), dim3(256), 0, st, n, m,
                       row, col, w, order, trow, tcol, tw, row2, col2, w2, order2);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_directed_split(int32_t n, int64_t total, const int64_t* off2, int32_t* hub2, const int32_t* dist2,
                          int64_t* out_off, int32_t* out_hub, int32_t* out_dist, hipStream_t st) {
    hipLaunchKernelGGL(k_dsplit, dim3(grid_for(std::max<int64_t>(total, (int64_t)n + 1), 256)), dim3(256), 0, st,
                       n, off2, hub2, dist2, out_off, out_hub, out_dist);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_check_symmetric(int32_t n, int64_t m, const int64_t* rrow, const uint64_t* rarc, int32_t* err,
                           hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(k_sym, dim3(grid_for(m, 256)), dim3(256), 0, st, n, m, rrow, rarc, err);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace chl
