// Exclusive prefix sums (int32 or int64 input, int64 output, out[n] = total):
// per-tile sums, a recursive scan of the tile sums, then per-tile scans.
#include "internal.h"

namespace chl {

namespace {

constexpr int SB = 256;            // threads per block
constexpr int SI = 8;              // items per thread
constexpr int TILE = SB * SI;

template <typename T>
__global__ __launch_bounds__(SB) void k_tile_sum(const T* __restrict__ in, int64_t n,
                                                 int64_t* __restrict__ sums) {
    __shared__ int64_t red[SB / 64];
    int64_t base = (int64_t)blockIdx.x * TILE;
    int64_t s = 0;
    for (int i = threadIdx.x; i < TILE; i += SB) {
        int64_t k = base + i;
        if (k < n) s += (int64_t)in[k];
    }
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int i = 0; i < SB / 64; i++) t += red[i];
        sums[blockIdx.x] = t;
    }
}

// scan TILE consecutive items of one block, adding prefix[block]
template <typename T>
__global__ __launch_bounds__(SB) void k_tile_scan(const T* __restrict__ in, int64_t n,
                                                  const int64_t* __restrict__ prefix,
                                                  int64_t* __restrict__ out) {
    __shared__ int64_t wsum[SB / 64];
    const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * SI;
    int64_t v[SI];
    int64_t run = 0;
#pragma unroll
    for (int j = 0; j < SI; j++) {
        int64_t k = base + j;
        v[j] = k < n ? (int64_t)in[k] : 0;
        run += v[j];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t inc = run;
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int64_t wpre = 0;
    for (int i = 0; i < w; i++) wpre += wsum[i];
    int64_t ex = prefix[blockIdx.x] + wpre + inc - run;
#pragma unroll
    for (int j = 0; j < SI; j++) {
        int64_t k = base + j;
        if (k < n) out[k] = ex;
        ex += v[j];
    }
    if (base <= n - 1 && n - 1 < base + SI) out[n] = ex;   // thread holding the last item
}

int64_t ntiles(int64_t n) { return (n + TILE - 1) / TILE; }

template <typename T>
int scan_rec(const T* in, int64_t* out, int64_t n, int64_t* temp, hipStream_t st) {
    if (n == 0) return hipMemsetAsync(out, 0, sizeof(int64_t), st) == hipSuccess ? 0 : -1;
    int64_t nt = ntiles(n);
    int64_t* sums = temp;               // nt
    int64_t* pre = temp + nt;           // nt + 1
    int64_t* rest = temp + 2 * nt + 1;
    hipLaunchKernelGGL((k_tile_sum<T>), dim3(nt), dim3(SB), 0, st, in, n, sums);
    if (nt == 1) {
        hipMemsetAsync(pre, 0, sizeof(int64_t), st);
    } else {
        if (scan_rec<int64_t>(sums, pre, nt, rest, st)) return -1;
    }
    hipLaunchKernelGGL((k_tile_scan<T>), dim3(nt), dim3(SB), 0, st, in, n, pre, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

size_t scan_temp_bytes(int64_t n) {
    size_t words = 2;
    while (true) {
        int64_t nt = ntiles(n);
        words += 2 * nt + 1;
        if (nt <= 1) break;
        n = nt;
    }
    return words * sizeof(int64_t);
}

int launch_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* temp, hipStream_t st) {
    return scan_rec<int64_t>(in, out, n, (int64_t*)temp, st);
}

int launch_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* temp, hipStream_t st) {
    return scan_rec<int32_t>(in, out, n, (int64_t*)temp, st);
}

}  // namespace chl
