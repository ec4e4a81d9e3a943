// Segmented ascending sort of 64-bit keys: every segment [off[i], off[i+1])
// is sorted on its own. Three tiers by segment length:
//   <= 64      one wave per segment, bitonic network across the lanes;
//   <= LCAP    one block per segment, bitonic network in LDS;
//   larger     one block per segment, bitonic network in global memory.
// The LDS and global tiers use the form of the bitonic network in which every
// comparator moves the smaller key to the lower index (the first step of each
// merge compares mirrored positions), so a length that is not a power of two
// is handled as if padded with all-ones keys that never move into range.
#include "internal.h"

namespace chl {

namespace {

constexpr int LCAP = 8192;
constexpr int BLK = 256;

__global__ __launch_bounds__(BLK) void k_sort_wave(uint64_t* __restrict__ keys,
                                                   const int64_t* __restrict__ off, int64_t nseg) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * BLK + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * BLK) >> 6;
    for (int64_t s = wave; s < nseg; s += nwaves) {
        const int64_t b = off[s];
        const int len = (int)(off[s + 1] - b);
        if (len <= 1 || len > 64) continue;
        uint64_t x = lane < len ? keys[b + lane] : ~0ull;
        for (int k = 2; k <= 64; k <<= 1) {
            for (int j = k >> 1; j >= 1; j >>= 1) {
                uint64_t y = __shfl_xor(x, j);
                bool up = (lane & k) == 0;            // ascending half
                bool lower = (lane & j) == 0;
                uint64_t mn = x < y ? x : y, mx = x < y ? y : x;
                x = (up == lower) ? mn : mx;
            }
        }
        if (lane < len) keys[b + lane] = x;
    }
}

__device__ __forceinline__ void cas(uint64_t* a, int i, int j) {
    uint64_t x = a[i], y = a[j];
    if (y < x) { a[i] = y; a[j] = x; }
}

__global__ __launch_bounds__(BLK) void k_sort_lds(uint64_t* __restrict__ keys,
                                                  const int64_t* __restrict__ off, int64_t nseg) {
    __shared__ uint64_t a[LCAP];
    for (int64_t s = blockIdx.x; s < nseg; s += gridDim.x) {
        const int64_t b = off[s];
        const int len = (int)(off[s + 1] - b);
        if (len <= 64 || len > LCAP) continue;
        int p2 = 128;
        while (p2 < len) p2 <<= 1;
        for (int i = threadIdx.x; i < p2; i += BLK) a[i] = i < len ? keys[b + i] : ~0ull;
        __syncthreads();
        for (int k = 2; k <= p2; k <<= 1) {
            // mirrored step: pairs (i, i ^ (k - 1)) inside blocks of k
            for (int t = threadIdx.x; t < p2 / 2; t += BLK) {
                int i = (t / (k >> 1)) * k + (t % (k >> 1));
                int j = i ^ (k - 1);
                cas(a, i, j);
            }
            __syncthreads();
            for (int j = k >> 2; j >= 1; j >>= 1) {
                for (int t = threadIdx.x; t < p2 / 2; t += BLK) {
                    int i = (t / j) * 2 * j + (t % j);
                    cas(a, i, i + j);
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < len; i += BLK) keys[b + i] = a[i];
        __syncthreads();
    }
}

__global__ __launch_bounds__(BLK) void k_sort_global(uint64_t* __restrict__ keys,
                                                     const int64_t* __restrict__ off, int64_t nseg) {
    for (int64_t s = blockIdx.x; s < nseg; s += gridDim.x) {
        const int64_t b = off[s];
        const int64_t len = off[s + 1] - b;
        if (len <= LCAP) continue;
        uint64_t* a = keys + b;
        int64_t p2 = 1;
        while (p2 < len) p2 <<= 1;
        for (int64_t k = 2; k <= p2; k <<= 1) {
            for (int64_t t = threadIdx.x; t < p2 / 2; t += BLK) {
                int64_t i = (t / (k >> 1)) * k + (t % (k >> 1));
                int64_t j = i ^ (k - 1);
                if (j < len) {                          // j >= len holds a virtual all-ones key
                    uint64_t x = a[i], y = a[j];
                    if (y < x) { a[i] = y; a[j] = x; }
                }
            }
            __threadfence_block();
            __syncthreads();
            for (int64_t j = k >> 2; j >= 1; j >>= 1) {
                for (int64_t t = threadIdx.x; t < p2 / 2; t += BLK) {
                    int64_t i = (t / j) * 2 * j + (t % j);
                    if (i + j < len) {
                        uint64_t x = a[i], y = a[i + j];
                        if (y < x) { a[i] = y; a[i + j] = x; }
                    }
                }
                __threadfence_block();
                __syncthreads();
            }
        }
    }
}

int grid_cap(int64_t work) {
    int64_t g = work < 1 ? 1 : work;
    return (int)(g > 4096 ? 4096 : g);   // grid-stride kernels
}

}  // namespace

size_t segsort_temp_bytes(int64_t) { return 0; }

int launch_segsort_u64(uint64_t* keys, const int64_t* off, int64_t nseg, int64_t total, void*,
                       hipStream_t st) {
    if (nseg <= 0 || total <= 1) return 0;
    hipLaunchKernelGGL(k_sort_wave, dim3(grid_cap((nseg + 3) / 4)), dim3(BLK), 0, st, keys, off, nseg);
    hipLaunchKernelGGL(k_sort_lds, dim3(grid_cap(nseg < 8192 ? nseg : 8192)), dim3(BLK), 0, st, keys, off, nseg);
    hipLaunchKernelGGL(k_sort_global, dim3(grid_cap(nseg < 1024 ? nseg : 1024)), dim3(BLK), 0, st, keys, off, nseg);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace chl
