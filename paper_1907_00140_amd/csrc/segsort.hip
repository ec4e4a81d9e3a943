// Segmented ascending sort of 64-bit keys: every segment [off[i], off[i+1])
// is sorted on its own. Three tiers by segment length:
//   <= 256     one wave per segment, bitonic network in registers: 1, 2 or 4
//              keys per lane, position e * 64 + lane for the lane's key e;
//              partners 64 or more positions apart sit in the same lane,
//              closer ones are exchanged with lane shuffles;
//   <= LCAP    one 1024-thread block per segment, bitonic network in LDS;
//   larger     one 1024-thread block per segment, bitonic network in global
//              memory.
// A length that is not a power of two is padded with all-ones keys, which
// sort to the end and are not stored. The LDS and global tiers use the form
// of the network in which every comparator moves the smaller key to the lower
// index (the first step of each merge compares mirrored positions), so their
// padding is virtual.
#include "internal.h"

namespace chl {

namespace {

constexpr int LCAP = 8192;
constexpr int BLK = 256;
constexpr int BLKL = 1024;
constexpr int BLKG = 1024;

template <int E>
__device__ __forceinline__ void wave_bitonic(uint64_t (&x)[E], int lane) {
#pragma unroll
    for (int k = 2; k <= 64 * E; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
            if (j >= 64) {
                const int je = j >> 6;
#pragma unroll
                for (int e = 0; e < E; e++) {
                    if (e & je) continue;
                    const bool up = ((e * 64 + lane) & k) == 0;
                    const uint64_t a = x[e], b = x[e | je];
                    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
                    x[e] = up ? lo : hi;
                    x[e | je] = up ? hi : lo;
                }
            } else {
                const bool lower = (lane & j) == 0;
#pragma unroll
                for (int e = 0; e < E; e++) {
                    const uint64_t y = __shfl_xor(x[e], j);
                    const bool up = ((e * 64 + lane) & k) == 0;
                    const uint64_t mn = x[e] < y ? x[e] : y, mx = x[e] < y ? y : x[e];
                    x[e] = (up == lower) ? mn : mx;
                }
            }
        }
    }
}

template <int E>
__device__ __forceinline__ void wave_sort(uint64_t* __restrict__ a, int len, int lane) {
    uint64_t x[E];
#pragma unroll
    for (int e = 0; e < E; e++) x[e] = e * 64 + lane < len ? a[e * 64 + lane] : ~0ull;
    wave_bitonic<E>(x, lane);
#pragma unroll
    for (int e = 0; e < E; e++)
        if (e * 64 + lane < len) a[e * 64 + lane] = x[e];
}

// Segments are dealt out interleaved: with G workers (waves or blocks) of W
// lanes each, worker w checks the segments w + G * (i * W + lane), i = 0, 1,
// ..., so the lengths of W segments are read in one parallel step and the
// long segments, which a rank order clusters at low ids, spread over workers.
__global__ __launch_bounds__(BLK) void k_sort_wave(uint64_t* __restrict__ keys,
                                                   const int64_t* __restrict__ off, int64_t nseg) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * BLK + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * BLK) >> 6;
    for (int64_t i0 = 0; wave + nwaves * i0 < nseg; i0 += 64) {
        const int64_t s = wave + nwaves * (i0 + lane);
        int64_t b = 0;
        int len = 0;
        if (s < nseg) {
            b = off[s];
            const int64_t l = off[s + 1] - b;
            len = l > 256 ? 257 : (int)l;
        }
        uint64_t m = __ballot(len > 1 && len <= 256);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int64_t sb = __shfl(b, src);
            const int sl = __shfl(len, src);
            if (sl <= 64) wave_sort<1>(keys + sb, sl, lane);
            else if (sl <= 128) wave_sort<2>(keys + sb, sl, lane);
            else wave_sort<4>(keys + sb, sl, lane);
        }
    }
}

__device__ __forceinline__ void cas(uint64_t* a, int i, int j) {
    uint64_t x = a[i], y = a[j];
    if (y < x) { a[i] = y; a[j] = x; }
}

__global__ __launch_bounds__(BLKL) void k_sort_lds(uint64_t* __restrict__ keys,
                                                   const int64_t* __restrict__ off, int64_t nseg) {
    __shared__ uint64_t a[LCAP];
    __shared__ int64_t lst[BLKL];
    __shared__ int cnt;
    const int64_t G = gridDim.x;
    for (int64_t i0 = 0; (int64_t)blockIdx.x + G * i0 < nseg; i0 += BLKL) {
        if (threadIdx.x == 0) cnt = 0;
        __syncthreads();
        {
            const int64_t s = (int64_t)blockIdx.x + G * (i0 + threadIdx.x);
            if (s < nseg) {
                const int64_t l = off[s + 1] - off[s];
                if (l > 256 && l <= LCAP) lst[atomicAdd(&cnt, 1)] = s;
            }
        }
        __syncthreads();
        const int c = cnt;
        for (int q = 0; q < c; q++) {
            const int64_t s = lst[q];
            const int64_t b = off[s];
            const int len = (int)(off[s + 1] - b);
            int lp = 9;
            while ((1 << lp) < len) lp++;
            const int p2 = 1 << lp;
            for (int i = threadIdx.x; i < p2; i += BLKL) a[i] = i < len ? keys[b + i] : ~0ull;
            __syncthreads();
            for (int lk = 1; lk <= lp; lk++) {
                const int k = 1 << lk;
                // mirrored step: pairs (i, i ^ (k - 1)) inside blocks of k
                for (int t = threadIdx.x; t < p2 / 2; t += BLKL) {
                    const int i = ((t >> (lk - 1)) << lk) | (t & ((k >> 1) - 1));
                    cas(a, i, i ^ (k - 1));
                }
                __syncthreads();
                for (int lj = lk - 2; lj >= 0; lj--) {
                    const int j = 1 << lj;
                    for (int t = threadIdx.x; t < p2 / 2; t += BLKL) {
                        const int i = ((t >> lj) << (lj + 1)) | (t & (j - 1));
                        cas(a, i, i + j);
                    }
                    __syncthreads();
                }
            }
            for (int i = threadIdx.x; i < len; i += BLKL) keys[b + i] = a[i];
            __syncthreads();
        }
        // every thread has read cnt and lst before the next round resets them
        __syncthreads();
    }
}

__global__ __launch_bounds__(BLKG) void k_sort_global(uint64_t* __restrict__ keys,
                                                      const int64_t* __restrict__ off, int64_t nseg) {
    __shared__ int64_t lst[BLKG];
    __shared__ int cnt;
    const int64_t G = gridDim.x;
    for (int64_t i0 = 0; (int64_t)blockIdx.x + G * i0 < nseg; i0 += BLKG) {
        if (threadIdx.x == 0) cnt = 0;
        __syncthreads();
        {
            const int64_t s = (int64_t)blockIdx.x + G * (i0 + threadIdx.x);
            if (s < nseg && off[s + 1] - off[s] > LCAP) lst[atomicAdd(&cnt, 1)] = s;
        }
        __syncthreads();
        const int c = cnt;
        for (int q = 0; q < c; q++) {
            const int64_t s = lst[q];
            const int64_t b = off[s];
            const int64_t len = off[s + 1] - b;
            uint64_t* a = keys + b;
            int lp = 0;
            while (((int64_t)1 << lp) < len) lp++;
            const int64_t half = (int64_t)1 << (lp - 1);
            for (int lk = 1; lk <= lp; lk++) {
                const int64_t k = (int64_t)1 << lk;
                for (int64_t t = threadIdx.x; t < half; t += BLKG) {
                    const int64_t i = ((t >> (lk - 1)) << lk) | (t & ((k >> 1) - 1));
                    const int64_t j = i ^ (k - 1);
                    if (j < len) {                          // j >= len holds a virtual all-ones key
                        uint64_t x = a[i], y = a[j];
                        if (y < x) { a[i] = y; a[j] = x; }
                    }
                }
                __threadfence_block();
                __syncthreads();
                for (int lj = lk - 2; lj >= 0; lj--) {
                    const int64_t j = (int64_t)1 << lj;
                    for (int64_t t = threadIdx.x; t < half; t += BLKG) {
                        const int64_t i = ((t >> lj) << (lj + 1)) | (t & (j - 1));
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
        __syncthreads();
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
    hipLaunchKernelGGL(k_sort_lds, dim3(grid_cap(nseg < 2048 ? nseg : 2048)), dim3(BLKL), 0, st, keys, off, nseg);
    hipLaunchKernelGGL(k_sort_global, dim3(grid_cap(nseg < 1024 ? nseg : 1024)), dim3(BLKG), 0, st, keys, off, nseg);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace chl
