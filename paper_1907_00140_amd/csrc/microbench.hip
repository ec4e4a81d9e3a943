// Measured ceiling of the relaxation's memory operation: random atomic
// minima on an array the size of the tree slots' keys (roots in flight x n
// keys of 32 or 64 bits). The tree kernels' arc relaxations per second are
// reported against it, beside the HBM bandwidth roofline: no atomic
// throughput is published for the chip.
//
// Every thread draws its addresses and values from its own splitmix64
// sequence; the address is the high half of a 64-bit product (a uniform
// index below `words` without a division).
#include "internal.h"

#include <algorithm>

namespace chl {

namespace {

__device__ __forceinline__ uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename K>
__global__ __launch_bounds__(256) void k_atomic_min(K* __restrict__ buf, uint64_t words, int64_t per_thread,
                                                    uint64_t seed) {
    uint64_t s = seed ^ ((uint64_t)(blockIdx.x * 256u + threadIdx.x) << 20);
    for (int64_t i = 0; i < per_thread; i++) {
        const uint64_t x = splitmix(s);
        const uint64_t idx = (uint64_t)(((unsigned __int128)(x >> 1) * words) >> 63);
        atomicMin(&buf[idx], (K)(x >> 40));
    }
}

}  // namespace

}  // namespace chl

using namespace chl;

extern "C" int chl_microbench_atomic_min(void* buf, int64_t words, int key_bits, int64_t ops, int64_t* done,
                                         double* ms, void* stream) {
    if (!buf || words < 1 || (key_bits != 32 && key_bits != 64) || ops < 1 || !ms || !done)
        return CHL_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();   // the launch below is checked with hipGetLastError
    const int64_t threads = 256 * 8192;
    const int64_t per = std::max<int64_t>(1, ops / threads);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return CHL_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CHL_ERR_HIP;
    }
    int rc = CHL_OK;
    if (hipMemsetAsync(buf, 0xFF, (size_t)words * (key_bits / 8), st) != hipSuccess ||
        hipEventRecord(e0, st) != hipSuccess) {
        rc = CHL_ERR_HIP;
    } else {
        if (key_bits == 32)
            hipLaunchKernelGGL(k_atomic_min<uint32_t>, dim3(8192), dim3(256), 0, st, (uint32_t*)buf, (uint64_t)words,
                               per, 0x5EEDull);
        else
            hipLaunchKernelGGL((k_atomic_min<unsigned long long>), dim3(8192), dim3(256), 0, st,
                               (unsigned long long*)buf, (uint64_t)words, per, 0x5EEDull);
        float t = 0;
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            rc = CHL_ERR_HIP;
        else {
            *ms = t;
            *done = per * threads;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
