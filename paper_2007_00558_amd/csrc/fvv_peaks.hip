// fvv_peaks.hip -- measured machine peaks for the roofline of the plain
// path: achievable HBM copy bandwidth and 64-bit atomicMin rates (global
// memory at distinct and at contended addresses, LDS at conflict-free
// addresses and at scattered addresses of one tile window), the operations
// the splat and the binning are built from.  Each figure is the best of a
// few timed launches (HIP events) after a warm-up launch.
#include <algorithm>
#include <string>

#include "fvv_internal.h"

namespace {

constexpr int PK_THREADS = 256;

// grid-stride copy of n 16-byte words, four independent words per step
__global__ void __launch_bounds__(PK_THREADS) k_pk_copy(const uint4 *__restrict__ a, uint4 *__restrict__ b, size_t n)
{
    const size_t nt = (size_t)gridDim.x * PK_THREADS;
    size_t i = (size_t)blockIdx.x * PK_THREADS + threadIdx.x;
    for (; i + 3 * nt < n; i += 4 * nt) {
        const uint4 x0 = a[i], x1 = a[i + nt], x2 = a[i + 2 * nt], x3 = a[i + 3 * nt];
        b[i] = x0;
        b[i + nt] = x1;
        b[i + 2 * nt] = x2;
        b[i + 3 * nt] = x3;
    }
    for (; i < n; i += nt) b[i] = a[i];
}

__device__ __forceinline__ unsigned long long pk_key(uint32_t a, uint32_t b)
{
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    return ((unsigned long long)(0x3F800000u + (h & 0xFFFFFu)) << 32) | h;
}

// global 64-bit atomicMin, no return value used.  distinct: lane-consecutive
// words, a fresh word for every operation (n >= threads * reps); contended:
// the 64 lanes of a wave on one word.
template <bool CONTENDED>
__global__ void __launch_bounds__(PK_THREADS) k_pk_gatomic(unsigned long long *__restrict__ z, size_t n, int reps)
{
    const size_t nt = (size_t)gridDim.x * PK_THREADS;
    const size_t tid = (size_t)blockIdx.x * PK_THREADS + threadIdx.x;
    for (int r = 0; r < reps; ++r) {
        const size_t i = CONTENDED ? (tid >> 6) + (size_t)r * (nt >> 6) : tid + (size_t)r * nt;
        if (i < n) atomicMin(z + i, pk_key((uint32_t)tid, (uint32_t)r));
    }
}

// LDS 64-bit atomicMin over a 34 x 34 key window (the tile kernel's
// z-buffer), eight waves per window.  distinct: lane l of wave w on word
// 64 w + l (no bank conflicts); scattered: pseudo-random words of the
// window (the splat's case: lanes of a wave land on nearby, overlapping
// footprints).  The window is reduced to one store so the atomics stay.
template <bool SCATTER>
__global__ void __launch_bounds__(PK_THREADS) k_pk_latomic(unsigned long long *__restrict__ sink, int reps)
{
    constexpr int NW = 34 * 34;
    __shared__ unsigned long long zk[NW];
    for (int e = threadIdx.x; e < NW; e += PK_THREADS) zk[e] = ~0ull;
    __syncthreads();
    const uint32_t t = threadIdx.x;
    uint32_t h = (blockIdx.x * PK_THREADS + t) * 0x9E3779B1u + 1u;
    for (int r = 0; r < reps; ++r) {
        uint32_t idx;
        if (SCATTER) {
            h ^= h << 13;
            h ^= h >> 17;
            h ^= h << 5;
            idx = h % NW;
        } else {
            idx = (t + (uint32_t)r * 256u) % (uint32_t)NW;
        }
        atomicMin(&zk[idx], pk_key(t, (uint32_t)r));
    }
    __syncthreads();
    if (t == 0) {
        unsigned long long m = ~0ull;
        for (int e = 0; e < NW; ++e) m = min(m, zk[e]);
        sink[blockIdx.x] = m;
    }
}

// best of `reps` timed launches of fn, in milliseconds
template <typename F>
hipError_t best_ms(F fn, int reps, float &best)
{
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    best = 1e30f;
    fn();   // warm-up
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        (void)hipEventRecord(e0, nullptr);
        fn();
        (void)hipEventRecord(e1, nullptr);
        if ((e = hipEventSynchronize(e1)) == hipSuccess && (e = hipGetLastError()) == hipSuccess) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, ms);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
}

}  // namespace

// out[0] copy GB/s (bytes read + written), out[1] global atomicMin/s at
// distinct addresses, out[2] at one address per wave, out[3] LDS
// atomicMin/s conflict-free, out[4] LDS atomicMin/s scattered over a tile
// window.  Runs on the current device with the null stream.
hipError_t fvv_measure_peaks_impl(double *out, std::string &err)
{
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t copy_bytes = (size_t)1 << 30;
    const size_t n16 = copy_bytes / 16;
    uint8_t *buf = nullptr;
    if ((e = hipMalloc((void **)&buf, 2 * copy_bytes)) != hipSuccess) {
        err = "device buffers for the copy";
        return e;
    }
    if ((e = hipMemset(buf, 1, 2 * copy_bytes)) != hipSuccess) {
        (void)hipFree(buf);
        return e;
    }
    float ms = 0.f;
    const int copy_blocks = cus * 16;
    e = best_ms([&] {
        hipLaunchKernelGGL(k_pk_copy, dim3(copy_blocks), dim3(PK_THREADS), 0, nullptr, (const uint4 *)buf,
                           (uint4 *)(buf + copy_bytes), n16);
    }, 5, ms);
    if (e == hipSuccess) out[0] = 2.0 * (double)copy_bytes / (ms * 1e-3) / 1e9;
    // global atomics: 1 M threads x 16 operations over 16 M words (128 MiB)
    const int g_blocks = 4096, g_reps = 16;
    const size_t g_words = (size_t)g_blocks * PK_THREADS * g_reps;
    unsigned long long *z = (unsigned long long *)buf;
    if (e == hipSuccess) e = hipMemset(z, 0xFF, g_words * 8);
    if (e == hipSuccess)
        e = best_ms([&] {
            hipLaunchKernelGGL((k_pk_gatomic<false>), dim3(g_blocks), dim3(PK_THREADS), 0, nullptr, z, g_words, g_reps);
        }, 5, ms);
    if (e == hipSuccess) out[1] = (double)g_words / (ms * 1e-3);
    if (e == hipSuccess)
        e = best_ms([&] {
            hipLaunchKernelGGL((k_pk_gatomic<true>), dim3(g_blocks), dim3(PK_THREADS), 0, nullptr, z, g_words, g_reps);
        }, 5, ms);
    if (e == hipSuccess) out[2] = (double)g_words / (ms * 1e-3);
    // LDS atomics: 8 blocks per CU, 4096 operations per thread
    const int l_blocks = cus * 8, l_reps = 4096;
    unsigned long long *sink = (unsigned long long *)(buf + copy_bytes);
    if (e == hipSuccess)
        e = best_ms([&] {
            hipLaunchKernelGGL((k_pk_latomic<false>), dim3(l_blocks), dim3(PK_THREADS), 0, nullptr, sink, l_reps);
        }, 5, ms);
    if (e == hipSuccess) out[3] = (double)l_blocks * PK_THREADS * l_reps / (ms * 1e-3);
    if (e == hipSuccess)
        e = best_ms([&] {
            hipLaunchKernelGGL((k_pk_latomic<true>), dim3(l_blocks), dim3(PK_THREADS), 0, nullptr, sink, l_reps);
        }, 5, ms);
    if (e == hipSuccess) out[4] = (double)l_blocks * PK_THREADS * l_reps / (ms * 1e-3);
    (void)hipFree(buf);
    return e;
}
