// Roofline microbenchmarks of the memory system (gfx950): the ceilings the build and lookup kernels
// are measured against.  The method's costs are streaming reads and writes of keys plus random
// accesses into bit arrays (one test-and-set per key and level during the build, Algorithm 2; one
// probe per visited level during a query, Algorithm 3), and the paper names random accesses as its
// limit (Section 3.2, "Parallelization"; Section 4.2).  Each probe isolates one of these:
//
//  * streaming read / copy of a buffer (16-byte loads and stores, grid-stride);
//  * random 8-byte reads and random 64-byte sector reads (four 16-byte loads of one aligned
//    sector, as a lookup probe issues them) over a footprint;
//  * random atomicOr with the old value returned (the global test-and-set) over a footprint;
//  * random atomicOr with return in LDS (the test-and-set of the partitioned levels);
//  * a kernel reading pinned host memory and writing pinned host memory over PCIe, 8 bytes a lane
//    (as the serving kernel reads request keys and writes their labels in place).
//
// Random indices come from a per-thread xorshift64 generator (Marsaglia 2003) reduced by a
// multiply-high, so that the address arithmetic stays a few instructions per access.  Each thread
// keeps U accesses in flight.  Loaded values are folded into a per-thread accumulator that one
// atomic per workgroup folds into a device word, so no load is dead.
#include "internal.h"
#include "mphf.h"
#include "api_internal.h"

namespace {

__device__ unsigned long long g_probe_sink;

constexpr int PT = 256;   // threads per workgroup
constexpr int U = 8;      // accesses per thread and iteration (atomics: all in flight together)
constexpr int UR = 2;     // random reads in flight per thread: the fastest depth measured for random
                          // 64-byte sector reads (5.5e10/s at 440 MB with 2 in flight, 3.8e10 with 8)

__device__ __forceinline__ uint64_t xorshift64(uint64_t& x) {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return x;
}

__device__ __forceinline__ uint64_t seed_thread(uint64_t seed) {
    uint64_t x = mphfk::fmix64(seed ^ (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 0x9E3779B97F4A7C15ull));
    return x ? x : 0x2545F4914F6CDD1Dull;
}

__device__ __forceinline__ void sink(uint64_t acc) {
    __shared__ unsigned long long part;
    if (threadIdx.x == 0) part = 0;
    __syncthreads();
    atomicXor(&part, (unsigned long long)acc);
    __syncthreads();
    if (threadIdx.x == 0) atomicXor(&g_probe_sink, part);
}

__global__ void __launch_bounds__(PT) k_probe_read(const uint4* __restrict__ p, uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * PT;
    uint64_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * PT + threadIdx.x; i < n16; i += stride) {
        const uint4 v = p[i];
        acc ^= ((uint64_t)v.x | ((uint64_t)v.y << 32)) + ((uint64_t)v.z | ((uint64_t)v.w << 32));
    }
    sink(acc);
}

__global__ void __launch_bounds__(PT) k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                   uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * PT;
    for (uint64_t i = (uint64_t)blockIdx.x * PT + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

__global__ void __launch_bounds__(PT) k_probe_rand8(const uint64_t* __restrict__ p, uint64_t nwords,
                                                    uint64_t per_thread, uint64_t seed) {
    uint64_t x = seed_thread(seed), acc = 0;
    for (uint64_t r = 0; r < per_thread; r += UR) {
        uint64_t v[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) v[u] = p[__umul64hi(xorshift64(x), nwords)];
#pragma unroll
        for (int u = 0; u < UR; ++u) acc += v[u];
    }
    sink(acc);
}

__global__ void __launch_bounds__(PT) k_probe_rand64(const uint4* __restrict__ p, uint64_t nsec,
                                                     uint64_t per_thread, uint64_t seed) {
    uint64_t x = seed_thread(seed), acc = 0;
    for (uint64_t r = 0; r < per_thread; r += UR) {
        uint4 v[UR][4];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const uint4* s = p + 4 * __umul64hi(xorshift64(x), nsec);
#pragma unroll
            for (int c = 0; c < 4; ++c) v[u][c] = s[c];
        }
#pragma unroll
        for (int u = 0; u < UR; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc += v[u][c].x ^ v[u][c].y ^ v[u][c].z ^ v[u][c].w;
    }
    sink(acc);
}

__global__ void __launch_bounds__(PT) k_probe_host(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                                                   uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * PT;
    for (uint64_t i = (uint64_t)blockIdx.x * PT + threadIdx.x; i < n; i += stride) dst[i] = src[i] + 1;
}

__global__ void __launch_bounds__(PT) k_probe_atomic(unsigned long long* __restrict__ p, uint64_t nwords,
                                                     uint64_t per_thread, uint64_t seed) {
    uint64_t x = seed_thread(seed), acc = 0;
    for (uint64_t r = 0; r < per_thread; r += U) {
        unsigned long long o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t h = xorshift64(x);
            o[u] = atomicOr(p + __umul64hi(h, nwords), 1ull << (h & 63));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += o[u];
    }
    sink(acc);
}

__global__ void __launch_bounds__(PT) k_probe_lds_atomic(uint32_t nwords, uint64_t per_thread, uint64_t seed) {
    extern __shared__ uint32_t w[];
    for (uint32_t i = threadIdx.x; i < nwords; i += PT) w[i] = 0;
    __syncthreads();
    uint64_t x = seed_thread(seed), acc = 0;
    for (uint64_t r = 0; r < per_thread; r += U) {
        uint32_t o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t h = xorshift64(x);
            o[u] = atomicOr(&w[(uint32_t)((h >> 32) * nwords >> 32)], 1u << (h & 31));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += o[u];
    }
    sink(acc);
}

// workgroups of a probe launch: eight per compute unit
constexpr unsigned GRID = 256 * 8;

}  // namespace

extern "C" {

mphf_status mphf_probe(uint32_t kind, void* buf, uint64_t bytes, void* dst, uint64_t ops, uint64_t seed,
                       void* stream) {
    const hipStream_t s = (hipStream_t)stream;
    const uint64_t threads = (uint64_t)GRID * PT;
    const uint64_t per_thread = ((ops + threads - 1) / threads + U - 1) / U * U;
    if (kind == MPHF_PROBE_LDS_ATOMIC_OR) {
        if (bytes < 4 || bytes > 49152) return mphf_api::set_error(MPHF_E_INVALID, "LDS footprint must be 4..49152 bytes");
        hipLaunchKernelGGL(k_probe_lds_atomic, dim3(GRID), dim3(PT), (size_t)(bytes / 4) * 4, s,
                           (uint32_t)(bytes / 4), per_thread, seed);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? MPHF_OK : mphf_api::hip_error(e, "probe");
    }
    if (kind == MPHF_PROBE_HOST_EXCHANGE) {
        if (bytes < 8 || bytes % 8) return mphf_api::set_error(MPHF_E_INVALID, "a positive multiple of 8 bytes");
        const void* src = buf ? mphf_api::pinned_alias(buf, bytes) : nullptr;
        void* out = dst ? const_cast<void*>(mphf_api::pinned_alias(dst, bytes)) : nullptr;
        if (!src || !out) return mphf_api::set_error(MPHF_E_INVALID, "buf and dst must be pinned host memory of `bytes`");
        hipLaunchKernelGGL(k_probe_host, dim3(GRID), dim3(PT), 0, s, (const uint64_t*)src, (uint64_t*)out, bytes / 8);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? MPHF_OK : mphf_api::hip_error(e, "probe");
    }
    if (!buf || !mphf_api::device_ptr(buf)) return mphf_api::set_error(MPHF_E_INVALID, "buf must be device memory");
    if ((uintptr_t)buf & 63) return mphf_api::set_error(MPHF_E_INVALID, "buf must be 64-byte aligned");
    switch (kind) {
        case MPHF_PROBE_STREAM_READ:
            if (bytes < 16) return mphf_api::set_error(MPHF_E_INVALID, "at least 16 bytes");
            hipLaunchKernelGGL(k_probe_read, dim3(GRID), dim3(PT), 0, s, (const uint4*)buf, bytes / 16);
            break;
        case MPHF_PROBE_STREAM_COPY:
            if (bytes < 16) return mphf_api::set_error(MPHF_E_INVALID, "at least 16 bytes");
            if (!dst || !mphf_api::device_ptr(dst) || ((uintptr_t)dst & 15))
                return mphf_api::set_error(MPHF_E_INVALID, "dst must be 16-byte aligned device memory");
            hipLaunchKernelGGL(k_probe_copy, dim3(GRID), dim3(PT), 0, s, (const uint4*)buf, (uint4*)dst, bytes / 16);
            break;
        case MPHF_PROBE_RANDOM_READ8:
            if (bytes < 8) return mphf_api::set_error(MPHF_E_INVALID, "at least 8 bytes");
            hipLaunchKernelGGL(k_probe_rand8, dim3(GRID), dim3(PT), 0, s, (const uint64_t*)buf, bytes / 8,
                               per_thread, seed);
            break;
        case MPHF_PROBE_RANDOM_SECTOR64:
            if (bytes < 64) return mphf_api::set_error(MPHF_E_INVALID, "at least 64 bytes");
            hipLaunchKernelGGL(k_probe_rand64, dim3(GRID), dim3(PT), 0, s, (const uint4*)buf, bytes / 64,
                               per_thread, seed);
            break;
        case MPHF_PROBE_RANDOM_ATOMIC_OR:
            if (bytes < 8) return mphf_api::set_error(MPHF_E_INVALID, "at least 8 bytes");
            hipLaunchKernelGGL(k_probe_atomic, dim3(GRID), dim3(PT), 0, s, (unsigned long long*)buf, bytes / 8,
                               per_thread, seed);
            break;
        default:
            return mphf_api::set_error(MPHF_E_INVALID, "unknown probe kind");
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MPHF_OK : mphf_api::hip_error(e, "probe");
}

uint64_t mphf_probe_ops(uint64_t ops) {
    const uint64_t threads = (uint64_t)GRID * PT;
    return ((ops + threads - 1) / threads + U - 1) / U * U * threads;
}

}  // extern "C"
