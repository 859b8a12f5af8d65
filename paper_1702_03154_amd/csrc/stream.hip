// Streaming build for key sets beyond device memory: the keys are never stored.  Each streamed
// level re-generates every key of the stream, skips the keys placed at an earlier level (their bit
// is set in A_j at their level-j position, Algorithm 3's walk), and marks the rest in the level's
// A and C bits with global test-and-set (Algorithm 2).  This is the second strategy of Section 3.4
// (every level re-reads the whole input and queries the finished levels instead of storing F_d),
// with device memory in the role of the disk.  Once the survivors fit the key budget they are
// collected and the in-memory levels take over; the result equals a build from the stored keys
// because the levels depend only on the key set.
//
// Key sources: a deterministic stream of pseudo-random keys generated on the fly, as for the
// trillion-key run of Section 4.5: key i is the SplitMix64 output (Steele, Lea and Flood, OOPSLA
// 2014) of seed + (i + 1) * 0x9E3779B97F4A7C15, a bijective mix, so the n keys are distinct; or a
// stored key set in host memory, copied to the device chunk by chunk at every re-scan (the kernels
// below then read the chunk's keys instead of generating them).
#include "internal.h"

namespace mphfk {

namespace {

constexpr int ZT = 256;

// True if x was placed at one of the levels 0..d-1 (its bit is set in A there).
__device__ __forceinline__ bool placed_before(uint64_t x, const DevLevel* __restrict__ lev, uint32_t d,
                                              const uint64_t* __restrict__ words) {
    for (uint32_t j = 0; j < d; ++j) {
        const DevLevel L = lev[j];
        const uint64_t g = L.bit_off + mod_invariant(fmix64(x ^ L.seed), L.m, L.magic, L.sh1, L.sh2);
        if ((words[g >> 6] >> (g & 63)) & 1ull) return true;
    }
    return false;
}

__device__ __forceinline__ void mark_pos(unsigned long long* W, uint64_t p) {
    unsigned long long* w = W + (p >> 5);
    const unsigned long long b = 1ull << (p & 31);
    const unsigned long long old = atomicOr(w, b);
    if (old & b) atomicOr(w, b << 32);
}

constexpr int ZI = 8;   // keys per thread per iteration: independent walks in flight

__global__ void __launch_bounds__(ZT)
k_stream_fill(uint64_t kseed, uint64_t kstart, const uint64_t* __restrict__ keys, uint64_t n,
              const DevLevel* __restrict__ lev, uint32_t d, const uint64_t* __restrict__ words, unsigned long long* W,
              LevelHash L) {
    const uint64_t stride = (uint64_t)gridDim.x * ZT * ZI;
    for (uint64_t i0 = (uint64_t)blockIdx.x * ZT * ZI; i0 < n; i0 += stride) {
        uint64_t x[ZI];
        bool live[ZI];
#pragma unroll
        for (int it = 0; it < ZI; ++it) {
            const uint64_t i = i0 + (uint64_t)it * ZT + threadIdx.x;
            live[it] = i < n;
            x[it] = live[it] ? (keys ? keys[i] : stream_key(kseed, kstart + i)) : 0;
        }
#pragma unroll
        for (int it = 0; it < ZI; ++it) live[it] = live[it] && !placed_before(x[it], lev, d, words);
#pragma unroll
        for (int it = 0; it < ZI; ++it)
            if (live[it]) mark_pos(W, level_pos(x[it], L));
    }
}

// Survivors appended with one counter update per block and iteration (ZT * ZI keys): a single
// counter updated by every wave would serialize on one address.  Order inside a block's chunk is
// thread-major; the build does not depend on the order of F_d.
__global__ void __launch_bounds__(ZT)
k_stream_collect(uint64_t kseed, uint64_t kstart, const uint64_t* __restrict__ keys, uint64_t n,
                 const DevLevel* __restrict__ lev, uint32_t d, const uint64_t* __restrict__ words,
                 uint64_t* __restrict__ out, uint64_t cap, unsigned long long* count) {
    __shared__ uint32_t wsum[ZT / 64 + 1];
    __shared__ unsigned long long s_base;
    const uint64_t stride = (uint64_t)gridDim.x * ZT * ZI;
    for (uint64_t i0 = (uint64_t)blockIdx.x * ZT * ZI; i0 < n; i0 += stride) {
        uint64_t x[ZI];
        uint32_t keep = 0;
#pragma unroll
        for (int it = 0; it < ZI; ++it) {
            const uint64_t i = i0 + (uint64_t)it * ZT + threadIdx.x;
            x[it] = i < n ? (keys ? keys[i] : stream_key(kseed, kstart + i)) : 0;
        }
#pragma unroll
        for (int it = 0; it < ZI; ++it) {
            const uint64_t i = i0 + (uint64_t)it * ZT + threadIdx.x;
            if (i < n && !placed_before(x[it], lev, d, words)) keep |= 1u << it;
        }
        uint32_t tot;
        const uint32_t ex = block_exclusive_sum<ZT>((uint32_t)__popc(keep), wsum, &tot);
        if (threadIdx.x == 0) s_base = tot ? atomicAdd(count, (unsigned long long)tot) : 0ull;
        __syncthreads();
        uint64_t j = s_base + ex;
#pragma unroll
        for (int it = 0; it < ZI; ++it) {
            if ((keep >> it) & 1u) {
                if (j < cap) out[j] = x[it];
                ++j;
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(ZT)
k_stream_keys(uint64_t kseed, uint64_t kstart, uint64_t n, uint64_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * ZT;
    for (uint64_t i = (uint64_t)blockIdx.x * ZT + threadIdx.x; i < n; i += stride) out[i] = stream_key(kseed, kstart + i);
}

unsigned zgrid(uint64_t n) {
    uint64_t g = (n + (uint64_t)ZI * ZT - 1) / ((uint64_t)ZI * ZT);
    if (g < 1) g = 1;
    if (g > 32768) g = 32768;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_stream_fill(uint64_t kseed, uint64_t kstart, const uint64_t* keys, uint64_t n, const DevLevel* lev,
                              uint32_t d, const uint64_t* words, uint64_t* W, const LevelHash& L, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_stream_fill, dim3(zgrid(n)), dim3(ZT), 0, s, kseed, kstart, keys, n, lev, d, words,
                       (unsigned long long*)W, L);
    return hipGetLastError();
}

hipError_t launch_stream_collect(uint64_t kseed, uint64_t kstart, const uint64_t* keys, uint64_t n,
                                 const DevLevel* lev, uint32_t d, const uint64_t* words, uint64_t* out, uint64_t cap,
                                 unsigned long long* count, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_stream_collect, dim3(zgrid(n)), dim3(ZT), 0, s, kseed, kstart, keys, n, lev, d, words, out,
                       cap, count);
    return hipGetLastError();
}

hipError_t launch_stream_keys(uint64_t kseed, uint64_t kstart, uint64_t n, uint64_t* out, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_stream_keys, dim3(zgrid(n)), dim3(ZT), 0, s, kseed, kstart, n, out);
    return hipGetLastError();
}

}  // namespace mphfk
