// Device primitives shared by the build and lookup kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mphfk {

// Level hash parameters as the kernels see them.  pos_d(x) = fmix64(x ^ seed) mod m, where the
// reduction is the paper's `mod` (Algorithms 1-3) done as an exact division by an invariant
// integer (Granlund and Montgomery, PLDI 1994, Figure 4.1): q = (t + ((n - t) >> sh1)) >> sh2
// with t = mulhi(magic, n), then r = n - q * m.
struct LevelHash {
    uint64_t seed;
    uint64_t m;
    uint64_t magic;
    uint64_t bit_off;   // offset of A_d inside the concatenated A (a multiple of 64)
    uint32_t sh1;
    uint32_t sh2;
};

// MurmurHash3's 64-bit finalizer (Appleby; public domain): a bijection of 64-bit words.
__device__ __forceinline__ uint64_t fmix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xFF51AFD7ED558CCDull;
    x ^= x >> 33;
    x *= 0xC4CEB9FE1A85EC53ull;
    x ^= x >> 33;
    return x;
}

// The inverse of fmix64: each x ^= x >> 33 undoes itself on 64 bits, and the multipliers are
// replaced by their inverses modulo 2^64.
__device__ __forceinline__ uint64_t unfmix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0x9CB4B2F8129337DBull;   // 0xC4CEB9FE1A85EC53^-1 mod 2^64
    x ^= x >> 33;
    x *= 0x4F74430C22A54005ull;   // 0xFF51AFD7ED558CCD^-1 mod 2^64
    x ^= x >> 33;
    return x;
}

__device__ __forceinline__ uint64_t mod_invariant(uint64_t n, uint64_t m, uint64_t magic,
                                                  uint32_t sh1, uint32_t sh2) {
    uint64_t t = __umul64hi(magic, n);
    uint64_t q = (t + ((n - t) >> sh1)) >> sh2;
    return n - q * m;
}

__device__ __forceinline__ uint64_t level_pos(uint64_t key, const LevelHash& L) {
    return mod_invariant(fmix64(key ^ L.seed), L.m, L.magic, L.sh1, L.sh2);
}

// ---------------------------------------------------------------- wave64 / block helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive prefix sum over the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if ((int)lane_id() >= o) v += u;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive prefix sum across a block of NT threads (NT a multiple of 64).  `sh` must hold
// NT/64 + 1 elements.  Returns the thread's exclusive prefix; *total gets the block sum.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* sh, T* total) {
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6;
    T inc = wave_inclusive_sum(v);
    if (lane_id() == 63) sh[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int i = 0; i < NW; ++i) {
            T t = sh[i];
            sh[i] = acc;
            acc += t;
        }
        sh[NW] = acc;
    }
    __syncthreads();
    T res = sh[w] + inc - v;
    *total = sh[NW];
    __syncthreads();
    return res;
}

}  // namespace mphfk
