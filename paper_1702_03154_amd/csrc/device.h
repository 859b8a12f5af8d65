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

// n mod m, with *q = floor(n / m) (the same exact division).
__device__ __forceinline__ uint64_t divmod_invariant(uint64_t n, uint64_t m, uint64_t magic, uint32_t sh1,
                                                     uint32_t sh2, uint64_t* q) {
    const uint64_t t = __umul64hi(magic, n);
    *q = (t + ((n - t) >> sh1)) >> sh2;
    return n - *q * m;
}

__device__ __forceinline__ uint64_t level_pos(uint64_t key, const LevelHash& L) {
    return mod_invariant(fmix64(key ^ L.seed), L.m, L.magic, L.sh1, L.sh2);
}

// level_pos for levels below 2^32 positions: the remainder h - q m is below 2^32, so its low 32
// bits (one 32-bit multiply) are all of it.
__device__ __forceinline__ uint32_t level_pos32(uint64_t key, const LevelHash& L) {
    const uint64_t h = fmix64(key ^ L.seed);
    const uint64_t t = __umul64hi(L.magic, h);
    const uint64_t q = (t + ((h - t) >> L.sh1)) >> L.sh2;
    return (uint32_t)h - (uint32_t)q * (uint32_t)L.m;
}

// Exact floor(a * 2^64 / m) for a < m (any m >= 1) by binary long division (one thread).  The
// remainder stays below m; when m > 2^63 a doubled remainder can pass 2^64, which the carry out of
// the shift records (the true remainder is then >= m, and the wrapped subtraction is exact).
__host__ __device__ inline uint64_t div_shift64(uint64_t a, uint64_t m) {
    if ((m >> 32) == 0) {   // two base-2^32 digits of the long division, each a 64-bit quotient
        const uint64_t t1 = a << 32;
        const uint64_t q1 = t1 / m;
        const uint64_t t2 = (t1 - q1 * m) << 32;
        return (q1 << 32) | (t2 / m);
    }
    uint64_t q = 0, r = a;
    for (int i = 0; i < 64; ++i) {
        const uint64_t carry = r >> 63;
        r <<= 1;
        q <<= 1;
        if (carry || r >= m) {
            r -= m;
            q |= 1;
        }
    }
    return q;
}

// Device-side twin of make_level_hash (Granlund-Montgomery Figure 4.1 constants) for any m >= 1:
// l = ceil(log2 m), magic = floor(2^64 (2^l - m) / m) + 1, sh1 = min(l, 1), sh2 = max(l - 1, 0),
// with 2^l - m taken modulo 2^64 when l = 64 (m > 2^63).
__host__ __device__ inline LevelHash device_level_hash(uint64_t seed, uint64_t m, uint64_t bit_off) {
    LevelHash L;
    L.seed = seed;
    L.m = m;
    L.bit_off = bit_off;
    uint32_t l = 0;
    while (l < 64 && (1ull << l) < m) ++l;   // l = 64 only when m > 2^63
    const uint64_t pow_l = l < 64 ? (1ull << l) : 0;   // 2^l mod 2^64
    L.magic = div_shift64(pow_l - m, m) + 1;
    L.sh1 = l < 1 ? l : 1;
    L.sh2 = l > 1 ? l - 1 : 0;
    return L;
}

// ---------------------------------------------------------------- lookup sectors
//
// The lookup reads A through a copy laid out in 64-byte sectors: u32 word 0 of sector s holds the
// ones of A before bit 480*s counted from the start of its superblock of 2^21 sectors, u32 words
// 1..15 hold bits [480*s, 480*s + 480) of A, and super[s >> 21] holds the ones before the
// superblock.  A probe reads the aligned 64 bytes of one sector (four 16-byte loads).
constexpr uint64_t SEC_BITS = 480;
constexpr uint32_t SEC_WORDS = 16;
constexpr uint32_t SUPER_SHIFT = 21;

// The 64 bytes of sector j (four 16-byte loads).
__device__ __forceinline__ void sector_load(const uint32_t* __restrict__ sec, uint64_t j, uint4 v[4]) {
    const uint4* s4 = (const uint4*)(sec + j * SEC_WORDS);
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = s4[c];
}

__host__ __device__ __forceinline__ uint32_t popc32(uint32_t x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __popc(x);
#else
    return (uint32_t)__builtin_popcount(x);
#endif
}

// If bit r (< 480) of the loaded sector is set: *count = the sector's counter plus the ones of the
// sector before bit r, and true.  Two forms with the same result:
// * CHAIN (the lookup kernel, two queries per lane): the word holding the bit (data word s = r / 32)
//   is picked by a 4-level select on the bits of s and tested before any counting; on a hit a
//   running sum of popcounts along the data words is picked by the same select.  Fewest
//   instructions (about 40% fewer VALU instructions per probe than the other form).
// * otherwise (kernels with one query per lane, where a probe's latency is not hidden by another):
//   one compare per word for the select, and the popcounts of the words before it added as they
//   come, which keeps the dependency chain short.  Measured faster there.
template <bool CHAIN = true>
__host__ __device__ __forceinline__ bool sector_count(const uint4 v[4], uint32_t r, uint32_t* count) {
    const uint32_t e[16] = {v[0].x, v[0].y, v[0].z, v[0].w, v[1].x, v[1].y, v[1].z, v[1].w,
                            v[2].x, v[2].y, v[2].z, v[2].w, v[3].x, v[3].y, v[3].z, v[3].w};
    const uint32_t s = r >> 5, b = r & 31u;
    if constexpr (CHAIN) {
        uint32_t W[16];   // data word i is e[i + 1]
#pragma unroll
        for (int i = 0; i < 16; ++i) W[i] = i < 15 ? e[i + 1] : 0u;
#pragma unroll
        for (int lvl = 0; lvl < 4; ++lvl) {   // halve the candidates on bit lvl of s
            const bool hi = (s >> lvl) & 1u;
#pragma unroll
            for (int i = 0; i < (8 >> lvl); ++i) W[i] = hi ? W[2 * i + 1] : W[2 * i];
        }
        if (!((W[0] >> b) & 1u)) return false;
        uint32_t P[16];   // the counter plus the ones of the data words before data word i
        P[0] = e[0];
#pragma unroll
        for (int i = 0; i < 15; ++i) P[i + 1] = P[i] + popc32(e[i + 1]);
#pragma unroll
        for (int lvl = 0; lvl < 4; ++lvl) {
            const bool hi = (s >> lvl) & 1u;
#pragma unroll
            for (int i = 0; i < (8 >> lvl); ++i) P[i] = hi ? P[2 * i + 1] : P[2 * i];
        }
        *count = P[0] + popc32(W[0] & ((1u << b) - 1u));
    } else {
        const uint32_t t = 1 + s;   // the bit's u32 word in the sector
        uint32_t w = 0;
#pragma unroll
        for (uint32_t k = 1; k < SEC_WORDS; ++k)
            if (k == t) w = e[k];
        if (!((w >> b) & 1u)) return false;
        // sector counter + whole words before t + bits of t below r
        uint32_t acc = e[0];
        const uint32_t mask = (1u << b) - 1u;
#pragma unroll
        for (uint32_t k = 1; k < SEC_WORDS; ++k) {
            if (k < t) acc += popc32(e[k]);
            else if (k == t) acc += popc32(e[k] & mask);
        }
        *count = acc;
    }
    return true;
}

// The empty asm statements below consume loaded values before the bit test, so that the compiler
// issues every load of a probe together instead of sinking the counter word and the superblock
// load behind the test (a second round trip on every hit).  They contain no instruction.

// If bit r (< 480) of sector j is set: *count = the sector's counter plus the ones before bit r.
__device__ __forceinline__ bool sector_probe(const uint32_t* __restrict__ sec, uint64_t j, uint32_t r,
                                             uint32_t* count) {
    uint4 v[4];
    sector_load(sec, j, v);
    asm volatile("" ::"v"(v[0].x));
    return sector_count<false>(v, r, count);
}

// If bit g of A is set: *rank = the ones of A before g, and true.
__device__ __forceinline__ bool sector_rank(const uint32_t* __restrict__ sec,
                                            const uint64_t* __restrict__ super, uint64_t g,
                                            uint64_t* rank) {
    const uint64_t j = g / SEC_BITS;
    const uint64_t base = super[j >> SUPER_SHIFT];
    uint4 v[4];
    sector_load(sec, j, v);
    asm volatile("" ::"v"(v[0].x), "v"(base));
    uint32_t c;
    if (!sector_count<false>(v, (uint32_t)(g - j * SEC_BITS), &c)) return false;
    *rank = base + c;
    return true;
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
