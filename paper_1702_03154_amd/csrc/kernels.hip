// HIP kernels of the cascading-bit-array MPHF for gfx950 (wave64), and their launchers.
//
// Layouts in HBM:
//  * W, the working array of the level being filled: 64-bit words, each holding 32 positions
//    as an A half (bits 0..31) and a C half (bits 32..63), so that the collision bit of a
//    position lives in the same word (and cache line) as its A bit.  Position p of the level
//    is A bit p%32 / C bit 32+p%32 of word p/32.  2*ceil(m/64) words.
//  * A, the concatenation of the finalized levels: bit p of level d is bit (o+p)%64 of word
//    (o+p)/64 with o the level's bit offset, a multiple of 64; padding bits stay 0.
//  * rank[b]: 64-bit count of the ones of A before position b*rank_sample.
#include "internal.h"

namespace mphfk {

namespace {

constexpr int NT = 256;          // threads per block for the streaming kernels
constexpr int MAX_GRID = 8192;   // grid-stride kernels: enough blocks to fill 256 CUs

// Blocks for a random-access kernel: one per per_block items, up to 2^24 - 1 (so that the grid's
// work-items stay below 2^32); more items than that are strided.
inline unsigned short_grid(uint64_t items, uint64_t per_block) {
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > (1ull << 24) - 1) b = (1ull << 24) - 1;
    return (unsigned)b;
}

inline unsigned grid_for(uint64_t items, uint64_t per_block) {
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > MAX_GRID) b = MAX_GRID;
    return (unsigned)b;
}

// Record one key landing on position p of the level held in W (Algorithm 2 with the
// collision array): the first key sets the A bit; any later key finds it set and sets the
// C bit.  The final state, A = exactly one key and C = two or more after the finalize step,
// does not depend on the order of the atomics.
__device__ __forceinline__ void mark(unsigned long long* W, uint64_t p) {
    unsigned long long* w = W + (p >> 5);
    const unsigned long long b = 1ull << (p & 31);
    const unsigned long long old = atomicOr(w, b);
    if (old & b) atomicOr(w, b << 32);
}

__global__ void k_zero(uint64_t* __restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

__global__ void k_zero32(uint32_t* __restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

__global__ void k_fill(const uint64_t* __restrict__ keys, uint64_t n, unsigned long long* W,
                       LevelHash L) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        mark(W, level_pos(keys[i], L));
}

// A_d = A & ~C over each pair of W words; weight(A_d) accumulated into *weight.
__global__ void k_finalize(const ulonglong2* __restrict__ W, uint64_t nwords,
                           uint64_t* __restrict__ A, uint64_t* __restrict__ C,
                           unsigned long long* weight) {
    __shared__ unsigned long long part[NT / 64];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long cnt = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nwords; j += stride) {
        const ulonglong2 v = W[j];
        const uint64_t a0 = (uint32_t)v.x & ~(uint32_t)(v.x >> 32);
        const uint64_t a1 = (uint32_t)v.y & ~(uint32_t)(v.y >> 32);
        const uint64_t a = a0 | (a1 << 32);
        A[j] = a;
        if (C) C[j] = (v.x >> 32) | ((v.y >> 32) << 32);
        cnt += __popcll(a);
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < NT / 64; ++i) s += part[i];
        if (s) atomicAdd(weight, s);
    }
}

// Filter of level d fused with the fill of level d+1 (Algorithm 1): a key whose A_d bit is 0
// collided at level d, so it goes to F_{d+1} (compacted into Fout) and, when there is a next
// level, is marked in W at its level d+1 position.  One block reserves its output range with
// one atomic on *count; the order of F_{d+1} does not affect any result.
template <int ITEMS>
__global__ void k_filter_fill(const uint64_t* __restrict__ Fin, uint64_t n,
                              const uint64_t* __restrict__ words, LevelHash Ld,
                              uint64_t* __restrict__ Fout, uint64_t cap,
                              unsigned long long* count, unsigned long long* W, LevelHash Ln,
                              int do_fill) {
    __shared__ uint32_t sh[NT / 64 + 1];
    __shared__ unsigned long long base_sh;
    constexpr uint64_t TILE = (uint64_t)NT * ITEMS;
    const uint64_t ntiles = (n + TILE - 1) / TILE;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint64_t t0 = t * TILE;
        uint64_t k[ITEMS];
        uint32_t surv = 0;
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint64_t i = t0 + (uint64_t)it * NT + threadIdx.x;
            k[it] = 0;
            if (i < n) {
                const uint64_t x = Fin[i];
                k[it] = x;
                const uint64_t g = Ld.bit_off + level_pos(x, Ld);
                if (!((words[g >> 6] >> (g & 63)) & 1ull)) {
                    surv |= 1u << it;
                    if (do_fill) mark(W, level_pos(x, Ln));
                }
            }
        }
        const uint32_t c = __popc(surv);
        uint32_t total;
        const uint32_t pre = block_exclusive_sum<NT>(c, sh, &total);
        if (threadIdx.x == 0) base_sh = total ? atomicAdd(count, (unsigned long long)total) : 0;
        __syncthreads();
        uint64_t o = base_sh + pre;
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            if ((surv >> it) & 1u) {
                if (o < cap) Fout[o] = k[it];
                ++o;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- scans

// Three-phase exclusive scan of u32 counts into u64 prefixes.
constexpr int SCAN_ITEMS = 16;
constexpr uint64_t SCAN_TILE = (uint64_t)NT * SCAN_ITEMS;

__global__ void k_scan_tile_sums(const uint32_t* __restrict__ in, uint64_t n,
                                 uint64_t* __restrict__ tile_sums, const uint64_t* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ uint64_t part[NT / 64];
    const uint64_t t = blockIdx.x;
    const uint64_t i0 = t * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t s = 0;
    for (int it = 0; it < SCAN_ITEMS; ++it)
        if (i0 + it < n) s += in[i0 + it];
    s = wave_sum(s);
    if (lane_id() == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0;
        for (int i = 0; i < NT / 64; ++i) a += part[i];
        tile_sums[t] = a;
    }
}

__global__ void k_scan_tiles(uint64_t* __restrict__ tile_sums, uint64_t ntiles, const uint64_t* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ uint64_t sh[NT / 64 + 1];
    uint64_t carry = 0;
    for (uint64_t c0 = 0; c0 < ntiles; c0 += NT) {
        const uint64_t i = c0 + threadIdx.x;
        const uint64_t v = i < ntiles ? tile_sums[i] : 0;
        uint64_t total;
        const uint64_t pre = block_exclusive_sum<NT>(v, sh, &total);
        if (i < ntiles) tile_sums[i] = carry + pre;
        carry += total;
    }
}

__global__ void k_scan_apply(const uint32_t* __restrict__ in, uint64_t* __restrict__ out, uint64_t n,
                             const uint64_t* __restrict__ tile_off, const uint64_t* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ uint64_t sh[NT / 64 + 1];
    const uint64_t t = blockIdx.x;
    const uint64_t i0 = t * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint64_t s = 0;
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        v[it] = i0 + it < n ? in[i0 + it] : 0;
        s += v[it];
    }
    uint64_t total;
    uint64_t run = tile_off[t] + block_exclusive_sum<NT>(s, sh, &total);
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        if (i0 + it < n) out[i0 + it] = run;
        run += v[it];
    }
}

// The whole scan in one workgroup, tile after tile, for inputs of at most SCAN_SINGLE entries (one
// launch instead of three; the per-level counts of the small levels).
constexpr uint64_t SCAN_SINGLE = 4 * SCAN_TILE;

__global__ void k_scan_single(const uint32_t* __restrict__ in, uint64_t* __restrict__ out, uint64_t n,
                              const uint64_t* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ uint64_t sh[NT / 64 + 1];
    uint64_t carry = 0;
    for (uint64_t t0 = 0; t0 < n; t0 += SCAN_TILE) {
        const uint64_t i0 = t0 + (uint64_t)threadIdx.x * SCAN_ITEMS;
        uint32_t v[SCAN_ITEMS];
        uint64_t s = 0;
        for (int it = 0; it < SCAN_ITEMS; ++it) {
            v[it] = i0 + it < n ? in[i0 + it] : 0;
            s += v[it];
        }
        uint64_t total;
        uint64_t run = carry + block_exclusive_sum<NT>(s, sh, &total);
        for (int it = 0; it < SCAN_ITEMS; ++it) {
            if (i0 + it < n) out[i0 + it] = run;
            run += v[it];
        }
        carry += total;
    }
}

// ---------------------------------------------------------------- radix sort (fallback keys)

constexpr int RADIX_ROUNDS = 8;
constexpr uint64_t RADIX_TILE = (uint64_t)NT * RADIX_ROUNDS;

__global__ void k_radix_hist(const uint64_t* __restrict__ in, uint64_t n, int shift,
                             uint32_t* __restrict__ counts, uint64_t ntiles) {
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t t = blockIdx.x;
    for (int r = 0; r < RADIX_ROUNDS; ++r) {
        const uint64_t i = t * RADIX_TILE + (uint64_t)r * NT + threadIdx.x;
        if (i < n) atomicAdd(&hist[(in[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(uint64_t)threadIdx.x * ntiles + t] = hist[threadIdx.x];
}

// Stable scatter: keys of a tile keep their order within each digit.
__global__ void k_radix_scatter(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                uint64_t n, int shift, const uint64_t* __restrict__ offsets,
                                uint64_t ntiles) {
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[NT / 64][256];
    running[threadIdx.x] = 0;
    for (int w = 0; w < NT / 64; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t t = blockIdx.x;
    const int w = threadIdx.x >> 6;
    const uint32_t lane = lane_id();
    const uint64_t lt = (1ull << lane) - 1;
    for (int r = 0; r < RADIX_ROUNDS; ++r) {
        const uint64_t i = t * RADIX_TILE + (uint64_t)r * NT + threadIdx.x;
        const bool valid = i < n;
        const uint64_t key = valid ? in[i] : 0;
        const uint32_t dig = (uint32_t)(key >> shift) & 255u;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t bb = __ballot(valid && bit);
            match &= bit ? bb : ~bb;
        }
        const uint32_t rank = __popcll(match & lt);
        if (valid && rank == 0) wcnt[w][dig] = __popcll(match);
        __syncthreads();
        if (valid) {
            uint64_t pos = offsets[(uint64_t)dig * ntiles + t] + running[dig] + rank;
            for (int v = 0; v < w; ++v) pos += wcnt[v][dig];
            out[pos] = key;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int v = 0; v < NT / 64; ++v) {
            add += wcnt[v][threadIdx.x];
            wcnt[v][threadIdx.x] = 0;
        }
        running[threadIdx.x] += add;
        __syncthreads();
    }
}

__global__ void k_find_duplicates(const uint64_t* __restrict__ s, uint64_t n,
                                  unsigned long long* flag) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i + 1 < n; i += stride)
        if (s[i] == s[i + 1]) atomicOr(flag, 1ull);
}

// ---------------------------------------------------------------- lookup layout
//
// A random read on gfx950 moves one 128-byte line from HBM whatever its width, and the L1/L2
// request rate caps how many 16-byte pieces a lane may load per probe, so a probe should touch one
// small aligned unit holding both the probed bit and what its rank needs: the 64-byte sectors of
// device.h (Section 3.1's counters, here one 32-bit counter per 480 positions plus superblocks).
//
// Sectors, superblocks and the rank table in two reads of A.  Workgroup g covers the 256 sectors
// 256 g .. 256 g + 255, i.e. the 3840 u32 words of bits [122880 g, 122880 (g+1)), which is exactly
// 240 rank blocks of 512 positions (120 of 1024).  The first kernel counts the ones of each
// workgroup's range; one scan of those counts gives every workgroup the ones before it; the second
// kernel loads its range into LDS again, counts its sectors and rank blocks there, scans them in
// the workgroup and writes its sectors, its rank entries and, at a superblock's first workgroup
// (2^21 sectors = 2^13 workgroups), the superblock entry.  Both read A with 16-byte coalesced loads.
constexpr uint32_t SR_SECTORS = 256;
constexpr uint64_t SR_BITS = SR_SECTORS * SEC_BITS;   // 122880
constexpr uint32_t SR_WORDS = SR_SECTORS * 15;        // 3840 u32 words of A per workgroup
constexpr uint32_t SUPER_GROUPS_SHIFT = SUPER_SHIFT - 8;   // workgroups per superblock: 2^13

// The u32 words [w0, w0 + 4) of A, words at or past nwords32 read as 0.
__device__ __forceinline__ uint4 load_a4(const uint32_t* __restrict__ A32, uint64_t nwords32, uint64_t w0) {
    if (w0 + 4 <= nwords32) return *(const uint4*)(A32 + w0);
    uint4 v;
    v.x = w0 < nwords32 ? A32[w0] : 0u;
    v.y = w0 + 1 < nwords32 ? A32[w0 + 1] : 0u;
    v.z = w0 + 2 < nwords32 ? A32[w0 + 2] : 0u;
    v.w = 0u;   // nwords32 is even, so w0 + 3 < nwords32 implies the whole vector is in range
    return v;
}

__global__ void __launch_bounds__(SR_SECTORS)
k_sector_group_sums(const uint32_t* __restrict__ A32, uint64_t nwords32, uint32_t* __restrict__ group_sums) {
    __shared__ uint32_t part[SR_SECTORS / 64];
    const uint64_t w0 = (uint64_t)blockIdx.x * SR_WORDS;
    uint32_t c = 0;
    for (uint32_t i = threadIdx.x; i < SR_WORDS / 4; i += SR_SECTORS) {
        const uint4 v = load_a4(A32, nwords32, w0 + 4ull * i);
        c += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
    }
    c = wave_sum(c);
    if (lane_id() == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t i = 0; i < SR_SECTORS / 64; ++i) t += part[i];
        group_sums[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(SR_SECTORS)
k_sector_layout(const uint32_t* __restrict__ A32, uint64_t nwords32, uint64_t nsec, uint32_t rshift, uint64_t nrank,
                const uint64_t* __restrict__ group_pre, uint32_t* __restrict__ sec, uint64_t* __restrict__ super,
                uint64_t* __restrict__ rank) {
    __shared__ uint4 w4[SR_WORDS / 4];
    __shared__ uint32_t cnt[SR_SECTORS];
    __shared__ uint32_t sh[SR_SECTORS / 64 + 1];
    const uint32_t* w = (const uint32_t*)w4;
    const uint64_t g = blockIdx.x;
    const uint64_t w0 = g * SR_WORDS;
    for (uint32_t i = threadIdx.x; i < SR_WORDS / 4; i += SR_SECTORS) w4[i] = load_a4(A32, nwords32, w0 + 4ull * i);
    __syncthreads();
    const uint64_t gp = group_pre[g];                                   // ones before this workgroup
    const uint64_t sp = group_pre[(g >> SUPER_GROUPS_SHIFT) << SUPER_GROUPS_SHIFT];   // ... its superblock
    // sector tid: words 15 tid .. 15 tid + 14 (stride 15: no bank conflicts)
    uint32_t c = 0;
#pragma unroll
    for (uint32_t k = 0; k < 15; ++k) c += __popc(w[15 * threadIdx.x + k]);
    uint32_t tot;
    const uint32_t ex = block_exclusive_sum<SR_SECTORS>(c, sh, &tot);
    cnt[threadIdx.x] = (uint32_t)(gp - sp) + ex;   // below 2^21 * 480
    // rank block tid (2^rshift positions = 2^(rshift-5) words), words read in a rotated order
    const uint32_t rw = 1u << (rshift - 5), nrb = (uint32_t)(SR_BITS >> rshift);
    uint32_t rc = 0;
    if (threadIdx.x < nrb)
        for (uint32_t q = 0; q < rw; ++q) rc += __popc(w[threadIdx.x * rw + ((q + threadIdx.x) & (rw - 1))]);
    const uint32_t rex = block_exclusive_sum<SR_SECTORS>(rc, sh, &tot);
    const uint64_t r = g * nrb + threadIdx.x;
    if (threadIdx.x < nrb && r < nrank) rank[r] = gp + rex;
    if (threadIdx.x == 0 && (g & ((1ull << SUPER_GROUPS_SHIFT) - 1)) == 0) super[g >> SUPER_GROUPS_SHIFT] = gp;
    // (block_exclusive_sum ends with a barrier, so cnt[] is complete)
    // the workgroup's 256 sectors as 1024 16-byte pieces: piece u is words 4(u&3) .. 4(u&3)+3 of
    // sector u>>2, word 0 of a sector being its counter and word k its A word k-1
    uint4* out4 = (uint4*)(sec + g * SR_SECTORS * SEC_WORDS);
    const uint64_t nsec_here = nsec - g * SR_SECTORS;
    for (uint32_t u = threadIdx.x; u < SR_SECTORS * 4; u += SR_SECTORS) {
        const uint32_t j = u >> 2, p = u & 3;
        if (j >= nsec_here) break;
        const uint32_t b = 15 * j + 4 * p;   // A word of this piece's second u32 (first when p > 0, minus 1)
        uint4 v;
        if (p == 0) {
            v.x = cnt[j];
            v.y = w[b];
            v.z = w[b + 1];
            v.w = w[b + 2];
        } else {
            v.x = w[b - 1];
            v.y = w[b];
            v.z = w[b + 1];
            v.w = w[b + 2];
        }
        out4[u] = v;
    }
}

// ---------------------------------------------------------------- lookup (Algorithm 3)

// Two queries per lane (i and i + stride) walked in lockstep, which doubles the independent sector
// loads a wave keeps in flight.  Queries and labels are streamed with non-temporal accesses so
// that they do not displace the structure's lines from the caches.
__global__ void k_lookup(const uint64_t* __restrict__ q, uint64_t n, uint64_t* __restrict__ out,
                         const DevLevel* __restrict__ lev, uint32_t nlev,
                         const uint32_t* __restrict__ sec, const uint64_t* __restrict__ super,
                         const uint64_t* __restrict__ fbk, uint64_t nfb, uint64_t N) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += 2 * stride) {
        const uint64_t i2 = i + stride;
        bool pend[2] = {true, i2 < n};
        const uint64_t x[2] = {__builtin_nontemporal_load(q + i), pend[1] ? __builtin_nontemporal_load(q + i2) : 0};
        uint64_t res[2] = {0, 0};
        walk_levels<2>(x, pend, res, lev, nlev, sec, super);
        __builtin_nontemporal_store(pend[0] ? fallback_label(x[0], fbk, nfb, N) : res[0], out + i);
        if (i2 < n) __builtin_nontemporal_store(pend[1] ? fallback_label(x[1], fbk, nfb, N) : res[1], out + i2);
    }
}

// A level's overflow flag and survivor total written to coherent host memory the device can write
// (one small kernel rather than two copies), then the sequence number `seq` after a system-scope
// fence, so that the host may poll out[2] instead of waiting for the stream; the flag is cleared
// for the next level.
__global__ void k_report(unsigned long long* flag, const uint64_t* __restrict__ total, uint64_t* out,
                         uint64_t seq, unsigned long long* last) {
    if (threadIdx.x == 0) {
        const unsigned long long f = *flag;
        out[0] = f;
        out[1] = *total;
        *last = f;   // for a level queued behind this one
        *flag = 0;
        __threadfence_system();
        __hip_atomic_store(out + 2, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__global__ void k_positions(const uint64_t* __restrict__ keys, uint64_t n, LevelHash L,
                            uint64_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = level_pos(keys[i], L);
}

}  // namespace

// ---------------------------------------------------------------- launchers

LevelHash make_level_hash(uint64_t seed, uint64_t m, uint64_t bit_off) {
    // Granlund-Montgomery 1994, Figure 4.1, for 64-bit words: l = ceil(log2 m),
    // magic = floor(2^64 (2^l - m) / m) + 1, sh1 = min(l, 1), sh2 = max(l - 1, 0).
    LevelHash L{};
    L.seed = seed;
    L.m = m;
    L.bit_off = bit_off;
    if (m == 0) return L;   // an empty level is never hashed
    uint32_t l = 0;
    while (l < 64 && ((unsigned __int128)1 << l) < (unsigned __int128)m) ++l;
    const unsigned __int128 num = (((unsigned __int128)1 << l) - m) << 64;
    L.magic = (uint64_t)(num / m) + 1;
    L.sh1 = l < 1 ? l : 1;
    L.sh2 = l > 1 ? l - 1 : 0;
    return L;
}

hipError_t launch_zero(uint64_t* p, uint64_t nwords, hipStream_t s) {
    if (!nwords) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(nwords, NT * 4)), dim3(NT), 0, s, p, nwords);
    return hipGetLastError();
}

hipError_t launch_zero32(uint32_t* p, uint64_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_zero32, dim3(grid_for(n, NT * 4)), dim3(NT), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fill(const uint64_t* keys, uint64_t n, uint64_t* W, const LevelHash& L,
                       hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, NT * 4)), dim3(NT), 0, s, keys, n,
                       (unsigned long long*)W, L);
    return hipGetLastError();
}

hipError_t launch_finalize(const uint64_t* W, uint64_t nwords, uint64_t* A, uint64_t* C,
                           unsigned long long* weight, hipStream_t s) {
    if (!nwords) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(nwords, NT * 4)), dim3(NT), 0, s,
                       (const ulonglong2*)W, nwords, A, C, weight);
    return hipGetLastError();
}

hipError_t launch_filter_fill(const uint64_t* Fin, uint64_t n, const uint64_t* words,
                              const LevelHash& Ld, uint64_t* Fout, uint64_t cap,
                              unsigned long long* count, uint64_t* W, const LevelHash& Lnext,
                              bool do_fill, hipStream_t s) {
    if (!n) return hipSuccess;
    constexpr int ITEMS = 16;
    hipLaunchKernelGGL(k_filter_fill<ITEMS>, dim3(grid_for(n, (uint64_t)NT * ITEMS)), dim3(NT), 0,
                       s, Fin, n, words, Ld, Fout, cap, count, (unsigned long long*)W, Lnext,
                       do_fill ? 1 : 0);
    return hipGetLastError();
}

uint64_t scan_tmp_tiles(uint64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t launch_exclusive_scan(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* tmp_tiles,
                                 hipStream_t s, const uint64_t* skip) {
    if (!n) return hipSuccess;
    if (n <= SCAN_SINGLE) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(NT), 0, s, in, out, n, skip);
        return hipGetLastError();
    }
    const uint64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)nt), dim3(NT), 0, s, in, n, tmp_tiles, skip);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(NT), 0, s, tmp_tiles, nt, skip);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(NT), 0, s, in, out, n, tmp_tiles, skip);
    return hipGetLastError();
}

uint64_t radix_tmp_counts(uint64_t n) { return 256 * ((n + RADIX_TILE - 1) / RADIX_TILE); }

hipError_t radix_sort_u64(uint64_t* a, uint64_t* b, uint64_t n, uint32_t* counts,
                          uint64_t* offsets, uint64_t* tmp_tiles, hipStream_t s) {
    if (n < 2) return hipSuccess;
    const uint64_t ntiles = (n + RADIX_TILE - 1) / RADIX_TILE;
    uint64_t* src = a;
    uint64_t* dst = b;
    for (int shift = 0; shift < 64; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(NT), 0, s, src, n, shift,
                           counts, ntiles);
        hipError_t e = launch_exclusive_scan(counts, offsets, 256 * ntiles, tmp_tiles, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(NT), 0, s, src, dst, n,
                           shift, offsets, ntiles);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t* t = src;
        src = dst;
        dst = t;
    }
    return hipSuccess;   // eight passes: the result is back in a
}

hipError_t launch_find_duplicates(const uint64_t* sorted, uint64_t n, unsigned long long* flag,
                                  hipStream_t s) {
    if (n < 2) return hipSuccess;
    hipLaunchKernelGGL(k_find_duplicates, dim3(grid_for(n, NT * 4)), dim3(NT), 0, s, sorted, n, flag);
    return hipGetLastError();
}

uint64_t sector_count(uint64_t total_bits) { return (total_bits + SEC_BITS - 1) / SEC_BITS; }
uint64_t super_count(uint64_t nsec) { return (nsec >> SUPER_SHIFT) + 1; }

hipError_t launch_rank_sectors(const uint64_t* words, uint64_t total_bits, uint32_t rank_sample, uint64_t* rank,
                               uint64_t nrank, uint32_t* sec, uint64_t* super, uint32_t* tmp_group_sums,
                               uint64_t* tmp_group_pre, uint64_t* tmp_tiles, hipStream_t s) {
    const uint64_t ns = sector_count(total_bits);
    if (!ns) return hipSuccess;
    if (rank_sample != 512 && rank_sample != 1024) return hipErrorInvalidValue;
    const uint64_t nw32 = total_bits / 32;
    const uint64_t ng = rank_sector_groups(total_bits);
    hipLaunchKernelGGL(k_sector_group_sums, dim3((unsigned)ng), dim3(SR_SECTORS), 0, s, (const uint32_t*)words, nw32,
                       tmp_group_sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_exclusive_scan(tmp_group_sums, tmp_group_pre, ng, tmp_tiles, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sector_layout, dim3((unsigned)ng), dim3(SR_SECTORS), 0, s, (const uint32_t*)words, nw32, ns,
                       rank_sample == 512 ? 9u : 10u, nrank, tmp_group_pre, sec, super, rank);
    return hipGetLastError();
}

uint64_t rank_sector_groups(uint64_t total_bits) { return (sector_count(total_bits) + SR_SECTORS - 1) / SR_SECTORS; }

hipError_t launch_lookup(const uint64_t* q, uint64_t n, uint64_t* out, const DevLevel* lev,
                         uint32_t nlev, const uint32_t* sec, const uint64_t* super,
                         const uint64_t* fb_keys, uint64_t nfb, uint64_t N, hipStream_t s) {
    if (!n) return hipSuccess;
    // short blocks (two passes of two queries per thread), as many as the queries need: measured
    // faster than a capped grid-stride grid (31.6-31.8 against 32.5 ms for 1e9 queries)
    hipLaunchKernelGGL(k_lookup, dim3(short_grid(n, NT * 4)), dim3(NT), 0, s, q, n, out, lev, nlev,
                       sec, super, fb_keys, nfb, N);
    return hipGetLastError();
}

hipError_t launch_report(unsigned long long* flag, const uint64_t* total, uint64_t* out, uint64_t seq,
                         unsigned long long* last, hipStream_t s) {
    hipLaunchKernelGGL(k_report, dim3(1), dim3(64), 0, s, flag, total, out, seq, last);
    return hipGetLastError();
}

hipError_t launch_positions(const uint64_t* keys, uint64_t n, const LevelHash& L, uint64_t* out,
                            hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_positions, dim3(grid_for(n, NT * 4)), dim3(NT), 0, s, keys, n, L, out);
    return hipGetLastError();
}

}  // namespace mphfk
