// Batched construction: many independent key sets built in one persistent launch.
//
// Each workgroup takes sets from an atomic work queue (largest first) and builds every level of
// its set by itself (Algorithms 1 and 2): the level's A and C bits live in LDS, the keys of the
// level are streamed from global memory (the set's own keys at level 0, its survivors in a scratch
// region after that, compacted in place), and the finalized A words go to the set's region of an
// unpacked bit buffer whose size per set is the worst case (every key surviving every level).
// A second kernel packs the sets' bits into one concatenated array; the rank table and the lookup
// sectors are then built over it like for a single function.  Set s gets labels 1..n_s: the ones of
// A before the key's bit minus the ones before the set's first bit, plus one.  Every set's levels,
// bits and labels equal those of a standalone build of that set, since the levels depend only on
// the set's keys, gamma and the level seeds.
#include <cmath>

#include "internal.h"

namespace mphfk {

namespace {

constexpr int BW = 256;   // threads per set-building workgroup

// One workgroup builds set s.
__global__ void __launch_bounds__(BW)
k_batch_build(const uint64_t* __restrict__ keys, const uint64_t* __restrict__ offsets,
              const uint32_t* __restrict__ order, uint64_t nsets, unsigned long long* next,
              uint64_t* __restrict__ scratch, const uint64_t* __restrict__ region_bit, double gamma,
              SeedTable seeds, uint32_t D, uint32_t left_cap, uint64_t* __restrict__ region,
              BatchSet* __restrict__ sets, BatchLevel* __restrict__ levels,
              uint64_t* __restrict__ left_sorted, uint32_t* __restrict__ bits32) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t wsum[BW / 64 + 1];
    __shared__ unsigned long long s_item;
    __shared__ LevelHash s_L;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(next, 1ull);
        __syncthreads();
        const uint64_t item = s_item;
        __syncthreads();
        if (item >= nsets) return;
        const uint32_t s = order[item];
        const uint64_t k0 = offsets[s];
        uint64_t n = offsets[s + 1] - k0;
        const uint64_t* F = keys + k0;
        uint64_t* scr = scratch + k0;
        uint64_t* A = region + region_bit[s] / 64;
        uint64_t off = 0;
        uint32_t d = 0;
        while (n > 0 && d < D) {
            const uint64_t m = (uint64_t)ceil(gamma * (double)n);
            const uint32_t aw = (uint32_t)((m + 31) >> 5);
            uint32_t* Ab = lds;
            uint32_t* Cb = lds + aw + (aw & 1);
            if (threadIdx.x == 0) s_L = device_level_hash(seeds.s[d], m, 0);
            for (uint32_t w = threadIdx.x; w < 2 * aw + 2; w += BW) lds[w] = 0;
            __syncthreads();
            const LevelHash L = s_L;
            for (uint64_t i = threadIdx.x; i < n; i += BW) {
                const uint32_t p = (uint32_t)level_pos(F[i], L);
                const uint32_t bit = 1u << (p & 31);
                const uint32_t old = atomicOr(&Ab[p >> 5], bit);
                if (old & bit) atomicOr(&Cb[p >> 5], bit);
            }
            __syncthreads();
            const uint64_t words = (m + 63) >> 6;
            for (uint32_t j = threadIdx.x; j < words; j += BW) {
                const uint32_t a0 = Ab[2 * j] & ~Cb[2 * j];
                const uint32_t a1 = Ab[2 * j + 1] & ~Cb[2 * j + 1];
                A[(off >> 6) + j] = (uint64_t)a0 | ((uint64_t)a1 << 32);
            }
            __syncthreads();
            for (uint32_t w = threadIdx.x; w < aw; w += BW) Ab[w] &= ~Cb[w];
            __syncthreads();
            // filter, compacted in place into the set's scratch region: each chunk is read into
            // registers before any of its survivors is written, and survivors only move left
            constexpr int FI = 8;
            uint64_t out = 0;
            for (uint64_t c0 = 0; c0 < n; c0 += BW * FI) {
                uint64_t kk[FI];
                uint32_t mask = 0;
#pragma unroll
                for (int it = 0; it < FI; ++it) {
                    const uint64_t i = c0 + it * BW + threadIdx.x;
                    kk[it] = 0;
                    if (i < n) {
                        kk[it] = F[i];
                        const uint32_t p = (uint32_t)level_pos(kk[it], L);
                        if (!((Ab[p >> 5] >> (p & 31)) & 1u)) mask |= 1u << it;
                    }
                }
                uint32_t tot;
                uint64_t o = out + block_exclusive_sum<BW>((uint32_t)__popc(mask), wsum, &tot);
#pragma unroll
                for (int it = 0; it < FI; ++it)
                    if ((mask >> it) & 1u) scr[o++] = kk[it];
                out += tot;
                __syncthreads();
            }
            if (threadIdx.x == 0) {
                BatchLevel& bl = levels[(uint64_t)s * D + d];
                bl.m = m;
                bl.magic = L.magic;
                bl.off = off;
                bl.n = (uint32_t)n;
                bl.sh = L.sh1 | (L.sh2 << 8);
            }
            n = out;
            off += 64 * words;
            F = scr;
            ++d;
        }
        // leftovers: sorted ascending by counting, in place of a general sort (there are almost
        // never more than a few; above left_cap the set is reported for a standalone build)
        uint32_t status = 0;
        if (n > left_cap) {
            status = 2;
        } else if (n > 0) {
            uint64_t* lk = (uint64_t*)lds;   // at most left_cap keys
            for (uint64_t i = threadIdx.x; i < n; i += BW) lk[i] = scr[i];
            __syncthreads();
            for (uint64_t i = threadIdx.x; i < n; i += BW) {
                const uint64_t x = lk[i];
                uint64_t r = 0;
                bool dup = false;
                for (uint64_t j = 0; j < n; ++j) {
                    const uint64_t y = lk[j];
                    r += (y < x) || (y == x && j < i);
                    dup |= (y == x && j != i);
                }
                left_sorted[k0 + r] = x;
                if (dup) atomicOr((unsigned int*)&sets[s].status, 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            sets[s].n = offsets[s + 1] - k0;
            sets[s].nlev = d;
            sets[s].nleft = (uint32_t)n;
            sets[s].bits = off;
            bits32[s] = (uint32_t)off;
            if (status) atomicOr((unsigned int*)&sets[s].status, status);
        }
        __syncthreads();
    }
}

// Packs every set's bits and fallback keys at their packed offsets; one workgroup per set.
__global__ void k_batch_pack(const uint64_t* __restrict__ region, const uint64_t* __restrict__ region_bit,
                             BatchSet* __restrict__ sets, const uint64_t* __restrict__ bit_pre,
                             const uint64_t* __restrict__ left_pre, const uint64_t* __restrict__ left_sorted,
                             const uint64_t* __restrict__ offsets, uint64_t* __restrict__ words,
                             uint64_t* __restrict__ left) {
    const uint64_t s = blockIdx.x;
    const uint64_t start = bit_pre[s];
    const uint64_t nw = sets[s].bits / 64;
    const uint64_t* src = region + region_bit[s] / 64;
    uint64_t* dst = words + start / 64;
    for (uint64_t j = threadIdx.x; j < nw; j += blockDim.x) dst[j] = src[j];
    const uint32_t nl = sets[s].nleft;
    for (uint32_t j = threadIdx.x; j < nl; j += blockDim.x) left[left_pre[s] + j] = left_sorted[offsets[s] + j];
    if (threadIdx.x == 0) {
        sets[s].start_bit = start;
        sets[s].left_off = left_pre[s];
    }
}

// u32 copy of one field of every set (0: bits, 1: nleft), the input of a prefix scan.
__global__ void k_u32_from_sets(const BatchSet* __restrict__ sets, uint64_t nsets, int field,
                                uint32_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s <= nsets; s += stride)
        out[s] = s < nsets ? (field == 0 ? (uint32_t)sets[s].bits : sets[s].nleft) : 0u;
}

__global__ void k_batch_ones_before(BatchSet* __restrict__ sets, const uint64_t* __restrict__ words,
                                    const uint64_t* __restrict__ rank, uint32_t rank_shift, uint64_t nsets) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nsets; s += stride) {
        const uint64_t g = sets[s].start_bit;   // a multiple of 64
        const uint64_t b = g >> rank_shift;
        uint64_t r = sets[s].bits ? rank[b] : 0;
        if (sets[s].bits)
            for (uint64_t k = (b << rank_shift) >> 6; k < (g >> 6); ++k) r += __popcll(words[k]);
        if (!sets[s].bits) {
            // an empty set has no bits; the value is never used
            r = 0;
        }
        sets[s].ones_before = r;
    }
}

// Lookup of (set, key) pairs: Algorithm 3 within the set, ranks through the sector layout.
__global__ void k_batch_lookup(const uint64_t* __restrict__ set_ids, const uint64_t* __restrict__ q, uint64_t n,
                               uint64_t* __restrict__ out, const BatchSet* __restrict__ sets,
                               const BatchLevel* __restrict__ levels, uint32_t D, uint64_t nsets,
                               const uint32_t* __restrict__ sec, const uint64_t* __restrict__ super,
                               const uint64_t* __restrict__ left, SeedTable seeds) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t s = set_ids[i];
        const uint64_t x = q[i];
        uint64_t label = 0;
        if (s < nsets) {
            const BatchSet st = sets[s];
            bool found = false;
            for (uint32_t d = 0; d < st.nlev; ++d) {
                const BatchLevel bl = levels[s * D + d];
                const uint64_t pos = mod_invariant(fmix64(x ^ seeds.s[d]), bl.m, bl.magic, bl.sh & 255u, bl.sh >> 8);
                const uint64_t g = st.start_bit + bl.off + pos;
                uint64_t rank;
                if (sector_rank(sec, super, g, &rank)) {
                    label = rank - st.ones_before + 1;
                    found = true;
                    break;
                }
            }
            if (!found && st.nleft) {
                const uint64_t* L = left + st.left_off;
                uint64_t lo = 0, hi = st.nleft;
                while (lo < hi) {
                    const uint64_t mid = (lo + hi) >> 1;
                    if (L[mid] < x) lo = mid + 1; else hi = mid;
                }
                if (lo < st.nleft && L[lo] == x) label = st.n - st.nleft + 1 + lo;
            }
        }
        out[i] = label;
    }
}

}  // namespace

hipError_t launch_batch_build(const uint64_t* keys, const uint64_t* offsets, const uint32_t* order,
                              uint64_t nsets, unsigned long long* next, uint64_t* scratch,
                              const uint64_t* region_bit, double gamma, const SeedTable& seeds,
                              uint32_t D, uint32_t left_cap, uint64_t* region, BatchSet* sets,
                              BatchLevel* levels, uint64_t* left_sorted, uint32_t* bits32,
                              uint64_t max_m, uint32_t grid, hipStream_t s) {
    const uint64_t lds = batch_lds_bytes(max_m, left_cap);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_batch_build,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_batch_build, dim3(grid), dim3(BW), (unsigned)lds, s, keys, offsets, order, nsets,
                       next, scratch, region_bit, gamma, seeds, D, left_cap, region, sets, levels,
                       left_sorted, bits32);
    return hipGetLastError();
}

uint64_t batch_lds_bytes(uint64_t max_m, uint32_t left_cap) {
    const uint64_t aw = (max_m + 31) / 32;
    uint64_t lds = (2 * aw + 4) * 4;
    if (lds < (uint64_t)left_cap * 8) lds = (uint64_t)left_cap * 8;
    return lds;
}

hipError_t launch_u32_from_sets(const BatchSet* sets, uint64_t nsets, int field, uint32_t* out,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_u32_from_sets, dim3((unsigned)((nsets + 256) / 256)), dim3(256), 0, s, sets, nsets,
                       field, out);
    return hipGetLastError();
}

hipError_t launch_batch_pack(const uint64_t* region, const uint64_t* region_bit, BatchSet* sets,
                             uint64_t nsets, const uint64_t* bit_pre, const uint64_t* left_pre,
                             const uint64_t* left_sorted, const uint64_t* offsets, uint64_t* words,
                             uint64_t* left, hipStream_t s) {
    if (!nsets) return hipSuccess;
    hipLaunchKernelGGL(k_batch_pack, dim3((unsigned)nsets), dim3(256), 0, s, region, region_bit, sets, bit_pre,
                       left_pre, left_sorted, offsets, words, left);
    return hipGetLastError();
}

hipError_t launch_batch_ones_before(BatchSet* sets, const uint64_t* words, const uint64_t* rank,
                                    uint32_t rank_shift, uint64_t nsets, hipStream_t s) {
    if (!nsets) return hipSuccess;
    hipLaunchKernelGGL(k_batch_ones_before, dim3((unsigned)((nsets + 255) / 256)), dim3(256), 0, s, sets,
                       words, rank, rank_shift, nsets);
    return hipGetLastError();
}

hipError_t launch_batch_lookup(const uint64_t* set_ids, const uint64_t* q, uint64_t n, uint64_t* out,
                               const BatchSet* sets, const BatchLevel* levels, uint32_t D, uint64_t nsets,
                               const uint32_t* sec, const uint64_t* super, const uint64_t* left,
                               const SeedTable& seeds, hipStream_t s) {
    if (!n) return hipSuccess;
    uint64_t blocks = (n + 1023) / 1024;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_batch_lookup, dim3((unsigned)blocks), dim3(256), 0, s, set_ids, q, n, out, sets,
                       levels, D, nsets, sec, super, left, seeds);
    return hipGetLastError();
}

}  // namespace mphfk
