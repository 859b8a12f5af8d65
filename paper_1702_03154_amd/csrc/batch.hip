// Batched construction: many independent key sets built in one persistent launch.
//
// A preparation pass checks the set offsets, sizes each set's worst-case regions (every key
// surviving every level) and orders the sets by size class, largest first.  Each workgroup of the
// build kernel then takes sets from an atomic work queue in that order and builds every level of
// its set by itself (Algorithms 1 and 2): the level's A and C bits live in LDS, the keys of the level
// are streamed from global memory (the set's own keys at level 0, its survivors in a scratch region
// after that, compacted in place), and the finalized A words go to the set's staging region.  When
// the set is done the workgroup writes the set's lookup sectors: 480 bits each with a counter of the
// ones of the set before the sector, so a label is the rank within the set plus one (Section 2.2,
// "Minimality", applied to the set alone).  Every set's levels, bits and labels equal those of a
// standalone build of that set, since the levels depend only on the set's keys, gamma and the
// level seeds.
//
// Nothing in a build after the preparation depends on a value read back by the host, so a planned
// batch rebuilds with a fixed sequence of launches (capturable in a HIP graph).  The one-shot build
// additionally packs the sectors and fallback keys densely once their sizes are known.
#include <cmath>

#include "internal.h"

namespace mphfk {

namespace {

constexpr int NCLASS = 65;          // size classes: 0 for an empty set, else floor(log2 n) + 1
constexpr int PT = 256;             // threads of the preparation kernels

__device__ __forceinline__ uint32_t size_class(uint64_t n) { return n ? 64u - (uint32_t)__clzll(n) : 0u; }

// Lanes below this one whose bit is set in mask.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Per set: staging words and lookup sectors (worst case, or the expected size with slack), size class
// histogram, offset checks and the largest set.  info[0]: largest n (atomicMax); info[1]: flags (1 offsets decrease, 2 offsets[0] != 0,
// 4 a set too large for the LDS levels).
__global__ void __launch_bounds__(PT)
k_batch_prepare(const uint64_t* __restrict__ offsets, uint64_t nsets, double gamma, uint32_t D, uint64_t max_m,
                double slack, uint32_t* __restrict__ bound, uint32_t* __restrict__ sbound, uint32_t* __restrict__ hist,
                unsigned long long* __restrict__ info) {
    __shared__ uint32_t lh[NCLASS];
    __shared__ unsigned long long smax;
    __shared__ uint32_t sflags;
    if (threadIdx.x < NCLASS) lh[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        smax = 0;
        sflags = 0;
    }
    __syncthreads();
    uint64_t my_max = 0;
    uint32_t flags = 0;
    const uint64_t stride = (uint64_t)gridDim.x * PT;
    for (uint64_t s = (uint64_t)blockIdx.x * PT + threadIdx.x; s <= nsets; s += stride) {
        if (s == nsets) {
            bound[s] = 0;
            sbound[s] = 0;
            continue;
        }
        const uint64_t a = offsets[s], b = offsets[s + 1];
        if (s == 0 && a != 0) flags |= 2;
        if (b < a) flags |= 1;
        const uint64_t n = b >= a ? b - a : 0;
        const double dm = ceil(gamma * (double)n);
        uint32_t w = 0, ns = 0;
        if (dm > (double)max_m) {
            flags |= 4;
        } else if (n) {
            // every level is at most m0 bits plus padding; with slack > 0, the expected total
            // (slack * m0 bits) plus one word of padding per level instead
            const uint64_t w0 = ((uint64_t)dm + 63) >> 6;
            const uint64_t tight = (uint64_t)ceil(slack * dm / 64.0) + D;
            w = (uint32_t)(slack > 0 && tight < D * w0 ? tight : D * w0);
            ns = (uint32_t)(((uint64_t)w * 64 + SEC_BITS - 1) / SEC_BITS);
        }
        bound[s] = w;
        sbound[s] = ns;
        my_max = n > my_max ? n : my_max;
        atomicAdd(&lh[size_class(n)], 1u);
    }
    atomicMax(&smax, (unsigned long long)my_max);
    if (flags) atomicOr(&sflags, flags);
    __syncthreads();
    if (threadIdx.x < NCLASS && lh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], lh[threadIdx.x]);
    if (threadIdx.x == 0) {
        atomicMax(&info[0], smax);
        if (sflags) atomicOr(&info[1], (unsigned long long)sflags);
    }
}

// The work queue: set indices in descending size class (any order within a class; the result does
// not depend on the order in which sets are built, only the load balance does).
__global__ void __launch_bounds__(PT)
k_batch_order(const uint64_t* __restrict__ offsets, uint64_t nsets, const uint32_t* __restrict__ hist,
              uint32_t* __restrict__ cursor, uint32_t* __restrict__ order) {
    __shared__ uint32_t gbase[NCLASS], lcnt[NCLASS], lbase[NCLASS];
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int c = NCLASS - 1; c >= 0; --c) {
            gbase[c] = acc;
            acc += hist[c];
        }
    }
    const uint64_t chunks = (nsets + PT - 1) / PT;
    for (uint64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        if (threadIdx.x < NCLASS) lcnt[threadIdx.x] = 0;
        __syncthreads();
        const uint64_t s = ch * PT + threadIdx.x;
        uint32_t c = 0, r = 0;
        if (s < nsets) {
            const uint64_t a = offsets[s], b = offsets[s + 1];
            c = size_class(b >= a ? b - a : 0);
            r = atomicAdd(&lcnt[c], 1u);
        }
        __syncthreads();
        if (threadIdx.x < NCLASS && lcnt[threadIdx.x])
            lbase[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], lcnt[threadIdx.x]);
        __syncthreads();
        if (s < nsets) order[gbase[c] + lbase[c] + r] = (uint32_t)s;
        __syncthreads();
    }
}

// Start of every build: empty work queues, no failure (fail[1] is the first failing set).
__global__ void k_batch_reset(unsigned long long* queue, uint32_t* fail) {
    if (threadIdx.x == 0) {
        queue[0] = 0;
        queue[1] = 0;
        fail[0] = 0;
        fail[1] = 0xFFFFFFFFu;
    }
}

// One workgroup of BW threads builds one set at a time, with FI keys per thread in flight in the
// level passes.  The sets come from two queues over `order` (descending size class): the large
// sets (class >= small_class) and after them the small ones.  Every small_every-th workgroup (none
// when 0) takes small sets first, so that their latency-bound levels run beside the large sets'
// streaming passes instead of after them; the others take large sets first.  A workgroup whose
// first queue is empty takes from the other.
template <int BW, int FI>
__global__ void __launch_bounds__(BW)
k_batch_build(const uint64_t* __restrict__ keys, const uint64_t* __restrict__ offsets,
              const uint32_t* __restrict__ order, uint64_t nsets, const uint32_t* __restrict__ hist,
              uint32_t small_class, uint32_t small_every, unsigned long long* next,
              uint64_t* __restrict__ scratch, const uint64_t* __restrict__ region_w, double gamma,
              SeedTable seeds, uint32_t D, uint32_t left_cap, uint64_t* __restrict__ region,
              uint32_t* __restrict__ sreg, const uint64_t* __restrict__ sreg_base,
              BatchSet* __restrict__ sets, BatchLevel* __restrict__ levels) {
    constexpr int NWAVE = BW / 64;
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t wsum[NWAVE + 1];
    __shared__ unsigned long long s_item;
    __shared__ uint32_t s_status;
    __shared__ LevelHash s_L;
    const uint32_t wave = threadIdx.x >> 6;
    // items [0, first_small) are the large sets
    uint64_t first_small = 0;
    if (threadIdx.x == 0)
        for (uint32_t c = small_class; c < (uint32_t)NCLASS; ++c) first_small += hist[c];
    const bool small_first = small_every && blockIdx.x % small_every == 0;
    bool large_left = true, small_left = true;   // (thread 0's view of the queues)
    for (;;) {
        if (threadIdx.x == 0) {
            uint64_t item = nsets;
            for (int t = 0; t < 2 && item == nsets; ++t) {
                if ((t == 0) == small_first) {
                    if (small_left) {
                        const uint64_t j = first_small + atomicAdd(&next[1], 1ull);
                        if (j < nsets) item = j; else small_left = false;
                    }
                } else if (large_left) {
                    const uint64_t i = atomicAdd(&next[0], 1ull);
                    if (i < first_small) item = i; else large_left = false;
                }
            }
            s_item = item;
            s_status = 0;
        }
        __syncthreads();
        const uint64_t item = s_item;
        __syncthreads();
        if (item >= nsets) return;
        const uint32_t s = order[item];
        const uint64_t k0 = offsets[s];
        uint64_t n = offsets[s + 1] - k0;
        const uint64_t* F = keys + k0;
        uint64_t* scr = scratch + k0;
        uint64_t* A = region + region_w[s];
        const uint64_t cap_bits = 64 * (region_w[s + 1] - region_w[s]);
        uint64_t off = 0;
        uint32_t d = 0;
        bool overflow = false;
        // A level's start: its size, its hash and A and C cleared in LDS; false (uniform) when the
        // set's staging region is too small, and the batch is redone larger.
        auto begin_level = [&](uint64_t& m, uint32_t*& Ab, uint32_t*& Cb, LevelHash& L) {
            m = (uint64_t)ceil(gamma * (double)n);
            if (off + 64 * ((m + 63) >> 6) > cap_bits) {
                overflow = true;
                return false;
            }
            const uint32_t aw = (uint32_t)((m + 31) >> 5);
            Ab = lds;
            Cb = lds + aw + (aw & 1);
            if (threadIdx.x == 0) s_L = device_level_hash(seeds.s[d], m, 0);
            for (uint32_t w = threadIdx.x; w < 2 * aw + 2; w += BW) lds[w] = 0;
            __syncthreads();
            L = s_L;
            return true;
        };
        // After the fill: the finalized A words to the set's staging region, and A &= ~C in LDS.
        auto finalize = [&](uint64_t m, uint32_t* Ab, const uint32_t* Cb) {
            __syncthreads();
            const uint64_t words = (m + 63) >> 6;
            for (uint32_t j = threadIdx.x; j < words; j += BW) {
                const uint32_t a0 = Ab[2 * j] & ~Cb[2 * j];
                const uint32_t a1 = Ab[2 * j + 1] & ~Cb[2 * j + 1];
                A[(off >> 6) + j] = (uint64_t)a0 | ((uint64_t)a1 << 32);
            }
            __syncthreads();
            for (uint32_t w = threadIdx.x; w < (uint32_t)((m + 31) >> 5); w += BW) Ab[w] &= ~Cb[w];
            __syncthreads();
        };
        auto test_and_set = [&](uint32_t* Ab, uint32_t* Cb, uint32_t p) {
            const uint32_t bit = 1u << (p & 31);
            const uint32_t old = atomicOr(&Ab[p >> 5], bit);
            if (old & bit) atomicOr(&Cb[p >> 5], bit);
        };
        // After the filter: the level's record, and the survivors become the next level's keys.
        auto end_level = [&](uint64_t m, const LevelHash& L, uint64_t nnext) {
            if (threadIdx.x == 0) {
                BatchLevel& bl = levels[(uint64_t)s * D + d];
                bl.m = m;
                bl.magic = L.magic;
                bl.off = off;
                bl.n = (uint32_t)n;
                bl.sh = L.sh1 | (L.sh2 << 8);
            }
            n = nnext;
            off += 64 * ((m + 63) >> 6);
            ++d;
        };
        // The kept items of every thread, in (wave, item, lane) order, to dst from base on (all
        // threads' values of wsum are read before it is written again).
        auto write_kept = [&](const uint64_t (&k)[FI], uint32_t kept, uint64_t* dst, uint64_t base) {
            uint32_t wc = 0;
#pragma unroll
            for (int it = 0; it < FI; ++it) wc += (uint32_t)__popcll(__ballot((kept >> it) & 1u));
            if (lane_id() == 0) wsum[wave] = wc;
            __syncthreads();
            uint32_t tot = 0;
#pragma unroll
            for (int w = 0; w < NWAVE; ++w) {
                const uint32_t v = wsum[w];
                if (w < (int)wave) base += v;
                tot += v;
            }
#pragma unroll
            for (int it = 0; it < FI; ++it) {
                const bool keep = (kept >> it) & 1u;
                const uint64_t bal = __ballot(keep);
                if (keep) dst[base + lanes_below(bal)] = k[it];
                base += (uint32_t)__popcll(bal);
            }
            __syncthreads();
            return tot;
        };
        auto load = [&](uint64_t (&k)[FI], uint64_t c0) {
#pragma unroll
            for (int it = 0; it < FI; ++it) {
                const uint64_t i = c0 + it * BW + threadIdx.x;
                k[it] = i < n ? F[i] : 0;
            }
        };

        // Levels of more than BW * FI keys: the keys streamed from global memory in chunks of
        // BW * FI, the next chunk's loads issued before the current one is processed.
        while (n > (uint64_t)(BW * FI) && d < D) {
            uint64_t m;
            uint32_t *Ab, *Cb;
            LevelHash L;
            if (!begin_level(m, Ab, Cb, L)) break;
            uint64_t kn[FI];
            load(kn, 0);
            for (uint64_t c0 = 0; c0 < n; c0 += BW * FI) {
                uint64_t kk[FI];
#pragma unroll
                for (int it = 0; it < FI; ++it) kk[it] = kn[it];
                if (c0 + BW * FI < n) load(kn, c0 + BW * FI);
#pragma unroll
                for (int it = 0; it < FI; ++it)
                    if (c0 + it * BW + threadIdx.x < n) test_and_set(Ab, Cb, level_pos32(kk[it], L));
            }
            finalize(m, Ab, Cb);
            // filter, compacted in place into the set's scratch region in key order: survivors only
            // move left, so the writes of chunk c stay below chunk c + 1, which every thread has
            // loaded (and waited for) before the barrier that precedes them
            uint64_t out = 0;
            load(kn, 0);
            for (uint64_t c0 = 0; c0 < n; c0 += BW * FI) {
                uint64_t kk[FI];
#pragma unroll
                for (int it = 0; it < FI; ++it) kk[it] = kn[it];
                if (c0 + BW * FI < n) load(kn, c0 + BW * FI);
                uint32_t sv = 0;
#pragma unroll
                for (int it = 0; it < FI; ++it) {
                    bool keep = false;
                    if (c0 + it * BW + threadIdx.x < n) {
                        const uint32_t p = level_pos32(kk[it], L);   // (a level in LDS: m < 2^32)
                        keep = !((Ab[p >> 5] >> (p & 31)) & 1u);
                    }
                    sv |= (uint32_t)keep << it;
                }
                out += write_kept(kk, sv, scr, out);
            }
            end_level(m, L, out);
            F = scr;
        }
        // The remaining levels (at most BW * FI keys) in registers: item it of a thread holds key
        // it * BW + thread while its bit in `live` is set, so no level reads or writes keys in
        // global memory; the keys left after the last level go to the front of the scratch region.
        if (n > 0 && d < D && !overflow) {
            uint64_t kr[FI];
            load(kr, 0);
            uint32_t live = 0;
#pragma unroll
            for (int it = 0; it < FI; ++it) live |= (uint32_t)(it * BW + threadIdx.x < n) << it;
            while (n > 0 && d < D) {
                uint64_t m;
                uint32_t *Ab, *Cb;
                LevelHash L;
                if (!begin_level(m, Ab, Cb, L)) break;
#pragma unroll
                for (int it = 0; it < FI; ++it)
                    if ((live >> it) & 1u) test_and_set(Ab, Cb, level_pos32(kr[it], L));
                finalize(m, Ab, Cb);
                uint32_t wc = 0, next = 0;
#pragma unroll
                for (int it = 0; it < FI; ++it) {
                    bool keep = false;
                    if ((live >> it) & 1u) {
                        const uint32_t p = level_pos32(kr[it], L);
                        keep = !((Ab[p >> 5] >> (p & 31)) & 1u);
                    }
                    next |= (uint32_t)keep << it;
                    wc += (uint32_t)__popcll(__ballot(keep));
                }
                live = next;
                if (lane_id() == 0) wsum[wave] = wc;
                __syncthreads();
                uint32_t tot = 0;
#pragma unroll
                for (int w = 0; w < NWAVE; ++w) tot += wsum[w];
                __syncthreads();
                end_level(m, L, tot);
            }
            if (n > 0 && !overflow) write_kept(kr, live, scr, 0);
        }
        // leftovers: sorted ascending by counting, back into the front of the set's scratch region
        // (there are almost never more than a few; above left_cap the set is reported and the batch
        // fails)
        if (n > 0 && n <= left_cap && !overflow) {
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
                scr[r] = x;
                if (dup) atomicOr(&s_status, 1u);
            }
        }
        __syncthreads();
        // the set's lookup sectors from its staged bits (written above by this workgroup)
        {
            const uint32_t* A32 = (const uint32_t*)A;
            const uint64_t w32 = off >> 5;
            const uint64_t nsec = (off + SEC_BITS - 1) / SEC_BITS;
            uint4* S = (uint4*)(sreg + sreg_base[s] * SEC_WORDS);
            uint32_t run = 0;
            for (uint64_t c0 = 0; c0 < nsec; c0 += BW) {
                const uint64_t k = c0 + threadIdx.x;
                uint32_t e[15];
                uint32_t c = 0;
#pragma unroll
                for (int j = 0; j < 15; ++j) {
                    const uint64_t idx = 15 * k + j;
                    e[j] = (k < nsec && idx < w32) ? A32[idx] : 0u;
                    c += __popc(e[j]);
                }
                uint32_t tot;
                const uint32_t ex = block_exclusive_sum<BW>(c, wsum, &tot);
                if (k < nsec) {
                    S[4 * k + 0] = make_uint4(run + ex, e[0], e[1], e[2]);
                    S[4 * k + 1] = make_uint4(e[3], e[4], e[5], e[6]);
                    S[4 * k + 2] = make_uint4(e[7], e[8], e[9], e[10]);
                    S[4 * k + 3] = make_uint4(e[11], e[12], e[13], e[14]);
                }
                run += tot;
            }
        }
        if (threadIdx.x == 0) {
            BatchSet& st = sets[s];
            st.n = offsets[s + 1] - k0;
            st.sec_base = sreg_base[s];
            st.bits = off;
            st.left_off = k0;
            st.nlev = d;
            st.nleft = (uint32_t)n;
            st.status = overflow ? 4u : (s_status | (n > left_cap ? 2u : 0u));
            st.pad = 0;
        }
        __syncthreads();
    }
}

// Per set: fallback-key and sector counts (inputs of the dense packing's prefix scans), and the OR
// of the statuses with the first failing set.  fail[0]: OR of statuses; fail[1]: first bad set.
__global__ void __launch_bounds__(PT)
k_batch_tally(const BatchSet* __restrict__ sets, uint64_t nsets, uint32_t* __restrict__ left32,
              uint32_t* __restrict__ sec32, uint32_t* __restrict__ fail) {
    const uint64_t stride = (uint64_t)gridDim.x * PT;
    for (uint64_t s = (uint64_t)blockIdx.x * PT + threadIdx.x; s <= nsets; s += stride) {
        if (s == nsets) {
            left32[s] = 0;
            sec32[s] = 0;
            continue;
        }
        const BatchSet st = sets[s];
        left32[s] = st.nleft;
        sec32[s] = (uint32_t)((st.bits + SEC_BITS - 1) / SEC_BITS);
        if (st.status) {
            atomicOr(&fail[0], st.status);
            atomicMin(&fail[1], (uint32_t)s);
        }
    }
}

// Dense copy of every set's sectors and fallback keys; one workgroup per set.
__global__ void k_batch_pack(const uint32_t* __restrict__ sreg, BatchSet* __restrict__ sets,
                             const uint64_t* __restrict__ sec_pre, const uint64_t* __restrict__ left_pre,
                             const uint64_t* __restrict__ scratch, uint32_t* __restrict__ sec,
                             uint64_t* __restrict__ left) {
    const uint64_t s = blockIdx.x;
    const BatchSet st = sets[s];
    const uint64_t n4 = 4 * ((st.bits + SEC_BITS - 1) / SEC_BITS);
    const uint4* src = (const uint4*)(sreg + st.sec_base * SEC_WORDS);
    uint4* dst = (uint4*)(sec + sec_pre[s] * SEC_WORDS);
    for (uint64_t j = threadIdx.x; j < n4; j += blockDim.x) dst[j] = src[j];
    for (uint32_t j = threadIdx.x; j < st.nleft; j += blockDim.x) left[left_pre[s] + j] = scratch[st.left_off + j];
    __syncthreads();
    if (threadIdx.x == 0) {
        sets[s].sec_base = sec_pre[s];
        sets[s].left_off = left_pre[s];
    }
}

// Per set: the lookup records: the 16-byte head, levels 2.. in the set's D - 2 slots, the fallback
// record.
__global__ void __launch_bounds__(PT)
k_batch_heads(const BatchSet* __restrict__ sets, const BatchLevel* __restrict__ levels, uint32_t D,
              uint64_t nsets, BatchHead* __restrict__ heads, BatchLev* __restrict__ lev, BatchAux* __restrict__ aux) {
    const uint64_t stride = (uint64_t)gridDim.x * PT;
    for (uint64_t s = (uint64_t)blockIdx.x * PT + threadIdx.x; s < nsets; s += stride) {
        const BatchSet st = sets[s];
        const BatchLevel* L = levels + s * D;
        const uint64_t m0 = st.nlev > 0 ? L[0].m : 0, m1 = st.nlev > 1 ? L[1].m : 0;
        BatchHead h;
        h.a = st.sec_base | (m0 << HEAD_BASE_BITS);
        h.b = m1 | ((uint64_t)st.nlev << HEAD_M_BITS);
        heads[s] = h;
        BatchAux x;
        x.left_off = st.left_off;
        x.n = (uint32_t)st.n;
        x.nleft = st.nleft;
        aux[s] = x;
        for (uint32_t d = 2; d < st.nlev; ++d) {
            BatchLev e;
            e.m = (uint32_t)L[d].m;
            e.off = (uint32_t)L[d].off;
            lev[s * (D - 2) + d - 2] = e;
        }
    }
}

// h mod m for 1 <= m < 2^20, exactly: two base-2^32 digits of the long division, each quotient
// estimated with the fp64 reciprocal rm = 1/m (error far below one unit) and corrected by one step.
// All intermediate remainders lie in (-m, 2m), so 32-bit wrapping arithmetic holds them exactly.
__device__ __forceinline__ uint32_t mod_small(uint64_t h, uint32_t m, double rm) {
    const uint32_t hi = (uint32_t)(h >> 32), lo = (uint32_t)h;
    uint32_t q = (uint32_t)((double)hi * rm);
    int32_t r = (int32_t)(hi - q * m);
    r += r < 0 ? (int32_t)m : 0;
    r -= r >= (int32_t)m ? (int32_t)m : 0;
    const double x = fma((double)(uint32_t)r, 4294967296.0, (double)lo);   // r * 2^32 + lo < 2^52
    q = (uint32_t)(x * rm);
    r = (int32_t)(lo - q * m);
    r += r < 0 ? (int32_t)m : 0;
    r -= r >= (int32_t)m ? (int32_t)m : 0;
    return (uint32_t)r;
}

// Lookup of (set, key) pairs: Algorithm 3 within the set, ranks through the set's sectors.
__global__ void __launch_bounds__(256)
k_batch_lookup(const uint64_t* __restrict__ set_ids, const uint64_t* __restrict__ q, uint64_t n,
               uint64_t* __restrict__ out, const BatchHead* __restrict__ heads, const BatchLev* __restrict__ lev,
               const BatchAux* __restrict__ aux, uint32_t D, uint64_t nsets, const uint32_t* __restrict__ sec,
               const uint64_t* __restrict__ left, SeedTable seeds) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t s = set_ids[i];
        const uint64_t x = q[i];
        uint64_t label = 0;
        if (s < nsets) {
            const BatchHead h = heads[s];
            const uint64_t base = h.a & ((1ull << HEAD_BASE_BITS) - 1);
            const uint32_t m0 = (uint32_t)(h.a >> HEAD_BASE_BITS);
            const uint32_t m1 = (uint32_t)h.b & ((1u << HEAD_M_BITS) - 1);
            const uint32_t nlev = (uint32_t)(h.b >> HEAD_M_BITS);
            bool found = false;
            for (uint32_t d = 0; d < nlev; ++d) {
                uint32_t m, off;
                if (d == 0) {
                    m = m0;
                    off = 0;
                } else if (d == 1) {
                    m = m1;
                    off = (m0 + 63u) & ~63u;
                } else {
                    const BatchLev e = lev[s * (D - 2) + d - 2];
                    m = e.m;
                    off = e.off;
                }
                const uint32_t g = off + mod_small(fmix64(x ^ seeds.s[d]), m, 1.0 / (double)m);
                const uint32_t j = g / (uint32_t)SEC_BITS;
                uint32_t c;
                if (sector_probe(sec, base + j, g - j * (uint32_t)SEC_BITS, &c)) {
                    label = (uint64_t)c + 1;
                    found = true;
                    break;
                }
            }
            if (!found) {
                const BatchAux ax = aux[s];
                if (ax.nleft) {
                    const uint64_t* L = left + ax.left_off;
                    uint32_t lo = 0, hi = ax.nleft;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (L[mid] < x) lo = mid + 1; else hi = mid;
                    }
                    if (lo < ax.nleft && L[lo] == x) label = ax.n - ax.nleft + 1 + lo;
                }
            }
        }
        out[i] = label;
    }
}

// The build kernel for a launch configuration, or null if it is not one of the compiled ones.
const void* batch_kernel(const BatchLaunch& cfg) {
#define MPHF_BATCH_CASE(T, I) \
    if (cfg.threads == T && cfg.items == I) return (const void*)k_batch_build<T, I>;
    MPHF_BATCH_CASE(128, 4)
    MPHF_BATCH_CASE(128, 8)
    MPHF_BATCH_CASE(128, 16)
    MPHF_BATCH_CASE(256, 4)
    MPHF_BATCH_CASE(256, 8)
    MPHF_BATCH_CASE(256, 16)
    MPHF_BATCH_CASE(512, 4)
    MPHF_BATCH_CASE(512, 8)
    MPHF_BATCH_CASE(512, 16)
#undef MPHF_BATCH_CASE
    return nullptr;
}

uint32_t prep_grid(uint64_t items) {
    const uint64_t g = (items + PT - 1) / PT;
    return (uint32_t)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

}  // namespace

uint32_t batch_classes() { return NCLASS; }

hipError_t launch_batch_prepare(const uint64_t* offsets, uint64_t nsets, double gamma, uint32_t D, uint64_t max_m,
                                double slack, uint32_t* bound, uint32_t* sbound, uint32_t* hist,
                                unsigned long long* info, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_prepare, dim3(prep_grid(nsets + 1)), dim3(PT), 0, s, offsets, nsets, gamma, D,
                       max_m, slack, bound, sbound, hist, info);
    return hipGetLastError();
}

hipError_t launch_batch_order(const uint64_t* offsets, uint64_t nsets, const uint32_t* hist, uint32_t* cursor,
                              uint32_t* order, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_order, dim3(prep_grid(nsets)), dim3(PT), 0, s, offsets, nsets, hist, cursor, order);
    return hipGetLastError();
}

hipError_t launch_batch_reset(unsigned long long* queue, uint32_t* fail, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, queue, fail);
    return hipGetLastError();
}

hipError_t launch_batch_build(const uint64_t* keys, const uint64_t* offsets, const uint32_t* order,
                              uint64_t nsets, const uint32_t* hist, unsigned long long* next, uint64_t* scratch,
                              const uint64_t* region_w, double gamma, const SeedTable& seeds,
                              uint32_t D, uint32_t left_cap, uint64_t* region, uint32_t* sreg,
                              const uint64_t* sreg_base, BatchSet* sets, BatchLevel* levels, uint64_t max_m,
                              const BatchLaunch& cfg, uint32_t grid, hipStream_t s) {
    const uint64_t lds = batch_lds_bytes(max_m, left_cap);
    const void* k = batch_kernel(cfg);
    if (!k) return hipErrorInvalidValue;
    uint32_t small_class = cfg.small_class, small_every = cfg.small_every;
    void* args[] = {(void*)&keys, (void*)&offsets, (void*)&order, (void*)&nsets, (void*)&hist,
                    (void*)&small_class, (void*)&small_every, (void*)&next, (void*)&scratch,
                    (void*)&region_w, (void*)&gamma, (void*)&seeds, (void*)&D, (void*)&left_cap, (void*)&region,
                    (void*)&sreg, (void*)&sreg_base, (void*)&sets, (void*)&levels};
    return hipLaunchKernel(k, dim3(grid), dim3(cfg.threads), args, (size_t)lds, s);
}

hipError_t batch_kernel_setup(const BatchLaunch& cfg, uint64_t max_m, uint32_t left_cap) {
    const void* k = batch_kernel(cfg);
    if (!k) return hipErrorInvalidValue;
    const uint64_t lds = batch_lds_bytes(max_m, left_cap);
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

uint64_t batch_lds_bytes(uint64_t max_m, uint32_t left_cap) {
    const uint64_t aw = (max_m + 31) / 32;
    uint64_t lds = (2 * aw + 4) * 4;
    if (lds < (uint64_t)left_cap * 8) lds = (uint64_t)left_cap * 8;
    return lds;
}

hipError_t launch_batch_tally(const BatchSet* sets, uint64_t nsets, uint32_t* left32, uint32_t* sec32,
                              uint32_t* fail, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_tally, dim3(prep_grid(nsets + 1)), dim3(PT), 0, s, sets, nsets, left32, sec32,
                       fail);
    return hipGetLastError();
}

hipError_t launch_batch_pack(const uint32_t* sreg, BatchSet* sets, uint64_t nsets, const uint64_t* sec_pre,
                             const uint64_t* left_pre, const uint64_t* scratch, uint32_t* sec, uint64_t* left,
                             hipStream_t s) {
    if (!nsets) return hipSuccess;
    hipLaunchKernelGGL(k_batch_pack, dim3((unsigned)nsets), dim3(256), 0, s, sreg, sets, sec_pre, left_pre, scratch,
                       sec, left);
    return hipGetLastError();
}

hipError_t launch_batch_heads(const BatchSet* sets, const BatchLevel* levels, uint32_t D, uint64_t nsets,
                              BatchHead* heads, BatchLev* lev, BatchAux* aux, hipStream_t s) {
    if (!nsets) return hipSuccess;
    hipLaunchKernelGGL(k_batch_heads, dim3(prep_grid(nsets)), dim3(PT), 0, s, sets, levels, D, nsets, heads, lev,
                       aux);
    return hipGetLastError();
}

hipError_t launch_batch_lookup(const uint64_t* set_ids, const uint64_t* q, uint64_t n, uint64_t* out,
                               const BatchHead* heads, const BatchLev* lev, const BatchAux* aux, uint32_t D,
                               uint64_t nsets, const uint32_t* sec, const uint64_t* left, const SeedTable& seeds,
                               hipStream_t s) {
    if (!n) return hipSuccess;
    // short blocks (four queries per thread), as many as the queries need, at most 2^24 - 1
    uint64_t blocks = (n + 1023) / 1024;
    if (blocks > (1ull << 24) - 1) blocks = (1ull << 24) - 1;
    hipLaunchKernelGGL(k_batch_lookup, dim3((unsigned)blocks), dim3(256), 0, s, set_ids, q, n, out, heads, lev, aux,
                       D, nsets, sec, left, seeds);
    return hipGetLastError();
}

}  // namespace mphfk
