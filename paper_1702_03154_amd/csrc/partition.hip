// Position-partitioned level construction for gfx950.
//
// Global atomics on MI355X run at a few tens of billions per second whatever the footprint,
// while LDS atomics and streaming reads are one to two orders of magnitude faster.  So a large
// level is not filled with global atomics: its keys are first radix-partitioned by position
// bucket (one or two streaming passes of at most 2^DBITS-way fan-out), then one workgroup per
// bucket runs the level's fill, finalize and filter (Algorithms 1 and 2) entirely in LDS:
// 2^pbits positions (A and C halves) plus the bucket's keys.  The bit arrays produced are the
// same as with any other order of insertion, because a bit of A_d survives iff exactly one key
// of F_d lands on it.
//
// The partition passes and the bucket pass carry, instead of the key x, the level hash
// h = fmix64(x ^ s_d) (one pass) or the pair (q, pos) with h = q m_d + pos (two passes, packed into
// 8 bytes below): the bucket pass gets h and then x back for the survivors with the exact inverse
// of fmix64, so every record stays 8 bytes and only the first pass divides by m_d.
//
// Data layout of a partitioned set: "regions" of fixed capacity `cap` keys, region r starting at
// base + r * cap, with its key count in cnt[r] (counts above cap mean the region overflowed and
// the level has to be redone another way).  A pass writes region (bin * S + slot): bin = output
// bucket (or coarse bin), slot = the writing workgroup's index within its group, so every
// region has exactly one writer and no global atomic is needed.
//
// The last levels, once the remaining keys fit in one workgroup's LDS, are all built by one
// workgroup in one launch (k_tail).
#include <cmath>

#include "internal.h"

#ifndef MPHF_WIDE_WC
#define MPHF_WIDE_WC 1
#endif

namespace mphfk {

namespace {

constexpr int PT = 768;               // threads of the partition kernel
constexpr int PITEMS = 4;             // keys per thread per tile
constexpr int PTILE = PT * PITEMS;    // keys per tile
constexpr int TSEG = 64;              // input segments one tile may span
constexpr int BT = 1024;              // threads of the tail kernel
constexpr int KT = 1024;              // threads of the bucket kernel
constexpr int POOL_WORDS = 19712;     // 154 KiB of LDS for the tail kernel's keys and bits
constexpr int BUCKET_LDS = 49152;     // bytes of LDS for a bucket's local positions and bits

// The segment holding dense index i: the last s in [s0, s1) with pre[s] <= i.
__device__ __forceinline__ uint32_t find_segment(const uint64_t* __restrict__ pre, uint32_t s0,
                                                 uint32_t s1, uint64_t i) {
    uint32_t lo = s0, hi = s1;   // pre[lo] <= i < pre[hi] is kept
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------- radix partition pass
//
// Workgroup g = group * K + slot reads the dense index range `slot` of K equal parts of its
// group's input segments [group*SG, group*SG + SG) (segment s: keys at in + s*in_stride, count
// pre[s+1] - pre[s]) and writes each key to output region (bin * S_out + slot), where
// bin = (pos_d(key) >> pbits) >> out_shift.  In a second pass every group is one coarse bin of
// the first, so its keys fall in bins (group << group_shift) + [0, 2^group_shift); otherwise
// the bins start at 0.  Either way a workgroup sees at most 2^DBITS bins, and a key outside the
// bins its group owns is a configuration error (flag 4), never written.  The input holds keys
// (HASHED = false: h = fmix64(x ^ s_d) is computed here) or the records of an earlier pass
// (HASHED = true); DIG says what the bins and the output records are: DIG = 0 bins by level
// position and writes h.
//
// A tile is counting-sorted by bin in LDS.  With lines combined (WC) a workgroup also keeps, per
// bin, the keys of its last unfinished line in LDS, and a tile writes only whole lines, each at a
// line boundary of the bin's region (out_cap is a multiple of 16) and written once, by adjacent
// lanes: 128-byte lines of 16 keys with 2^8 bins, 64-byte half lines of 8 keys with 2^10 bins
// (whose 128-byte lines would not fit in LDS beside the tile; the workgroup then holds a whole
// compute unit's LDS).  The runs of a tile average 12 or 3 keys per bin, so writing them where
// they fall would split most lines between tiles and writes.  The unfinished lines go out at the
// end.  Without WC (one-pass levels of 2^10 bins, or WIDE_WC off) the runs are written as they are.
//
// Tiles: with SPAN = false a tile is up to PTILE keys from the segment holding its start and the
// next segment, and the next tile's keys are loaded while the current one is sorted and written.  With
// SPAN = true (inputs of small segments) a tile is a dense range across up to TSEG segments, each
// key found in the segment boundaries staged in LDS.
//
// DIG = 3 or 5 (first of two passes; 5 when m < 2^32) writes, instead of h, the packed record
// (q << pack_shift) | (pos mod 2^pack_shift) where h = q m + pos: with pack_shift = the coarse
// bin's bits the record keeps everything the later passes need (q < 2^64 / m fits above them, the
// bin is the region) and spares them the division.  DIG = 4 (second pass) reads such records and writes
// (q << pbits) | (pos mod 2^pbits) for the bucket pass, which forms h = q m + pos again and
// recovers the surviving keys from it.
//
// DIG = 1 or 2 partitions by the top bits of h instead of its level position: pos = h >> L.sh1
// (the hash-set partition of a key set into 2^(64 - sh1) independent sets).  DIG = 2 writes the
// keys themselves (not their hashes) densely: bin d of this workgroup starts at dbase[(bin_base +
// d) * S_out + slot] of out, counted beforehand by k_slice_counts over the same slices.  With
// lines combined (WC) the bin's lines are counted from the line holding that start, and only the
// workgroup's own keys of its first and last lines are written.

// Keys per combined line: a 128-byte line with 2^8 bins, a 64-byte half line with 2^10 bins.
template <int NB>
constexpr int line_keys() { return NB > 256 ? 8 : 16; }
// 2^10-bin passes with combined lines (else their runs are written as they fall).
constexpr bool WIDE_WC = MPHF_WIDE_WC;

// Keys generated instead of read (a first pass over a chunk of a generated stream): the key of
// dense index i is stream_key(seed, start + i).
struct GenKeys {
    uint64_t seed, start;
    uint32_t on;
};

template <int NB, bool WC, bool DENSE>
struct PartLds {
    static constexpr int LW = line_keys<NB>();
    static constexpr int MAXL = WC ? (PTILE + NB * (LW - 1)) / LW + 1 : 1;
    // the tile sorted by bin in kbuf[0, PTILE); with WC, the unfinished line of bin d in
    // kbuf[PTILE + d * LW, PTILE + d * LW + LW) (one array, so a key is read from either by index)
    uint64_t kbuf[PTILE + (WC ? NB * LW : 0)];
    uint16_t sdig[WC ? 1 : PTILE];  // bin of each sorted key (runs written as they are)
    uint32_t hist[NB];              // keys of the tile per bin
    uint32_t hoff[NB];              // first sorted position of the bin
    uint32_t run[NB];               // keys of the bin so far, this tile included once scanned
    uint32_t rold[WC ? NB : 1];     // run[] before the tile
    uint32_t fpre[WC ? NB : 1];     // first key of the bin in the tile's flush order
    uint16_t lbin[MAXL];            // bin of each whole line the tile writes
    uint32_t wsum[PT / 64 + 1];
    uint32_t nf;                    // keys in whole lines this tile
    uint64_t sp[TSEG + 1];          // pre[s .. s + TSEG] of a spanning tile
    uint64_t dst[NB];               // the bin's output at obase + dst (dense: first key at dst + a0, dst on a line)
    uint32_t a0[DENSE ? NB : 1];
};

// One tile of tn keys.  k[] holds a value for every item (items j >= tn hold copies and are
// ignored); every value goes through the digit computation, so that the tile's loads are
// consumed on every path.
template <int NB, bool WC, bool HASHED, int DIG>
__device__ __forceinline__ void part_tile(PartLds<NB, WC, DIG == 2>& S, uint64_t (&k)[PITEMS], uint32_t tn,
                                          const LevelHash& L, uint32_t pbits, uint32_t out_shift,
                                          uint32_t pack_shift, uint64_t bin_base, uint64_t lim,
                                          uint64_t* __restrict__ obase, uint64_t out_cap,
                                          unsigned long long* overflow) {
    constexpr int LW = line_keys<NB>();
    uint32_t dg[PITEMS], rk[PITEMS];
    bool bad = false;
#pragma unroll
    for (int it = 0; it < PITEMS; ++it) {
        const uint32_t j = it * PT + threadIdx.x;
        uint64_t bin;
        bool in_range;   // the bin is one this workgroup may write
        if constexpr (DIG == 5) {
            // m < 2^32 (first of two passes, never grouped): pos < 2^32, so the low 32 bits of
            // h - q m are all of it, and the bin is a 32-bit shift of it
            const uint64_t h = HASHED ? k[it] : fmix64(k[it] ^ L.seed);
            const uint64_t t = __umul64hi(L.magic, h);
            const uint64_t q = (t + ((h - t) >> L.sh1)) >> L.sh2;
            const uint32_t pos = (uint32_t)h - (uint32_t)q * (uint32_t)L.m;
            const uint32_t b32 = pos >> (pbits + out_shift);
            bin = b32;
            in_range = b32 < (uint32_t)lim;
            k[it] = (q << pack_shift) | (pos & ((1ull << pack_shift) - 1));
        } else if constexpr (DIG == 4) {
            // packed input (q << pack_shift) | (position inside the group's coarse bin): the
            // bucket is known without a division; the output keeps q and the position inside the
            // bucket
            const uint64_t local = k[it] & ((1ull << pack_shift) - 1);
            bin = bin_base + (local >> pbits);
            k[it] = ((k[it] >> pack_shift) << pbits) | (local & ((1ull << pbits) - 1));
        } else if constexpr (DIG == 3) {
            // level position of h = q * m + pos, written as (q << pack_shift) | (pos mod 2^pack_shift)
            const uint64_t h = HASHED ? k[it] : fmix64(k[it] ^ L.seed);
            uint64_t q;
            const uint64_t pos = divmod_invariant(h, L.m, L.magic, L.sh1, L.sh2, &q);
            bin = (pos >> pbits) >> out_shift;
            k[it] = (q << pack_shift) | (pos & ((1ull << pack_shift) - 1));
        } else {
            const uint64_t h = HASHED ? k[it] : fmix64(k[it] ^ L.seed);
            const uint64_t pos = DIG ? h >> L.sh1 : mod_invariant(h, L.m, L.magic, L.sh1, L.sh2);
            bin = (pos >> pbits) >> out_shift;
            if (DIG == 2) {   // dense output holds the keys
                if (HASHED) k[it] = unfmix64(h) ^ L.seed;
            } else {
                k[it] = h;
            }
        }
        // bin - bin_base wraps above lim (<= 2^DBITS) for a bin below the group's first
        const uint64_t rel = DIG == 5 ? bin : bin - bin_base;
        if constexpr (DIG != 5) in_range = rel < lim;
        const bool ok = j < tn && in_range;
        bad |= j < tn && !ok;
        dg[it] = ok ? (uint32_t)rel : (uint32_t)NB;
        rk[it] = 0;
        if (ok) rk[it] = atomicAdd(&S.hist[dg[it]], 1u);
    }
    if (bad) atomicOr(overflow, 4ull);   // a configuration error: never silently dropped
    __syncthreads();
    if constexpr (WC) {
        // One scan gives both the tile's sorted offsets (low half) and the flush order of the
        // lines it completes (high half): bin d completes the lines between floor(run/LW) and
        // floor((run + h)/LW).  Both sums stay below 2^16 (PTILE keys; PTILE + NB (LW - 1) at
        // most in whole lines).  A thread takes BPT consecutive bins.
        constexpr int BPT = (NB + PT - 1) / PT;
        uint32_t h[BPT], r[BPT], f[BPT], sum = 0;
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int d = threadIdx.x * BPT + b;
            h[b] = r[b] = f[b] = 0;
            if (d < NB) {
                h[b] = S.hist[d];
                r[b] = S.run[d];
                f[b] = ((r[b] + h[b]) & ~(uint32_t)(LW - 1)) - (r[b] & ~(uint32_t)(LW - 1));
            }
            sum += h[b] | (f[b] << 16);
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_sum<PT>(sum, S.wsum, &tot);
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int d = threadIdx.x * BPT + b;
            if (d < NB) {
                S.hoff[d] = ex & 0xFFFFu;
                S.fpre[d] = ex >> 16;
                S.rold[d] = r[b];
                S.run[d] = r[b] + h[b];
                S.hist[d] = 0;
                const uint32_t l0 = (ex >> 16) / LW;
                for (uint32_t q = 0; q < f[b] / LW; ++q) S.lbin[l0 + q] = (uint16_t)d;
            }
            ex += h[b] | (f[b] << 16);
        }
        if (threadIdx.x == 0) S.nf = tot >> 16;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < PITEMS; ++it)
            if (dg[it] < (uint32_t)NB) S.kbuf[S.hoff[dg[it]] + rk[it]] = k[it];
        __syncthreads();
        // whole lines: key g of bin d comes from the unfinished line (g < run before the tile)
        // or from the tile's sorted run
        const uint32_t nf = S.nf;
        if constexpr (DIG == 2) {
            for (uint32_t f = threadIdx.x; f < nf; f += PT) {
                const uint32_t d = S.lbin[f / LW];
                const uint32_t r = S.rold[d];
                const uint32_t g = (r & ~(uint32_t)(LW - 1)) + (f - S.fpre[d]);
                // the key's index in the unfinished line (g < r) or in the sorted tile, blended with a
                // mask rather than a branch (the lanes of a line take both sides)
                const uint32_t ic = PTILE + d * LW + (g & (LW - 1));
                const uint32_t it = S.hoff[d] + (g - r);
                const uint64_t v = S.kbuf[ic + ((it - ic) & (0u - (uint32_t)(g >= r)))];
                if (g >= S.a0[d]) obase[S.dst[d] + g] = v;
            }
        } else {
            // four consecutive keys of a line per lane (two 16-byte stores; four lanes per line): the
            // line's bookkeeping is read and computed once per four keys
            for (uint32_t f = 4 * threadIdx.x; f < nf; f += 4 * PT) {
                const uint32_t d = S.lbin[f / LW];
                const uint32_t r = S.rold[d];
                const uint32_t g = (r & ~(uint32_t)(LW - 1)) + (f - S.fpre[d]);   // a multiple of 4
                const uint32_t ic = PTILE + d * LW + (g & (LW - 1));
                const uint32_t it = S.hoff[d] + (g - r);
                uint64_t v[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u)
                    v[u] = S.kbuf[(g + u >= r) ? it + u : ic + u];
                if (g < out_cap) {   // out_cap is a multiple of 16: the four keys are in or out together
                    ulonglong2* o = (ulonglong2*)(obase + S.dst[d] + g);
                    o[0] = make_ulonglong2(v[0], v[1]);
                    o[1] = make_ulonglong2(v[2], v[3]);
                }
            }
        }
        __syncthreads();
        // keys past the last whole line start the bin's next unfinished line (run[] already
        // counts the tile)
#pragma unroll
        for (int it = 0; it < PITEMS; ++it) {
            if (dg[it] < (uint32_t)NB) {
                const uint32_t g = S.rold[dg[it]] + rk[it];
                if (g >= (S.run[dg[it]] & ~(uint32_t)(LW - 1))) S.kbuf[PTILE + dg[it] * LW + (g & (LW - 1))] = k[it];
            }
        }
    } else {
        {   // exclusive scan of the tile histogram
            constexpr int PER = (NB + PT - 1) / PT;   // bins per thread
            uint32_t v[PER];
            uint32_t sum = 0;
            const int b0 = threadIdx.x * PER;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                v[q] = (b0 + q < NB) ? S.hist[b0 + q] : 0;
                sum += v[q];
            }
            uint32_t tot;
            uint32_t ex = block_exclusive_sum<PT>(sum, S.wsum, &tot);
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (b0 + q < NB) {
                    S.hoff[b0 + q] = ex;
                    ex += v[q];
                }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < PITEMS; ++it) {
            if (dg[it] < (uint32_t)NB) {
                const uint32_t p = S.hoff[dg[it]] + rk[it];
                S.kbuf[p] = k[it];
                S.sdig[p] = (uint16_t)dg[it];
            }
        }
        __syncthreads();
        // write the runs: position p of the sorted tile goes to its bin's region
        for (uint32_t p = threadIdx.x; p < tn; p += PT) {
            const uint32_t d = S.sdig[p];
            const uint64_t o = (uint64_t)S.run[d] + (p - S.hoff[d]);
            if (DIG == 2 || o < out_cap) obase[S.dst[d] + o] = S.kbuf[p];
        }
        __syncthreads();
        for (int d = threadIdx.x; d < NB; d += PT) {
            S.run[d] += S.hist[d];
            S.hist[d] = 0;
        }
        __syncthreads();
    }
}

// Loads a tile of tn >= 1 keys: its first n1 from src1, the rest from src2 (the start of the next
// segment); items past the tile load the last key again.
__device__ __forceinline__ void load_tile(uint64_t (&k)[PITEMS], const uint64_t* __restrict__ src1, uint32_t n1,
                                          const uint64_t* __restrict__ src2, uint32_t tn) {
#pragma unroll
    for (int it = 0; it < PITEMS; ++it) {
        const uint32_t j0 = it * PT + threadIdx.x;
        const uint32_t j = j0 < tn ? j0 : tn - 1;
        k[it] = j < n1 ? src1[j] : src2[j - n1];
    }
}

// (6 waves per SIMD: two workgroups of 12 waves per compute unit, as the LDS allows, at 80 VGPRs)
template <int DBITS, bool HASHED, bool SPAN, int DIG, bool GEN = false>
__global__ void __launch_bounds__(PT, 6)
k_partition(const uint64_t* __restrict__ in, uint64_t in_stride, const uint64_t* __restrict__ pre,
            uint32_t SG, uint32_t K, LevelHash L, uint32_t pbits, uint32_t out_shift, uint32_t pack_shift,
            uint32_t grouped, uint32_t group_shift, uint64_t nbins, uint64_t* __restrict__ out,
            uint64_t out_cap, uint32_t S_out, uint32_t* __restrict__ out_cnt,
            unsigned long long* overflow, const uint64_t* __restrict__ dbase, SpecArgs spec, GenKeys gk) {
    if (spec.mode) {   // a level queued ahead: its hash from the device, or nothing to do
        __shared__ SpecLevel sl;
        if (threadIdx.x == 0) {
            if (spec.mode == 1) {   // m = ceil(gamma n) in IEEE double, as the host computes it
                const uint64_t n = *spec.total;
                const bool skip = *spec.prev_flag != 0 || n < spec.lo || n > spec.hi;
                sl.L = device_level_hash(spec.seed, skip ? 1 : (uint64_t)ceil(spec.gamma * (double)n), spec.bit_off);
                sl.n = n;
                sl.skip = skip ? 1 : 0;
                if (blockIdx.x == 0) *spec.out = sl;
            } else {
                sl = *spec.out;
            }
        }
        __syncthreads();
        if (sl.skip) return;
        L = sl.L;
    }
    constexpr int NB = 1 << DBITS;
    // (a one-pass level of 2^9..2^10 buckets is small: it keeps two workgroups per CU instead)
    constexpr bool WC = DBITS == 8 || (WIDE_WC && DIG != 0);
    constexpr int LW = line_keys<NB>();
    constexpr bool DENSE = DIG == 2;
    static_assert(PTILE + NB * (LW - 1) < 65536, "tile sums in 16 bits");
    __shared__ PartLds<NB, WC, DENSE> S;

    const uint32_t group = blockIdx.x / K;
    const uint32_t slot = blockIdx.x % K;
    const uint32_t s0 = group * SG, s1 = s0 + SG;
    const uint64_t g0 = pre[s0], g1 = pre[s1];
    const uint64_t part = (g1 - g0 + K - 1) / K;
    const uint64_t lo = g0 + (uint64_t)slot * part < g1 ? g0 + (uint64_t)slot * part : g1;
    const uint64_t hi = lo + part < g1 ? lo + part : g1;
    const uint64_t bin_base = grouped ? (uint64_t)group << group_shift : 0;
    // bins this workgroup may write: those its group owns, and only existing ones
    const uint64_t owned = grouped ? (1ull << group_shift) : (uint64_t)NB;
    const uint64_t lim = bin_base >= nbins ? 0 : (nbins - bin_base < owned ? nbins - bin_base : owned);
    // regions: digit d writes at obase + dst[d] = obase + d * ostride; dense: at out + dst[d] (+ a0[d]
    // for the first)
    uint64_t* const obase = DENSE ? out : out + (bin_base * S_out + slot) * out_cap;
    const uint64_t ostride = (uint64_t)S_out * out_cap;

    for (int d = threadIdx.x; d < NB; d += PT) {
        S.hist[d] = 0;
        S.run[d] = 0;
        if constexpr (DENSE) {
            // this workgroup's keys of bin d go to [dbase, dbase + count) of out; whole lines are
            // counted from the line holding dbase, whose keys before dbase are not written
            const uint64_t B = (uint64_t)d < lim ? dbase[(bin_base + d) * S_out + slot] : 0;
            const uint32_t a = WC ? (uint32_t)(B & (LW - 1)) : 0u;
            S.dst[d] = B - a;
            S.a0[d] = a;
            S.run[d] = a;
        } else {
            S.dst[d] = (uint64_t)d * ostride;
        }
    }
    __syncthreads();

    // s: the segment holding the tile start (its bounds sb, se are reloaded only when s moves)
    uint32_t s = lo < hi ? find_segment(pre, s0, s1, lo) : s0;
    uint64_t sb = pre[s], se = pre[s + 1];
    if constexpr (!SPAN) {
        // the tile starting at t (< hi): up to PTILE keys from the segment holding t and the next
        // one (segments average at least half a tile here, so tiles stay nearly full)
        auto tile_end = [&](uint64_t t) {
            while (se <= t) {   // pre[s1] >= hi > t ends it
                ++s;
                sb = se;
                se = pre[s + 1];
            }
            uint64_t e = t + PTILE < hi ? t + PTILE : hi;
            if (e > se) {   // then s + 1 < s1, and pre[s + 2] ends the next segment
                const uint64_t se2 = pre[s + 2];
                if (e > se2) e = se2;
            }
            return e;
        };
        // the tile [t, e) from segment s and, past se, segment s + 1
        auto load = [&](uint64_t (&k)[PITEMS], uint64_t t, uint64_t e) {
            if constexpr (GEN) {   // one segment of generated keys: dense index = stream index
#pragma unroll
                for (int it = 0; it < PITEMS; ++it) {
                    const uint64_t j = it * PT + threadIdx.x;
                    k[it] = stream_key(gk.seed, gk.start + t + (t + j < e ? j : e - 1 - t));
                }
            } else {
                const uint64_t n1 = (se < e ? se : e) - t;
                load_tile(k, in + (uint64_t)s * in_stride + (t - sb), (uint32_t)n1,
                          in + (uint64_t)(s + 1) * in_stride, (uint32_t)(e - t));
            }
        };
        uint64_t kn[PITEMS];
        uint64_t t0 = lo, te = lo;
        if (t0 < hi) {
            te = tile_end(t0);
            load(kn, t0, te);
        }
        while (t0 < hi) {
            uint64_t k[PITEMS];
#pragma unroll
            for (int it = 0; it < PITEMS; ++it) k[it] = kn[it];
            const uint32_t tn = (uint32_t)(te - t0);
            const uint64_t t1 = te;
            uint64_t te1 = t1;
            if (t1 < hi) {   // the next tile's loads overlap this tile's sort and writes
                te1 = tile_end(t1);
                load(kn, t1, te1);
            }
            part_tile<NB, WC, HASHED, DIG>(S, k, tn, L, pbits, out_shift, pack_shift, bin_base, lim, obase,
                                      out_cap, overflow);
            t0 = t1;
            te = te1;
        }
    } else {
        uint64_t t0 = lo;
        while (t0 < hi) {
            while (se <= t0) {
                ++s;
                sb = se;
                se = pre[s + 1];
            }
            for (uint32_t q = threadIdx.x; q <= (uint32_t)TSEG; q += PT) S.sp[q] = pre[s + q < s1 ? s + q : s1];
            __syncthreads();
            uint64_t te = t0 + PTILE < hi ? t0 + PTILE : hi;
            if (S.sp[TSEG] < te) te = S.sp[TSEG];
            const uint32_t tn = (uint32_t)(te - t0);
            uint64_t k[PITEMS];
            {
                // segment of the thread's first key by binary search, later keys by stepping
                // forward; items past the tile read key t0 again
                const uint64_t i0 = t0 + threadIdx.x;
                uint32_t q = 0;
                for (uint32_t b = TSEG / 2; b > 0; b >>= 1)
                    if (S.sp[q + b] <= i0) q += b;
#pragma unroll
                for (int it = 0; it < PITEMS; ++it) {
                    const uint32_t j = it * PT + threadIdx.x;
                    uint64_t i = t0;
                    uint32_t qi = 0;
                    if (j < tn) {
                        i = t0 + j;
                        while (S.sp[q + 1] <= i) ++q;
                        qi = q;
                    }
                    k[it] = in[(uint64_t)(s + qi) * in_stride + (i - S.sp[qi])];
                }
            }
            part_tile<NB, WC, HASHED, DIG>(S, k, tn, L, pbits, out_shift, pack_shift, bin_base, lim, obase,
                                      out_cap, overflow);
            t0 = te;
        }
    }
    if constexpr (WC) {
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < NB * LW; e += PT) {   // the unfinished lines
            const uint32_t d = e / LW;
            const uint32_t r = S.run[d];
            const uint32_t g = (r & ~(uint32_t)(LW - 1)) + (e & (LW - 1));
            if (g < r && (DENSE ? g >= S.a0[d] : g < out_cap)) obase[S.dst[d] + g] = S.kbuf[PTILE + e];
        }
    }
    if constexpr (!DENSE) {
        // the entry after the last region is 0, so an exclusive scan of the counts ends in the total
        if (blockIdx.x == 0 && threadIdx.x == 0) out_cnt[nbins * S_out] = 0;
        for (uint64_t d = threadIdx.x; d < lim; d += PT) {
            out_cnt[(bin_base + d) * S_out + slot] = S.run[d] < out_cap ? S.run[d] : (uint32_t)out_cap;
            if (S.run[d] > out_cap) atomicOr(overflow, 1ull);
        }
    }
}

// Keys per (bin, workgroup) of the top-bits partition that k_partition would write, over the same
// input slices: cnt[(bin_base + d) * K + slot], bin = top bits of h (h = x, or fmix64(x ^ seed)
// for keys).  The exclusive prefix of cnt gives every workgroup's dense output start per bin.
__global__ void __launch_bounds__(256)
k_slice_counts(const uint64_t* __restrict__ in, uint64_t in_stride, const uint64_t* __restrict__ pre,
               uint32_t SG, uint32_t K, uint64_t seed, uint32_t sh, uint32_t hashed, uint32_t grouped,
               uint32_t group_shift, uint64_t nbins, uint32_t* __restrict__ cnt) {
    __shared__ uint32_t hist[1024];
    const uint32_t group = blockIdx.x / K;
    const uint32_t slot = blockIdx.x % K;
    const uint32_t s0 = group * SG, s1 = s0 + SG;
    const uint64_t g0 = pre[s0], g1 = pre[s1];
    const uint64_t part = (g1 - g0 + K - 1) / K;
    const uint64_t lo = g0 + (uint64_t)slot * part < g1 ? g0 + (uint64_t)slot * part : g1;
    const uint64_t hi = lo + part < g1 ? lo + part : g1;
    const uint64_t bin_base = grouped ? (uint64_t)group << group_shift : 0;
    const uint64_t owned = grouped ? (1ull << group_shift) : 1024ull;
    const uint64_t lim = bin_base >= nbins ? 0 : (nbins - bin_base < owned ? nbins - bin_base : owned);
    for (uint32_t d = threadIdx.x; d < 1024; d += 256) hist[d] = 0;
    __syncthreads();
    uint32_t s = lo < hi ? find_segment(pre, s0, s1, lo) : s0;
    for (uint64_t t = lo; t < hi; ++s) {
        const uint64_t sb = pre[s], se = pre[s + 1] < hi ? pre[s + 1] : hi;
        const uint64_t* src = in + (uint64_t)s * in_stride;
        for (uint64_t i = t + threadIdx.x; i < se; i += 256) {
            const uint64_t x = src[i - sb];
            const uint64_t d = ((hashed ? x : fmix64(x ^ seed)) >> sh) - bin_base;
            if (d < lim) atomicAdd(&hist[d], 1u);
        }
        if (se > t) t = se;
    }
    __syncthreads();
    for (uint64_t d = threadIdx.x; d < lim; d += 256) cnt[(bin_base + d) * K + slot] = hist[d];
}

// offsets[i] = base[i * K] for i <= nsets (every K-th entry of the (set, workgroup) prefix).
__global__ void k_take_every(const uint64_t* __restrict__ base, uint32_t K, uint64_t nsets,
                             uint64_t* __restrict__ offsets) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= nsets) offsets[i] = base[i * K];
}

// The segment q < S holding index i of a bucket, from the LDS prefix off[0..S].
__device__ __forceinline__ uint32_t seg_of(const uint32_t* off, uint32_t S, uint32_t i) {
    uint32_t lo = 0, hi = S;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------- bucket pass
//
// Workgroup b owns positions [b << pbits, (b+1) << pbits) of level d.  It reads the records of
// the bucket's keys (regions b*S .. b*S+S-1) once into registers, writes their positions inside
// the bucket to LDS, fills A and C there with LDS atomics, writes the finalized A words of its
// positions, and writes the keys whose A bit is 0 (F_{d+1}, recovered from their hashes) into
// output region b of capacity ycap, with their number in surv[b].  A record is the level hash h,
// or with PACKED the pair (q << pbits) | (pos mod 2^pbits) of h = q m + pos.
// 1024 threads holding 18 records each: at 62 VGPRs two workgroups fill a CU with 8 waves per SIMD
// (512 threads with 36 records each needed 91 VGPRs and ran 4 waves per SIMD).
constexpr int BI = 18;   // hashes held per thread: KT * BI >= the largest kcap

template <bool PACKED>
__global__ void __launch_bounds__(KT)
k_bucket(const uint64_t* __restrict__ in, uint64_t in_cap, const uint32_t* __restrict__ cnt,
         uint32_t S, LevelHash L, uint32_t pbits, uint32_t kcap, uint64_t* __restrict__ A,
         uint64_t* __restrict__ Cout, uint64_t level_words, uint64_t* __restrict__ Y, uint64_t ycap,
         uint32_t* __restrict__ surv, unsigned long long* overflow, const SpecLevel* __restrict__ spec) {
    __shared__ uint32_t pool[BUCKET_LDS / 4];
    __shared__ uint32_t wsum[KT / 64 + 1];
    __shared__ uint32_t segoff[257];
    const uint64_t b = blockIdx.x;
    const uint32_t P = 1u << pbits;
    if (spec) {   // a level queued ahead: its hash and size from the device; buckets past it are empty
        if (spec->skip) return;
        L = spec->L;
        level_words = (L.m + 63) / 64;
        if (b >= (L.m + P - 1) >> pbits) {
            if (threadIdx.x == 0) {
                surv[b] = 0;
                if (b == 0) surv[gridDim.x] = 0;
            }
            return;
        }
    }
    uint32_t* Abits = pool;
    uint32_t* Cbits = pool + (P >> 5);
    uint16_t* lps = (uint16_t*)(pool + 2 * (P >> 5));

    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t q = 0; q < S; ++q) {
            segoff[q] = acc;
            acc += cnt[b * S + q];
        }
        segoff[S] = acc;
    }
    for (uint32_t w = threadIdx.x; w < 2 * (P >> 5); w += KT) pool[w] = 0;
    __syncthreads();
    const uint32_t nb = segoff[S];
    if (nb > kcap || nb > (uint32_t)(KT * BI)) {
        if (threadIdx.x == 0) {
            atomicOr(overflow, 2ull);
            surv[b] = 0;
            if (b == 0) surv[gridDim.x] = 0;
        }
        return;
    }
    const uint64_t pbase = b << pbits;
    bool bad = false;
    uint64_t h[BI];
    {
        // segment of the thread's first key by binary search, later keys (KT further on each)
        // by stepping forward; segoff[S] = nb ends every step
        uint32_t q = threadIdx.x < nb ? seg_of(segoff, S, threadIdx.x) : 0;
#pragma unroll
        for (int it = 0; it < BI; ++it) {
            const uint32_t i = it * KT + threadIdx.x;
            h[it] = 0;
            if (i < nb) {
                while (segoff[q + 1] <= i) ++q;
                h[it] = in[(b * S + q) * in_cap + (i - segoff[q])];
            }
        }
    }
#pragma unroll
    for (int it = 0; it < BI; ++it) {
        const uint32_t i = it * KT + threadIdx.x;
        if (i < nb) {
            uint64_t p;
            if (PACKED) {   // the position inside the bucket; the hash q m + pos kept for survivors
                p = h[it] & (P - 1);
                lps[i] = (uint16_t)p;
                h[it] = (h[it] >> pbits) * L.m + pbase + p;
            } else {
                p = mod_invariant(h[it], L.m, L.magic, L.sh1, L.sh2) - pbase;
                // not this bucket's key: the partition was wrong; never touch LDS with it
                const bool out = p >= P;
                bad |= out;
                lps[i] = out ? 0 : (uint16_t)p;
                if (out) continue;
            }
            const uint32_t bit = 1u << (p & 31);
            const uint32_t old = atomicOr(&Abits[p >> 5], bit);
            if (old & bit) atomicOr(&Cbits[p >> 5], bit);
        }
    }
    if (bad) atomicOr(overflow, 8ull);
    __syncthreads();
    // finalize: A &= ~C, written as 64-bit words of the level
    const uint64_t w0 = b << (pbits - 6);
    for (uint32_t j = threadIdx.x; j < (P >> 6); j += KT) {
        const uint32_t a0 = Abits[2 * j] & ~Cbits[2 * j];
        const uint32_t a1 = Abits[2 * j + 1] & ~Cbits[2 * j + 1];
        if (w0 + j < level_words) {
            A[w0 + j] = (uint64_t)a0 | ((uint64_t)a1 << 32);
            if (Cout) Cout[w0 + j] = (uint64_t)Cbits[2 * j] | ((uint64_t)Cbits[2 * j + 1] << 32);
        }
    }
    __syncthreads();
    for (uint32_t w = threadIdx.x; w < (P >> 5); w += KT) Abits[w] &= ~Cbits[w];
    __syncthreads();
    // filter: keys whose A bit is 0 collided and go on to F_{d+1}
    uint64_t mask = 0;
#pragma unroll
    for (int it = 0; it < BI; ++it) {
        const uint32_t i = it * KT + threadIdx.x;
        if (i < nb) {
            const uint32_t p = lps[i];
            if (!((Abits[p >> 5] >> (p & 31)) & 1u)) mask |= 1ull << it;
        }
    }
    uint32_t tot;
    const uint32_t o = block_exclusive_sum<KT>((uint32_t)__popcll(mask), wsum, &tot);
    // survivors in (wave, item, lane) order, so that each store of a wave is one contiguous run
    uint32_t wo = __shfl(o, 0, 64);
    const uint64_t below = (1ull << lane_id()) - 1;
    uint64_t* dst = Y + b * ycap;
#pragma unroll
    for (int it = 0; it < BI; ++it) {
        const bool keep = (mask >> it) & 1ull;
        const uint64_t bal = __ballot(keep);
        if (keep) dst[wo + __popcll(bal & below)] = unfmix64(h[it]) ^ L.seed;
        wo += (uint32_t)__popcll(bal);
    }
    if (threadIdx.x == 0) {
        surv[b] = tot;
        if (b == 0) surv[gridDim.x] = 0;   // the entry after the last bucket, for the scan's total
    }
}

// ---------------------------------------------------------------- accumulating a level by chunks
//
// Workgroup b owns positions [b << pbits, (b+1) << pbits) of a level held in interleaved A/C words
// W (word p >> 5: the A bits of 32 positions in bits 0..31, their C bits in 32..63).  It reads the
// bucket's words into LDS, applies the test-and-set of Algorithm 2 for every key of its regions,
// and writes the words back.  The final A and C do not depend on the order of the keys, so a
// level's keys can be added chunk by chunk, each chunk partitioned by bucket first: a level whose
// keys are never all in memory is filled without global atomics.
constexpr int AT = 512;

template <bool PACKED>
__global__ void __launch_bounds__(AT)
k_accumulate(const uint64_t* __restrict__ in, uint64_t in_cap, const uint32_t* __restrict__ cnt, uint32_t S,
             LevelHash L, uint32_t pbits, uint64_t* __restrict__ W, uint64_t wwords,
             unsigned long long* overflow) {
    extern __shared__ uint32_t acc[];   // A bits [0, nw), C bits [nw, 2 nw)
    const uint64_t b = blockIdx.x;
    const uint32_t P = 1u << pbits;
    const uint32_t nw = P >> 5;
    uint32_t* Ab = acc;
    uint32_t* Cb = acc + nw;
    const uint64_t w0 = b * nw;
    for (uint32_t j = threadIdx.x; j < nw; j += AT) {
        const uint64_t v = w0 + j < wwords ? W[w0 + j] : 0;
        Ab[j] = (uint32_t)v;
        Cb[j] = (uint32_t)(v >> 32);
    }
    __syncthreads();
    const uint64_t pbase = b << pbits;
    bool bad = false;   // a key outside the bucket: the partition was wrong; never touch LDS with it
    for (uint32_t q = 0; q < S; ++q) {
        const uint32_t c = cnt[b * S + q];
        const uint64_t* src = in + (b * S + q) * in_cap;
        for (uint32_t i0 = 0; i0 < c; i0 += 4 * AT) {
            uint64_t h[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t i = i0 + u * AT + threadIdx.x;
                h[u] = i < c ? src[i] : 0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (i0 + u * AT + threadIdx.x >= c) continue;
                uint32_t p;
                if (PACKED) {
                    p = (uint32_t)h[u] & (P - 1);
                } else {
                    const uint64_t pl = mod_invariant(h[u], L.m, L.magic, L.sh1, L.sh2) - pbase;
                    bad |= pl >= P;
                    if (pl >= P) continue;
                    p = (uint32_t)pl;
                }
                const uint32_t bit = 1u << (p & 31);
                const uint32_t old = atomicOr(&Ab[p >> 5], bit);
                if (old & bit) atomicOr(&Cb[p >> 5], bit);
            }
        }
    }
    if (bad) atomicOr(overflow, 8ull);
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < nw; j += AT)
        if (w0 + j < wwords) W[w0 + j] = (uint64_t)Ab[j] | ((uint64_t)Cb[j] << 32);
}

// ---------------------------------------------------------------- testing keys against a finished level
//
// The walk over finished levels (Algorithm 3's loop, used by the streaming build to skip keys
// placed earlier) done by bucket instead of by random reads: workgroup b reads the 2^pbits A bits
// of its positions of finished level d (A_d at bit offset `off` of words) into LDS once, tests
// every key of its regions, and writes the keys whose bit is 0 (not placed at d) into output
// region b (capacity ycap) with their number in surv[b].  Records as in k_bucket.
constexpr int TT = 512;

template <bool PACKED>
__global__ void __launch_bounds__(TT)
k_bucket_test(const uint64_t* __restrict__ in, uint64_t in_cap, const uint32_t* __restrict__ cnt, uint32_t S,
              LevelHash L, uint32_t pbits, const uint64_t* __restrict__ words, uint64_t off, uint64_t level_words,
              uint64_t* __restrict__ Y, uint64_t ycap, uint32_t* __restrict__ surv,
              unsigned long long* overflow) {
    extern __shared__ uint32_t abits[];   // 2^pbits bits of A_d
    __shared__ uint32_t wsum[TT / 64 + 1];
    const uint64_t b = blockIdx.x;
    const uint32_t P = 1u << pbits;
    const uint64_t w0 = (off >> 6) + (b << (pbits - 6));   // off and b * 2^pbits are multiples of 64
    const uint64_t wend = (off >> 6) + level_words;
    for (uint32_t j = threadIdx.x; j < (P >> 6); j += TT) {
        const uint64_t w = w0 + j < wend ? words[w0 + j] : 0;
        abits[2 * j] = (uint32_t)w;
        abits[2 * j + 1] = (uint32_t)(w >> 32);
    }
    __syncthreads();
    const uint64_t pbase = b << pbits;
    uint64_t* dst = Y + b * ycap;
    uint32_t o = 0;   // survivors written so far (uniform)
    bool full = false;
    bool bad = false;   // a key outside the bucket: the partition was wrong
    for (uint32_t q = 0; q < S && !full; ++q) {
        const uint32_t c = cnt[b * S + q];
        const uint64_t* src = in + (b * S + q) * in_cap;
        for (uint32_t i0 = 0; i0 < c; i0 += 4 * TT) {
            uint64_t h[4];
            uint32_t keep = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t i = i0 + u * TT + threadIdx.x;
                h[u] = i < c ? src[i] : 0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (i0 + u * TT + threadIdx.x >= c) continue;
                uint64_t p;
                if (PACKED) {
                    p = h[u] & (P - 1);
                    h[u] = (h[u] >> pbits) * L.m + pbase + p;
                } else {
                    p = mod_invariant(h[u], L.m, L.magic, L.sh1, L.sh2) - pbase;
                    bad |= p >= P;
                    if (p >= P) continue;
                }
                if (!((abits[p >> 5] >> (p & 31)) & 1u)) keep |= 1u << u;
            }
            uint32_t tot;
            uint32_t e = block_exclusive_sum<TT>((uint32_t)__popc(keep), wsum, &tot);
            if (o + tot > ycap) {   // cannot happen: survivors are at most the bucket's records
                if (threadIdx.x == 0) atomicOr(overflow, 2ull);
                full = true;   // uniform: the count below stays within the region
                break;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if ((keep >> u) & 1u) dst[o + e++] = unfmix64(h[u]) ^ L.seed;
            o += tot;
        }
    }
    if (bad) atomicOr(overflow, 8ull);
    if (threadIdx.x == 0) surv[b] = o;
}

// ---------------------------------------------------------------- small levels in one workgroup
//
// Builds levels d0, d0+1, ... of a set of n <= kcap keys (segments of the partitioned layout or a
// dense array) in one workgroup: m_d = ceil(gamma n_d) in IEEE double, the level's hash
// constants, fill, finalize and filter in LDS, A written at the running bit offset.  Stops when
// no key is left or after level D-1; the leftover keys are written to `left`.
__global__ void __launch_bounds__(BT)
k_tail(const uint64_t* __restrict__ in, uint64_t in_stride, const uint64_t* __restrict__ pre,
       uint32_t nseg, uint32_t kcap, double gamma, SeedTable seeds, uint32_t d0, uint32_t D,
       uint64_t bit_off, uint64_t* __restrict__ A, uint64_t* __restrict__ Cout,
       TailLevel* __restrict__ rec, uint64_t* __restrict__ left, TailSummary* __restrict__ sum) {
    __shared__ uint64_t pool[POOL_WORDS];
    __shared__ uint32_t wsum[BT / 64 + 1];
    __shared__ LevelHash Ls;
    __shared__ unsigned long long wacc;
    uint64_t* keys = pool;
    uint32_t* Abits = (uint32_t*)(pool + kcap);
    const uint64_t n0 = pre[nseg];
    // load
    for (uint64_t i = threadIdx.x; i < n0; i += BT) {
        const uint32_t s = find_segment(pre, 0, nseg, i);
        keys[i] = in[(uint64_t)s * in_stride + (i - pre[s])];
    }
    uint64_t n = n0;
    uint32_t d = d0;
    uint64_t off = bit_off;
    constexpr int FI = (POOL_WORDS + BT - 1) / BT;
    while (n > 0 && d < D) {
        const uint64_t m = (uint64_t)ceil(gamma * (double)n);
        const uint32_t aw = (uint32_t)((m + 31) >> 5);   // u32 words of A (and of C)
        uint32_t* Cbits = Abits + aw + (aw & 1);
        if (threadIdx.x == 0) {
            Ls = device_level_hash(seeds.s[d], m, off);
            wacc = 0;
        }
        for (uint32_t w = threadIdx.x; w < 2 * aw + 2; w += BT) Abits[w] = 0;
        __syncthreads();
        const LevelHash L = Ls;
        for (uint32_t i = threadIdx.x; i < n; i += BT) {
            const uint32_t p = level_pos32(keys[i], L);   // (a level in LDS: m < 2^32)
            const uint32_t bit = 1u << (p & 31);
            const uint32_t old = atomicOr(&Abits[p >> 5], bit);
            if (old & bit) atomicOr(&Cbits[p >> 5], bit);
        }
        __syncthreads();
        const uint64_t words = (m + 63) >> 6;
        unsigned long long wt = 0;
        for (uint32_t j = threadIdx.x; j < words; j += BT) {
            const uint32_t a0 = Abits[2 * j] & ~Cbits[2 * j];
            const uint32_t a1 = Abits[2 * j + 1] & ~Cbits[2 * j + 1];
            const uint64_t a = (uint64_t)a0 | ((uint64_t)a1 << 32);
            A[(off >> 6) + j] = a;
            if (Cout) Cout[(off >> 6) + j] = (uint64_t)Cbits[2 * j] | ((uint64_t)Cbits[2 * j + 1] << 32);
            wt += __popcll(a);
        }
        wt = wave_sum(wt);
        if (lane_id() == 0 && wt) atomicAdd(&wacc, wt);
        __syncthreads();
        for (uint32_t w = threadIdx.x; w < aw; w += BT) Abits[w] &= ~Cbits[w];
        __syncthreads();
        // filter and compact in place
        uint32_t mask = 0;
        uint64_t kk[FI];
#pragma unroll
        for (int it = 0; it < FI; ++it) {
            const uint32_t i = it * BT + threadIdx.x;
            kk[it] = 0;
            if (i < n) {
                kk[it] = keys[i];
                const uint32_t p = level_pos32(kk[it], L);   // (a level in LDS: m < 2^32)
                if (!((Abits[p >> 5] >> (p & 31)) & 1u)) mask |= 1u << it;
            }
        }
        uint32_t tot;
        uint32_t o = block_exclusive_sum<BT>((uint32_t)__popc(mask), wsum, &tot);
#pragma unroll
        for (int it = 0; it < FI; ++it)
            if ((mask >> it) & 1u) keys[o++] = kk[it];
        if (threadIdx.x == 0) {
            rec[d].n = n;
            rec[d].m = m;
            rec[d].weight = wacc;
            rec[d].offset = off;
        }
        __syncthreads();
        n = tot;
        off += 64 * words;
        ++d;
    }
    for (uint64_t i = threadIdx.x; i < n; i += BT) left[i] = keys[i];
    if (threadIdx.x == 0) {
        sum->end_level = d;
        sum->n_left = n;
        sum->bit_end = off;
    }
}

__global__ void k_pair(uint64_t* p, uint64_t a, uint64_t b) {
    if (threadIdx.x == 0) {
        p[0] = a;
        p[1] = b;
    }
}

// Dense copy of a segmented set (used before falling back to the global-atomic levels).
__global__ void k_gather(const uint64_t* __restrict__ in, uint64_t in_stride,
                         const uint64_t* __restrict__ pre, uint32_t nseg, uint64_t* __restrict__ out) {
    const uint64_t n = pre[nseg];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t s = find_segment(pre, 0, nseg, i);
        out[i] = in[(uint64_t)s * in_stride + (i - pre[s])];
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers

uint32_t tail_capacity(double gamma) {
    // keys (8 B each) + A and C halves (gamma * kcap / 16 bytes... in u32 words, rounded up)
    uint32_t k = 16384;
    while (k > 64) {
        const double m = std::ceil(gamma * k);
        const double aw = std::ceil(m / 32.0);
        const double bytes = 8.0 * k + 4.0 * (2 * aw + 4);
        if (bytes <= 8.0 * POOL_WORDS) break;
        k -= 64;
    }
    return k;
}

hipError_t launch_tail(const uint64_t* in, uint64_t in_stride, const uint64_t* pre, uint32_t nseg,
                       uint32_t kcap, double gamma, const SeedTable& seeds, uint32_t d0, uint32_t D,
                       uint64_t bit_off, uint64_t* A, uint64_t* Cout, TailLevel* rec, uint64_t* left,
                       TailSummary* sum, hipStream_t s) {
    hipLaunchKernelGGL(k_tail, dim3(1), dim3(BT), 0, s, in, in_stride, pre, nseg, kcap, gamma, seeds,
                       d0, D, bit_off, A, Cout, rec, left, sum);
    return hipGetLastError();
}

BucketGeometry bucket_geometry(double gamma, uint32_t pbits) {
    // Largest power-of-two bucket (at most 2^16 positions, so a local position fits 16 bits)
    // whose expected keys (P / gamma, plus 8 standard deviations and a margin) fit the LDS
    // budget together with the bucket's A and C bits; with pbits != 0, that size if it fits.
    BucketGeometry g{};
    const uint32_t hi = pbits ? pbits : 16, lo = pbits ? pbits : 10;
    if (pbits && (pbits < 6 || pbits > 16)) return g;
    for (uint32_t pb = hi; pb >= lo; --pb) {
        const double P = (double)(1u << pb);
        const double mu = P / gamma;
        const double kc = std::ceil(mu + 8.0 * std::sqrt(mu) + 128.0);
        const double bytes = 2.0 * kc + P / 4.0;
        if (bytes <= (double)BUCKET_LDS && mu <= 16384.0 && kc <= (double)(KT * BI)) {
            g.pbits = pb;
            g.kcap = (uint32_t)kc;
            return g;
        }
    }
    g.pbits = 0;
    return g;
}

hipError_t launch_partition(int dbits, bool hashed, const uint64_t* in, uint64_t in_stride,
                            const uint64_t* pre, uint32_t groups, uint32_t SG, uint32_t K,
                            const LevelHash& L, uint32_t pbits, uint32_t out_shift, bool grouped,
                            uint32_t group_shift, uint64_t nbins, uint64_t* out, uint64_t out_cap,
                            uint32_t S_out, uint32_t* out_cnt, unsigned long long* overflow,
                            uint64_t n_in, uint64_t nseg_in, hipStream_t s, int dig, const uint64_t* dbase,
                            uint32_t pack_shift, const SpecArgs& spec, const uint64_t* gen) {
    const dim3 grid(groups * K);
    GenKeys gk{0, 0, 0};
    if (gen) {   // generated keys: one segment, never records
        if (hashed || nseg_in != 1 || (dig != 0 && dig != 3)) return hipErrorInvalidValue;
        gk = GenKeys{gen[0], gen[1], 1};
    }
    const uint32_t gr = grouped ? 1u : 0u;
    // segments averaging under half a tile: tiles span segments
    const bool span = !gen && nseg_in > 0 && n_in / nseg_in < (uint64_t)(PTILE / 2);
#define MPHF_PART_G(DB, HS, SP, DG, GN)                                                                   \
    hipLaunchKernelGGL((k_partition<DB, HS, SP, DG, GN>), grid, dim3(PT), 0, s, in, in_stride, pre, SG, K, L, \
                       pbits, out_shift, pack_shift, gr, group_shift, nbins, out, out_cap, S_out, out_cnt,      \
                       overflow, dbase, spec, gk)
#define MPHF_PART(DB, HS, SP, DG) MPHF_PART_G(DB, HS, SP, DG, false)
    if (dig == 1) {
        // regions by the top bits: the first pass over a dense key array
        if (hashed || dbits > 8 || span) return hipErrorInvalidValue;
        MPHF_PART(8, false, false, 1);
    } else if (dig == 2) {
        // dense output by the top bits: one pass over dense keys, or a grouped pass over regions
        if (!hashed) {
            if (dbits > 8 || span) return hipErrorInvalidValue;
            MPHF_PART(8, false, false, 2);
        } else if (dbits <= 8) {
            if (span) MPHF_PART(8, true, true, 2); else MPHF_PART(8, true, false, 2);
        } else {
            if (span) MPHF_PART(10, true, true, 2); else MPHF_PART(10, true, false, 2);
        }
    } else if (dig == 3) {
        // packed records: the first of two passes over keys
        if (hashed || dbits > 8 || pack_shift > 56) return hipErrorInvalidValue;
        const uint64_t m_max = spec.mode ? (uint64_t)std::ceil(spec.gamma * (double)spec.hi) : L.m;
        if (grouped) return hipErrorInvalidValue;
        if ((m_max >> 32) == 0) {   // pos < m < 2^32: its low 32 bits suffice
            if (gk.on) MPHF_PART_G(8, false, false, 5, true);
            else if (span) MPHF_PART(8, false, true, 5); else MPHF_PART(8, false, false, 5);
        } else {
            if (gk.on) MPHF_PART_G(8, false, false, 3, true);
            else if (span) MPHF_PART(8, false, true, 3); else MPHF_PART(8, false, false, 3);
        }
    } else if (dig == 4) {
        // packed records in and out: the second pass
        if (!hashed || pack_shift > 56 || pack_shift < pbits) return hipErrorInvalidValue;
        if (dbits <= 8) { if (span) MPHF_PART(8, true, true, 4); else MPHF_PART(8, true, false, 4); }
        else { if (span) MPHF_PART(10, true, true, 4); else MPHF_PART(10, true, false, 4); }
    } else {
        // level hashes: one pass over keys
        if (hashed) return hipErrorInvalidValue;
        if (gk.on) {
            if (dbits <= 8) MPHF_PART_G(8, false, false, 0, true); else MPHF_PART_G(10, false, false, 0, true);
        } else if (dbits <= 8) { if (span) MPHF_PART(8, false, true, 0); else MPHF_PART(8, false, false, 0); }
        else { if (span) MPHF_PART(10, false, true, 0); else MPHF_PART(10, false, false, 0); }
    }
#undef MPHF_PART
#undef MPHF_PART_G
    return hipGetLastError();
}

hipError_t launch_bucket(const uint64_t* in, uint64_t in_cap, const uint32_t* cnt, uint32_t S,
                         uint64_t nbuckets, const LevelHash& L, uint32_t pbits, bool packed, uint32_t kcap,
                         uint64_t* A, uint64_t* Cout, uint64_t level_words, uint64_t* Y, uint64_t ycap,
                         uint32_t* surv, unsigned long long* overflow, hipStream_t s, const SpecLevel* spec) {
    // local positions are 16-bit, and the A and C bits and the positions must fit the LDS pool
    if (pbits < 6 || pbits > 16 || kcap > (uint32_t)(KT * BI) ||
        (1u << pbits) / 4 + 2ull * kcap > (uint64_t)BUCKET_LDS)
        return hipErrorInvalidValue;
    if (packed)
        hipLaunchKernelGGL(k_bucket<true>, dim3((unsigned)nbuckets), dim3(KT), 0, s, in, in_cap, cnt, S, L,
                           pbits, kcap, A, Cout, level_words, Y, ycap, surv, overflow, spec);
    else
        hipLaunchKernelGGL(k_bucket<false>, dim3((unsigned)nbuckets), dim3(KT), 0, s, in, in_cap, cnt, S, L,
                           pbits, kcap, A, Cout, level_words, Y, ycap, surv, overflow, spec);
    return hipGetLastError();
}

hipError_t accumulate_setup() {
    // up to 2^18 positions per bucket: 64 KiB of A and C bits
    hipError_t e = hipFuncSetAttribute((const void*)k_accumulate<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       65536);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_accumulate<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
}

hipError_t launch_accumulate(const uint64_t* in, uint64_t in_cap, const uint32_t* cnt, uint32_t S,
                             uint64_t nbuckets, const LevelHash& L, uint32_t pbits, bool packed, uint64_t* W,
                             uint64_t wwords, unsigned long long* overflow, hipStream_t s) {
    if (pbits < 5 || pbits > 18) return hipErrorInvalidValue;
    if (!nbuckets) return hipSuccess;
    const size_t lds = (size_t)(1u << pbits) / 4;   // 2 bits per position
    if (packed)
        hipLaunchKernelGGL(k_accumulate<true>, dim3((unsigned)nbuckets), dim3(AT), lds, s, in, in_cap, cnt, S, L,
                           pbits, W, wwords, overflow);
    else
        hipLaunchKernelGGL(k_accumulate<false>, dim3((unsigned)nbuckets), dim3(AT), lds, s, in, in_cap, cnt, S, L,
                           pbits, W, wwords, overflow);
    return hipGetLastError();
}

hipError_t bucket_test_setup() {
    hipError_t e = hipFuncSetAttribute((const void*)k_bucket_test<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       32768);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_bucket_test<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 32768);
}

hipError_t launch_bucket_test(const uint64_t* in, uint64_t in_cap, const uint32_t* cnt, uint32_t S,
                              uint64_t nbuckets, const LevelHash& L, uint32_t pbits, bool packed,
                              const uint64_t* words, uint64_t off, uint64_t level_words, uint64_t* Y, uint64_t ycap,
                              uint32_t* surv, unsigned long long* overflow, hipStream_t s) {
    if (pbits < 6 || pbits > 18 || (off & 63)) return hipErrorInvalidValue;
    if (!nbuckets) return hipSuccess;
    const size_t lds = (size_t)(1u << pbits) / 8;
    if (packed)
        hipLaunchKernelGGL(k_bucket_test<true>, dim3((unsigned)nbuckets), dim3(TT), lds, s, in, in_cap, cnt, S, L,
                           pbits, words, off, level_words, Y, ycap, surv, overflow);
    else
        hipLaunchKernelGGL(k_bucket_test<false>, dim3((unsigned)nbuckets), dim3(TT), lds, s, in, in_cap, cnt, S, L,
                           pbits, words, off, level_words, Y, ycap, surv, overflow);
    return hipGetLastError();
}

hipError_t launch_slice_counts(const uint64_t* in, uint64_t in_stride, const uint64_t* pre, uint32_t groups,
                               uint32_t SG, uint32_t K, uint64_t seed, uint32_t sh, bool hashed, bool grouped,
                               uint32_t group_shift, uint64_t nbins, uint32_t* cnt, hipStream_t s) {
    if (!grouped && nbins > 1024) return hipErrorInvalidValue;
    if (grouped && group_shift > 10) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_slice_counts, dim3(groups * K), dim3(256), 0, s, in, in_stride, pre, SG, K, seed, sh,
                       hashed ? 1u : 0u, grouped ? 1u : 0u, group_shift, nbins, cnt);
    return hipGetLastError();
}

hipError_t launch_take_every(const uint64_t* base, uint32_t K, uint64_t nsets, uint64_t* offsets, hipStream_t s) {
    hipLaunchKernelGGL(k_take_every, dim3((unsigned)((nsets + 256) / 256)), dim3(256), 0, s, base, K, nsets, offsets);
    return hipGetLastError();
}

hipError_t launch_pair(uint64_t* p, uint64_t a, uint64_t b, hipStream_t s) {
    hipLaunchKernelGGL(k_pair, dim3(1), dim3(64), 0, s, p, a, b);
    return hipGetLastError();
}

hipError_t launch_gather(const uint64_t* in, uint64_t in_stride, const uint64_t* pre, uint32_t nseg,
                         uint64_t n, uint64_t* out, hipStream_t s) {
    if (!n) return hipSuccess;
    uint64_t blocks = (n + 1023) / 1024;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(256), 0, s, in, in_stride, pre, nseg, out);
    return hipGetLastError();
}

}  // namespace mphfk
