// Host-side declarations shared by the runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace mphfk {

// Per-level record kept by the handle; the device copy drives the lookup kernel.
struct DevLevel {
    uint64_t seed;
    uint64_t m;
    uint64_t magic;
    uint64_t bit_off;
    uint32_t sh1;
    uint32_t sh2;
};

LevelHash make_level_hash(uint64_t seed, uint64_t m, uint64_t bit_off);

// The function a served request queries (device pointers owned by the handle, as the single
// lookup kernel takes them).
struct SegDesc {
    const DevLevel* lev;
    const uint32_t* sec;
    const uint64_t* super;
    const uint64_t* fbk;
    uint64_t nfb;
    uint64_t N;
    uint32_t nlev;
    uint32_t pad;
};

// The label of x in the fallback table (ascending keys, labels N - nfb + 1 ..), else 0.
__device__ __forceinline__ uint64_t fallback_label(uint64_t x, const uint64_t* __restrict__ fbk, uint64_t nfb,
                                                   uint64_t N) {
    if (nfb) {
        uint64_t lo = 0, hi = nfb;   // first index with fbk[idx] >= x
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (fbk[mid] < x) lo = mid + 1; else hi = mid;
        }
        if (lo < nfb && fbk[lo] == x) return N - nfb + 1 + lo;
    }
    return 0;
}

// The label of query x (Algorithm 3): the first level whose bit is set gives the ones of A before
// it plus one; else the fallback table; else 0.
__device__ __forceinline__ uint64_t label_of(uint64_t x, const DevLevel* __restrict__ lev, uint32_t nlev,
                                             const uint32_t* __restrict__ sec, const uint64_t* __restrict__ super,
                                             const uint64_t* __restrict__ fbk, uint64_t nfb, uint64_t N) {
    for (uint32_t d = 0; d < nlev; ++d) {
        const DevLevel L = lev[d];
        const uint64_t g = L.bit_off + mod_invariant(fmix64(x ^ L.seed), L.m, L.magic, L.sh1, L.sh2);
        uint64_t rank;
        if (sector_rank(sec, super, g, &rank)) return rank + 1;
    }
    return fallback_label(x, fbk, nfb, N);
}

// The labels of QP queries of one function walked level by level in lockstep (Algorithm 3 for
// each): every level's probes of the still pending queries are issued together, so a lane keeps
// QP independent sector loads in flight.  res[u] gets the label when pend[u] (pend[u] false on
// entry skips x[u]); queries that find no set bit stay pending for the fallback table.
template <int QP>
__device__ __forceinline__ void walk_levels(const uint64_t (&x)[QP], bool (&pend)[QP], uint64_t (&res)[QP],
                                            const DevLevel* __restrict__ lev, uint32_t nlev,
                                            const uint32_t* __restrict__ sec,
                                            const uint64_t* __restrict__ super) {
    for (uint32_t d = 0; d < nlev; ++d) {
        bool any = false;
#pragma unroll
        for (int u = 0; u < QP; ++u) any |= pend[u];
        if (!any) return;
        const DevLevel L = lev[d];
        uint4 v[QP][4];
        uint64_t base[QP];
        uint32_t r[QP];
#pragma unroll
        for (int u = 0; u < QP; ++u) {
            const uint64_t g = L.bit_off + mod_invariant(fmix64(x[u] ^ L.seed), L.m, L.magic, L.sh1, L.sh2);
            const uint64_t j = g / SEC_BITS;
            r[u] = (uint32_t)(g - j * SEC_BITS);
            base[u] = 0;
            if (pend[u]) {
                base[u] = super[j >> SUPER_SHIFT];
                sector_load(sec, j, v[u]);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) v[u][c] = make_uint4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < QP; ++u) {
            uint32_t c;
            if (pend[u] && sector_count(v[u], r[u], &c)) {
                res[u] = base[u] + c + 1;
                pend[u] = false;
            }
        }
    }
}

// Key i of a generated stream: output i of SplitMix64 (Steele, Lea and Flood 2014) started at
// `seed`; the streaming build generates its chunks (and a first radix pass its keys) from it.
__device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct SeedTable {
    uint64_t s[64];
};

// What the one-workgroup kernel for the last levels reports per level and at the end.
struct TailLevel {
    uint64_t n, m, weight, offset;
};
struct TailSummary {
    uint64_t end_level;   // first level not built
    uint64_t n_left;      // keys left for the fallback table
    uint64_t bit_end;     // bit offset after the last level built
};

// A level queued before the host knows its key count: its first partition pass derives the level
// hash from the previous level's survivor total on the device.  The host sized the launches for n
// in [lo, hi]; if the total falls outside, or the previous level overflowed, skip is set and every
// kernel of the level returns at once (the host then queues the level again with its exact size).
struct SpecLevel {
    LevelHash L;
    uint64_t n;
    uint64_t skip;
};

// How a partition pass of such a level gets it: mode 1 (the level's first pass) derives it from the
// survivor total at `total`, every workgroup for itself and workgroup 0 also into *out, with n in
// [lo, hi] and *prev_flag == 0 required; mode 2 (a later pass) reads *out; mode 0: an exact level.
struct SpecArgs {
    uint32_t mode = 0;
    const uint64_t* total = nullptr;
    const unsigned long long* prev_flag = nullptr;
    double gamma = 0;
    uint64_t seed = 0, bit_off = 0, lo = 0, hi = 0;
    SpecLevel* out = nullptr;
};

// Batched builds: per set and per (set, level) records.
struct BatchSet {
    uint64_t n;            // keys of the set
    uint64_t sec_base;     // first of the set's lookup sectors
    uint64_t bits;         // bits of the set's levels (64-bit padded)
    uint64_t left_off;     // first of the set's fallback keys in the fallback array
    uint32_t nlev;
    uint32_t nleft;
    uint32_t status;       // bit 0: duplicate keys; bit 1: too many leftovers; bit 2: region too small
    uint32_t pad;
};
struct BatchLevel {
    uint64_t m;
    uint64_t magic;
    uint64_t off;          // bit offset of the level inside the set
    uint32_t n;            // keys of the set at this level
    uint32_t sh;           // sh1 | sh2 << 8
};

// What a batched lookup reads first for set s: 16 bytes with the set's first lookup sector
// (44 bits) and m0 (20 bits) in word a, and m1 (20 bits) and the level count (7 bits) in word b.
// A set's sectors hold its own bits with counters of the ones of the set before each sector, so a
// label is that rank plus one.  Level 1 starts at bit (m0 + 63) & ~63 of the set; levels 2.. are
// BatchLev records in D - 2 slots per set, and the fallback table is described by BatchAux.
struct __attribute__((aligned(16))) BatchHead {
    uint64_t a, b;
};
constexpr uint32_t HEAD_BASE_BITS = 44, HEAD_M_BITS = 20;
struct BatchLev {
    uint32_t m;
    uint32_t off;          // bit offset of the level inside the set
};
struct BatchAux {
    uint64_t left_off;     // first of the set's fallback keys in the fallback array
    uint32_t n;
    uint32_t nleft;
};

// Bucket size of the partitioned levels: 2^pbits positions and room for kcap keys in LDS.
struct BucketGeometry {
    uint32_t pbits;
    uint32_t kcap;
};
// pbits = 0: the largest bucket that fits; else exactly 2^pbits positions (a result with pbits = 0
// if that does not fit).
BucketGeometry bucket_geometry(double gamma, uint32_t pbits = 0);
uint32_t tail_capacity(double gamma);

hipError_t launch_partition(int dbits, bool hashed, const uint64_t* in, uint64_t in_stride,
                            const uint64_t* pre, uint32_t groups, uint32_t SG, uint32_t K,
                            const LevelHash& L, uint32_t pbits, uint32_t out_shift, bool grouped,
                            uint32_t group_shift, uint64_t nbins, uint64_t* out, uint64_t out_cap,
                            uint32_t S_out, uint32_t* out_cnt, unsigned long long* overflow,
                            uint64_t n_in, uint64_t nseg_in, hipStream_t s, int dig = 0,
                            const uint64_t* dbase = nullptr, uint32_t pack_shift = 0,
                            const SpecArgs& spec = SpecArgs(), const uint64_t* gen = nullptr);
// Hash-set partition helpers: keys per (set, workgroup) over the slices of a partition pass, every
// K-th entry of their prefix (the set offsets), and a two-word device write.
hipError_t launch_slice_counts(const uint64_t* in, uint64_t in_stride, const uint64_t* pre, uint32_t groups,
                               uint32_t SG, uint32_t K, uint64_t seed, uint32_t sh, bool hashed, bool grouped,
                               uint32_t group_shift, uint64_t nbins, uint32_t* cnt, hipStream_t s);
hipError_t launch_take_every(const uint64_t* base, uint32_t K, uint64_t nsets, uint64_t* offsets, hipStream_t s);
hipError_t launch_pair(uint64_t* p, uint64_t a, uint64_t b, hipStream_t s);
// Keys partitioned by bucket of 2^pbits positions (6 <= pbits <= 18) tested against the finished
// level whose A starts at bit `off` of words (level_words words): the keys whose bit is 0 go to
// region b of Y (ycap keys each), their number to surv[b] (bucket_test_setup once per device first).
hipError_t bucket_test_setup();
hipError_t launch_bucket_test(const uint64_t* in, uint64_t in_cap, const uint32_t* cnt, uint32_t S,
                              uint64_t nbuckets, const LevelHash& L, uint32_t pbits, bool packed,
                              const uint64_t* words, uint64_t off, uint64_t level_words, uint64_t* Y, uint64_t ycap,
                              uint32_t* surv, unsigned long long* overflow, hipStream_t s);
// Keys partitioned by bucket of 2^pbits positions (5 <= pbits <= 18) added to the interleaved A/C
// words W of a level, one workgroup per bucket (accumulate_setup once per device first).
hipError_t accumulate_setup();
hipError_t launch_accumulate(const uint64_t* in, uint64_t in_cap, const uint32_t* cnt, uint32_t S,
                             uint64_t nbuckets, const LevelHash& L, uint32_t pbits, bool packed, uint64_t* W,
                             uint64_t wwords, unsigned long long* overflow, hipStream_t s);
hipError_t launch_bucket(const uint64_t* in, uint64_t in_cap, const uint32_t* cnt, uint32_t S,
                         uint64_t nbuckets, const LevelHash& L, uint32_t pbits, bool packed, uint32_t kcap,
                         uint64_t* A, uint64_t* Cout, uint64_t level_words, uint64_t* Y, uint64_t ycap,
                         uint32_t* surv, unsigned long long* overflow, hipStream_t s,
                         const SpecLevel* spec = nullptr);
hipError_t launch_gather(const uint64_t* in, uint64_t in_stride, const uint64_t* pre, uint32_t nseg,
                         uint64_t n, uint64_t* out, hipStream_t s);
hipError_t launch_tail(const uint64_t* in, uint64_t in_stride, const uint64_t* pre, uint32_t nseg,
                       uint32_t kcap, double gamma, const SeedTable& seeds, uint32_t d0, uint32_t D,
                       uint64_t bit_off, uint64_t* A, uint64_t* Cout, TailLevel* rec, uint64_t* left,
                       TailSummary* sum, hipStream_t s);

// ---- launchers (all asynchronous on `s`) ----
hipError_t launch_zero(uint64_t* p, uint64_t nwords, hipStream_t s);
hipError_t launch_zero32(uint32_t* p, uint64_t n, hipStream_t s);
hipError_t launch_fill(const uint64_t* keys, uint64_t n, uint64_t* W, const LevelHash& L,
                       hipStream_t s);
hipError_t launch_finalize(const uint64_t* W, uint64_t nwords, uint64_t* A, uint64_t* C,
                           unsigned long long* weight, hipStream_t s);
hipError_t launch_filter_fill(const uint64_t* Fin, uint64_t n, const uint64_t* words,
                              const LevelHash& Ld, uint64_t* Fout, uint64_t cap,
                              unsigned long long* count, uint64_t* W, const LevelHash& Lnext,
                              bool do_fill, hipStream_t s);
uint64_t scan_tmp_tiles(uint64_t n);
// (skip: a device word; nonzero when the kernels run makes them return at once)
hipError_t launch_exclusive_scan(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* tmp_tiles,
                                 hipStream_t s, const uint64_t* skip = nullptr);
// streaming build (stream.hip)
// keys = NULL: key i of the range is output kstart + i of the generated stream; else keys[i] (a chunk of a
// stored key set on the device).
hipError_t launch_stream_fill(uint64_t kseed, uint64_t kstart, const uint64_t* keys, uint64_t n, const DevLevel* lev,
                              uint32_t d, const uint64_t* words, uint64_t* W, const LevelHash& L, hipStream_t s);
hipError_t launch_stream_collect(uint64_t kseed, uint64_t kstart, const uint64_t* keys, uint64_t n,
                                 const DevLevel* lev, uint32_t d, const uint64_t* words, uint64_t* out, uint64_t cap,
                                 unsigned long long* count, hipStream_t s);
hipError_t launch_stream_keys(uint64_t kseed, uint64_t kstart, uint64_t n, uint64_t* out, hipStream_t s);

// k-mer workload (kmer.hip)
hipError_t launch_kmers(const uint64_t* seq, uint64_t npos, uint32_t k, uint64_t* out, hipStream_t s);
hipError_t launch_repeated(const uint64_t* sorted, uint64_t n, uint64_t* out, uint64_t cap,
                           unsigned long long* count, hipStream_t s);
hipError_t launch_first_pos(const uint64_t* keys, uint64_t n, const uint64_t* rep, uint64_t nrep,
                            unsigned long long* first, hipStream_t s);
hipError_t launch_later_pos(const uint64_t* keys, uint64_t n, const uint64_t* rep, uint64_t nrep,
                            const unsigned long long* first, uint64_t* out, uint64_t cap, unsigned long long* count,
                            hipStream_t s);
hipError_t launch_drop_positions(const uint64_t* keys, uint64_t n, const uint64_t* removed, uint64_t nrem,
                                 uint64_t* out, hipStream_t s);
hipError_t launch_set_partition(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t bits, uint32_t* counts,
                                uint64_t* offsets, unsigned long long* cursor, uint64_t* tiles, uint64_t* out,
                                hipStream_t s);
hipError_t launch_set_ids(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t bits, uint64_t* out,
                          hipStream_t s);

// LSD radix sort of n keys; `a` holds the input and receives the sorted keys, `b` is scratch.
uint64_t radix_tmp_counts(uint64_t n);
hipError_t radix_sort_u64(uint64_t* a, uint64_t* b, uint64_t n, uint32_t* counts,
                          uint64_t* offsets, uint64_t* tmp_tiles, hipStream_t s);
hipError_t launch_find_duplicates(const uint64_t* sorted, uint64_t n, unsigned long long* flag,
                                  hipStream_t s);
uint64_t sector_count(uint64_t total_bits);
uint64_t super_count(uint64_t nsec);
// The rank table (counters every rank_sample positions) and the lookup sectors from one counting
// read of A: tmp_counts holds a u32 per sector, tmp_rank_counts a u32 per rank entry, tmp_pre a u64
// per sector, tmp_tiles scan_tmp_tiles(max(sectors, rank entries)).
hipError_t launch_rank_sectors(const uint64_t* words, uint64_t total_bits, uint32_t rank_sample, uint64_t* rank,
                               uint64_t nrank, uint32_t* sec, uint64_t* super, uint32_t* tmp_group_sums,
                               uint64_t* tmp_group_pre, uint64_t* tmp_tiles, hipStream_t s);
// Workgroups of the sector layout (256 sectors each): the sizes of the two temporaries above.
uint64_t rank_sector_groups(uint64_t total_bits);
hipError_t launch_lookup(const uint64_t* q, uint64_t n, uint64_t* out, const DevLevel* lev,
                         uint32_t nlev, const uint32_t* sec, const uint64_t* super,
                         const uint64_t* fb_keys, uint64_t nfb, uint64_t N, hipStream_t s);
hipError_t launch_positions(const uint64_t* keys, uint64_t n, const LevelHash& L, uint64_t* out,
                            hipStream_t s);
// out[0] = *flag, out[1] = *total (out: host memory mapped for the device), *last = *flag, then
// *flag = 0 and out[2] = seq.
hipError_t launch_report(unsigned long long* flag, const uint64_t* total, uint64_t* out, uint64_t seq,
                         unsigned long long* last, hipStream_t s);


// Launch configuration of the batched build kernel: threads per workgroup (128, 256 or 512), keys
// per thread in flight (4, 8 or 16) and workgroups per CU (1..8, further bounded by LDS).
struct BatchLaunch {
    uint32_t threads = 256;
    uint32_t items = 4;
    uint32_t wgs_per_cu = 0;     // 0: as many as the LDS allows, at most 8
    uint32_t small_class = 13;   // sets of fewer than 2^(small_class - 1) keys are small
    uint32_t small_every = 2;    // every small_every-th workgroup takes small sets first (0: none)
};

uint32_t batch_classes();
hipError_t launch_batch_prepare(const uint64_t* offsets, uint64_t nsets, double gamma, uint32_t D, uint64_t max_m,
                                double slack, uint32_t* bound, uint32_t* sbound, uint32_t* hist,
                                unsigned long long* info, hipStream_t s);
hipError_t launch_batch_order(const uint64_t* offsets, uint64_t nsets, const uint32_t* hist, uint32_t* cursor,
                              uint32_t* order, hipStream_t s);
hipError_t launch_batch_reset(unsigned long long* queue, uint32_t* fail, hipStream_t s);
hipError_t launch_batch_build(const uint64_t* keys, const uint64_t* offsets, const uint32_t* order,
                              uint64_t nsets, const uint32_t* hist, unsigned long long* next, uint64_t* scratch,
                              const uint64_t* region_w, double gamma, const SeedTable& seeds,
                              uint32_t D, uint32_t left_cap, uint64_t* region, uint32_t* sreg,
                              const uint64_t* sreg_base, BatchSet* sets, BatchLevel* levels, uint64_t max_m,
                              const BatchLaunch& cfg, uint32_t grid, hipStream_t s);
uint64_t batch_lds_bytes(uint64_t max_m, uint32_t left_cap);
// Once per configuration and size, before any launch (and so outside a graph capture).
hipError_t batch_kernel_setup(const BatchLaunch& cfg, uint64_t max_m, uint32_t left_cap);
hipError_t launch_batch_tally(const BatchSet* sets, uint64_t nsets, uint32_t* left32, uint32_t* sec32,
                              uint32_t* fail, hipStream_t s);
hipError_t launch_batch_pack(const uint32_t* sreg, BatchSet* sets, uint64_t nsets, const uint64_t* sec_pre,
                             const uint64_t* left_pre, const uint64_t* scratch, uint32_t* sec, uint64_t* left,
                             hipStream_t s);
hipError_t launch_batch_heads(const BatchSet* sets, const BatchLevel* levels, uint32_t D, uint64_t nsets,
                              BatchHead* heads, BatchLev* lev, BatchAux* aux, hipStream_t s);
hipError_t launch_batch_lookup(const uint64_t* set_ids, const uint64_t* q, uint64_t n, uint64_t* out,
                               const BatchHead* heads, const BatchLev* lev, const BatchAux* aux, uint32_t D,
                               uint64_t nsets, const uint32_t* sec, const uint64_t* left, const SeedTable& seeds,
                               hipStream_t s);

}  // namespace mphfk
