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

// ---- launchers (all asynchronous on `s`) ----
hipError_t launch_zero(uint64_t* p, uint64_t nwords, hipStream_t s);
hipError_t launch_fill(const uint64_t* keys, uint64_t n, uint64_t* W, const LevelHash& L,
                       hipStream_t s);
hipError_t launch_finalize(const uint64_t* W, uint64_t nwords, uint64_t* A, uint64_t* C,
                           unsigned long long* weight, hipStream_t s);
hipError_t launch_filter_fill(const uint64_t* Fin, uint64_t n, const uint64_t* words,
                              const LevelHash& Ld, uint64_t* Fout, uint64_t cap,
                              unsigned long long* count, uint64_t* W, const LevelHash& Lnext,
                              bool do_fill, hipStream_t s);
hipError_t launch_rank(const uint64_t* words, uint64_t total_words, uint32_t rank_sample,
                       uint64_t* rank, uint64_t nrank, uint32_t* tmp_counts, uint64_t* tmp_tiles,
                       hipStream_t s);
uint64_t scan_tmp_tiles(uint64_t n);
hipError_t launch_exclusive_scan(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* tmp_tiles,
                                 hipStream_t s);
// LSD radix sort of n keys; `a` holds the input and receives the sorted keys, `b` is scratch.
uint64_t radix_tmp_counts(uint64_t n);
hipError_t radix_sort_u64(uint64_t* a, uint64_t* b, uint64_t n, uint32_t* counts,
                          uint64_t* offsets, uint64_t* tmp_tiles, hipStream_t s);
hipError_t launch_find_duplicates(const uint64_t* sorted, uint64_t n, unsigned long long* flag,
                                  hipStream_t s);
hipError_t launch_lookup(const uint64_t* q, uint64_t n, uint64_t* out, const DevLevel* lev,
                         uint32_t nlev, const uint64_t* words, const uint64_t* rank,
                         uint32_t rank_shift, const uint64_t* fb_keys, uint64_t nfb, uint64_t N,
                         hipStream_t s);
hipError_t launch_positions(const uint64_t* keys, uint64_t n, const LevelHash& L, uint64_t* out,
                            hipStream_t s);

}  // namespace mphfk
