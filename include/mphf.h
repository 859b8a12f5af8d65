/*
 * mphf.h -- C ABI of the MI355X (gfx950) cascading-bit-array minimal perfect
 * hash function of Limasset, Rizk, Chikhi and Peterlongo, "Fast and scalable
 * minimal perfect hashing for massive key sets" (arXiv 1702.03154).
 *
 * Given N distinct 64-bit keys, the build computes a bijection of the keys
 * onto [1, N] (Section 1, first paragraph).  Level d hashes every key of the
 * set F_d into a bit array A_d of m_d = ceil(gamma * |F_d|) positions; a
 * position keeps a 1 iff exactly one key lands on it, and the keys that
 * collided form F_{d+1} (Section 2.1; Section 2.2, "Collision detection";
 * Algorithms 1 and 2).  After at most max_levels levels the leftover keys go
 * to a fallback table (Section 3, "Termination").  A query walks the levels
 * until its bit is 1 and returns the number of ones before that bit in the
 * concatenation of all A_d, plus one (Section 2.1, query paragraph;
 * Section 2.2, "Minimality"; Algorithm 3), using 64-bit counters sampled
 * every 512 positions (Section 3.1, "Rank structure").
 *
 * Conventions for every entry point:
 *  - Key, query and label arrays are DEVICE pointers (hipMalloc memory or a
 *    ROCm tensor's storage) on the current HIP device.  The caller owns them;
 *    keys and queries are only read.  A host pointer is rejected with
 *    MPHF_E_INVALID.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - An mphf_t owns all the device memory of one function and is immutable
 *    after the build, so lookups on one handle from several streams or host
 *    threads at once are safe.  mphf_destroy must not overlap any of them.
 *  - Errors return a status; mphf_last_error() gives this thread's message
 *    for the last failing call.  On error nothing is leaked and *out is NULL.
 */
#ifndef MPHF_H
#define MPHF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPHF_MAX_LEVELS 64

typedef struct mphf mphf_t;

typedef enum mphf_status {
    MPHF_OK = 0,
    MPHF_E_INVALID = 1,        /* bad argument: gamma < 1 or NaN, NULL or host pointer, bad option */
    MPHF_E_NOMEM = 2,          /* device allocation failed or mem_budget exceeded */
    MPHF_E_DUPLICATE_KEYS = 3, /* two input keys are equal (they collide at every level) */
    MPHF_E_DEVICE = 4          /* a HIP call failed; the message carries hipGetErrorString */
} mphf_status;

/* Build options.  mphf_default_opts() fills the defaults. */
typedef struct mphf_opts {
    uint32_t max_levels;      /* D, the number of levels before the fallback table:
                                 1..MPHF_MAX_LEVELS, default 25 (Section 3, "Termination") */
    uint32_t rank_sample;     /* positions per rank counter: 512 (default, Section 3.1) or
                                 1024 (the "minirank" row of Table 1) */
    uint64_t mem_budget;      /* upper bound on the device bytes the build holds at once
                                 (workspace plus the structure); 0 = no bound */
    uint32_t keep_collisions; /* nonzero: keep every C_d so that mphf_export_collisions works */
    uint32_t flags;           /* 0, or MPHF_FLAG_ATOMIC_LEVELS */
    /* Launch configuration of the batched build (0 = default; ignored by single builds):
     * threads per workgroup 128/256/512 (default 256), keys in flight per thread 4/8/16
     * (default 4), workgroups per CU 1..8 (default: as many as the LDS allows, at most 8).
     * The size-class split of its work queue is at the end of this struct. */
    uint32_t batch_threads;
    uint32_t batch_items;
    uint32_t batch_wgs_per_cu;
    uint32_t bucket_bits;     /* log2 of the positions per bucket of the partitioned levels of a
                                 single build: 0 (default) = the largest bucket whose keys fit one
                                 workgroup's LDS (2^14 positions at gamma = 1, 2^15 at gamma = 2,
                                 2^16 from gamma = 4.3),
                                 else 6..16 and at most that default.  Smaller buckets make a level
                                 take more buckets and wider partition passes with the same result;
                                 for checks of those paths on small key sets. */
    /* Work queues of the batched build (0 = default; ignored by single builds).  Sets of fewer
     * than 2^(batch_small_class - 1) keys are small (1..64; default 13: below 4096 keys; 1: none,
     * one queue, largest sets first); every batch_small_every-th workgroup (default 2) takes
     * small sets first and the others large sets first, so that the small sets' short,
     * latency-bound levels overlap the large sets' streaming passes.  Same result either way. */
    uint32_t batch_small_class;
    uint32_t batch_small_every;
} mphf_opts;

/* Build every level by global atomic test-and-set on the interleaved A/C words instead of the
 * default position-partitioned LDS passes.  Same result, slower; for comparison and tests. */
#define MPHF_FLAG_ATOMIC_LEVELS 1u

/* Per-level sizes and totals of a built function (all host values). */
typedef struct mphf_stats {
    uint64_t n;                               /* N */
    double gamma;
    uint64_t seed;
    uint32_t num_levels;                      /* levels actually built (last + 1) */
    uint32_t rank_sample;
    uint64_t level_n[MPHF_MAX_LEVELS];        /* |F_d| */
    uint64_t level_m[MPHF_MAX_LEVELS];        /* |A_d| = ceil(gamma |F_d|) */
    uint64_t level_weight[MPHF_MAX_LEVELS];   /* ones in A_d = keys placed at level d */
    uint64_t level_offset[MPHF_MAX_LEVELS];   /* bit offset of A_d in the concatenated A */
    uint64_t level_seed[MPHF_MAX_LEVELS];     /* s_d */
    uint64_t n_fallback;                      /* |L|, keys in the fallback table */
    uint64_t total_bits;                      /* M, bits of the concatenated A (64-bit padded levels) */
    uint64_t rank_entries;                    /* ceil(M / rank_sample) */
    uint64_t structure_bytes;                 /* A + rank counters + fallback keys */
    double bits_per_key;                      /* (M + 64 * rank_entries + 128 * n_fallback) / N */
    uint64_t peak_bytes;                      /* most device bytes the build held at once */
    uint64_t lookup_bytes;                    /* the lookup's copy of A: 64-byte sectors that each hold a
                                                 32-bit rank counter and 480 bits, plus superblock counters */
    uint32_t level_path[MPHF_MAX_LEVELS];     /* how level d was built: one of MPHF_PATH_* */
    uint32_t bucket_bits;                     /* log2 of the bucket size of the partitioned levels */
    uint32_t reserved;
} mphf_stats_t;

/* Values of mphf_stats_t.level_path.  Every path gives the same bits (a position keeps its 1 iff
 * exactly one key lands on it, whatever the order of insertion).  A level of m positions in buckets
 * of 2^b positions (b = bucket_bits) has B = ceil(m / 2^b) buckets:
 *   B <= 1024: one radix pass into the buckets;
 *   1024 < B <= 2^16: a pass into coarse bins, then 2^8 buckets per bin;
 *   2^16 < B <= 2^18: the same with 2^9 or 2^10 buckets per bin (the wide second pass);
 *   B > 2^18 (more than 2^(18+b) positions, e.g. about 4.3e9 keys per level at gamma = 2):
 *   global atomic test-and-set over the whole level, also used after a region overflow (adversarial
 *   key sets) and with MPHF_FLAG_ATOMIC_LEVELS. */
#define MPHF_PATH_TAIL 1            /* every remaining level in one workgroup's LDS (small levels) */
#define MPHF_PATH_ONE_PASS 2
#define MPHF_PATH_TWO_PASS 3
#define MPHF_PATH_TWO_PASS_WIDE 4
#define MPHF_PATH_ATOMIC 5
#define MPHF_PATH_STREAMED 6        /* streaming build: chunks partitioned and added in LDS */
#define MPHF_PATH_STREAMED_ATOMIC 7 /* streaming build: global test-and-set over the stream */

/* Read-only device views of a built function (owned by the handle). */
typedef struct mphf_view {
    const uint64_t* words;          /* concatenated A: bit p of level d is bit (o+p)%64 of word (o+p)/64,
                                       o = level_offset[d]; padding bits are 0 */
    const uint64_t* rank;           /* rank[b] = ones of A before bit b * rank_sample */
    const uint64_t* fallback_keys;  /* ascending; key i has label N - n_fallback + 1 + i */
    const uint64_t* collisions;     /* C of every level laid out like A, or NULL without keep_collisions */
    uint64_t total_words;
    uint64_t rank_entries;
    uint64_t n_fallback;
} mphf_view_t;

/* Fill *opts with the defaults (max_levels 25, rank_sample 512, no budget). */
mphf_status mphf_default_opts(mphf_opts* opts);

/* Build from n distinct device keys with parameter gamma (Section 2.2: |A_d| = gamma |F_d|,
 * gamma >= 1) and hash seed `seed` (the level seeds s_d are the outputs of a SplitMix64
 * stream started at `seed`).  Default options, null stream; returns once the function is
 * complete.  NULL on error (see mphf_last_error). */
mphf_t* mphf_build(const uint64_t* keys, uint64_t n, double gamma, uint64_t seed);

/* Label each of the n device queries into the device array out (Algorithm 3): a key of the
 * set gets its label in [1, N]; any other key gets a deterministic value, which is 0 when it
 * falls through every level and is not in the fallback table (the footnote of Algorithm 3
 * allows any value).  Synchronous on the null stream.  Returns an mphf_status. */
int mphf_lookup(const mphf_t* h, const uint64_t* keys, uint64_t n, uint64_t* out);

/* mphf_build with options (NULL = defaults) on `stream`.  The build reads the level sizes back
 * to the host once per level, so it returns only when the function is complete on `stream`. */
mphf_status mphf_build_ex(const uint64_t* keys, uint64_t n, double gamma, uint64_t seed,
                          const mphf_opts* opts, void* stream, mphf_t** out);

/* mphf_lookup enqueued on `stream`; returns without waiting.  `out` may not alias `keys`. */
mphf_status mphf_lookup_ex(const mphf_t* h, const uint64_t* keys, uint64_t n, uint64_t* out,
                           void* stream);

/* Free every device buffer of h.  NULL is allowed. */
void mphf_destroy(mphf_t* h);

/* Sizes and per-level counts of h. */
mphf_status mphf_stats(const mphf_t* h, mphf_stats_t* st);

/* Device pointers to the structure of h, valid until mphf_destroy(h). */
mphf_status mphf_view(const mphf_t* h, mphf_view_t* v);

/* Copy the structure to host arrays (synchronous): `words` receives total_words words of the
 * concatenated A, `rank` rank_entries counters, `fallback_keys` n_fallback keys.  Each size must
 * equal the one mphf_stats reports; a NULL array with size 0 skips that part. */
mphf_status mphf_export(const mphf_t* h, uint64_t* words, uint64_t nwords, uint64_t* rank,
                        uint64_t nrank, uint64_t* fallback_keys, uint64_t nfb);

/* Copy C_d (the collision array of level d, Section 2.2) into the host array out of
 * ceil(level_m[d] / 64) words, packed like A_d.  Needs keep_collisions at build time. */
mphf_status mphf_export_collisions(const mphf_t* h, uint32_t level, uint64_t* out, uint64_t nwords);

/* The level-d position of each device key: fmix64(key XOR level_seed) mod m, the reduction of
 * Algorithms 1-3, exactly as the build and lookup kernels compute it (m >= 1).  For checks of the
 * hash and of the exact division by m; out is a device array of n words. */
mphf_status mphf_positions(const uint64_t* keys, uint64_t n, uint64_t level_seed, uint64_t m,
                           uint64_t* out, void* stream);

/* ---- Streaming build: key sets generated on the fly, beyond device memory -------------------
 * The keys are never stored: key i (0 <= i < n) is output start + i of the SplitMix64 stream
 * seeded with `seed` (Steele, Lea and Flood, OOPSLA 2014): the mix of seed + (start+i+1) *
 * 0x9E3779B97F4A7C15, so the n keys are distinct (as the generated stream of Section 4.5). */
typedef struct mphf_key_stream {
    uint64_t seed;
    uint64_t start;
} mphf_key_stream;

/* Build over the n keys of `src`.  While more than resident_keys keys are left, a level re-generates
 * every key and skips those placed at an earlier level (a lookup walk over the finished levels):
 * the re-scan strategy of Section 3.4, which stores no F_d.  The stream is taken in chunks of
 * max(resident_keys, 2^20) keys: a chunk's keys are radix-partitioned by bucket of each finished
 * level and tested against its bits in LDS, and the unplaced ones partitioned by bucket of the
 * current level and added to its A and C bits in LDS.  Levels beyond 2^36 positions, or flags =
 * MPHF_FLAG_ATOMIC_LEVELS, walk by random reads and mark with global test-and-set instead.
 * Then the survivors are collected (8 bytes each) and the build continues in memory.  The
 * function, its levels and labels equal those of mphf_build_ex on the materialized keys.  Device
 * memory: the structure, 2 gamma n bits for the first level's A and C, the survivors and, for a
 * chunk, its keys and two partition buffers of about 9 bytes per key.  flags: 0 or
 * MPHF_FLAG_ATOMIC_LEVELS.  Synchronous, like mphf_build_ex. */
mphf_status mphf_build_stream(const mphf_key_stream* src, uint64_t n, double gamma, uint64_t seed,
                              const mphf_opts* opts, uint64_t resident_keys, void* stream, mphf_t** out);

/* The same streaming build over n keys stored in HOST memory (pinned memory from mphf_host_alloc is
 * copied fastest; any host array works): the re-scan strategy of Section 3.4 for a stored key set
 * larger than device memory.  Every streamed level copies the keys to the device chunk by chunk
 * (max(resident_keys, 2^20) keys at a time, over PCIe) and treats them as mphf_build_stream treats its
 * generated keys; no F_d is stored until the survivors fit resident_keys.  The keys must stay
 * unchanged until the call returns; a device pointer is rejected with MPHF_E_INVALID (mphf_build_ex
 * builds from device keys).  The function, its levels and labels equal those of mphf_build_ex on the
 * same keys; duplicate keys give MPHF_E_DUPLICATE_KEYS.  Synchronous. */
mphf_status mphf_build_host(const uint64_t* keys, uint64_t n, double gamma, uint64_t seed, const mphf_opts* opts,
                            uint64_t resident_keys, void* stream, mphf_t** out);

/* Keys first .. first+count-1 of the stream into the device array out (queries of a streamed build). */
mphf_status mphf_stream_keys(const mphf_key_stream* src, uint64_t first, uint64_t count, uint64_t* out,
                             void* stream);

/* ---- Batched builds: many independent key sets built in one launch ---------------------------
 * Set s holds the device keys keys[offsets[s] .. offsets[s+1]) (offsets: nsets+1 device u64,
 * non-decreasing, offsets[0] = 0).  Every set is an independent function with labels 1..n_s whose
 * levels, bits and labels are those of a standalone build of that set with the same gamma, seed
 * and options (Section 2; the levels of a set depend only on its keys, gamma and the level seeds).
 * A set may have at most 2^19 / gamma keys (ceil(gamma n) <= 2^19: its A and C bits live in one
 * workgroup's LDS).  A set that keeps more than 2048 keys after its last level fails the whole
 * batch with MPHF_E_INVALID, and duplicate keys within a set with MPHF_E_DUPLICATE_KEYS; keys
 * of different sets may be equal.  flags must be 0, rank_sample 512; keep_collisions is ignored.
 * A batch handle owns its device memory and is immutable between builds; lookups follow the
 * rules of mphf_lookup_ex. */
typedef struct mphf_batch mphf_batch_t;

typedef struct mphf_set_info {
    uint64_t n;
    uint32_t num_levels;
    uint32_t n_fallback;
    uint64_t level_n[MPHF_MAX_LEVELS];
    uint64_t level_m[MPHF_MAX_LEVELS];
    uint64_t level_offset[MPHF_MAX_LEVELS];   /* bit offset inside the set's own bits */
    uint64_t total_bits;                      /* the set's bits (64-bit padded levels) */
} mphf_set_info_t;

/* One-shot batched build on `stream`; returns when the batch is complete.  The structure is
 * packed: each set's lookup sectors (64 bytes per 480 bits of the set, with a 32-bit count of the
 * set's ones before them), a 16-byte head per set and the sets' fallback keys. */
mphf_status mphf_build_batch(const uint64_t* keys, const uint64_t* offsets, uint64_t nsets,
                             double gamma, uint64_t seed, const mphf_opts* opts, void* stream,
                             mphf_batch_t** out);

/* A planned batch for repeated builds of sets of these sizes: checks the offsets (copied) and
 * allocates, for the worst case of these sizes (every key surviving every level), every buffer a
 * build needs.  Synchronous.  The handle holds no function until mphf_batch_rebuild. */
mphf_status mphf_batch_plan(const uint64_t* offsets, uint64_t nsets, double gamma, uint64_t seed,
                            const mphf_opts* opts, void* stream, mphf_batch_t** out);

/* Build a planned batch from `keys` (laid out by the plan's offsets): only kernel launches on
 * `stream`, with no allocation and no host synchronization, so the call can be captured in a HIP
 * graph and replayed (the graph keeps the keys pointer).  The function is ready when the stream
 * reaches this point; a failed build (duplicate keys, a set with too many leftovers) is reported
 * by mphf_batch_status.  MPHF_E_INVALID for a handle that was not planned. */
mphf_status mphf_batch_rebuild(mphf_batch_t* b, const uint64_t* keys, void* stream);

/* Wait for `stream` and report the last build of a planned batch (MPHF_OK for a one-shot one). */
mphf_status mphf_batch_status(mphf_batch_t* b, void* stream);

/* Label each (set_ids[i], keys[i]) device pair into out[i] (Algorithm 3 within set set_ids[i]);
 * a set id out of range gives 0.  Asynchronous on `stream`. */
mphf_status mphf_batch_lookup(const mphf_batch_t* b, const uint64_t* set_ids, const uint64_t* keys,
                              uint64_t n, uint64_t* out, void* stream);

/* Sizes of set `set` (host values, synchronous). */
mphf_status mphf_batch_set_info(const mphf_batch_t* b, uint64_t set, mphf_set_info_t* info);

/* Host copies of set `set`'s bits (info.total_bits / 64 words, laid out like mphf_export's A) and
 * fallback keys (ascending). */
mphf_status mphf_batch_export_set(const mphf_batch_t* b, uint64_t set, uint64_t* words, uint64_t nwords,
                                  uint64_t* fallback_keys, uint64_t nfb);

/* Host copy of set `set`'s lookup sectors: ceil(total_bits / 480) sectors of 16 u32, word 0 the
 * ones of the set before the sector, words 1..15 the next 480 bits of the set. */
mphf_status mphf_batch_export_sectors(const mphf_batch_t* b, uint64_t set, uint32_t* sectors,
                                      uint64_t nsectors);

/* Sets, total keys, total bits of the sets' levels and bits/key of the packed structure. */
mphf_status mphf_batch_totals(const mphf_batch_t* b, uint64_t* nsets, uint64_t* nkeys,
                              uint64_t* total_bits, double* bits_per_key);

/* Free every device buffer of b.  NULL is allowed; must not overlap a lookup or build on b. */
void mphf_batch_destroy(mphf_batch_t* b);

/* ---- Serving: many resident functions, lookup requests batched as they arrive ---------------
 * A server keeps registered functions resident and answers lookup requests from host memory.
 * Requests wait in arrival order and are admitted while their device memory (16 bytes per key:
 * the key in, the label out) fits the server's HBM budget; every admitted group of requests is one
 * batch: one segmented lookup kernel labels all of them (each request against its own function,
 * Algorithm 3).  Arrays in pinned host memory (mphf_host_alloc) are read and written by that kernel
 * in place over PCIe; other arrays are copied into the batch's device buffers and back.  The budget
 * counts 16 bytes per key for every request alike.  Up to max_inflight
 * batches are on the device at once on their own streams, so requests arriving while a batch runs
 * form the next one and its copies overlap the running kernels (continuous batching).  A request's
 * labels are exactly those of mphf_lookup on its function, alone or in any mix.
 * The server's threads issue all device work; the API calls are thread-safe. */
typedef struct mphf_server mphf_server_t;

typedef struct mphf_server_opts {
    uint64_t hbm_budget;           /* device bytes for requests in flight (default 1 GiB); split
                                      evenly over the in-flight batches */
    uint32_t max_inflight;         /* batches on the device at once, 1..8 (default 2) */
    uint32_t max_batch_requests;   /* requests per batch (default 1024) */
} mphf_server_opts;

typedef struct mphf_request_info {
    uint32_t done;                 /* 1 once the labels are in the caller's array */
    uint32_t batch_requests;       /* requests in the batch that served this one */
    uint64_t batch;                /* sequence number of that batch */
    double submit_us, start_us, done_us;   /* server clock: submitted, batch launched, labels out */
} mphf_request_info;

typedef struct mphf_server_stats {
    uint64_t requests, keys, batches;      /* completed */
    uint64_t max_batch_requests_seen;
    uint64_t peak_bytes_in_flight;
} mphf_server_stats;

/* Fill *opts with the defaults. */
mphf_status mphf_server_default_opts(mphf_server_opts* opts);

/* A server on the current device (NULL opts = defaults). */
mphf_status mphf_server_create(const mphf_server_opts* opts, mphf_server_t** out);

/* Make a built function resident: its id is written to *id.  h must be on the server's device and
 * outlive the server (the server does not own it). */
mphf_status mphf_server_register(mphf_server_t* s, const mphf_t* h, uint32_t* id);

/* Queue a request: label keys[0..n) (host memory) against function `id` into out[0..n) (host
 * memory).  Both arrays must stay valid until the request is done; pinned memory from
 * mphf_host_alloc is used in place (no copies).  *ticket identifies the request.  MPHF_E_INVALID for an unknown
 * id or a request larger than one batch's share of the budget. */
mphf_status mphf_server_submit(mphf_server_t* s, uint32_t id, const uint64_t* keys, uint64_t n,
                               uint64_t* out, uint64_t* ticket);

/* State of a request; with wait != 0, block until it is done.  A done request is forgotten after
 * it has been reported (poll each ticket until done once). */
mphf_status mphf_server_poll(mphf_server_t* s, uint64_t ticket, int wait, mphf_request_info* info);

mphf_status mphf_server_get_stats(const mphf_server_t* s, mphf_server_stats* st);

/* Finish every queued request, stop the server's threads and free its memory.  NULL is allowed. */
void mphf_server_destroy(mphf_server_t* s);

/* Pinned host memory for request arrays (and its release). */
mphf_status mphf_host_alloc(uint64_t bytes, void** out);
void mphf_host_free(void* p);

/* ---- k-mer keys (the de Bruijn graph use of Section 1) -----------------------------------------
 * A DNA sequence of nbases bases packed 2 bits per base (A=0, C=1, G=2, T=3): base i is bits
 * 63-2(i%32) .. 62-2(i%32) of seq[i/32] (first base of a word in its most significant pair). */

/* out[p] = canonical k-mer at p for p in [0, nbases-k]: the smaller of the forward k-mer (bases
 * p..p+k-1, first base most significant, 2k bits) and its reverse complement (bases reversed, each
 * x -> 3-x).  1 <= k <= 32; device arrays; asynchronous on `stream`. */
mphf_status mphf_kmers(const uint64_t* seq, uint64_t nbases, uint32_t k, uint64_t* out, void* stream);

/* The first min(target, distinct) distinct keys of keys[0..n) in order of first occurrence, into the
 * device array out (room for target keys); *nout gets their number.  Synchronous.  Uses about
 * 17.5 n bytes of temporary device memory (a sorted copy finds the keys that repeat). */
mphf_status mphf_first_occurrences(const uint64_t* keys, uint64_t n, uint64_t target, uint64_t* out,
                                   uint64_t* nout, void* stream);

/* Hash partition of n keys into 2^bits sets (set of x = top `bits` bits of fmix64(x XOR seed)):
 * out gets the keys grouped by set (any order within a set), offsets (2^bits + 1 device u64) the
 * start of each set: the input of mphf_build_batch.  Synchronous.  1 <= bits <= 24. */
mphf_status mphf_partition_sets(const uint64_t* keys, uint64_t n, uint32_t bits, uint64_t seed,
                                uint64_t* out, uint64_t* offsets, void* stream);

/* out[i] = the set of keys[i] under the same partition (the set ids of batched lookups). */
mphf_status mphf_set_ids(const uint64_t* keys, uint64_t n, uint32_t bits, uint64_t seed, uint64_t* out,
                         void* stream);

/* mphf_partition_sets for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same sets and offsets, with no device
 * allocation and no host synchronization.  Its scratch (per-set counts and cursors, about 770 KiB)
 * is a fixed array of the library that each device holds until the process ends, so 1 <= bits <= 16
 * (MPHF_E_INVALID beyond).  The caller passes the keys, out (n keys) and offsets (2^bits + 1 u64),
 * all device memory.  Asynchronous on `stream`.  Every call on a device shares that device's
 * scratch: calls that overlap on one device (on different streams or threads) race and must be
 * serialized by the caller.  The order of the keys inside a set is unspecified. */
mphf_status mphf_partition_sets_noalloc(const uint64_t* keys, uint64_t n, uint32_t bits, uint64_t seed,
                                        uint64_t* out, uint64_t* offsets, void* stream);

/* ---- Roofline microbenchmarks ----------------------------------------------------------------
 * The memory-system ceilings the build and lookup are measured against: the method streams keys and
 * makes random accesses into bit arrays (a test-and-set per key and level while building,
 * Algorithm 2; a probe per visited level while querying, Algorithm 3), and random accesses are what
 * limits it (Section 3.2, "Parallelization"; Section 4.2).  mphf_probe enqueues one probe kernel on
 * `stream` (asynchronous; time it with events on that stream):
 *   MPHF_PROBE_STREAM_READ       read `bytes` of buf once (16-byte loads);
 *   MPHF_PROBE_STREAM_COPY       copy `bytes` from buf to dst;
 *   MPHF_PROBE_RANDOM_READ8      about `ops` 8-byte reads at random words of the `bytes` of buf;
 *   MPHF_PROBE_RANDOM_SECTOR64   about `ops` reads of a random aligned 64-byte sector of buf (four
 *                                16-byte loads, as a lookup probe issues them);
 *   MPHF_PROBE_RANDOM_ATOMIC_OR  about `ops` atomicOr with the old value returned at random words of
 *                                buf (the global test-and-set); buf's contents change;
 *   MPHF_PROBE_LDS_ATOMIC_OR     about `ops` atomicOr with return at random words of `bytes`
 *                                (4..49152) of each workgroup's LDS; buf and dst are unused;
 *   MPHF_PROBE_HOST_EXCHANGE     a kernel reads `bytes` (a multiple of 8) of buf and writes them
 *                                to dst, 8 bytes a lane, both pinned host memory (mphf_host_alloc)
 *                                reached over PCIe: the ceiling of a lookup fed from host memory.
 * buf (and dst) are caller-owned device memory, buf 64-byte aligned, except for
 * MPHF_PROBE_HOST_EXCHANGE.  `seed` seeds the random
 * indices.  mphf_probe_ops(ops) is the exact number of random operations a probe of `ops` performs
 * (rounded up to whole rounds of the launch). */
#define MPHF_PROBE_STREAM_READ 0
#define MPHF_PROBE_STREAM_COPY 1
#define MPHF_PROBE_RANDOM_READ8 2
#define MPHF_PROBE_RANDOM_SECTOR64 3
#define MPHF_PROBE_RANDOM_ATOMIC_OR 4
#define MPHF_PROBE_LDS_ATOMIC_OR 5
#define MPHF_PROBE_HOST_EXCHANGE 6
mphf_status mphf_probe(uint32_t kind, void* buf, uint64_t bytes, void* dst, uint64_t ops, uint64_t seed,
                       void* stream);
uint64_t mphf_probe_ops(uint64_t ops);

/* Free the build temporaries the library keeps per device between builds (a few times the
 * largest key set built so far).  Must not overlap a build. */
mphf_status mphf_trim(void);

/* Message of the last failing call on this thread ("" if none). */
const char* mphf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MPHF_H */
