// Host runtime and C ABI: the level driver of the build (Algorithm 1), the fallback table,
// the rank table and the lookup entry points.  Every step of the method runs in the kernels of
// kernels.hip and partition.hip (batch.hip, stream.hip, kmer.hip and server.hip for the batched,
// streamed, k-mer and serving paths); the host only sizes levels, allocates, and reads one count
// back per level.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "api_internal.h"
#include "internal.h"
#include "mphf.h"

using namespace mphfk;

// The streams a handle's device work was enqueued on after its build (lookups, rebuilds), each with
// an event recorded after its latest use there, so that destroying the handle waits for exactly that
// work rather than for the whole device (a serving loop's other batches keep running).  Work
// recorded into a HIP graph under capture is not tracked: the caller finishes its replays first.
class UseTracker {
  public:
    hipError_t note(hipStream_t s) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess) return hipGetLastError();
        if (cs != hipStreamCaptureStatusNone) return hipSuccess;
        std::lock_guard<std::mutex> g(mu_);
        for (auto& u : uses_)
            if (u.first == s) return hipEventRecord(u.second, s);
        hipEvent_t e = nullptr;
        hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r != hipSuccess) return r;
        uses_.push_back({s, e});
        return hipEventRecord(e, s);
    }
    void wait_all() {
        std::lock_guard<std::mutex> g(mu_);
        for (auto& u : uses_) {
            (void)hipEventSynchronize(u.second);
            (void)hipEventDestroy(u.second);
        }
        uses_.clear();
        (void)hipGetLastError();
    }

  private:
    std::mutex mu_;
    std::vector<std::pair<hipStream_t, hipEvent_t>> uses_;
};

// Frees device memory of a destroyed handle in stream order on a library-owned stream of the
// device (non-blocking, default priority), so that no other stream is waited for.
void free_on_device(int dev, const std::vector<void*>& ptrs) {
    static std::mutex mu;
    static hipStream_t fs[64] = {};
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (dev != cur) (void)hipSetDevice(dev);
    hipStream_t s = nullptr;
    {
        std::lock_guard<std::mutex> g(mu);
        if (dev >= 0 && dev < 64) {
            if (!fs[dev] && hipStreamCreateWithFlags(&fs[dev], hipStreamNonBlocking) != hipSuccess) fs[dev] = nullptr;
            s = fs[dev];
        }
    }
    for (void* p : ptrs)
        if (p) (void)(s ? hipFreeAsync(p, s) : hipFree(p));
    if (s) (void)hipStreamSynchronize(s);
    (void)hipGetLastError();
    if (dev != cur) (void)hipSetDevice(cur);
}

struct mphf {
    int device = 0;
    uint64_t n = 0;
    double gamma = 0;
    uint64_t seed = 0;
    mphf_opts opts{};
    uint32_t num_levels = 0;
    uint64_t level_n[MPHF_MAX_LEVELS] = {};
    uint64_t level_m[MPHF_MAX_LEVELS] = {};
    uint64_t level_weight[MPHF_MAX_LEVELS] = {};
    uint64_t level_offset[MPHF_MAX_LEVELS] = {};
    uint64_t level_seed[MPHF_MAX_LEVELS] = {};
    uint32_t level_path[MPHF_MAX_LEVELS] = {};   // MPHF_PATH_* of each level
    uint32_t bucket_bits = 0;
    uint64_t total_bits = 0;
    uint64_t total_words = 0;
    uint64_t* words = nullptr;
    uint64_t* rank = nullptr;
    uint64_t nrank = 0;
    uint32_t rank_shift = 9;
    uint64_t* fb_keys = nullptr;
    uint64_t nfb = 0;
    uint32_t* sec = nullptr;        // lookup layout: 64-byte sectors of (rank counter, 480 bits of A)
    uint64_t* super = nullptr;
    void* layout = nullptr;         // the one allocation holding sec, super and rank
    uint64_t nsec = 0;
    DevLevel* dlev = nullptr;
    uint64_t* coll_all = nullptr;   // C of every level, laid out like A (keep_collisions)
    uint64_t peak_bytes = 0;
    mutable UseTracker uses;
};

namespace {

thread_local std::string g_err;

// Optional host-side phase trace of the build (MPHF_TRACE=1 in the environment): wall time of
// each phase after a stream synchronisation, printed to stderr.
struct Trace {
    bool on;
    hipStream_t s;
    std::chrono::steady_clock::time_point t0, last;
    explicit Trace(hipStream_t st) : s(st) {
        const char* e = std::getenv("MPHF_TRACE");
        on = e && *e && *e != '0';
        t0 = last = std::chrono::steady_clock::now();
    }
    void mark(const char* what, long a = -1) {
        if (!on) return;
        (void)hipStreamSynchronize(s);
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[mphf] %-22s %9.3f ms (total %9.3f)  %ld\n", what,
                     std::chrono::duration<double, std::milli>(now - last).count(),
                     std::chrono::duration<double, std::milli>(now - t0).count(), a);
        last = now;
    }
};

mphf_status fail(mphf_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

mphf_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? MPHF_E_NOMEM : MPHF_E_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                        \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

bool is_device_ptr(const void* p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.isManaged;
}

// SplitMix64 stream (Steele, Lea and Flood 2014): s_d is its output d, the state starting at
// the build seed.
void level_seeds(uint64_t seed, uint32_t count, uint64_t* out) {
    uint64_t s = seed;
    for (uint32_t d = 0; d < count; ++d) {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        out[d] = z ^ (z >> 31);
    }
}

// |A_d| = gamma |F_d| (Section 2.2), rounded up; the product is taken in IEEE double.
uint64_t level_size(double gamma, uint64_t n) { return (uint64_t)std::ceil(gamma * (double)n); }

// Device memory comes from the stream-ordered allocator (hipMallocAsync) with the device's
// default pool set to keep freed memory, so repeated builds reuse their workspace instead of
// paying hipMalloc each time.
void configure_pool(int dev) {
    static std::mutex mu;
    static bool done[64] = {};
    std::lock_guard<std::mutex> g(mu);
    if (dev < 0 || dev >= 64 || done[dev]) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t keep = ~0ull;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    done[dev] = true;
}

// Temporaries of the partitioned levels (a few times the key set) and the pinned readback buffer,
// kept per device between builds so that repeated builds reuse them.  A build takes its device's
// workspace if no other build holds it, else it allocates private temporaries; a build with a
// memory budget always uses private temporaries so that the budget counts them.
struct WsBufs {
    uint64_t *Z = nullptr, *X = nullptr, *Y[2] = {nullptr, nullptr}, *preZ = nullptr,
             *preY[2] = {nullptr, nullptr}, *tiles = nullptr, *host = nullptr;
    uint32_t *cntZ = nullptr, *cntX = nullptr, *surv[2] = {nullptr, nullptr};
    uint64_t capZ = 0, capX = 0, capCntZ = 0, capCntX = 0, capTiles = 0, capPreZ = 0;
    uint64_t capY[2] = {0, 0}, capSurv[2] = {0, 0}, capPreY[2] = {0, 0};
};

struct Workspace {
    std::mutex mu;
    WsBufs b;
    void release() {
        void* bufs[] = {b.Z, b.X, b.Y[0], b.Y[1], b.preZ, b.preY[0], b.preY[1], b.tiles, b.cntZ,
                        b.cntX, b.surv[0], b.surv[1]};
        for (void* q : bufs)
            if (q) (void)hipFree(q);
        if (b.host) (void)hipHostFree(b.host);
        b = WsBufs();
    }
};
Workspace g_ws[64];

// The batched build's temporaries (slot 0: per-set queue and prefixes; slot 1: survivors, unpacked
// bits and per-set counts), kept per device like the single build's workspace.
struct BatchWorkspace {
    std::mutex mu;
    void* buf[2] = {nullptr, nullptr};
    uint64_t cap[2] = {0, 0};
    void release() {
        for (int i = 0; i < 2; ++i) {
            if (buf[i]) (void)hipFree(buf[i]);
            buf[i] = nullptr;
            cap[i] = 0;
        }
    }
};
BatchWorkspace g_bws[64];

// Device memory of one build: every buffer is released when the builder goes out of scope
// unless it was handed to the finished function.  Tracks the bytes held against mem_budget.
class Arena {
  public:
    Arena(uint64_t budget, hipStream_t s) : budget_(budget), s_(s) {}
    ~Arena() {
        for (auto& b : bufs_)
            if (b.first) (void)hipFreeAsync(b.first, s_);
    }
    template <typename T>
    mphf_status alloc(T** p, uint64_t count, const char* what) {
        *p = nullptr;
        const uint64_t bytes = count * sizeof(T);
        if (!bytes) return MPHF_OK;
        if (budget_ && held_ + bytes > budget_)
            return fail(MPHF_E_NOMEM, std::string(what) + ": mem_budget exceeded");
        void* q = nullptr;
        hipError_t e = hipMallocAsync(&q, bytes, s_);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return hip_fail(e, what);
        }
        bufs_.push_back({q, bytes});
        held_ += bytes;
        if (held_ > peak_) peak_ = held_;
        *p = (T*)q;
        return MPHF_OK;
    }
    void release(void* p) {   // free (in stream order)
        if (!p) return;
        for (auto& b : bufs_)
            if (b.first == p) {
                (void)hipFreeAsync(p, s_);
                held_ -= b.second;
                b.first = nullptr;
                return;
            }
    }
    void keep(void* p) {      // hand over to the finished function
        for (auto& b : bufs_)
            if (b.first == p) b.first = nullptr;
    }
    uint64_t peak() const { return peak_; }

  private:
    uint64_t budget_;
    hipStream_t s_;
    uint64_t held_ = 0, peak_ = 0;
    std::vector<std::pair<void*, uint64_t>> bufs_;
};

void free_handle(mphf* h) {
    if (!h) return;
    // lookups may still be in flight on the streams that used h: wait for those, then free
    h->uses.wait_all();
    free_on_device(h->device, {h->words, h->fb_keys, h->dlev, h->coll_all, h->layout});
    delete h;
}

mphf_status check_opts(const mphf_opts& o) {
    if (o.max_levels < 1 || o.max_levels > MPHF_MAX_LEVELS)
        return fail(MPHF_E_INVALID, "max_levels must be in 1..64");
    if (o.rank_sample != 512 && o.rank_sample != 1024)
        return fail(MPHF_E_INVALID, "rank_sample must be 512 or 1024");
    if (o.flags & ~(uint32_t)MPHF_FLAG_ATOMIC_LEVELS) return fail(MPHF_E_INVALID, "unknown flags");
    if (o.bucket_bits && (o.bucket_bits < 6 || o.bucket_bits > 16))
        return fail(MPHF_E_INVALID, "bucket_bits must be 0 or 6..16");
    return MPHF_OK;
}

// A key set on the device: dense (one segment of stride 0) or partitioned into segments
// s = 0..nseg-1 holding keys base[s*stride ..], with exclusive prefix pre[0..nseg] of their sizes.
struct KeySet {
    const uint64_t* base = nullptr;
    uint64_t stride = 0;
    const uint64_t* pre = nullptr;
    uint32_t nseg = 0;
    uint64_t n = 0;
    uint64_t gen[2] = {0, 0};   // with base == nullptr: one segment of generated keys (seed, first index)
};

// Capacity of a region expected to receive e keys: 8 standard deviations and a margin above e,
// rounded up to whole 16-key (128-byte) lines, so that every region starts on a line.
uint64_t region_cap(double e) { return ((uint64_t)std::ceil(e + 8.0 * std::sqrt(e) + 64.0) + 15) & ~15ull; }

// The first 128-byte boundary at or after p (a buffer allocated 16 words longer).
uint64_t* line_align(uint64_t* p) { return (uint64_t*)(((uintptr_t)p + 127) & ~(uintptr_t)127); }

// Workgroups of a partition pass: two fit on a compute unit (LDS), 256 compute units.
constexpr uint64_t PART_WGS = 512;

// Workgroups per coarse bin in the second partition pass over n keys (the bucket pass then reads
// that many regions per bucket).  The C * K workgroups run in ceil(C * K / PART_WGS) rounds, each
// doing 1 / (C * K) of the keys, so K minimizes rounds / (C * K): C = 188 gives K = 8 (1504
// workgroups in 3 rounds) rather than K = 2 (376 workgroups, a quarter of the slots idle).  A
// workgroup keeps at least 16 tiles of work while there are more workgroups than slots.
uint64_t slots_per_group(uint64_t C, uint64_t n) {
    const uint64_t cap = std::max<uint64_t>(PART_WGS, n / 65536) / C;
    const uint64_t kmax = std::max<uint64_t>(1, std::min<uint64_t>(16, cap));
    uint64_t best = 1;
    double best_t = 1e300;
    for (uint64_t K = 1; K <= kmax; ++K) {
        const double t = (double)((C * K + PART_WGS - 1) / PART_WGS) / (double)(C * K);
        if (t < best_t * 0.999) {
            best_t = t;
            best = K;
        }
    }
    return best;
}

uint32_t ceil_log2(uint64_t x) {
    uint32_t l = 0;
    while (l < 64 && (1ull << l) < x) ++l;
    return l;
}

class Builder {
  public:
    Builder(mphf* h, const mphf_opts& o, hipStream_t s)
        : h_(h), o_(o), s_(s), ar_(o.mem_budget, s), tr_(s) {}
    ~Builder() {
        if (host_ && !cached_) (void)hipHostFree(host_);
    }

    mphf_status run(const uint64_t* keys, uint64_t n, double gamma) {
        mphf_status st;
        defer_ = true;   // the first level's radix passes are queued before the structure is allocated
        if ((st = setup(n, gamma)) != MPHF_OK) return st;
        return levels_and_finish(keys, n, 0, 0);
    }

    // Streamed levels over a generated key stream, or over a key set in host memory (host_keys set),
    // while the survivors exceed `budget` keys (no F_d is stored), then the survivors are collected
    // and the in-memory levels continue.
    void use_host_keys(const uint64_t* keys) { host_keys_ = keys; }

    mphf_status run_stream(uint64_t kseed, uint64_t kstart, uint64_t n, double gamma, uint64_t budget) {
        mphf_status st;
        if ((st = setup(n, gamma)) != MPHF_OK) return st;
        const uint32_t D = o_.max_levels;
        DevLevel* lev = nullptr;
        if ((st = ar_.alloc(&lev, MPHF_MAX_LEVELS, "stream levels")) != MPHF_OK) return st;
        unsigned long long* counters = (unsigned long long*)dev_;
        HIP_TRY(launch_zero(dev_, 256, s_), "zero counters");
        uint64_t* W = nullptr;
        uint32_t d = 0;
        uint64_t off = 0, nd = n;
        uint64_t* chunk = nullptr;   // the keys of one chunk of the stream
        uint64_t* pre0 = nullptr;
        bool walkable = true;        // every finished level has a bucket geometry (no atomic fill)
        while (nd > 0 && d < D && nd > budget) {
            const uint64_t m = level_size(gamma_, nd);
            const uint64_t wd = (m + 63) / 64;
            if (!W && (st = ar_.alloc(&W, 2 * wd + 2, "stream W")) != MPHF_OK) return st;
            const LevelHash L = make_level_hash(seeds_.s[d], m, off);
            if ((st = ensure_words(off / 64 + wd + 1)) != MPHF_OK) return st;
            HIP_TRY(launch_zero(W, 2 * wd, s_), "zero W");
            // Buckets of 2^pb positions, at most 2^18 of them, so that each chunk takes two radix
            // passes at most; a level beyond 2^36 positions, or the atomic-only option, takes
            // global atomics over the whole stream instead.
            const uint32_t pb = stream_bucket_bits(m);
            bool accumulated = false;
            if (!(o_.flags & MPHF_FLAG_ATOMIC_LEVELS) && pb && walkable) {
                if ((st = accumulate_stream_level(kseed, kstart, n, d, L, m, pb, budget, W, wd, &chunk, &pre0,
                                                  &accumulated)) != MPHF_OK)
                    return st;
            }
            if (!accumulated) {
                walkable = false;   // the later scans walk by random reads too
                HIP_TRY(launch_zero(W, 2 * wd, s_), "zero W");
                if (!host_keys_) {
                    HIP_TRY(launch_stream_fill(kseed, kstart, nullptr, n, lev, d, words_, W, L, s_), "stream fill");
                } else {   // the stored keys, chunk by chunk
                    const uint64_t ch = chunk_keys(n, budget);
                    if (!chunk && (st = ar_.alloc(&chunk, ch, "stream chunk")) != MPHF_OK) return st;
                    for (uint64_t c0 = 0; c0 < n; c0 += ch) {
                        const uint64_t c = std::min<uint64_t>(ch, n - c0);
                        if ((st = load_chunk(kseed, kstart, c0, c, chunk)) != MPHF_OK) return st;
                        HIP_TRY(launch_stream_fill(0, 0, chunk, c, lev, d, words_, W, L, s_), "stream fill");
                    }
                }
            }
            HIP_TRY(launch_finalize(W, wd, words_ + off / 64, coll_ ? coll_ + off / 64 : nullptr, counters + d, s_),
                    "finalize");
            if ((st = read_back(counters + d, 8)) != MPHF_OK) return st;
            const uint64_t weight = host_[0];
            if (weight > nd) return fail(MPHF_E_DEVICE, "level weight exceeds the level's keys");
            record(d, nd, m, weight, off, accumulated ? MPHF_PATH_STREAMED : MPHF_PATH_STREAMED_ATOMIC);
            // the level joins the walk of the next scans
            DevLevel* hl = (DevLevel*)(host_ + 64);
            *hl = DevLevel{L.seed, L.m, L.magic, L.bit_off, L.sh1, L.sh2};
            HIP_TRY(hipMemcpyAsync(lev + d, hl, sizeof(DevLevel), hipMemcpyHostToDevice, s_), "copy level");
            HIP_TRY(hipStreamSynchronize(s_), "level sync");
            off += 64 * wd;
            nd -= weight;
            ++d;
            tr_.mark("streamed level", (long)(d - 1));
        }
        if (W) ar_.release(W);
        if (!nd) {
            if (chunk) ar_.release(chunk);
            h_->total_words = h_->total_bits / 64;
            return finish();
        }
        // the survivors of the streamed levels, in any order (the levels do not depend on it)
        uint64_t* dense = nullptr;
        if ((st = ar_.alloc(&dense, nd, "streamed survivors")) != MPHF_OK) return st;
        tr_.mark("collect alloc", (long)nd);
        bool collected = false;
        if (pre0 && walkable && !(o_.flags & MPHF_FLAG_ATOMIC_LEVELS)) {   // (pre0: the chunked scans ran)
            // chunk by chunk, the levels walked by bucket
            unsigned long long* ovf = (unsigned long long*)(dev_ + 129);
            HIP_TRY(launch_zero(dev_ + 129, 1, s_), "zero overflow");
            const uint64_t ch = chunk_keys(n, budget);
            uint64_t got = 0;
            bool fits = true;
            for (uint64_t c0 = 0; c0 < n && fits; c0 += ch) {
                const uint64_t c = std::min<uint64_t>(ch, n - c0);
                KeySet in;
                if ((st = stream_unplaced(kseed, kstart, c0, c, d, chunk, pre0, &in, ovf)) != MPHF_OK) return st;
                if (got + in.n > nd) {
                    fits = false;
                    break;
                }
                if (in.n && !in.base) return fail(MPHF_E_DEVICE, "collect before any streamed level");
                if (in.n) HIP_TRY(launch_gather(in.base, in.stride, in.pre, in.nseg, in.n, dense + got, s_), "gather");
                got += in.n;
            }
            if ((st = read_back(dev_ + 129, 8)) != MPHF_OK) return st;
            collected = fits && host_[0] == 0 && got == nd;
        }
        if (!collected) {
            HIP_TRY(launch_zero(dev_ + 200, 1, s_), "zero count");
            if (!host_keys_) {
                HIP_TRY(launch_stream_collect(kseed, kstart, nullptr, n, lev, d, words_, dense, nd, counters + 200, s_),
                        "collect");
            } else {   // the stored keys, chunk by chunk, appended at the running count
                const uint64_t ch = chunk_keys(n, budget);
                if (!chunk && (st = ar_.alloc(&chunk, ch, "stream chunk")) != MPHF_OK) return st;
                for (uint64_t c0 = 0; c0 < n; c0 += ch) {
                    const uint64_t c = std::min<uint64_t>(ch, n - c0);
                    if ((st = load_chunk(kseed, kstart, c0, c, chunk)) != MPHF_OK) return st;
                    HIP_TRY(launch_stream_collect(0, 0, chunk, c, lev, d, words_, dense, nd, counters + 200, s_),
                            "collect");
                }
            }
            if ((st = read_back(counters + 200, 8)) != MPHF_OK) return st;
            if (host_[0] != nd) return fail(MPHF_E_DEVICE, "collected survivors differ from the level counts");
        }
        if (chunk) ar_.release(chunk);
        tr_.mark("collect", (long)nd);
        return levels_and_finish(dense, nd, d, off);
    }

    // Keys per chunk of a streamed scan: the survivor budget, at least 2^20, at most the set.
    static uint64_t chunk_keys(uint64_t n, uint64_t budget) {
        return std::min<uint64_t>(n, std::max<uint64_t>(budget, 1ull << 20));
    }

    // Keys c0 .. c0 + c - 1 of the key source into the device array chunk: generated, or copied from
    // the host array (over PCIe, in stream order).
    mphf_status load_chunk(uint64_t kseed, uint64_t kstart, uint64_t c0, uint64_t c, uint64_t* chunk) {
        if (host_keys_) {
            HIP_TRY(hipMemcpyAsync(chunk, host_keys_ + c0, 8 * c, hipMemcpyHostToDevice, s_), "chunk copy");
        } else {
            HIP_TRY(launch_stream_keys(kseed, kstart + c0, c, chunk, s_), "chunk keys");
        }
        return MPHF_OK;
    }

    // Bucket bits for a level of m positions: the bucket geometry's, raised until two radix passes
    // reach every bucket (at most 2^18 buckets); 0 if no bucket of at most 2^18 positions does.
    uint32_t stream_bucket_bits(uint64_t m) const {
        uint32_t pb = geo_.pbits ? geo_.pbits : 15;
        while (pb < 18 && ceil_log2((m + (1ull << pb) - 1) >> pb) > 18) ++pb;
        return ceil_log2((m + (1ull << pb) - 1) >> pb) <= 18 ? pb : 0;
    }

    // The keys of stream chunk [c0, c0 + c) that no finished level 0..d-1 placed (the walk of
    // Algorithm 3 over those levels), found by bucket: the chunk is copied into `chunk` (a stored key
    // set) or generated by the first radix pass (a generated stream), and for
    // each finished level j its keys are partitioned by bucket of level j and tested against A_j
    // in LDS (k_bucket_test).  *out gets them as the regions of ws_->Y[0] with prefix ws_->preY[0].
    // Region overflows (adversarial streams only) are flagged in *ovf.
    mphf_status stream_unplaced(uint64_t kseed, uint64_t kstart, uint64_t c0, uint64_t c, uint32_t d,
                                uint64_t* chunk, uint64_t* pre0, KeySet* out, unsigned long long* ovf) {
        mphf_status st;
        KeySet cur;
        if (host_keys_) {
            if ((st = load_chunk(kseed, kstart, c0, c, chunk)) != MPHF_OK) return st;
            cur.base = chunk;
        } else {   // generated keys: the first radix pass makes them itself
            cur.gen[0] = kseed;
            cur.gen[1] = kstart + c0;
        }
        HIP_TRY(launch_pair(pre0, 0, c, s_), "chunk prefix");
        cur.pre = pre0;
        cur.nseg = 1;
        cur.n = c;
        for (uint32_t j = 0; j < d && cur.n > 0; ++j) {
            const uint64_t m = h_->level_m[j];
            const uint32_t pb = stream_bucket_bits(m);
            if (!pb || pb < 6) return fail(MPHF_E_INVALID, "no bucket geometry for a streamed level");
            const LevelHash L = make_level_hash(seeds_.s[j], m, h_->level_offset[j]);
            uint64_t* X = nullptr;
            uint64_t xcap = 0;
            uint32_t S = 0;
            bool packed = false;
            if ((st = partition_buckets(cur, L, m, pb, &X, &xcap, &S, &packed, ovf)) != MPHF_OK) return st;
            const uint64_t B = (m + (1ull << pb) - 1) >> pb;
            const uint64_t ycap = (uint64_t)S * xcap;   // a bucket keeps at most its records
            if ((st = ensure(&ws_->Y[0], &ws_->capY[0], B * ycap, "unplaced keys")) != MPHF_OK) return st;
            if ((st = ensure(&ws_->surv[0], &ws_->capSurv[0], B + 1, "unplaced counts")) != MPHF_OK) return st;
            if ((st = ensure(&ws_->preY[0], &ws_->capPreY[0], B + 1, "unplaced prefix")) != MPHF_OK) return st;
            HIP_TRY(launch_bucket_test(X, xcap, ws_->cntX, S, B, L, pb, packed, words_, h_->level_offset[j],
                                       (m + 63) / 64, ws_->Y[0], ycap, ws_->surv[0], ovf, s_),
                    "bucket test");
            HIP_TRY(launch_zero32(ws_->surv[0] + B, 1, s_), "zero count tail");
            if ((st = prefix(ws_->surv[0], B, ws_->preY[0])) != MPHF_OK) return st;
            if ((st = read_back(ws_->preY[0] + B, 8)) != MPHF_OK) return st;
            cur.base = ws_->Y[0];
            cur.stride = ycap;
            cur.pre = ws_->preY[0];
            cur.nseg = (uint32_t)B;
            cur.n = host_[0];
            if (cur.n > c) return fail(MPHF_E_DEVICE, "more unplaced keys than the chunk holds");
        }
        *out = cur;
        return MPHF_OK;
    }

    // Level d of a generated stream added to W chunk by chunk: the unplaced keys of up to `budget`
    // stream keys at a time are collected, partitioned by bucket of 2^pb positions and accumulated
    // (no global atomics).  *done = false if a region overflowed (adversarial streams only): W is
    // then partial and the caller fills the level with global atomics.
    mphf_status accumulate_stream_level(uint64_t kseed, uint64_t kstart, uint64_t n, uint32_t d,
                                        const LevelHash& L, uint64_t m, uint32_t pb, uint64_t budget, uint64_t* W,
                                        uint64_t wd, uint64_t** chunk, uint64_t** pre0, bool* done) {
        mphf_status st;
        *done = false;
        const uint64_t ch = chunk_keys(n, budget);
        // (a generated chunk is never stored: its first radix pass makes the keys)
        if (host_keys_ && !*chunk && (st = ar_.alloc(chunk, ch, "stream chunk")) != MPHF_OK) return st;
        if (!*pre0 && (st = ar_.alloc(pre0, 2, "chunk prefix")) != MPHF_OK) return st;
        HIP_TRY(accumulate_setup(), "accumulate setup");
        HIP_TRY(bucket_test_setup(), "bucket test setup");
        unsigned long long* ovf = (unsigned long long*)(dev_ + 129);
        HIP_TRY(launch_zero(dev_ + 129, 1, s_), "zero overflow");
        const uint64_t B = (m + (1ull << pb) - 1) >> pb;
        for (uint64_t c0 = 0; c0 < n; c0 += ch) {
            const uint64_t c = std::min<uint64_t>(ch, n - c0);
            KeySet in;
            if ((st = stream_unplaced(kseed, kstart, c0, c, d, *chunk, *pre0, &in, ovf)) != MPHF_OK) return st;
            const uint64_t nc = in.n;
            if (!nc) continue;
            uint64_t* X = nullptr;
            uint64_t xcap = 0;
            uint32_t S = 0;
            bool packed = false;
            if ((st = partition_buckets(in, L, m, pb, &X, &xcap, &S, &packed, ovf)) != MPHF_OK) return st;
            HIP_TRY(launch_accumulate(X, xcap, ws_->cntX, S, B, L, pb, packed, W, 2 * wd, ovf, s_), "accumulate");
            tr_.mark("accumulated chunk", (long)nc);
        }
        if ((st = read_back(dev_ + 129, 8)) != MPHF_OK) return st;
        *done = host_[0] == 0;
        return MPHF_OK;
    }

    // Sizes, seeds, counters and the concatenated A reserved for n keys.
    mphf_status setup(uint64_t n, double gamma) {
        mphf_status st;
        gamma_ = gamma;
        geo_ = bucket_geometry(gamma, o_.bucket_bits);
        if (o_.bucket_bits && !geo_.pbits)
            return fail(MPHF_E_INVALID, "bucket_bits: the keys of such a bucket do not fit one workgroup at this gamma");
        h_->bucket_bits = geo_.pbits;
        acquire_workspace();
        level_seeds(h_->seed, o_.max_levels, seeds_.s);
        if (cached_ && ws_->host) {
            host_ = ws_->host;
        } else {
            HIP_TRY(hipHostMalloc((void**)&host_, 4096, hipHostMallocCoherent), "hipHostMalloc");
            if (cached_) ws_->host = host_;
        }
        HIP_TRY(hipHostGetDevicePointer((void**)&host_dev_, host_, 0), "hipHostGetDevicePointer");
        // counters, flags and the tail's level records in one small allocation
        static_assert(sizeof(TailLevel) * MPHF_MAX_LEVELS <= 8 * 256, "tail records after the counters");
        if ((st = ar_.alloc(&dev_, 512 + 256, "counters")) != MPHF_OK) return st;
        HIP_TRY(launch_zero(dev_, 512 + 256, s_), "zero counters");
        tail_rec_ = (TailLevel*)(dev_ + 512);
        // The concatenated A: reserve the expected gamma e^{1/gamma} N bits (Section 2.3) plus
        // slack; grown by copying in the rare case the levels need more.
        {
            const double expect = gamma * std::exp(1.0 / gamma) * (double)n;
            const uint64_t w0 = (level_size(gamma, n) + 63) / 64;
            uint64_t cap = (uint64_t)(expect * 1.02 / 64.0) + 4 * (uint64_t)o_.max_levels + 1024;
            if (cap < w0 + 1) cap = w0 + 1;
            reserve_words_ = cap;
            if (!defer_ && (st = reserve()) != MPHF_OK) return st;
        }
        tr_.mark("setup");
        return MPHF_OK;
    }

    // Levels d.. of the n keys at `keys` (the whole set when d = 0), starting at bit `off` of A,
    // then the fallback table, rank table, lookup layout and level table.
    mphf_status levels_and_finish(const uint64_t* keys, uint64_t n, uint32_t d, uint64_t off) {
        mphf_status st;
        const bool atomic_only = o_.flags & MPHF_FLAG_ATOMIC_LEVELS;
        KeySet cur;
        uint64_t* pre0 = dev_ + 400;   // the one-segment prefix {0, n} of the input
        HIP_TRY(launch_zero(dev_ + 129, 1, s_), "zero overflow");   // the partitioned levels' flag
        HIP_TRY(launch_pair(pre0, 0, n, s_), "prefix");
        cur.base = keys;
        cur.pre = pre0;
        cur.nseg = 1;
        cur.n = n;
        const uint32_t D = o_.max_levels;
        const double gamma = gamma_;
        const uint32_t tk = tail_capacity(gamma);
        const BucketGeometry geo = geo_;
        bool fallback = atomic_only || geo.pbits == 0;
        // Level d is queued (exactly, or ahead of its key count and then accepted) before the host
        // waits for level d - 1's report, so that the device never waits for the host between levels.
        SpecLevel* const spec = (SpecLevel*)(dev_ + 144);
        QueuedLevel q;
        bool have = false;   // q holds level d, queued
        while (!fallback && cur.n > 0 && d < D) {
            if (!have) {
                if (cur.n <= tk) {
                    if ((st = tail(cur, d, off, tk)) != MPHF_OK) return st;
                    tr_.mark("tail", (long)h_->num_levels);
                    cur.n = 0;   // the tail built every remaining level and wrote the leftovers
                    d = h_->num_levels;
                    break;
                }
                bool queued = false;
                if ((st = queue_level(cur, d, off, geo, SpecArgs(), 0, 0, &q, &queued)) != MPHF_OK) return st;
                if (!queued) {
                    fallback = true;
                    break;
                }
            }
            const uint64_t m_d = level_size(gamma, cur.n);
            const uint64_t off_next = off + 64 * ((m_d + 63) / 64);
            // level d + 1 queued ahead, when its key count is sure to stay above the tail's
            QueuedLevel q2;
            bool ahead = false;
            uint64_t lo = 0, hi = 0;
            if (ahead_ != AHEAD_OFF && d + 1 < D) {
                survivor_bounds(cur.n, m_d, &lo, &hi);
                if (ahead_ == AHEAD_REJECT) hi = lo;   // (a test mode: nearly every level queued ahead is redone)
                if (lo > tk) {
                    KeySet nin;
                    nin.base = ws_->Y[q.yp];
                    nin.stride = geo.kcap;
                    nin.pre = ws_->preY[q.yp];
                    nin.nseg = (uint32_t)((m_d + (1ull << geo.pbits) - 1) >> geo.pbits);
                    nin.n = hi;
                    SpecArgs sa;
                    sa.mode = 1;
                    sa.total = ws_->preY[q.yp] + q.B;
                    sa.prev_flag = (const unsigned long long*)(dev_ + 140);
                    sa.gamma = gamma;
                    sa.seed = seeds_.s[d + 1];
                    sa.bit_off = off_next;
                    sa.lo = lo;
                    sa.hi = hi;
                    sa.out = spec;
                    if ((st = queue_level(nin, d + 1, off_next, geo, sa, lo, hi, &q2, &ahead)) != MPHF_OK) return st;
                }
            }
            KeySet next;
            bool ok = false;
            if ((st = finish_level(q, geo, &next, &ok)) != MPHF_OK) return st;
            tr_.mark("partitioned level", (long)d);
            if (!ok) {   // (a level queued ahead saw the flag and did nothing)
                fallback = true;
                break;
            }
            off = off_next;
            ++d;
            cur = next;
            have = ahead && cur.n >= lo && cur.n <= hi;   // else it did nothing and is queued again
            if (have) {
                q = q2;
                q.n = cur.n;
            }
        }
        if (cur.n > 0) {
            // dense copy of what is left: either the input of the global-atomic levels, or the
            // leftovers after D levels
            uint64_t* dense = nullptr;
            if (cur.nseg == 1 && cur.stride == 0) {
                dense = const_cast<uint64_t*>(cur.base);
            } else {
                if ((st = ar_.alloc(&dense, cur.n, "dense keys")) != MPHF_OK) return st;
                HIP_TRY(launch_gather(cur.base, cur.stride, cur.pre, cur.nseg, cur.n, dense, s_), "gather");
            }
            if (d < D) {
                if ((st = atomic_levels(dense, cur.n, d, off)) != MPHF_OK) return st;
            } else {
                left_ = dense;
                nleft_ = cur.n;
                h_->total_bits = off;
            }
        } else if (h_->num_levels == d) {
            h_->total_bits = std::max(h_->total_bits, off);
        }
        h_->total_words = h_->total_bits / 64;
        tr_.mark("levels done");
        return finish();
    }

    mphf_status finish() {
        mphf_status st;
        if ((st = reserve()) != MPHF_OK) return st;
        if ((st = fallback_table()) != MPHF_OK) return st;
        tr_.mark("fallback table", (long)nleft_);
        if ((st = rank_and_lookup_layout()) != MPHF_OK) return st;
        tr_.mark("rank table and lookup layout");
        if ((st = level_table()) != MPHF_OK) return st;
        tr_.mark("level table");
        h_->words = words_;
        ar_.keep(words_);
        if (coll_) {
            h_->coll_all = coll_;
            ar_.keep(coll_);
        }
        HIP_TRY(hipStreamSynchronize(s_), "final sync");
        h_->peak_bytes = ar_.peak();
        tr_.mark("done");
        return MPHF_OK;
    }

  private:
    mphf* h_;
    mphf_opts o_;
    hipStream_t s_;
    Arena ar_;
    Trace tr_;
    double gamma_ = 0;
    BucketGeometry geo_{};
    SeedTable seeds_{};
    uint64_t* host_ = nullptr;
    uint64_t* host_dev_ = nullptr;   // host_ as the device sees it (pinned, device-writable)
    uint64_t* dev_ = nullptr;        // [0..63] weights, [64..127] survivor counts, [128] dup flag,
                                     // [129] overflow flag, [130..132] tail summary, [200] streamed
                                     // survivors, [300] keys collected from a stream chunk, [400..401]
                                     // the input's prefix, [512..767] the tail's level records
    TailLevel* tail_rec_ = nullptr;
    uint64_t* words_ = nullptr;
    uint64_t* coll_ = nullptr;
    uint64_t cap_words_ = 0;
    uint64_t* left_ = nullptr;
    uint64_t nleft_ = 0;
    // partition temporaries: the device's cached workspace, or a private one
    WsBufs priv_;
    WsBufs* ws_ = &priv_;
    bool cached_ = false;
    const uint64_t* host_keys_ = nullptr;   // streaming build over a stored key set in host memory
    std::unique_lock<std::mutex> lock_;

    // The structure's memory: A (reserve_words_ words, the expected size plus slack) and, sized for
    // that many bits, the lookup sectors, superblocks and rank table with their temporaries.  Its
    // host-side cost (large stream-ordered allocations) is paid once the first level's passes are
    // queued, so that it overlaps them.
    // Levels queued ahead of their key count: on, off, or (a test mode) with bounds that nearly
    // every level misses, so that the redo runs; from MPHF_LEVELS_AHEAD (unset or 1, 0, "reject").
    enum { AHEAD_ON, AHEAD_OFF, AHEAD_REJECT };
    int ahead_ = ahead_mode();
    static int ahead_mode() {
        const char* e = std::getenv("MPHF_LEVELS_AHEAD");
        if (!e || !*e || std::strcmp(e, "1") == 0) return AHEAD_ON;
        if (std::strcmp(e, "reject") == 0) return AHEAD_REJECT;
        return AHEAD_OFF;
    }

    bool defer_ = false, reserved_ = false;
    uint64_t reserve_words_ = 0;
    uint8_t *pre_keep_ = nullptr, *pre_tmp_ = nullptr;
    uint64_t pre_keep_bytes_ = 0, pre_tmp_bytes_ = 0;

    static uint64_t up256(uint64_t b) { return (b + 255) & ~uint64_t(255); }
    uint64_t layout_keep_bytes(uint64_t bits) const {
        const uint64_t ns = sector_count(bits), nr = (bits + o_.rank_sample - 1) / o_.rank_sample;
        return ns ? up256(ns * 64) + up256(super_count(ns) * 8) + up256(nr * 8) : 0;
    }
    static uint64_t layout_tmp_bytes(uint64_t bits) {
        const uint64_t ng = rank_sector_groups(bits);
        return ng ? up256(ng * 4) + up256(ng * 8) + up256(scan_tmp_tiles(ng) * 8) : 0;
    }

    mphf_status reserve() {
        if (reserved_) return MPHF_OK;
        reserved_ = true;
        mphf_status st;
        if ((st = ensure_words(reserve_words_)) != MPHF_OK) return st;
        const uint64_t bits = 64 * cap_words_;
        pre_keep_bytes_ = layout_keep_bytes(bits);
        pre_tmp_bytes_ = layout_tmp_bytes(bits);
        if ((st = ar_.alloc(&pre_keep_, pre_keep_bytes_, "lookup sectors and rank table")) != MPHF_OK) return st;
        if ((st = ar_.alloc(&pre_tmp_, pre_tmp_bytes_, "rank and sector temporaries")) != MPHF_OK) return st;
        return MPHF_OK;
    }

    // Report sequence numbers: distinct per report of this process, so that a value left in the
    // (cached, reused) pinned buffer by an earlier build is never taken for a new one.
    static uint64_t next_seq() {
        static std::atomic<uint64_t> c{1};
        return c.fetch_add(1);
    }

    // Waits until the report kernel has written `seq` (and so its values) into word 2 of its slot,
    // polling the coherent pinned buffer; every 256 polls the stream is queried, so that a failed or
    // finished stream ends the wait.  Report slots (four words each, two of them) sit past every
    // other use of the buffer.
    static constexpr uint32_t REPORT_WORDS = 280;
    static_assert(REPORT_WORDS * 8 >= 8 * 8 + sizeof(TailLevel) * MPHF_MAX_LEVELS && (REPORT_WORDS + 8) * 8 <= 4096,
                  "report slots after the tail's records, inside the pinned buffer");
    mphf_status wait_report(uint64_t seq, uint32_t slot) {
        volatile uint64_t* const flag = host_ + REPORT_WORDS + 4 * slot + 2;
        for (uint32_t i = 1;; ++i) {
            if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == seq) return MPHF_OK;
            if ((i & 255) == 0) {
                const hipError_t e = hipStreamQuery(s_);
                if (e == hipErrorNotReady) continue;
                if (e != hipSuccess) return hip_fail(e, "level report");
                if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == seq) return MPHF_OK;
                return fail(MPHF_E_DEVICE, "level report not written");
            }
        }
    }

    void record(uint32_t d, uint64_t n, uint64_t m, uint64_t weight, uint64_t off, uint32_t path) {
        h_->level_path[d] = path;
        h_->level_n[d] = n;
        h_->level_m[d] = m;
        h_->level_weight[d] = weight;
        h_->level_offset[d] = off;
        h_->level_seed[d] = seeds_.s[d];
        h_->num_levels = d + 1;
        h_->total_bits = off + 64 * ((m + 63) / 64);
    }

    mphf_status ensure_words(uint64_t need) {
        if (need <= cap_words_) return MPHF_OK;
        mphf_status st;
        const uint64_t ncap = cap_words_ ? need * 5 / 4 + 64 : need;
        uint64_t* nw = nullptr;
        if ((st = ar_.alloc(&nw, ncap, "A")) != MPHF_OK) return st;
        if (words_) {   // (every word below total_bits is written by its level; no zeroing needed)
            HIP_TRY(hipMemcpyAsync(nw, words_, cap_words_ * 8, hipMemcpyDeviceToDevice, s_), "grow A");
        }
        uint64_t* nc = nullptr;
        if (o_.keep_collisions) {
            if ((st = ar_.alloc(&nc, ncap, "C")) != MPHF_OK) return st;
            HIP_TRY(launch_zero(nc, ncap, s_), "zero C");
            if (coll_) HIP_TRY(hipMemcpyAsync(nc, coll_, cap_words_ * 8, hipMemcpyDeviceToDevice, s_), "grow C");
        }
        // the old arrays are freed in stream order, after the copies
        ar_.release(words_);
        ar_.release(coll_);
        words_ = nw;
        coll_ = nc;
        cap_words_ = ncap;
        return MPHF_OK;
    }

    template <typename T>
    mphf_status ensure(T** buf, uint64_t* cap, uint64_t need, const char* what) {
        if (need <= *cap) return MPHF_OK;
        if (!cached_) {
            ar_.release(*buf);
            *buf = nullptr;
            *cap = 0;
            mphf_status st = ar_.alloc(buf, need, what);
            if (st == MPHF_OK) *cap = need;
            return st;
        }
        // cached workspace: plain device allocations that outlive the build
        HIP_TRY(hipStreamSynchronize(s_), "workspace sync");
        if (*buf) (void)hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
        const uint64_t grown = need + need / 8;
        hipError_t e = hipMalloc((void**)buf, grown * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *buf = nullptr;
            return hip_fail(e, what);
        }
        *cap = grown;
        return MPHF_OK;
    }

    void acquire_workspace() {
        if (o_.mem_budget) return;   // a budgeted build counts its own temporaries
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
        std::unique_lock<std::mutex> lk(g_ws[dev].mu, std::try_to_lock);
        if (!lk.owns_lock()) return;
        lock_ = std::move(lk);
        ws_ = &g_ws[dev].b;
        cached_ = true;
    }

    mphf_status read_back(const void* dev, uint64_t bytes) {
        HIP_TRY(hipMemcpyAsync(host_, dev, bytes, hipMemcpyDeviceToHost, s_), "read back");
        HIP_TRY(hipStreamSynchronize(s_), "level sync");
        return MPHF_OK;
    }

    // Exclusive prefix of `n` u32 counts (the array has a trailing 0 at index n) into pre[0..n].
    mphf_status prefix(const uint32_t* cnt, uint64_t n, uint64_t* pre, const uint64_t* skip = nullptr) {
        mphf_status st;
        if ((st = ensure(&ws_->tiles, &ws_->capTiles, scan_tmp_tiles(n + 1), "scan tiles")) != MPHF_OK) return st;
        HIP_TRY(launch_exclusive_scan(cnt, pre, n + 1, ws_->tiles, s_, skip), "prefix");
        return MPHF_OK;
    }

    // The keys of `in` radix-partitioned by bucket of 2^pb positions of a level of m positions
    // (ceil(m / 2^pb) <= 2^18 buckets): one pass, or coarse bins then buckets.  *X gets the
    // regions (xcap records each, *S per bucket) with their counts in ws_->cntX; region overflows
    // and configuration errors are flagged in *ovf.  A record is the level hash h (one pass) or,
    // *packed, (q << pb) | (pos mod 2^pb) for h = q m + pos (two passes).
    //
    // For a level queued ahead of its key count (spec.mode != 0), in.n and m are the upper bounds the
    // launches are sized for, m_lo the lower bound of m (region capacities take the larger density),
    // and the kernels take the level hash from the device.
    mphf_status partition_buckets(const KeySet& in, const LevelHash& L, uint64_t m, uint32_t pb, uint64_t** X,
                                  uint64_t* xcap, uint32_t* S, bool* packed, unsigned long long* ovf,
                                  const SpecArgs& spec = SpecArgs(), uint64_t m_lo = 0) {
        mphf_status st;
        const uint64_t n = in.n;
        const uint64_t md = spec.mode ? m_lo : m;   // positions for the key density
        const uint64_t* skip = spec.mode ? &spec.out->skip : nullptr;
        SpecArgs later = spec;   // the second pass reads what the first derived
        if (spec.mode) later.mode = 2;
        const uint64_t P = 1ull << pb;
        const uint64_t B = (m + P - 1) / P;
        const uint32_t lb = ceil_log2(B);
        if (lb > 18) return fail(MPHF_E_INVALID, "more than 2^18 buckets");
        if (B <= 1024) {
            // one pass: every workgroup scatters its share straight into the buckets
            uint64_t W = (n + 8191) / 8192;
            W = std::max<uint64_t>(1, std::min<uint64_t>(W, 256));
            const uint64_t cap = region_cap((double)n / W * (double)P / (double)md);
            if ((st = ensure(&ws_->X, &ws_->capX, B * W * cap + 16, "partition X")) != MPHF_OK) return st;
            *X = line_align(ws_->X);
            if ((st = ensure(&ws_->cntX, &ws_->capCntX, B * W + 1, "counts X")) != MPHF_OK) return st;
            HIP_TRY(launch_partition(B <= 256 ? 8 : 10, false, in.base, in.stride, in.pre, 1, in.nseg,
                                     (uint32_t)W, L, pb, 0, false, 0, B, *X, cap, (uint32_t)W,
                                     ws_->cntX, ovf, n, in.nseg, s_, 0, nullptr, 0, spec, in.base ? nullptr : in.gen),
                    "partition");
            *xcap = cap;
            *S = (uint32_t)W;
            *packed = false;
        } else {
            // two passes: coarse bins of 2^fb buckets, then the buckets of each coarse bin
            const uint32_t fb = lb - 8;
            const uint64_t C = (B + (1ull << fb) - 1) >> fb;
            uint64_t W = (n + 65535) / 65536;
            W = std::max<uint64_t>(1, std::min<uint64_t>(W, PART_WGS));
            const double pc = (double)(P << fb) / (double)md;
            const uint64_t cap1 = region_cap((double)n / W * pc);
            if ((st = ensure(&ws_->Z, &ws_->capZ, C * W * cap1 + 16, "partition Z")) != MPHF_OK) return st;
            uint64_t* const Z = line_align(ws_->Z);
            if ((st = ensure(&ws_->cntZ, &ws_->capCntZ, C * W + 1, "counts Z")) != MPHF_OK) return st;
            // records (q << (pb + fb)) | (pos mod 2^(pb + fb)): B > 1024 buckets make m at least
            // 2^7 times the coarse bin, so q < 2^64 / m fits above it
            HIP_TRY(launch_partition(8, false, in.base, in.stride, in.pre, 1, in.nseg, (uint32_t)W, L, pb,
                                     fb, false, 0, C, Z, cap1, (uint32_t)W, ws_->cntZ, ovf, n, in.nseg, s_,
                                     3, nullptr, pb + fb, spec, in.base ? nullptr : in.gen),
                    "partition 1");
            // (the pass writes the count after the last region as 0, for the scan's total)
            if ((st = ensure(&ws_->preZ, &ws_->capPreZ, C * W + 1, "prefix Z")) != MPHF_OK) return st;
            if ((st = prefix(ws_->cntZ, C * W, ws_->preZ, skip)) != MPHF_OK) return st;
            const uint64_t K = slots_per_group(C, n);
            const double bin_keys = (double)n * pc;
            const double e2 = bin_keys / (double)K / (double)(1ull << fb) * (1.0 + 8.0 / std::sqrt(bin_keys));
            const uint64_t cap2 = region_cap(e2);
            if ((st = ensure(&ws_->X, &ws_->capX, B * K * cap2 + 16, "partition X")) != MPHF_OK) return st;
            *X = line_align(ws_->X);
            if ((st = ensure(&ws_->cntX, &ws_->capCntX, B * K + 1, "counts X")) != MPHF_OK) return st;
            HIP_TRY(launch_partition(fb <= 8 ? 8 : 10, true, Z, cap1, ws_->preZ, (uint32_t)C, (uint32_t)W,
                                     (uint32_t)K, L, pb, 0, true, fb, B, *X, cap2, (uint32_t)K,
                                     ws_->cntX, ovf, n, C * W, s_, 4, nullptr, pb + fb, later),
                    "partition 2");
            *xcap = cap2;
            *S = (uint32_t)K;
            *packed = true;
        }
        return MPHF_OK;
    }

    // A partitioned level on the stream: its geometry, where its survivors go and its report.
    struct QueuedLevel {
        uint32_t d = 0;
        uint64_t off = 0;
        uint64_t n = 0;      // the level's keys (for a level queued ahead: set once known)
        uint64_t B = 0;      // buckets launched (for a level queued ahead: for its largest size)
        uint32_t lb = 0;
        int yp = 0;          // survivor buffers (by level parity)
        uint64_t seq = 0;    // its report's sequence number
        uint32_t slot = 0;   // its report's slot in the pinned buffer
    };

    // Queues level d by radix partition + per-bucket LDS pass over `in`.  Exact (sa.mode == 0):
    // in.n keys.  Ahead of its key count: between lo and hi keys, the level hash derived on the
    // device by the level's first pass from the survivor total before it (sa), the launches sized for
    // hi keys.  *queued = false when the level would need more than 2^18 buckets (nothing queued).
    mphf_status queue_level(const KeySet& in, uint32_t d, uint64_t off, const BucketGeometry& g,
                            const SpecArgs& sa, uint64_t lo, uint64_t hi, QueuedLevel* q, bool* queued) {
        const SpecLevel* spec = sa.mode ? sa.out : nullptr;
        mphf_status st;
        *queued = false;
        const uint64_t m = level_size(gamma_, spec ? hi : in.n);
        const uint64_t m_lo = spec ? level_size(gamma_, lo) : m;
        const uint64_t wd = (m + 63) / 64;
        const LevelHash L = spec ? LevelHash{} : make_level_hash(seeds_.s[d], m, off);
        const uint32_t pb = g.pbits;
        const uint64_t P = 1ull << pb;
        const uint64_t B = (m + P - 1) / P;
        const uint32_t lb = ceil_log2(B);
        if (lb > 18) return MPHF_OK;   // beyond two passes: use the atomic levels
        unsigned long long* ovf = (unsigned long long*)(dev_ + 129);   // zero here (cleared by each report)
        uint64_t xcap;
        uint32_t S;
        uint64_t* X = nullptr;   // regions of the buckets, on a 128-byte line
        bool packed = false;
        KeySet sized = in;
        if (spec) sized.n = hi;
        if ((st = partition_buckets(sized, L, m, pb, &X, &xcap, &S, &packed, ovf, sa, m_lo)) != MPHF_OK) return st;
        if ((st = reserve()) != MPHF_OK) return st;
        if ((st = ensure_words(off / 64 + wd + 1)) != MPHF_OK) return st;
        // buckets: fill, finalize and filter in LDS
        const int yp = (int)(d & 1);
        if ((st = ensure(&ws_->Y[yp], &ws_->capY[yp], B * g.kcap, "survivors")) != MPHF_OK) return st;
        if ((st = ensure(&ws_->surv[yp], &ws_->capSurv[yp], B + 1, "survivor counts")) != MPHF_OK) return st;
        if ((st = ensure(&ws_->preY[yp], &ws_->capPreY[yp], B + 1, "survivor prefix")) != MPHF_OK) return st;
        uint64_t* C_level = coll_ ? coll_ + off / 64 : nullptr;
        HIP_TRY(launch_bucket(X, xcap, ws_->cntX, S, B, L, pb, packed, g.kcap, words_ + off / 64, C_level, wd,
                              ws_->Y[yp], g.kcap, ws_->surv[yp], ovf, s_, spec),
                "bucket");
        // (the bucket pass writes the count after the last bucket as 0, for the scan's total)
        if ((st = prefix(ws_->surv[yp], B, ws_->preY[yp], spec ? &spec->skip : nullptr)) != MPHF_OK) return st;
        // the overflow flag and the survivor total, written to pinned host memory by one small kernel
        // (which also clears the flag for the next level and keeps it for a level queued behind)
        q->d = d;
        q->off = off;
        q->n = spec ? 0 : in.n;
        q->B = B;
        q->lb = lb;
        q->yp = yp;
        q->seq = next_seq();
        q->slot = d & 1;
        HIP_TRY(launch_report(ovf, ws_->preY[yp] + B, host_dev_ + REPORT_WORDS + 4 * q->slot, q->seq,
                              (unsigned long long*)(dev_ + 140), s_),
                "report");
        *queued = true;
        return MPHF_OK;
    }

    // Waits for a queued level's report.  *ok = false means a region or a bucket overflowed its
    // capacity (only for adversarial key sets): nothing of the level is kept and the caller redoes
    // it with global atomics.  Else the level is recorded and *out describes its survivors.
    mphf_status finish_level(const QueuedLevel& q, const BucketGeometry& g, KeySet* out, bool* ok) {
        mphf_status st;
        *ok = false;
        if ((st = wait_report(q.seq, q.slot)) != MPHF_OK) return st;
        const uint64_t* r = host_ + REPORT_WORDS + 4 * q.slot;
        if (r[0]) return MPHF_OK;   // overflow: redo with atomics
        const uint64_t nnext = r[1];
        if (nnext > q.n) return fail(MPHF_E_DEVICE, "survivors exceed the level's keys");
        const uint64_t m = level_size(gamma_, q.n);
        record(q.d, q.n, m, q.n - nnext, q.off,
               q.B <= 1024 ? MPHF_PATH_ONE_PASS : q.lb - 8 > 8 ? MPHF_PATH_TWO_PASS_WIDE : MPHF_PATH_TWO_PASS);
        out->base = ws_->Y[q.yp];
        out->stride = g.kcap;
        out->pre = ws_->preY[q.yp];
        out->nseg = (uint32_t)((m + (1ull << g.pbits) - 1) >> g.pbits);   // buckets past m hold no survivors
        out->n = nnext;
        *ok = true;
        return MPHF_OK;
    }

    // Bounds on the survivors of a level of n keys in m positions for queueing the next level ahead:
    // the expected number of keys sharing a position, n (1 - (1 - 1/m)^(n-1)), within 10 sqrt(n) + 64
    // (the standard deviation is below sqrt(n) / 2).
    static void survivor_bounds(uint64_t n, uint64_t m, uint64_t* lo, uint64_t* hi) {
        const double e = (double)n * -std::expm1((double)(n - 1) * std::log1p(-1.0 / (double)m));
        const double w = 10.0 * std::sqrt((double)n) + 64.0;
        *lo = e - w > 1.0 ? (uint64_t)(e - w) : 1;
        *hi = (uint64_t)std::ceil(e + w);
        if (*hi > n) *hi = n;
    }

    // Every remaining level in one workgroup (the set fits in its LDS).
    mphf_status tail(const KeySet& in, uint32_t d0, uint64_t off, uint32_t tk) {
        mphf_status st;
        if ((st = reserve()) != MPHF_OK) return st;
        const uint32_t D = o_.max_levels;
        const uint64_t per = (uint64_t)std::ceil(gamma_ * tk) / 64 + 2;
        if ((st = ensure_words(off / 64 + (uint64_t)(D - d0) * per + 1)) != MPHF_OK) return st;
        uint64_t* left = nullptr;
        if ((st = ar_.alloc(&left, in.n, "leftovers")) != MPHF_OK) return st;
        HIP_TRY(launch_tail(in.base, in.stride, in.pre, in.nseg, tk, gamma_, seeds_, d0, D, off, words_,
                            coll_, tail_rec_, left, (TailSummary*)(dev_ + 130), s_),
                "tail");
        // the summary and the per-level records in one read-back into the pinned buffer
        static_assert(8 * 8 + sizeof(TailLevel) * MPHF_MAX_LEVELS <= 4096, "pinned read-back buffer");
        HIP_TRY(hipMemcpyAsync(host_, dev_ + 130, 24, hipMemcpyDeviceToHost, s_), "read back");
        HIP_TRY(hipMemcpyAsync(host_ + 8, tail_rec_, sizeof(TailLevel) * MPHF_MAX_LEVELS, hipMemcpyDeviceToHost, s_),
                "read tail records");
        HIP_TRY(hipStreamSynchronize(s_), "tail sync");
        const uint64_t end = host_[0], nleft = host_[1], bit_end = host_[2];
        const TailLevel* rec = (const TailLevel*)(host_ + 8);
        for (uint64_t d = d0; d < end; ++d)
            record((uint32_t)d, rec[d].n, rec[d].m, rec[d].weight, rec[d].offset, MPHF_PATH_TAIL);
        h_->total_bits = bit_end;
        if (nleft) {
            left_ = left;
            nleft_ = nleft;
        }
        return MPHF_OK;
    }

    // Levels d.. built with global atomics on the interleaved A/C words (used when a level's
    // partition overflows, or on request).  F is dense.
    mphf_status atomic_levels(const uint64_t* F, uint64_t n, uint32_t d0, uint64_t off) {
        mphf_status st;
        if ((st = reserve()) != MPHF_OK) return st;
        const uint32_t D = o_.max_levels;
        const uint64_t m0 = level_size(gamma_, n);
        const uint64_t w0 = (m0 + 63) / 64;
        uint64_t* W = nullptr;
        if ((st = ar_.alloc(&W, 2 * w0 + 2, "W")) != MPHF_OK) return st;
        unsigned long long* counters = (unsigned long long*)dev_;
        HIP_TRY(launch_zero(dev_, 128, s_), "zero counters");
        uint64_t* Fbuf[2] = {nullptr, nullptr};
        const uint64_t* Fin = F;
        uint64_t nd = n;
        LevelHash L = make_level_hash(seeds_.s[d0], m0, off);
        if ((st = ensure_words(off / 64 + w0 + 1)) != MPHF_OK) return st;
        HIP_TRY(launch_zero(W, 2 * w0, s_), "zero W");
        HIP_TRY(launch_fill(Fin, nd, W, L, s_), "fill");
        for (uint32_t d = d0; nd > 0; ++d) {
            const uint64_t m = L.m;
            const uint64_t wd = (m + 63) / 64;
            HIP_TRY(launch_finalize(W, wd, words_ + off / 64, coll_ ? coll_ + off / 64 : nullptr,
                                    counters + d, s_),
                    "finalize");
            if ((st = read_back(counters + d, 8)) != MPHF_OK) return st;
            const uint64_t weight = host_[0];
            if (weight > nd) return fail(MPHF_E_DEVICE, "level weight exceeds the level's keys");
            record(d, nd, m, weight, off, MPHF_PATH_ATOMIC);
            const uint64_t nnext = nd - weight;
            const uint64_t off_next = off + 64 * wd;
            off = off_next;
            if (nnext == 0) break;
            const bool last = d + 1 == D;
            LevelHash Ln{};
            if (!last) {
                const uint64_t mn = level_size(gamma_, nnext);
                const uint64_t wn = (mn + 63) / 64;
                Ln = make_level_hash(seeds_.s[d + 1], mn, off_next);
                if ((st = ensure_words(off_next / 64 + wn + 1)) != MPHF_OK) return st;
                HIP_TRY(launch_zero(W, 2 * wn, s_), "zero W");
            }
            uint64_t*& Fo = Fbuf[(d - d0) & 1];
            if (!Fo && (st = ar_.alloc(&Fo, nnext, "F")) != MPHF_OK) return st;
            const LevelHash Ld = make_level_hash(seeds_.s[d], m, h_->level_offset[d]);
            HIP_TRY(launch_filter_fill(Fin, nd, words_, Ld, Fo, nnext, counters + 64 + d, W, Ln, !last, s_),
                    "filter");
            Fin = Fo;
            nd = nnext;
            L = Ln;
            if (last) {
                left_ = Fo;
                nleft_ = nnext;
                break;
            }
        }
        return MPHF_OK;
    }

    // Fallback table (Section 3, "Termination"): leftovers sorted ascending get N-|L|+1 .. N.
    mphf_status fallback_table() {
        if (!nleft_) return MPHF_OK;
        mphf_status st;
        uint64_t *fb = nullptr, *tmp = nullptr, *roffs = nullptr, *rtiles = nullptr;
        uint32_t* rcounts = nullptr;
        const uint64_t nc = radix_tmp_counts(nleft_);
        if ((st = ar_.alloc(&fb, nleft_, "fallback keys")) != MPHF_OK) return st;
        if ((st = ar_.alloc(&tmp, nleft_, "sort scratch")) != MPHF_OK) return st;
        if ((st = ar_.alloc(&rcounts, nc, "sort counts")) != MPHF_OK) return st;
        if ((st = ar_.alloc(&roffs, nc, "sort offsets")) != MPHF_OK) return st;
        if ((st = ar_.alloc(&rtiles, scan_tmp_tiles(nc), "sort tiles")) != MPHF_OK) return st;
        HIP_TRY(hipMemcpyAsync(fb, left_, nleft_ * 8, hipMemcpyDeviceToDevice, s_), "copy leftovers");
        HIP_TRY(radix_sort_u64(fb, tmp, nleft_, rcounts, roffs, rtiles, s_), "sort");
        HIP_TRY(launch_zero(dev_ + 128, 1, s_), "zero flag");
        HIP_TRY(launch_find_duplicates(fb, nleft_, (unsigned long long*)(dev_ + 128), s_), "duplicates");
        if ((st = read_back(dev_ + 128, 8)) != MPHF_OK) return st;
        if (host_[0]) return fail(MPHF_E_DUPLICATE_KEYS, "duplicate keys in the input");
        h_->fb_keys = fb;
        h_->nfb = nleft_;
        ar_.keep(fb);
        return MPHF_OK;
    }

    // Rank table (Section 3.1) and the lookup's copy of A in 64-byte sectors with embedded rank
    // counters, both from one counting read of A.
    mphf_status rank_and_lookup_layout() {
        h_->nrank = (h_->total_bits + o_.rank_sample - 1) / o_.rank_sample;
        h_->nsec = sector_count(h_->total_bits);
        if (!h_->nsec) return MPHF_OK;   // no bits: no rank entries either
        mphf_status st;
        // one allocation for what the function keeps (sectors, superblocks, rank table) and one for
        // the temporaries, each part on a 256-byte boundary
        auto up = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
        const uint64_t sec_b = up(h_->nsec * 64), sup_b = up(super_count(h_->nsec) * 8), rank_b = up(h_->nrank * 8);
        const uint64_t ng = rank_sector_groups(h_->total_bits);
        const uint64_t cnt_b = up(ng * 4), pre_b = up(ng * 8), tiles_b = up(scan_tmp_tiles(ng) * 8);
        uint8_t *keep = nullptr, *tmp = nullptr;
        if (pre_keep_ && sec_b + sup_b + rank_b <= pre_keep_bytes_ && cnt_b + pre_b + tiles_b <= pre_tmp_bytes_) {
            keep = pre_keep_;   // reserved with A (the levels stayed within the reservation)
            tmp = pre_tmp_;
        } else {
            ar_.release(pre_keep_);
            ar_.release(pre_tmp_);
            if ((st = ar_.alloc(&keep, sec_b + sup_b + rank_b, "lookup sectors and rank table")) != MPHF_OK)
                return st;
            if ((st = ar_.alloc(&tmp, cnt_b + pre_b + tiles_b, "rank and sector temporaries")) != MPHF_OK) return st;
        }
        pre_keep_ = pre_tmp_ = nullptr;
        h_->sec = (uint32_t*)keep;
        h_->super = (uint64_t*)(keep + sec_b);
        h_->rank = (uint64_t*)(keep + sec_b + sup_b);
        h_->layout = keep;
        uint32_t* cnt = (uint32_t*)tmp;
        uint64_t* pre = (uint64_t*)(tmp + cnt_b);
        uint64_t* tiles = (uint64_t*)(tmp + cnt_b + pre_b);
        HIP_TRY(launch_rank_sectors(words_, h_->total_bits, o_.rank_sample, h_->rank, h_->nrank, h_->sec, h_->super,
                                    cnt, pre, tiles, s_),
                "rank and sectors");
        ar_.keep(keep);
        return MPHF_OK;
    }

    // Level table for the lookup kernel.
    mphf_status level_table() {
        if (!h_->num_levels) return MPHF_OK;
        mphf_status st;
        DevLevel hl[MPHF_MAX_LEVELS];
        for (uint32_t d = 0; d < h_->num_levels; ++d) {
            const LevelHash x = make_level_hash(h_->level_seed[d], h_->level_m[d], h_->level_offset[d]);
            hl[d] = DevLevel{x.seed, x.m, x.magic, x.bit_off, x.sh1, x.sh2};
        }
        if ((st = ar_.alloc(&h_->dlev, h_->num_levels, "level table")) != MPHF_OK) return st;
        HIP_TRY(hipMemcpyAsync(h_->dlev, hl, sizeof(DevLevel) * h_->num_levels, hipMemcpyHostToDevice, s_),
                "copy level table");
        HIP_TRY(hipStreamSynchronize(s_), "level table sync");
        ar_.keep(h_->dlev);
        return MPHF_OK;
    }
};

mphf_status build_impl(const uint64_t* keys, uint64_t n, double gamma, uint64_t seed,
                       const mphf_opts& opts, hipStream_t s, mphf** out) {
    if (!(gamma >= 1.0) || !std::isfinite(gamma))
        return fail(MPHF_E_INVALID, "gamma must be a finite number >= 1");
    if (n && !keys) return fail(MPHF_E_INVALID, "keys is NULL");
    if (n && !is_device_ptr(keys)) return fail(MPHF_E_INVALID, "keys is not device memory");
    if (gamma * (double)n >= 9.2e18) return fail(MPHF_E_INVALID, "gamma * n too large");
    mphf_status st = check_opts(opts);
    if (st != MPHF_OK) return st;
    mphf* h = new mphf();
    HIP_TRY(hipGetDevice(&h->device), "hipGetDevice");
    configure_pool(h->device);
    h->n = n;
    h->gamma = gamma;
    h->seed = seed;
    h->opts = opts;
    h->rank_shift = opts.rank_sample == 1024 ? 10 : 9;
    {
        Builder b(h, opts, s);
        st = b.run(keys, n, gamma);
    }
    if (st != MPHF_OK) {
        free_handle(h);
        return st;
    }
    *out = h;
    return MPHF_OK;
}

mphf_status build_stream_impl(uint64_t kseed, uint64_t kstart, const uint64_t* host_keys, uint64_t n, double gamma,
                              uint64_t seed, const mphf_opts& opts, uint64_t budget, hipStream_t s, mphf** out) {
    if (!(gamma >= 1.0) || !std::isfinite(gamma))
        return fail(MPHF_E_INVALID, "gamma must be a finite number >= 1");
    if (gamma * (double)n >= 9.2e18) return fail(MPHF_E_INVALID, "gamma * n too large");
    mphf_status st = check_opts(opts);
    if (st != MPHF_OK) return st;
    mphf* h = new mphf();
    HIP_TRY(hipGetDevice(&h->device), "hipGetDevice");
    configure_pool(h->device);
    h->n = n;
    h->gamma = gamma;
    h->seed = seed;
    h->opts = opts;
    h->rank_shift = opts.rank_sample == 1024 ? 10 : 9;
    {
        Builder b(h, opts, s);
        b.use_host_keys(host_keys);
        st = b.run_stream(kseed, kstart, n, gamma, budget);
    }
    if (st != MPHF_OK) {
        free_handle(h);
        return st;
    }
    *out = h;
    return MPHF_OK;
}

}  // namespace

extern "C" {

mphf_status mphf_build_stream(const mphf_key_stream* src, uint64_t n, double gamma, uint64_t seed,
                              const mphf_opts* opts, uint64_t resident_keys, void* stream, mphf_t** out) {
    if (!out || !src) return fail(MPHF_E_INVALID, "NULL argument");
    *out = nullptr;
    mphf_opts o;
    if (opts) o = *opts;
    else mphf_default_opts(&o);
    if (o.flags & ~MPHF_FLAG_ATOMIC_LEVELS) return fail(MPHF_E_INVALID, "unknown flags");
    return build_stream_impl(src->seed, src->start, nullptr, n, gamma, seed, o, resident_keys, (hipStream_t)stream,
                             out);
}

mphf_status mphf_build_host(const uint64_t* keys, uint64_t n, double gamma, uint64_t seed, const mphf_opts* opts,
                            uint64_t resident_keys, void* stream, mphf_t** out) {
    if (!out) return fail(MPHF_E_INVALID, "NULL argument");
    *out = nullptr;
    if (n && !keys) return fail(MPHF_E_INVALID, "keys is NULL");
    if (n && is_device_ptr(keys)) return fail(MPHF_E_INVALID, "keys must be host memory (mphf_build_ex takes device keys)");
    mphf_opts o;
    if (opts) o = *opts;
    else mphf_default_opts(&o);
    if (o.flags & ~MPHF_FLAG_ATOMIC_LEVELS) return fail(MPHF_E_INVALID, "unknown flags");
    return build_stream_impl(0, 0, keys, n, gamma, seed, o, resident_keys, (hipStream_t)stream, out);
}

mphf_status mphf_stream_keys(const mphf_key_stream* src, uint64_t first, uint64_t count, uint64_t* out,
                             void* stream) {
    if (!src) return fail(MPHF_E_INVALID, "src is NULL");
    if (!count) return MPHF_OK;
    if (!out || !is_device_ptr(out)) return fail(MPHF_E_INVALID, "out must be device memory");
    HIP_TRY(launch_stream_keys(src->seed, src->start + first, count, out, (hipStream_t)stream), "stream keys");
    return MPHF_OK;
}

mphf_status mphf_default_opts(mphf_opts* o) {
    if (!o) return fail(MPHF_E_INVALID, "opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->max_levels = 25;
    o->rank_sample = 512;
    return MPHF_OK;
}

mphf_status mphf_build_ex(const uint64_t* keys, uint64_t n, double gamma, uint64_t seed,
                          const mphf_opts* opts, void* stream, mphf_t** out) {
    if (!out) return fail(MPHF_E_INVALID, "out is NULL");
    *out = nullptr;
    mphf_opts o;
    if (opts) o = *opts;
    else mphf_default_opts(&o);
    return build_impl(keys, n, gamma, seed, o, (hipStream_t)stream, out);
}

mphf_t* mphf_build(const uint64_t* keys, uint64_t n, double gamma, uint64_t seed) {
    mphf_t* h = nullptr;
    if (mphf_build_ex(keys, n, gamma, seed, nullptr, nullptr, &h) != MPHF_OK) return nullptr;
    return h;
}

mphf_status mphf_lookup_ex(const mphf_t* h, const uint64_t* keys, uint64_t n, uint64_t* out,
                           void* stream) {
    if (!h) return fail(MPHF_E_INVALID, "handle is NULL");
    if (!n) return MPHF_OK;
    if (!keys || !out) return fail(MPHF_E_INVALID, "keys or out is NULL");
    if (!is_device_ptr(keys) || !is_device_ptr(out))
        return fail(MPHF_E_INVALID, "keys and out must be device memory");
    if (keys == out) return fail(MPHF_E_INVALID, "out may not alias keys");
    HIP_TRY(launch_lookup(keys, n, out, h->dlev, h->num_levels, h->sec, h->super, h->fb_keys, h->nfb,
                          h->n, (hipStream_t)stream),
            "lookup");
    HIP_TRY(h->uses.note((hipStream_t)stream), "lookup event");
    return MPHF_OK;
}

int mphf_lookup(const mphf_t* h, const uint64_t* keys, uint64_t n, uint64_t* out) {
    mphf_status st = mphf_lookup_ex(h, keys, n, out, nullptr);
    if (st != MPHF_OK) return st;
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return hip_fail(e, "lookup sync");
    return MPHF_OK;
}

void mphf_destroy(mphf_t* h) { free_handle(h); }

mphf_status mphf_stats(const mphf_t* h, mphf_stats_t* st) {
    if (!h || !st) return fail(MPHF_E_INVALID, "NULL argument");
    std::memset(st, 0, sizeof(*st));
    st->n = h->n;
    st->gamma = h->gamma;
    st->seed = h->seed;
    st->num_levels = h->num_levels;
    st->rank_sample = h->opts.rank_sample;
    for (uint32_t d = 0; d < h->num_levels; ++d) {
        st->level_n[d] = h->level_n[d];
        st->level_m[d] = h->level_m[d];
        st->level_weight[d] = h->level_weight[d];
        st->level_offset[d] = h->level_offset[d];
        st->level_seed[d] = h->level_seed[d];
        st->level_path[d] = h->level_path[d];
    }
    st->bucket_bits = h->bucket_bits;
    st->n_fallback = h->nfb;
    st->total_bits = h->total_bits;
    st->rank_entries = h->nrank;
    st->structure_bytes = h->total_words * 8 + h->nrank * 8 + h->nfb * 8;
    st->lookup_bytes = h->nsec * 64 + (h->nsec ? super_count(h->nsec) * 8 : 0) + h->nfb * 8;
    st->bits_per_key = h->n ? (double)(h->total_bits + 64 * h->nrank + 128 * h->nfb) / (double)h->n : 0.0;
    st->peak_bytes = h->peak_bytes;
    return MPHF_OK;
}

mphf_status mphf_view(const mphf_t* h, mphf_view_t* v) {
    if (!h || !v) return fail(MPHF_E_INVALID, "NULL argument");
    v->words = h->words;
    v->rank = h->rank;
    v->fallback_keys = h->fb_keys;
    v->collisions = h->coll_all;
    v->total_words = h->total_words;
    v->rank_entries = h->nrank;
    v->n_fallback = h->nfb;
    return MPHF_OK;
}

mphf_status mphf_export(const mphf_t* h, uint64_t* words, uint64_t nwords, uint64_t* rank,
                        uint64_t nrank, uint64_t* fallback_keys, uint64_t nfb) {
    if (!h) return fail(MPHF_E_INVALID, "handle is NULL");
    if ((words && nwords != h->total_words) || (rank && nrank != h->nrank) ||
        (fallback_keys && nfb != h->nfb))
        return fail(MPHF_E_INVALID, "export sizes differ from the structure's");
    if (words && nwords) HIP_TRY(hipMemcpy(words, h->words, nwords * 8, hipMemcpyDeviceToHost), "copy A");
    if (rank && nrank) HIP_TRY(hipMemcpy(rank, h->rank, nrank * 8, hipMemcpyDeviceToHost), "copy rank");
    if (fallback_keys && nfb)
        HIP_TRY(hipMemcpy(fallback_keys, h->fb_keys, nfb * 8, hipMemcpyDeviceToHost), "copy fallback");
    return MPHF_OK;
}

mphf_status mphf_export_collisions(const mphf_t* h, uint32_t level, uint64_t* out, uint64_t nwords) {
    if (!h || !out) return fail(MPHF_E_INVALID, "NULL argument");
    if (level >= h->num_levels) return fail(MPHF_E_INVALID, "no such level");
    if (!h->coll_all) return fail(MPHF_E_INVALID, "collisions were not kept (keep_collisions)");
    const uint64_t need = (h->level_m[level] + 63) / 64;
    if (nwords < need) return fail(MPHF_E_INVALID, "output too small");
    HIP_TRY(hipMemcpy(out, h->coll_all + h->level_offset[level] / 64, need * 8, hipMemcpyDeviceToHost),
            "copy C");
    return MPHF_OK;
}

mphf_status mphf_positions(const uint64_t* keys, uint64_t n, uint64_t level_seed, uint64_t m,
                           uint64_t* out, void* stream) {
    if (m < 1 || m >= (1ull << 63)) return fail(MPHF_E_INVALID, "m must be in [1, 2^63)");
    if (!n) return MPHF_OK;
    if (!keys || !out || !is_device_ptr(keys) || !is_device_ptr(out))
        return fail(MPHF_E_INVALID, "keys and out must be device memory");
    HIP_TRY(launch_positions(keys, n, make_level_hash(level_seed, m, 0), out, (hipStream_t)stream),
            "positions");
    return MPHF_OK;
}

mphf_status mphf_trim(void) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (int d = 0; d < 64; ++d) {
        std::lock_guard<std::mutex> g(g_ws[d].mu);
        std::lock_guard<std::mutex> gb(g_bws[d].mu);
        if (!g_ws[d].b.host && !g_ws[d].b.Z && !g_ws[d].b.X && !g_ws[d].b.Y[0] && !g_ws[d].b.tiles &&
            !g_bws[d].buf[0] && !g_bws[d].buf[1])
            continue;
        if (hipSetDevice(d) != hipSuccess) continue;
        (void)hipDeviceSynchronize();
        g_ws[d].release();
        g_bws[d].release();
    }
    (void)hipSetDevice(cur);
    return MPHF_OK;
}

const char* mphf_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------- k-mer workload

namespace {

// Hash-set partition by radix passes over the top bits of h = fmix64(x ^ seed), written densely
// into out: with bits <= 8 one pass over the keys; with 8 < bits <= 18 a pass into 2^8 coarse bins
// (line-aligned regions of hashes) and a grouped pass over each coarse bin into its 2^(bits - 8)
// sets.  The dense pass writes each workgroup's keys of a set at an offset counted beforehand over
// the same input slices.  *ok = false if a region of the first pass overflowed (adversarial key
// sets only): out is then incomplete and the caller redoes the partition another way.
mphf_status partition_sets_radix(Arena& ar, const uint64_t* keys, uint64_t n, uint32_t bits, uint64_t seed,
                                 uint64_t* out, uint64_t* offsets, hipStream_t s, bool* ok) {
    mphf_status st;
    *ok = false;
    const uint64_t nb = 1ull << bits;
    const uint32_t sh = 64 - bits;   // set of x = fmix64(x ^ seed) >> sh
    LevelHash L{};
    L.seed = seed;
    L.sh1 = sh;
    uint64_t *pre0, *flag;
    if ((st = ar.alloc(&pre0, 2, "partition prefix")) != MPHF_OK) return st;
    if ((st = ar.alloc(&flag, 1, "overflow flag")) != MPHF_OK) return st;
    HIP_TRY(launch_pair(pre0, 0, n, s), "prefix");
    HIP_TRY(launch_zero(flag, 1, s), "zero flag");
    unsigned long long* ovf = (unsigned long long*)flag;
    const uint64_t W = std::max<uint64_t>(1, std::min<uint64_t>(n / 65536, PART_WGS));
    // the dense pass: input (in, stride, pre), groups x K workgroups
    const uint64_t* in = keys;
    uint64_t stride = 0, ngroups = 1, SG = 1, K = W, nseg = 1;
    const uint64_t* pre = pre0;
    uint32_t fb = 0;
    if (bits > 8) {
        fb = bits - 8;
        const uint64_t C = 256;
        const uint64_t cap1 = region_cap((double)n / (double)W / (double)C);
        uint64_t *Zb, *preZ, *tz;
        uint32_t* cntZ;
        if ((st = ar.alloc(&Zb, C * W * cap1 + 16, "coarse regions")) != MPHF_OK) return st;
        if ((st = ar.alloc(&cntZ, C * W + 1, "coarse counts")) != MPHF_OK) return st;
        if ((st = ar.alloc(&preZ, C * W + 1, "coarse prefix")) != MPHF_OK) return st;
        if ((st = ar.alloc(&tz, scan_tmp_tiles(C * W + 1), "scan tiles")) != MPHF_OK) return st;
        uint64_t* const Z = line_align(Zb);
        HIP_TRY(launch_partition(8, false, keys, 0, pre0, 1, 1, (uint32_t)W, L, 0, fb, false, 0, C, Z, cap1,
                                 (uint32_t)W, cntZ, ovf, n, 1, s, 1),
                "partition 1");
        HIP_TRY(launch_zero32(cntZ + C * W, 1, s), "zero count tail");
        HIP_TRY(launch_exclusive_scan(cntZ, preZ, C * W + 1, tz, s), "coarse prefix");
        in = Z;
        stride = cap1;
        pre = preZ;
        ngroups = C;
        SG = W;
        K = slots_per_group(C, n);
        nseg = C * W;
    }
    uint32_t* cnt;
    uint64_t *base, *tiles;
    if ((st = ar.alloc(&cnt, nb * K + 1, "slice counts")) != MPHF_OK) return st;
    if ((st = ar.alloc(&base, nb * K + 1, "slice offsets")) != MPHF_OK) return st;
    if ((st = ar.alloc(&tiles, scan_tmp_tiles(nb * K + 1), "scan tiles")) != MPHF_OK) return st;
    HIP_TRY(launch_slice_counts(in, stride, pre, (uint32_t)ngroups, (uint32_t)SG, (uint32_t)K, seed, sh, bits > 8,
                                bits > 8, fb, nb, cnt, s),
            "slice counts");
    HIP_TRY(launch_zero32(cnt + nb * K, 1, s), "zero count tail");
    HIP_TRY(launch_exclusive_scan(cnt, base, nb * K + 1, tiles, s), "slice offsets");
    HIP_TRY(launch_partition(bits > 8 && fb > 8 ? 10 : 8, bits > 8, in, stride, pre, (uint32_t)ngroups, (uint32_t)SG,
                             (uint32_t)K, L, 0, 0, bits > 8, fb, nb, out, 0, (uint32_t)K, nullptr, ovf, n, nseg, s,
                             2, base),
            "dense partition");
    HIP_TRY(launch_take_every(base, (uint32_t)K, nb, offsets, s), "offsets");
    uint64_t h_flag = 0;
    HIP_TRY(hipMemcpyAsync(&h_flag, flag, 8, hipMemcpyDeviceToHost, s), "read flag");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    *ok = h_flag == 0;
    return MPHF_OK;
}

}  // namespace

extern "C" {

mphf_status mphf_kmers(const uint64_t* seq, uint64_t nbases, uint32_t k, uint64_t* out, void* stream) {
    if (k < 1 || k > 32) return fail(MPHF_E_INVALID, "k must be 1..32");
    if (nbases < k) return MPHF_OK;
    if (!seq || !out || !is_device_ptr(seq) || !is_device_ptr(out))
        return fail(MPHF_E_INVALID, "seq and out must be device memory");
    HIP_TRY(launch_kmers(seq, nbases - k + 1, k, out, (hipStream_t)stream), "kmers");
    return MPHF_OK;
}

mphf_status mphf_first_occurrences(const uint64_t* keys, uint64_t n, uint64_t target, uint64_t* out,
                                   uint64_t* nout, void* stream) {
    if (!nout) return fail(MPHF_E_INVALID, "nout is NULL");
    *nout = 0;
    if (!n || !target) return MPHF_OK;
    if (!keys || !out || !is_device_ptr(keys) || !is_device_ptr(out))
        return fail(MPHF_E_INVALID, "keys and out must be device memory");
    const hipStream_t s = (hipStream_t)stream;
    mphf_status st;
    Arena ar(0, s);
    // keys that repeat: adjacent equal keys after a sort of a copy
    uint64_t *a, *b, *offs, *tiles, *cnt64;
    uint32_t* counts;
    const uint64_t nc = radix_tmp_counts(n);
    if ((st = ar.alloc(&a, n, "sort copy")) != MPHF_OK) return st;
    if ((st = ar.alloc(&b, n, "sort scratch")) != MPHF_OK) return st;
    if ((st = ar.alloc(&counts, nc, "sort counts")) != MPHF_OK) return st;
    if ((st = ar.alloc(&offs, nc, "sort offsets")) != MPHF_OK) return st;
    if ((st = ar.alloc(&tiles, scan_tmp_tiles(nc), "sort tiles")) != MPHF_OK) return st;
    if ((st = ar.alloc(&cnt64, 2, "counters")) != MPHF_OK) return st;
    HIP_TRY(hipMemcpyAsync(a, keys, 8 * n, hipMemcpyDeviceToDevice, s), "copy keys");
    HIP_TRY(radix_sort_u64(a, b, n, counts, offs, tiles, s), "sort");
    ar.release(b);
    ar.release(counts);
    ar.release(offs);
    const uint64_t cap = std::min<uint64_t>(n, 1ull << 24);
    uint64_t* rep;
    if ((st = ar.alloc(&rep, cap, "repeated keys")) != MPHF_OK) return st;
    HIP_TRY(launch_zero(cnt64, 2, s), "zero counters");
    HIP_TRY(launch_repeated(a, n, rep, cap, (unsigned long long*)cnt64, s), "repeated");
    uint64_t nrep = 0;
    HIP_TRY(hipMemcpyAsync(&nrep, cnt64, 8, hipMemcpyDeviceToHost, s), "read back");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    ar.release(a);
    if (nrep > cap) return fail(MPHF_E_INVALID, "more than 2^24 distinct keys repeat");
    std::vector<uint64_t> removed;
    if (nrep) {
        std::vector<uint64_t> h(nrep);
        HIP_TRY(hipMemcpy(h.data(), rep, 8 * nrep, hipMemcpyDeviceToHost), "copy repeated");
        std::sort(h.begin(), h.end());
        HIP_TRY(hipMemcpy(rep, h.data(), 8 * nrep, hipMemcpyHostToDevice), "copy repeated");
        unsigned long long* first;
        uint64_t* later;
        const uint64_t cap2 = std::min<uint64_t>(n, 1ull << 25);
        if ((st = ar.alloc(&first, nrep, "first positions")) != MPHF_OK) return st;
        if ((st = ar.alloc(&later, cap2, "later positions")) != MPHF_OK) return st;
        HIP_TRY(launch_first_pos(keys, n, rep, nrep, first, s), "first positions");
        HIP_TRY(launch_later_pos(keys, n, rep, nrep, first, later, cap2, (unsigned long long*)cnt64 + 1, s),
                "later positions");
        uint64_t nrem = 0;
        HIP_TRY(hipMemcpyAsync(&nrem, cnt64 + 1, 8, hipMemcpyDeviceToHost, s), "read back");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        if (nrem > cap2) return fail(MPHF_E_INVALID, "more than 2^25 repeated positions");
        removed.resize(nrem);
        HIP_TRY(hipMemcpy(removed.data(), later, 8 * nrem, hipMemcpyDeviceToHost), "copy positions");
        std::sort(removed.begin(), removed.end());
    }
    // the first `target` kept positions end at P: every removed position below P moves P by one
    uint64_t j = 0;
    uint64_t P = n, kept = n - removed.size();
    if (kept > target) {
        while (j < removed.size() && removed[j] < target + j) ++j;
        P = target + j;
        kept = target;
    } else {
        j = removed.size();
    }
    uint64_t* drem = nullptr;
    if (j) {
        if ((st = ar.alloc(&drem, j, "removed positions")) != MPHF_OK) return st;
        HIP_TRY(hipMemcpyAsync(drem, removed.data(), 8 * j, hipMemcpyHostToDevice, s), "copy positions");
    }
    HIP_TRY(launch_drop_positions(keys, P, drem, j, out, s), "compact");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    *nout = kept;
    return MPHF_OK;
}

mphf_status mphf_partition_sets(const uint64_t* keys, uint64_t n, uint32_t bits, uint64_t seed, uint64_t* out,
                                uint64_t* offsets, void* stream) {
    if (bits < 1 || bits > 24) return fail(MPHF_E_INVALID, "bits must be 1..24");
    if (!offsets || !is_device_ptr(offsets) || (n && (!keys || !out || !is_device_ptr(keys) || !is_device_ptr(out))))
        return fail(MPHF_E_INVALID, "keys, out and offsets must be device memory");
    const hipStream_t s = (hipStream_t)stream;
    mphf_status st;
    Arena ar(0, s);
    if (bits <= 18 && n >= 65536) {
        bool ok = false;
        if ((st = partition_sets_radix(ar, keys, n, bits, seed, out, offsets, s, &ok)) != MPHF_OK) return st;
        if (ok) {
            HIP_TRY(hipStreamSynchronize(s), "sync");
            return MPHF_OK;
        }
        // a region overflowed: the scatter below is exact for any key set
    }
    const uint64_t nb = 1ull << bits;
    uint32_t* counts;
    unsigned long long* cursor;
    uint64_t* tiles;
    if ((st = ar.alloc(&counts, nb + 1, "set counts")) != MPHF_OK) return st;
    if ((st = ar.alloc(&cursor, nb, "set cursors")) != MPHF_OK) return st;
    if ((st = ar.alloc(&tiles, scan_tmp_tiles(nb + 1), "scan tiles")) != MPHF_OK) return st;
    HIP_TRY(launch_set_partition(keys, n, seed, bits, counts, offsets, cursor, tiles, out, s), "partition");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    return MPHF_OK;
}

mphf_status mphf_set_ids(const uint64_t* keys, uint64_t n, uint32_t bits, uint64_t seed, uint64_t* out,
                         void* stream) {
    if (bits < 1 || bits > 24) return fail(MPHF_E_INVALID, "bits must be 1..24");
    if (n && (!keys || !out || !is_device_ptr(keys) || !is_device_ptr(out)))
        return fail(MPHF_E_INVALID, "keys and out must be device memory");
    HIP_TRY(launch_set_ids(keys, n, seed, bits, out, (hipStream_t)stream), "set ids");
    return MPHF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- shared with the serving loop

namespace mphf_api {

mphf_status set_error(mphf_status st, const std::string& msg) { return fail(st, msg); }

mphf_status hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }

bool device_ptr(const void* p) { return is_device_ptr(p); }

void lookup_desc(const mphf_t* h, SegDesc* d, int* device) {
    d->lev = h->dlev;
    d->sec = h->sec;
    d->super = h->super;
    d->fbk = h->fb_keys;
    d->nfb = h->nfb;
    d->N = h->n;
    d->nlev = h->num_levels;
    d->pad = 0;
    *device = h->device;
}

}  // namespace mphf_api

// ---------------------------------------------------------------- batched builds

struct mphf_batch {
    int device = 0;
    bool planned = false;
    uint64_t nsets = 0, nkeys = 0, total_bits = 0, nsec = 0, nleft = 0;
    uint64_t used_sec = 0, used_left = 0;   // sectors and fallback keys the sets use (packed sizes)
    double gamma = 0;
    uint32_t D = 25;
    SeedTable seeds{};
    std::vector<void*> mem;     // device allocations owned by the handle
    // per set (valid after a build)
    BatchSet* sets = nullptr;
    BatchLevel* levels = nullptr;
    BatchHead* heads = nullptr;
    BatchLev* lev = nullptr;
    BatchAux* aux = nullptr;
    uint32_t* sec = nullptr;    // lookup sectors: dense, or the worst-case region of a planned batch
    uint64_t* left = nullptr;   // fallback keys: packed, or in the survivors' scratch of a planned batch
    // what a planned batch keeps for its rebuilds
    uint64_t* offsets = nullptr;
    uint32_t* order = nullptr;
    uint32_t* hist = nullptr;   // sets per size class
    uint64_t* region_w = nullptr;
    uint64_t* sreg_base = nullptr;
    unsigned long long* queue = nullptr;
    uint32_t* fail32 = nullptr;
    uint32_t *left32 = nullptr, *sec32 = nullptr;
    uint64_t* scratch = nullptr;
    uint64_t* region = nullptr;
    uint64_t max_m = 0;
    uint32_t grid = 0;
    BatchLaunch cfg;
    bool retried = false;   // the one-shot build was redone with worst-case regions
    mutable UseTracker uses;
};

namespace {

void free_batch(mphf_batch* b) {
    if (!b) return;
    b->uses.wait_all();
    free_on_device(b->device, b->mem);
    delete b;
}

constexpr uint32_t BATCH_LEFT_CAP = 2048;
constexpr uint64_t BATCH_MAX_M = 1ull << 19;   // A and C of the level in LDS: 128 KiB

// A small pinned host buffer per thread and device for the batched build's read-backs.
uint64_t* batch_pinned(int dev) {
    thread_local uint64_t* buf[64] = {};
    if (dev < 0 || dev >= 64) return nullptr;
    if (!buf[dev] && hipHostMalloc((void**)&buf[dev], 256, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        buf[dev] = nullptr;
    }
    return buf[dev];
}

// Lays typed arrays out in one byte range, each 256-byte aligned.  With a null base it only
// measures (the pointers it returns are then offsets and must not be used).
struct Carver {
    uint8_t* base;
    uint64_t off = 0;
    template <typename T>
    T* take(uint64_t count) {
        off = (off + 255) & ~uint64_t(255);
        T* p = (T*)(base + off);
        off += count * sizeof(T);
        return p;
    }
};

// Device memory for a batch: the handle's own allocations (kept), or temporaries from the device's
// cached workspace when this build can take it, else from the arena (always so with a memory budget,
// so that the budget counts them).
class BatchMem {
  public:
    BatchMem(Arena& ar, int dev, bool cache) : ar_(ar) {
        if (!cache || dev < 0 || dev >= 64) return;
        std::unique_lock<std::mutex> lk(g_bws[dev].mu, std::try_to_lock);
        if (!lk.owns_lock()) return;
        lock_ = std::move(lk);
        ws_ = &g_bws[dev];
    }
    template <typename F>
    mphf_status temp(int slot, F lay) {
        Carver m{nullptr};
        lay(m);
        uint8_t* p = nullptr;
        mphf_status st = ws_ ? ws_get(slot, m.off, &p) : ar_.alloc(&p, m.off + 256, "batch temporaries");
        if (st != MPHF_OK) return st;
        Carver c{p};
        lay(c);
        return MPHF_OK;
    }
    template <typename F>
    mphf_status transient(F lay, const char* what) {   // freed when the build returns
        Carver m{nullptr};
        lay(m);
        uint8_t* p = nullptr;
        mphf_status st = ar_.alloc(&p, m.off + 256, what);
        if (st != MPHF_OK) return st;
        Carver c{p};
        lay(c);
        return MPHF_OK;
    }
    template <typename F>
    mphf_status own(mphf_batch* b, F lay, const char* what) {
        Carver m{nullptr};
        lay(m);
        uint8_t* p = nullptr;
        mphf_status st = ar_.alloc(&p, m.off + 256, what);
        if (st != MPHF_OK) return st;
        b->mem.push_back(p);
        Carver c{p};
        lay(c);
        return MPHF_OK;
    }

  private:
    mphf_status ws_get(int slot, uint64_t bytes, uint8_t** p) {
        if (ws_->cap[slot] < bytes) {
            if (ws_->buf[slot]) {
                HIP_TRY(hipDeviceSynchronize(), "workspace sync");
                (void)hipFree(ws_->buf[slot]);
                ws_->buf[slot] = nullptr;
                ws_->cap[slot] = 0;
            }
            const uint64_t want = bytes + bytes / 8 + 4096;
            const hipError_t e = hipMalloc(&ws_->buf[slot], want);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                ws_->buf[slot] = nullptr;
                return hip_fail(e, "batch workspace");
            }
            ws_->cap[slot] = want;
        }
        *p = (uint8_t*)ws_->buf[slot];
        return MPHF_OK;
    }
    Arena& ar_;
    BatchWorkspace* ws_ = nullptr;
    std::unique_lock<std::mutex> lock_;
};

mphf_status check_batch_args(const uint64_t* offsets, uint64_t nsets, double gamma, const mphf_opts& o) {
    if (!(gamma >= 1.0) || !std::isfinite(gamma)) return fail(MPHF_E_INVALID, "gamma must be a finite number >= 1");
    if (!nsets) return fail(MPHF_E_INVALID, "nsets must be positive");
    if (nsets >= (1ull << 32)) return fail(MPHF_E_INVALID, "at most 2^32 - 1 sets");
    if (!offsets || !is_device_ptr(offsets)) return fail(MPHF_E_INVALID, "offsets must be device memory");
    mphf_status st = check_opts(o);
    if (st != MPHF_OK) return st;
    if (o.flags) return fail(MPHF_E_INVALID, "flags are not supported for batched builds");
    if (o.rank_sample != 512) return fail(MPHF_E_INVALID, "batched builds use rank_sample 512");
    const uint32_t t = o.batch_threads, it = o.batch_items;
    if ((t && t != 128 && t != 256 && t != 512) || (it && it != 4 && it != 8 && it != 16) || o.batch_wgs_per_cu > 8)
        return fail(MPHF_E_INVALID, "batch launch: threads 128/256/512, items 4/8/16, at most 8 workgroups per CU");
    if (o.batch_small_class > 64) return fail(MPHF_E_INVALID, "batch_small_class: 0 (default) or 1..64");
    return MPHF_OK;
}

// Offsets checked, worst-case regions sized, size-ordered work queue, and every buffer a build needs.
// `keep` = a planned batch: everything lives in the handle; else the temporaries are borrowed.
mphf_status batch_setup(mphf_batch* b, const uint64_t* keys, const uint64_t* offsets, uint64_t nsets, double gamma,
                        uint64_t seed, const mphf_opts& o, bool keep, double slack, hipStream_t s, BatchMem& mem,
                        uint64_t* pin) {
    mphf_status st;
    b->nsets = nsets;
    b->gamma = gamma;
    b->D = o.max_levels;
    b->planned = keep;
    level_seeds(seed, o.max_levels, b->seeds.s);
    const uint32_t ncls = batch_classes();
    const uint64_t S1 = nsets + 1;
    uint32_t *bound, *sbound, *hist;
    uint64_t *tiles, *off_copy;
    unsigned long long* info;   // [0] largest set, [1] offset flags, [2] queue head
    auto lay1 = [&](Carver& c) {
        b->order = c.take<uint32_t>(nsets);
        b->region_w = c.take<uint64_t>(S1);
        b->sreg_base = c.take<uint64_t>(S1);
        info = c.take<unsigned long long>(4);
        hist = c.take<uint32_t>(2 * ncls + 2);
        bound = c.take<uint32_t>(S1);
        sbound = c.take<uint32_t>(S1);
        tiles = c.take<uint64_t>(scan_tmp_tiles(S1));
        b->left32 = c.take<uint32_t>(S1);
        b->sec32 = c.take<uint32_t>(S1);
        off_copy = keep ? c.take<uint64_t>(S1) : nullptr;
    };
    if ((st = keep ? mem.own(b, lay1, "batch plan") : mem.temp(0, lay1)) != MPHF_OK) return st;
    b->queue = info + 2;   // (two counters)
    b->hist = hist;
    b->fail32 = hist + 2 * ncls;
    if (keep) {
        HIP_TRY(hipMemcpyAsync(off_copy, offsets, S1 * 8, hipMemcpyDeviceToDevice, s), "copy offsets");
        b->offsets = off_copy;
    } else {
        b->offsets = const_cast<uint64_t*>(offsets);
    }
    HIP_TRY(launch_zero32(hist, 2 * ncls + 2, s), "zero classes");
    HIP_TRY(launch_zero((uint64_t*)info, 4, s), "zero counters");
    HIP_TRY(launch_batch_prepare(b->offsets, nsets, gamma, o.max_levels, BATCH_MAX_M, slack, bound, sbound, hist,
                                 info, s),
            "prepare");
    HIP_TRY(launch_exclusive_scan(bound, b->region_w, S1, tiles, s), "region prefix");
    HIP_TRY(launch_exclusive_scan(sbound, b->sreg_base, S1, tiles, s), "sector prefix");
    HIP_TRY(launch_batch_order(b->offsets, nsets, hist, hist + ncls, b->order, s), "order");
    HIP_TRY(hipMemcpyAsync(pin, info, 16, hipMemcpyDeviceToHost, s), "read back");
    HIP_TRY(hipMemcpyAsync(pin + 2, b->offsets + nsets, 8, hipMemcpyDeviceToHost, s), "read back");
    HIP_TRY(hipMemcpyAsync(pin + 3, b->region_w + nsets, 8, hipMemcpyDeviceToHost, s), "read back");
    HIP_TRY(hipMemcpyAsync(pin + 4, b->sreg_base + nsets, 8, hipMemcpyDeviceToHost, s), "read back");
    HIP_TRY(hipStreamSynchronize(s), "batch sync");
    const uint64_t max_n = pin[0], flags = pin[1], total = pin[2], region_words = pin[3], sreg_total = pin[4];
    if (flags & 2) return fail(MPHF_E_INVALID, "offsets[0] must be 0");
    if (flags & 1) return fail(MPHF_E_INVALID, "offsets must be non-decreasing");
    if (flags & 4) return fail(MPHF_E_INVALID, "a set is too large for a batched build (ceil(gamma n) > 2^19)");
    if (keys && total && !is_device_ptr(keys)) return fail(MPHF_E_INVALID, "keys must be device memory");
    if (sreg_total >= (1ull << HEAD_BASE_BITS)) return fail(MPHF_E_INVALID, "batch too large for the lookup records");
    b->nkeys = total;
    b->max_m = level_size(gamma, max_n);

    // survivors (then fallback keys), staged bits and worst-case sectors: the planned batch keeps them
    auto lay2 = [&](Carver& c) {
        b->scratch = c.take<uint64_t>(total + 1);
        b->region = c.take<uint64_t>(region_words + 1);
        b->sec = c.take<uint32_t>((sreg_total + 1) * SEC_WORDS);
    };
    if ((st = keep ? mem.own(b, lay2, "batch survivors and sectors") : mem.temp(1, lay2)) != MPHF_OK) return st;
    const uint64_t lev_slots = o.max_levels > 2 ? nsets * (o.max_levels - 2) : 0;
    auto lay3 = [&](Carver& c) {
        b->sets = c.take<BatchSet>(nsets);
        b->levels = c.take<BatchLevel>(nsets * o.max_levels);
        b->heads = c.take<BatchHead>(nsets);
        b->lev = c.take<BatchLev>(lev_slots + 1);
        b->aux = c.take<BatchAux>(nsets);
    };
    if ((st = mem.own(b, lay3, "set records")) != MPHF_OK) return st;
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device), "CU count");
    b->cfg.threads = o.batch_threads ? o.batch_threads : 256;
    b->cfg.items = o.batch_items ? o.batch_items : 4;
    b->cfg.wgs_per_cu = o.batch_wgs_per_cu;
    b->cfg.small_class = o.batch_small_class ? o.batch_small_class : 13;
    b->cfg.small_every = o.batch_small_every ? o.batch_small_every : 2;
    HIP_TRY(batch_kernel_setup(b->cfg, b->max_m, BATCH_LEFT_CAP), "batch kernel setup");
    const uint64_t lds = batch_lds_bytes(b->max_m, BATCH_LEFT_CAP);
    uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(8, 155000 / (lds + 1024)));
    if (b->cfg.wgs_per_cu) per_cu = std::min<uint64_t>(per_cu, b->cfg.wgs_per_cu);
    b->grid = (uint32_t)std::min<uint64_t>(nsets, (uint64_t)cus * per_cu);
    if (keep) {
        b->left = b->scratch;
        b->nsec = sreg_total;
    }
    return MPHF_OK;
}

// Every set's levels, sectors and status: a fixed sequence of launches, no allocation and no host
// synchronization (capturable).
hipError_t batch_levels(const mphf_batch* b, const uint64_t* keys, hipStream_t s) {
    hipError_t e;
    if ((e = launch_batch_reset(b->queue, b->fail32, s)) != hipSuccess) return e;
    if ((e = launch_batch_build(keys, b->offsets, b->order, b->nsets, b->hist, b->queue, b->scratch, b->region_w, b->gamma,
                                b->seeds, b->D, BATCH_LEFT_CAP, b->region, b->sec, b->sreg_base, b->sets, b->levels,
                                b->max_m, b->cfg, b->grid, s)) != hipSuccess)
        return e;
    return launch_batch_tally(b->sets, b->nsets, b->left32, b->sec32, b->fail32, s);
}

mphf_status batch_failure(uint64_t word) {
    const uint32_t bad = (uint32_t)word, first_bad = (uint32_t)(word >> 32);
    if (bad & 4u) return fail(MPHF_E_DEVICE, "set " + std::to_string(first_bad) + " outgrew its region");
    if (bad & 1u) return fail(MPHF_E_DUPLICATE_KEYS, "duplicate keys in set " + std::to_string(first_bad));
    if (bad & 2u)
        return fail(MPHF_E_INVALID, "set " + std::to_string(first_bad) +
                                        " keeps more than 2048 keys after its last level (duplicates, or too few levels)");
    return MPHF_OK;
}

mphf_status build_batch_impl(const uint64_t* keys, const uint64_t* offsets, uint64_t nsets, double gamma,
                             uint64_t seed, const mphf_opts& o, bool planned, hipStream_t s, mphf_batch** out) {
    mphf_status st = check_batch_args(offsets, nsets, gamma, o);
    if (st != MPHF_OK) return st;
    Trace tr(s);
    mphf_batch* b = new mphf_batch();
    struct Guard {   // on failure the arena frees the buffers; only the handle itself is deleted here
        mphf_batch* b;
        ~Guard() { delete b; }
    } guard{b};
    HIP_TRY(hipGetDevice(&b->device), "hipGetDevice");
    configure_pool(b->device);
    uint64_t* pin = batch_pinned(b->device);
    if (!pin) return fail(MPHF_E_NOMEM, "pinned read-back buffer");
    Arena ar(o.mem_budget, s);
    BatchMem mem(ar, b->device, !planned && o.mem_budget == 0);
    // a one-shot build first sizes each set's regions for the expected level sizes (with slack);
    // a set that outgrows them (vanishingly rare but possible) makes the batch run again with the
    // worst case.  A planned batch always takes the worst case.
    const double slack = planned ? 0.0 : 1.5 * std::exp(1.0 / gamma) * 1.0;
    if ((st = batch_setup(b, keys, offsets, nsets, gamma, seed, o, planned, slack, s, mem, pin)) != MPHF_OK) return st;
    tr.mark("batch setup", (long)b->nkeys);
    if (!planned) {
        if (b->nkeys && !keys) return fail(MPHF_E_INVALID, "keys is NULL");
        HIP_TRY(batch_levels(b, keys, s), "batch levels");
        HIP_TRY(hipMemcpyAsync(pin + 5, b->fail32, 8, hipMemcpyDeviceToHost, s), "read back");
        HIP_TRY(hipStreamSynchronize(s), "batch sync");
        if (((uint32_t)pin[5] & 4u) && !((uint32_t)pin[5] & 3u)) {
            for (void* p : b->mem) ar.release(p);
            b->mem.clear();
            if ((st = batch_setup(b, keys, offsets, nsets, gamma, seed, o, false, 0.0, s, mem, pin)) != MPHF_OK)
                return st;
            HIP_TRY(batch_levels(b, keys, s), "batch levels");
            b->retried = true;
        }
        const uint64_t S1 = nsets + 1;
        uint64_t *spre, *lpre, *tiles;
        auto lay = [&](Carver& c) {
            spre = c.take<uint64_t>(S1);
            lpre = c.take<uint64_t>(S1);
            tiles = c.take<uint64_t>(scan_tmp_tiles(S1));
        };
        if ((st = mem.transient(lay, "pack prefixes")) != MPHF_OK) return st;
        HIP_TRY(launch_exclusive_scan(b->sec32, spre, S1, tiles, s), "sector prefix");
        HIP_TRY(launch_exclusive_scan(b->left32, lpre, S1, tiles, s), "fallback prefix");
        HIP_TRY(hipMemcpyAsync(pin + 5, b->fail32, 8, hipMemcpyDeviceToHost, s), "read back");
        HIP_TRY(hipMemcpyAsync(pin + 6, spre + nsets, 8, hipMemcpyDeviceToHost, s), "read back");
        HIP_TRY(hipMemcpyAsync(pin + 7, lpre + nsets, 8, hipMemcpyDeviceToHost, s), "read back");
        HIP_TRY(hipStreamSynchronize(s), "batch sync");
        tr.mark("batch levels", (long)b->grid);
        if ((st = batch_failure(pin[5])) != MPHF_OK) return st;
        b->nsec = pin[6];
        b->nleft = pin[7];
        uint32_t* dsec;
        uint64_t* dleft;
        auto lay4 = [&](Carver& c) {
            dsec = c.take<uint32_t>((b->nsec + 1) * SEC_WORDS);
            dleft = c.take<uint64_t>(b->nleft + 1);
        };
        if ((st = mem.own(b, lay4, "batch structure")) != MPHF_OK) return st;
        HIP_TRY(launch_batch_pack(b->sec, b->sets, nsets, spre, lpre, b->scratch, dsec, dleft, s), "pack");
        HIP_TRY(launch_batch_heads(b->sets, b->levels, b->D, nsets, b->heads, b->lev, b->aux, s), "heads");
        HIP_TRY(hipStreamSynchronize(s), "batch final sync");
        tr.mark("batch structure");
        b->sec = dsec;
        b->left = dleft;
        // the borrowed temporaries go back with the workspace lock
        b->scratch = b->region = nullptr;
        b->order = nullptr;
        b->region_w = b->sreg_base = nullptr;
        b->queue = nullptr;
        b->fail32 = b->left32 = b->sec32 = nullptr;
        b->offsets = nullptr;
    } else {
        HIP_TRY(hipStreamSynchronize(s), "plan sync");
    }
    for (void* p : b->mem) ar.keep(p);
    guard.b = nullptr;
    *out = b;
    return MPHF_OK;
}

mphf_status batch_totals_of(mphf_batch* b, hipStream_t s) {
    // sum of the sets' bits, their fallback keys and sectors (a planned batch: after a rebuild)
    std::vector<BatchSet> hs(b->nsets);
    HIP_TRY(hipMemcpyAsync(hs.data(), b->sets, b->nsets * sizeof(BatchSet), hipMemcpyDeviceToHost, s), "copy sets");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    uint64_t tb = 0, tl = 0, ts = 0;
    for (const BatchSet& x : hs) {
        tb += x.bits;
        tl += x.nleft;
        ts += (x.bits + SEC_BITS - 1) / SEC_BITS;
    }
    b->total_bits = tb;
    b->used_left = tl;
    b->used_sec = ts;
    return MPHF_OK;
}

}  // namespace

extern "C" {

mphf_status mphf_build_batch(const uint64_t* keys, const uint64_t* offsets, uint64_t nsets, double gamma,
                             uint64_t seed, const mphf_opts* opts, void* stream, mphf_batch_t** out) {
    if (!out) return fail(MPHF_E_INVALID, "out is NULL");
    *out = nullptr;
    mphf_opts o;
    if (opts) o = *opts;
    else mphf_default_opts(&o);
    mphf_status st = build_batch_impl(keys, offsets, nsets, gamma, seed, o, false, (hipStream_t)stream, out);
    if (st == MPHF_OK && (st = batch_totals_of(*out, (hipStream_t)stream)) != MPHF_OK) {
        free_batch(*out);
        *out = nullptr;
    }
    return st;
}

mphf_status mphf_batch_plan(const uint64_t* offsets, uint64_t nsets, double gamma, uint64_t seed,
                            const mphf_opts* opts, void* stream, mphf_batch_t** out) {
    if (!out) return fail(MPHF_E_INVALID, "out is NULL");
    *out = nullptr;
    mphf_opts o;
    if (opts) o = *opts;
    else mphf_default_opts(&o);
    return build_batch_impl(nullptr, offsets, nsets, gamma, seed, o, true, (hipStream_t)stream, out);
}

mphf_status mphf_batch_rebuild(mphf_batch_t* b, const uint64_t* keys, void* stream) {
    if (!b) return fail(MPHF_E_INVALID, "handle is NULL");
    if (!b->planned) return fail(MPHF_E_INVALID, "the batch was not planned");
    if (b->nkeys && !keys) return fail(MPHF_E_INVALID, "keys is NULL");
    const hipStream_t s = (hipStream_t)stream;
    HIP_TRY(batch_levels(b, keys, s), "batch levels");
    HIP_TRY(launch_batch_heads(b->sets, b->levels, b->D, b->nsets, b->heads, b->lev, b->aux, s), "heads");
    HIP_TRY(b->uses.note(s), "rebuild event");
    return MPHF_OK;
}

mphf_status mphf_batch_status(mphf_batch_t* b, void* stream) {
    if (!b) return fail(MPHF_E_INVALID, "handle is NULL");
    if (!b->planned) return MPHF_OK;
    uint64_t* pin = batch_pinned(b->device);
    if (!pin) return fail(MPHF_E_NOMEM, "pinned read-back buffer");
    HIP_TRY(hipMemcpyAsync(pin, b->fail32, 8, hipMemcpyDeviceToHost, (hipStream_t)stream), "read back");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream), "sync");
    mphf_status st = batch_failure(pin[0]);
    if (st != MPHF_OK) return st;
    return batch_totals_of(b, (hipStream_t)stream);
}

mphf_status mphf_batch_lookup(const mphf_batch_t* b, const uint64_t* set_ids, const uint64_t* keys,
                              uint64_t n, uint64_t* out, void* stream) {
    if (!b) return fail(MPHF_E_INVALID, "handle is NULL");
    if (!n) return MPHF_OK;
    if (!set_ids || !keys || !out || !is_device_ptr(set_ids) || !is_device_ptr(keys) || !is_device_ptr(out))
        return fail(MPHF_E_INVALID, "set_ids, keys and out must be device memory");
    HIP_TRY(launch_batch_lookup(set_ids, keys, n, out, b->heads, b->lev, b->aux, b->D, b->nsets, b->sec, b->left,
                                b->seeds, (hipStream_t)stream),
            "batch lookup");
    HIP_TRY(b->uses.note((hipStream_t)stream), "batch lookup event");
    return MPHF_OK;
}

mphf_status mphf_batch_set_info(const mphf_batch_t* b, uint64_t set, mphf_set_info_t* info) {
    if (!b || !info) return fail(MPHF_E_INVALID, "NULL argument");
    if (set >= b->nsets) return fail(MPHF_E_INVALID, "no such set");
    BatchSet bs;
    std::vector<BatchLevel> lv(b->D);
    HIP_TRY(hipMemcpy(&bs, b->sets + set, sizeof(bs), hipMemcpyDeviceToHost), "copy set");
    HIP_TRY(hipMemcpy(lv.data(), b->levels + set * b->D, sizeof(BatchLevel) * b->D, hipMemcpyDeviceToHost),
            "copy levels");
    std::memset(info, 0, sizeof(*info));
    info->n = bs.n;
    info->num_levels = bs.nlev;
    info->n_fallback = bs.nleft;
    info->total_bits = bs.bits;
    for (uint32_t d = 0; d < bs.nlev; ++d) {
        info->level_n[d] = lv[d].n;
        info->level_m[d] = lv[d].m;
        info->level_offset[d] = lv[d].off;
    }
    return MPHF_OK;
}

mphf_status mphf_batch_export_set(const mphf_batch_t* b, uint64_t set, uint64_t* words, uint64_t nwords,
                                  uint64_t* fallback_keys, uint64_t nfb) {
    if (!b) return fail(MPHF_E_INVALID, "handle is NULL");
    if (set >= b->nsets) return fail(MPHF_E_INVALID, "no such set");
    BatchSet bs;
    HIP_TRY(hipMemcpy(&bs, b->sets + set, sizeof(bs), hipMemcpyDeviceToHost), "copy set");
    if ((words && nwords != bs.bits / 64) || (fallback_keys && nfb != bs.nleft))
        return fail(MPHF_E_INVALID, "export sizes differ from the set's");
    if (words && nwords) {
        // the set's bits are words 1..15 of each of its sectors
        const uint64_t ns = (bs.bits + SEC_BITS - 1) / SEC_BITS;
        std::vector<uint32_t> secs(ns * SEC_WORDS);
        HIP_TRY(hipMemcpy(secs.data(), b->sec + bs.sec_base * SEC_WORDS, secs.size() * 4, hipMemcpyDeviceToHost),
                "copy sectors");
        uint32_t* w32 = (uint32_t*)words;
        for (uint64_t i = 0; i < 2 * nwords; ++i) w32[i] = secs[(i / 15) * SEC_WORDS + 1 + i % 15];
    }
    if (fallback_keys && nfb)
        HIP_TRY(hipMemcpy(fallback_keys, b->left + bs.left_off, nfb * 8, hipMemcpyDeviceToHost), "copy fallback");
    return MPHF_OK;
}

mphf_status mphf_batch_export_sectors(const mphf_batch_t* b, uint64_t set, uint32_t* sectors, uint64_t nsectors) {
    if (!b || !sectors) return fail(MPHF_E_INVALID, "NULL argument");
    if (set >= b->nsets) return fail(MPHF_E_INVALID, "no such set");
    BatchSet bs;
    HIP_TRY(hipMemcpy(&bs, b->sets + set, sizeof(bs), hipMemcpyDeviceToHost), "copy set");
    if (nsectors != (bs.bits + SEC_BITS - 1) / SEC_BITS) return fail(MPHF_E_INVALID, "export size differs");
    if (nsectors)
        HIP_TRY(hipMemcpy(sectors, b->sec + bs.sec_base * SEC_WORDS, nsectors * SEC_WORDS * 4, hipMemcpyDeviceToHost),
                "copy sectors");
    return MPHF_OK;
}

mphf_status mphf_batch_totals(const mphf_batch_t* b, uint64_t* nsets, uint64_t* nkeys, uint64_t* total_bits,
                              double* bits_per_key) {
    if (!b) return fail(MPHF_E_INVALID, "handle is NULL");
    if (nsets) *nsets = b->nsets;
    if (nkeys) *nkeys = b->nkeys;
    if (total_bits) *total_bits = b->total_bits;
    if (bits_per_key) {
        // the packed structure: lookup sectors, 16-byte heads and fallback keys
        const double bits = 512.0 * (double)b->used_sec + 128.0 * (double)b->nsets + 64.0 * (double)b->used_left;
        *bits_per_key = b->nkeys ? bits / (double)b->nkeys : 0.0;
    }
    return MPHF_OK;
}

void mphf_batch_destroy(mphf_batch_t* b) { free_batch(b); }

}  // extern "C"
