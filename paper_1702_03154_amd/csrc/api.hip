// Host runtime and C ABI: the level driver of the build (Algorithm 1), the fallback table,
// the rank table and the lookup entry points.  Every step of the method runs in the kernels of
// kernels.hip; the host only sizes levels, allocates, and reads one count back per level.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "mphf.h"

using namespace mphfk;

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
    uint64_t total_bits = 0;
    uint64_t total_words = 0;
    uint64_t* words = nullptr;
    uint64_t* rank = nullptr;
    uint64_t nrank = 0;
    uint32_t rank_shift = 9;
    uint64_t* fb_keys = nullptr;
    uint64_t nfb = 0;
    DevLevel* dlev = nullptr;
    std::vector<uint64_t*> coll;
    uint64_t peak_bytes = 0;
};

namespace {

thread_local std::string g_err;

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

// Device memory of one build: every buffer is released when the builder goes out of scope
// unless it was handed to the finished function.  Tracks the bytes held against mem_budget.
class Arena {
  public:
    explicit Arena(uint64_t budget) : budget_(budget) {}
    ~Arena() {
        for (auto& b : bufs_)
            if (b.first) (void)hipFree(b.first);
    }
    template <typename T>
    mphf_status alloc(T** p, uint64_t count, const char* what) {
        *p = nullptr;
        const uint64_t bytes = count * sizeof(T);
        if (!bytes) return MPHF_OK;
        if (budget_ && held_ + bytes > budget_)
            return fail(MPHF_E_NOMEM, std::string(what) + ": mem_budget exceeded");
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, bytes);
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
    void release(void* p) {   // free now
        if (!p) return;
        for (auto& b : bufs_)
            if (b.first == p) {
                (void)hipFree(p);
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
    uint64_t budget_, held_ = 0, peak_ = 0;
    std::vector<std::pair<void*, uint64_t>> bufs_;
};

void free_handle(mphf* h) {
    if (!h) return;
    (void)hipFree(h->words);
    (void)hipFree(h->rank);
    (void)hipFree(h->fb_keys);
    (void)hipFree(h->dlev);
    for (uint64_t* c : h->coll) (void)hipFree(c);
    delete h;
}

mphf_status check_opts(const mphf_opts& o) {
    if (o.max_levels < 1 || o.max_levels > MPHF_MAX_LEVELS)
        return fail(MPHF_E_INVALID, "max_levels must be in 1..64");
    if (o.rank_sample != 512 && o.rank_sample != 1024)
        return fail(MPHF_E_INVALID, "rank_sample must be 512 or 1024");
    if (o.flags) return fail(MPHF_E_INVALID, "flags must be 0");
    return MPHF_OK;
}

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
    struct Guard {
        mphf* h;
        ~Guard() { free_handle(h); }
    } guard{h};
    HIP_TRY(hipGetDevice(&h->device), "hipGetDevice");
    h->n = n;
    h->gamma = gamma;
    h->seed = seed;
    h->opts = opts;
    h->rank_shift = opts.rank_sample == 1024 ? 10 : 9;
    uint64_t seeds[MPHF_MAX_LEVELS];
    level_seeds(seed, opts.max_levels, seeds);

    Arena ar(opts.mem_budget);
    const uint64_t m0 = level_size(gamma, n);
    const uint64_t w0 = (m0 + 63) / 64;

    // The concatenated A: reserve the expected gamma e^{1/gamma} N bits (Section 2.3) plus slack;
    // grown by copying in the rare case the levels need more.
    uint64_t cap_words = 0;
    uint64_t* words = nullptr;
    {
        const double expect = gamma * std::exp(1.0 / gamma) * (double)n;
        cap_words = (uint64_t)(expect * 1.02 / 64.0) + 2 * (uint64_t)opts.max_levels + 64;
        if (cap_words < w0 + 1) cap_words = w0 + 1;
        if ((st = ar.alloc(&words, cap_words, "A")) != MPHF_OK) return st;
    }
    uint64_t* W = nullptr;                 // working A/C pairs of the level being filled
    unsigned long long* counters = nullptr;  // [0..63] weights, [64..127] survivor counts, [128] dup flag
    if ((st = ar.alloc(&W, 2 * w0 + 2, "W")) != MPHF_OK) return st;
    if ((st = ar.alloc(&counters, 160, "counters")) != MPHF_OK) return st;
    HIP_TRY(launch_zero((uint64_t*)counters, 160, s), "zero counters");

    uint64_t* host_cnt = nullptr;
    HIP_TRY(hipHostMalloc((void**)&host_cnt, 64, hipHostMallocDefault), "hipHostMalloc");
    struct HostGuard {
        uint64_t* p;
        ~HostGuard() { (void)hipHostFree(p); }
    } hg{host_cnt};

    uint64_t* Fbuf[2] = {nullptr, nullptr};
    const uint64_t* Fin = keys;
    uint64_t nd = n;
    uint64_t off_bits = 0;
    uint64_t* leftovers = nullptr;
    uint64_t nleft = 0;

    LevelHash L{};
    if (n) {
        L = make_level_hash(seeds[0], m0, 0);
        HIP_TRY(launch_zero(W, 2 * w0, s), "zero W");
        HIP_TRY(launch_fill(keys, n, W, L, s), "fill");
    }
    for (uint32_t d = 0; nd > 0; ++d) {
        const uint64_t m = L.m;
        const uint64_t wd = (m + 63) / 64;
        uint64_t* C = nullptr;
        if (opts.keep_collisions) {
            if ((st = ar.alloc(&C, wd, "C")) != MPHF_OK) return st;
            h->coll.push_back(C);
        }
        HIP_TRY(launch_finalize(W, wd, words + off_bits / 64, C, counters + d, s), "finalize");
        HIP_TRY(hipMemcpyAsync(host_cnt, counters + d, 8, hipMemcpyDeviceToHost, s), "copy weight");
        HIP_TRY(hipStreamSynchronize(s), "level sync");
        const uint64_t weight = host_cnt[0];
        if (weight > nd) return fail(MPHF_E_DEVICE, "level weight exceeds the level's keys");
        h->level_n[d] = nd;
        h->level_m[d] = m;
        h->level_weight[d] = weight;
        h->level_offset[d] = off_bits;
        h->level_seed[d] = seeds[d];
        h->num_levels = d + 1;
        const uint64_t nnext = nd - weight;
        const uint64_t off_next = off_bits + 64 * wd;
        if (nnext == 0) {
            off_bits = off_next;
            break;
        }
        const bool last = d + 1 == opts.max_levels;
        LevelHash Ln{};
        if (!last) {
            const uint64_t mn = level_size(gamma, nnext);
            const uint64_t wn = (mn + 63) / 64;
            Ln = make_level_hash(seeds[d + 1], mn, off_next);
            if (off_next / 64 + wn > cap_words) {   // grow A
                uint64_t ncap = (off_next / 64 + wn) * 5 / 4 + 64;
                uint64_t* nw = nullptr;
                if ((st = ar.alloc(&nw, ncap, "A (grown)")) != MPHF_OK) return st;
                HIP_TRY(hipMemcpyAsync(nw, words, off_next / 8, hipMemcpyDeviceToDevice, s), "grow A");
                HIP_TRY(hipStreamSynchronize(s), "grow sync");
                ar.release(words);
                words = nw;
                cap_words = ncap;
            }
            HIP_TRY(launch_zero(W, 2 * wn, s), "zero W");
        }
        // F_{d+1}: ping-pong buffers, the one for odd levels sized by n_1 and the other by n_2
        // (sizes only shrink from level to level).
        uint64_t*& Fo = Fbuf[d & 1];
        if (!Fo && (st = ar.alloc(&Fo, nnext, "F")) != MPHF_OK) return st;
        {
            const LevelHash Ld = make_level_hash(seeds[d], m, off_bits);
            HIP_TRY(launch_filter_fill(Fin, nd, words, Ld, Fo, nnext, counters + 64 + d, W, Ln,
                                       !last, s),
                    "filter");
        }
        off_bits = off_next;
        Fin = Fo;
        nd = nnext;
        L = Ln;
        if (last) {
            leftovers = Fo;
            nleft = nnext;
            break;
        }
    }
    h->total_bits = off_bits;
    h->total_words = off_bits / 64;

    // Fallback table (Section 3, "Termination"): leftovers sorted ascending get N-|L|+1 .. N.
    if (nleft) {
        uint64_t* fb = nullptr;
        uint64_t* tmp = nullptr;
        uint32_t* rcounts = nullptr;
        uint64_t* roffs = nullptr;
        uint64_t* rtiles = nullptr;
        const uint64_t nc = radix_tmp_counts(nleft);
        if ((st = ar.alloc(&fb, nleft, "fallback keys")) != MPHF_OK) return st;
        if ((st = ar.alloc(&tmp, nleft, "sort scratch")) != MPHF_OK) return st;
        if ((st = ar.alloc(&rcounts, nc, "sort counts")) != MPHF_OK) return st;
        if ((st = ar.alloc(&roffs, nc, "sort offsets")) != MPHF_OK) return st;
        if ((st = ar.alloc(&rtiles, scan_tmp_tiles(nc), "sort tiles")) != MPHF_OK) return st;
        HIP_TRY(hipMemcpyAsync(fb, leftovers, nleft * 8, hipMemcpyDeviceToDevice, s), "copy leftovers");
        HIP_TRY(radix_sort_u64(fb, tmp, nleft, rcounts, roffs, rtiles, s), "sort");
        HIP_TRY(launch_find_duplicates(fb, nleft, counters + 128, s), "duplicates");
        HIP_TRY(hipMemcpyAsync(host_cnt, counters + 128, 8, hipMemcpyDeviceToHost, s), "copy flag");
        HIP_TRY(hipStreamSynchronize(s), "fallback sync");
        if (host_cnt[0]) return fail(MPHF_E_DUPLICATE_KEYS, "duplicate keys in the input");
        h->fb_keys = fb;
        h->nfb = nleft;
        ar.keep(fb);
    }

    // Rank table (Section 3.1).
    h->nrank = (h->total_bits + opts.rank_sample - 1) / opts.rank_sample;
    if (h->nrank) {
        uint32_t* rc = nullptr;
        uint64_t* rt = nullptr;
        if ((st = ar.alloc(&h->rank, h->nrank, "rank")) != MPHF_OK) return st;
        if ((st = ar.alloc(&rc, h->nrank, "rank counts")) != MPHF_OK) return st;
        if ((st = ar.alloc(&rt, scan_tmp_tiles(h->nrank), "rank tiles")) != MPHF_OK) return st;
        HIP_TRY(launch_rank(words, h->total_words, opts.rank_sample, h->rank, h->nrank, rc, rt, s),
                "rank");
        ar.keep(h->rank);
    }

    // Level table for the lookup kernel.
    if (h->num_levels) {
        DevLevel hl[MPHF_MAX_LEVELS];
        for (uint32_t d = 0; d < h->num_levels; ++d) {
            const LevelHash x = make_level_hash(h->level_seed[d], h->level_m[d], h->level_offset[d]);
            hl[d] = DevLevel{x.seed, x.m, x.magic, x.bit_off, x.sh1, x.sh2};
        }
        if ((st = ar.alloc(&h->dlev, h->num_levels, "level table")) != MPHF_OK) return st;
        HIP_TRY(hipMemcpyAsync(h->dlev, hl, sizeof(DevLevel) * h->num_levels, hipMemcpyHostToDevice, s),
                "copy level table");
        ar.keep(h->dlev);
    }
    h->words = words;
    ar.keep(words);
    for (uint64_t* c : h->coll) ar.keep(c);
    HIP_TRY(hipStreamSynchronize(s), "final sync");
    h->peak_bytes = ar.peak();
    guard.h = nullptr;
    *out = h;
    return MPHF_OK;
}

}  // namespace

extern "C" {

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
    HIP_TRY(launch_lookup(keys, n, out, h->dlev, h->num_levels, h->words, h->rank, h->rank_shift,
                          h->fb_keys, h->nfb, h->n, (hipStream_t)stream),
            "lookup");
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
    }
    st->n_fallback = h->nfb;
    st->total_bits = h->total_bits;
    st->rank_entries = h->nrank;
    st->structure_bytes = h->total_words * 8 + h->nrank * 8 + h->nfb * 8;
    st->bits_per_key = h->n ? (double)(h->total_bits + 64 * h->nrank + 128 * h->nfb) / (double)h->n : 0.0;
    st->peak_bytes = h->peak_bytes;
    return MPHF_OK;
}

mphf_status mphf_view(const mphf_t* h, mphf_view_t* v) {
    if (!h || !v) return fail(MPHF_E_INVALID, "NULL argument");
    v->words = h->words;
    v->rank = h->rank;
    v->fallback_keys = h->fb_keys;
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
    if (level >= h->coll.size()) return fail(MPHF_E_INVALID, "collisions were not kept (keep_collisions)");
    const uint64_t need = (h->level_m[level] + 63) / 64;
    if (nwords < need) return fail(MPHF_E_INVALID, "output too small");
    HIP_TRY(hipMemcpy(out, h->coll[level], need * 8, hipMemcpyDeviceToHost), "copy C");
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

const char* mphf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
