// Multithreaded CPU build and lookup in the paper's own style: TEST INFRASTRUCTURE ONLY.
//
// Only the tests and the cpu_baseline leg of bench.py load this library; nothing in the product
// path does.  It shares no code with the HIP library (its hash, sizes, rank and lookup are written
// here), and it is the timed multithreaded CPU baseline: the keys of a level are split into equal
// chunks over T std::threads, which set the bits of the shared arrays A_d and C_d with atomic
// fetch-or (Section 3.2, "Parallelization"):
//
//  * level d: m_d = ceil(gamma * |F_d|) positions (Section 2.2, parameter gamma); a thread's key x
//    at p = h_d(x) mod m_d does old = fetch_or(A_d[p / 64], bit); if the bit was already set it
//    marks C_d (Section 2.2, "Collision detection"; Algorithm 2); then A_d &= ~C_d;
//  * F_{d+1} is every key whose A_d bit is 0, each thread writing its chunk's survivors to its own
//    buffer (Algorithm 1); the loop stops when no key is left or after D levels, and the leftovers,
//    sorted ascending, get the labels N - |L| + 1 .. N (Section 3, "Termination");
//  * the rank table holds the ones before every 512th position (Section 3.1), and a query walks the
//    levels until its bit is set and returns the ones before that bit plus one (Algorithm 3).
//
// The hash is the project's: h_d(x) = fmix64(x XOR s_d) (MurmurHash3's finalizer), s_d output d of
// a SplitMix64 stream seeded with the build seed; each level starts on a 64-bit word boundary of the
// concatenated array.  Results equal the sequential oracle's bit for bit (the fill does not depend
// on the order of the atomics).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

uint64_t fmix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xFF51AFD7ED558CCDull;
    x ^= x >> 33;
    x *= 0xC4CEB9FE1A85EC53ull;
    x ^= x >> 33;
    return x;
}

struct Structure {
    uint64_t n = 0;
    uint32_t levels = 0;
    uint64_t level_n[64], level_m[64], level_off[64], level_seed[64];
    std::vector<uint64_t> words;      // concatenated A
    std::vector<uint64_t> rank;       // ones before every 512th position
    std::vector<uint64_t> fallback;   // leftover keys, ascending
};

template <typename F>
void parallel(uint32_t threads, uint64_t n, F f) {
    std::vector<std::thread> ts;
    const uint64_t chunk = (n + threads - 1) / threads;
    for (uint32_t t = 0; t < threads; ++t) {
        const uint64_t a = std::min<uint64_t>(n, t * chunk), b = std::min<uint64_t>(n, a + chunk);
        ts.emplace_back([=] { f(t, a, b); });
    }
    for (auto& th : ts) th.join();
}

}  // namespace

extern "C" {

// Build over n keys; returns an opaque handle (NULL on error or duplicate keys, with *status 1 for
// bad arguments, 3 for duplicates).
void* tb_build(const uint64_t* keys, uint64_t n, double gamma, uint64_t seed, uint32_t max_levels,
               uint32_t threads, int* status) {
    *status = 0;
    if (!(gamma >= 1.0) || max_levels < 1 || max_levels > 64 || threads < 1) {
        *status = 1;
        return nullptr;
    }
    Structure* S = new Structure();
    S->n = n;
    std::vector<uint64_t> cur(keys, keys + n), next;
    uint64_t s = seed, off = 0;
    std::vector<std::vector<uint64_t>> surv(threads);
    while (!cur.empty() && S->levels < max_levels) {
        const uint32_t d = S->levels;
        s += 0x9E3779B97F4A7C15ull;   // SplitMix64 output d
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        const uint64_t sd = z ^ (z >> 31);
        const uint64_t nd = cur.size();
        const uint64_t m = (uint64_t)std::ceil(gamma * (double)nd);
        const uint64_t wd = (m + 63) / 64;
        std::vector<uint64_t> A(wd, 0), C(wd, 0);
        parallel(threads, nd, [&](uint32_t, uint64_t a, uint64_t b) {
            for (uint64_t i = a; i < b; ++i) {
                const uint64_t p = fmix64(cur[i] ^ sd) % m;
                const uint64_t bit = 1ull << (p & 63);
                if (__atomic_fetch_or(&A[p >> 6], bit, __ATOMIC_RELAXED) & bit)
                    __atomic_fetch_or(&C[p >> 6], bit, __ATOMIC_RELAXED);
            }
        });
        parallel(threads, wd, [&](uint32_t, uint64_t a, uint64_t b) {
            for (uint64_t w = a; w < b; ++w) A[w] &= ~C[w];
        });
        parallel(threads, nd, [&](uint32_t t, uint64_t a, uint64_t b) {
            std::vector<uint64_t>& o = surv[t];
            o.clear();
            for (uint64_t i = a; i < b; ++i) {
                const uint64_t p = fmix64(cur[i] ^ sd) % m;
                if (!((A[p >> 6] >> (p & 63)) & 1)) o.push_back(cur[i]);
            }
        });
        next.clear();
        for (auto& o : surv) next.insert(next.end(), o.begin(), o.end());
        S->level_n[d] = nd;
        S->level_m[d] = m;
        S->level_off[d] = off;
        S->level_seed[d] = sd;
        S->words.insert(S->words.end(), A.begin(), A.end());
        off += 64 * wd;
        S->levels = d + 1;
        cur.swap(next);
    }
    std::sort(cur.begin(), cur.end());
    for (size_t i = 1; i < cur.size(); ++i)
        if (cur[i] == cur[i - 1]) {
            *status = 3;
            delete S;
            return nullptr;
        }
    S->fallback = cur;
    const uint64_t nb = (off + 511) / 512;
    S->rank.assign(nb, 0);
    std::vector<uint64_t> blk(nb, 0);
    parallel(threads, nb, [&](uint32_t, uint64_t a, uint64_t b) {
        for (uint64_t r = a; r < b; ++r) {
            uint64_t c = 0;
            for (uint64_t w = 8 * r; w < std::min<uint64_t>(8 * r + 8, S->words.size()); ++w)
                c += (uint64_t)__builtin_popcountll(S->words[w]);
            blk[r] = c;
        }
    });
    uint64_t acc = 0;
    for (uint64_t r = 0; r < nb; ++r) {
        S->rank[r] = acc;
        acc += blk[r];
    }
    return S;
}

// Labels of n queries (Algorithm 3): 1-based rank of the first set bit, else the fallback label,
// else 0.
void tb_lookup(const void* h, const uint64_t* q, uint64_t n, uint64_t* out, uint32_t threads) {
    const Structure* S = (const Structure*)h;
    parallel(threads, n, [&](uint32_t, uint64_t a, uint64_t b) {
        for (uint64_t i = a; i < b; ++i) {
            const uint64_t x = q[i];
            uint64_t lab = 0;
            bool found = false;
            for (uint32_t d = 0; d < S->levels && !found; ++d) {
                const uint64_t g = S->level_off[d] + fmix64(x ^ S->level_seed[d]) % S->level_m[d];
                const uint64_t w = S->words[g >> 6];
                if ((w >> (g & 63)) & 1) {
                    uint64_t r = S->rank[g >> 9];
                    for (uint64_t v = (g >> 9) << 3; v < (g >> 6); ++v) r += (uint64_t)__builtin_popcountll(S->words[v]);
                    r += (uint64_t)__builtin_popcountll(w & ((1ull << (g & 63)) - 1));
                    lab = r + 1;
                    found = true;
                }
            }
            if (!found) {
                auto it = std::lower_bound(S->fallback.begin(), S->fallback.end(), x);
                if (it != S->fallback.end() && *it == x) lab = S->n - S->fallback.size() + 1 + (it - S->fallback.begin());
            }
            out[i] = lab;
        }
    });
}

// Sizes: levels, total words of A, rank entries, fallback keys.
void tb_sizes(const void* h, uint64_t* sizes) {
    const Structure* S = (const Structure*)h;
    sizes[0] = S->levels;
    sizes[1] = S->words.size();
    sizes[2] = S->rank.size();
    sizes[3] = S->fallback.size();
}

// Copies of the concatenated A, the rank table, the fallback keys and the per-level n, m, offsets.
void tb_export(const void* h, uint64_t* words, uint64_t* rank, uint64_t* fallback, uint64_t* level_n,
               uint64_t* level_m, uint64_t* level_off) {
    const Structure* S = (const Structure*)h;
    std::memcpy(words, S->words.data(), 8 * S->words.size());
    std::memcpy(rank, S->rank.data(), 8 * S->rank.size());
    std::memcpy(fallback, S->fallback.data(), 8 * S->fallback.size());
    for (uint32_t d = 0; d < S->levels; ++d) {
        level_n[d] = S->level_n[d];
        level_m[d] = S->level_m[d];
        level_off[d] = S->level_off[d];
    }
}

void tb_free(void* h) { delete (Structure*)h; }

}  // extern "C"
