// k-mer keys for the bioinformatics workload the method targets (de Bruijn graph nodes, Section 1):
// canonical k-mers of a 2-bit packed DNA sequence, the first occurrence of every distinct key in
// sequence order, and a hash partition of a key set into independent sets for the batched build.
//
// Sequence layout: base i is bits (63 - 2 (i mod 32)) .. (62 - 2 (i mod 32)) of word i / 32, with
// A = 0, C = 1, G = 2, T = 3 (the first base of a word is its most significant pair).  The forward
// k-mer at p packs bases p .. p+k-1 with the first base most significant (2k bits); its reverse
// complement reverses the bases and complements each (x -> 3 - x, i.e. x XOR 3); the canonical
// k-mer is the smaller of the two.
#include "internal.h"

namespace mphfk {

namespace {

constexpr int KT = 256;

__device__ __forceinline__ uint64_t reverse_pairs(uint64_t x) {
    // reverse the order of the 32 two-bit groups of x
    x = ((x >> 2) & 0x3333333333333333ull) | ((x & 0x3333333333333333ull) << 2);
    x = ((x >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((x & 0x0F0F0F0F0F0F0F0Full) << 4);
    x = ((x >> 8) & 0x00FF00FF00FF00FFull) | ((x & 0x00FF00FF00FF00FFull) << 8);
    x = ((x >> 16) & 0x0000FFFF0000FFFFull) | ((x & 0x0000FFFF0000FFFFull) << 16);
    return (x >> 32) | (x << 32);
}

__global__ void __launch_bounds__(KT)
k_kmers(const uint64_t* __restrict__ seq, uint64_t npos, uint32_t k, uint64_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * KT;
    const uint32_t drop = 64 - 2 * k;
    for (uint64_t p = (uint64_t)blockIdx.x * KT + threadIdx.x; p < npos; p += stride) {
        const uint64_t w = p >> 5;
        const uint32_t o = (uint32_t)(p & 31);
        uint64_t win = seq[w] << (2 * o);                       // bases p .. p+31-o at the top
        if (o + k > 32) win |= seq[w + 1] >> (64 - 2 * o);      // the k-mer spans the next word
        const uint64_t fwd = win >> drop;
        // complement every group, reverse the 32 groups; the k-mer's k groups land on top
        const uint64_t rc = reverse_pairs(~fwd) >> drop;
        out[p] = fwd < rc ? fwd : rc;
    }
}

// Each key that occurs more than once in the sorted array, once (at the start of its run).
__global__ void __launch_bounds__(KT)
k_repeated(const uint64_t* __restrict__ sorted, uint64_t n, uint64_t* __restrict__ out, uint64_t cap,
           unsigned long long* __restrict__ count) {
    const uint64_t stride = (uint64_t)gridDim.x * KT;
    for (uint64_t i = (uint64_t)blockIdx.x * KT + threadIdx.x; i + 1 < n; i += stride) {
        if (sorted[i] == sorted[i + 1] && (i == 0 || sorted[i - 1] != sorted[i])) {
            const unsigned long long j = atomicAdd(count, 1ull);
            if (j < cap) out[j] = sorted[i];
        }
    }
}

__device__ __forceinline__ int64_t find_sorted(const uint64_t* __restrict__ a, uint64_t n, uint64_t x) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo < n && a[lo] == x ? (int64_t)lo : -1;
}

// first[j] = the smallest position of repeated key j (first[] starts at all ones).
__global__ void __launch_bounds__(KT)
k_first_pos(const uint64_t* __restrict__ keys, uint64_t n, const uint64_t* __restrict__ rep, uint64_t nrep,
            unsigned long long* __restrict__ first) {
    const uint64_t stride = (uint64_t)gridDim.x * KT;
    for (uint64_t p = (uint64_t)blockIdx.x * KT + threadIdx.x; p < n; p += stride) {
        const int64_t j = find_sorted(rep, nrep, keys[p]);
        if (j >= 0) atomicMin(&first[j], (unsigned long long)p);
    }
}

// Positions that repeat an earlier key.
__global__ void __launch_bounds__(KT)
k_later_pos(const uint64_t* __restrict__ keys, uint64_t n, const uint64_t* __restrict__ rep, uint64_t nrep,
            const unsigned long long* __restrict__ first, uint64_t* __restrict__ out, uint64_t cap,
            unsigned long long* __restrict__ count) {
    const uint64_t stride = (uint64_t)gridDim.x * KT;
    for (uint64_t p = (uint64_t)blockIdx.x * KT + threadIdx.x; p < n; p += stride) {
        const int64_t j = find_sorted(rep, nrep, keys[p]);
        if (j >= 0 && first[j] != p) {
            const unsigned long long i = atomicAdd(count, 1ull);
            if (i < cap) out[i] = p;
        }
    }
}

// out[p - (removed positions below p)] = keys[p] for every kept p < n (removed: sorted positions).
__global__ void __launch_bounds__(KT)
k_drop_positions(const uint64_t* __restrict__ keys, uint64_t n, const uint64_t* __restrict__ removed,
                 uint64_t nrem, uint64_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * KT;
    for (uint64_t p = (uint64_t)blockIdx.x * KT + threadIdx.x; p < n; p += stride) {
        uint64_t lo = 0, hi = nrem;   // removed positions below p
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (removed[mid] < p) lo = mid + 1; else hi = mid;
        }
        if (lo < nrem && removed[lo] == p) continue;
        out[p - lo] = keys[p];
    }
}

// Hash partition: the set of key x is the top `bits` bits of fmix64(x XOR seed).
__device__ __forceinline__ uint32_t set_of(uint64_t x, uint64_t seed, uint32_t bits) {
    return (uint32_t)(fmix64(x ^ seed) >> (64 - bits));
}

__global__ void __launch_bounds__(KT)
k_set_counts(const uint64_t* __restrict__ keys, uint64_t n, uint64_t seed, uint32_t bits,
             uint32_t* __restrict__ counts) {
    extern __shared__ uint32_t lh[];
    const uint32_t nb = 1u << bits;
    for (uint32_t b = threadIdx.x; b < nb; b += KT) lh[b] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * KT;
    for (uint64_t i = (uint64_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride)
        atomicAdd(&lh[set_of(keys[i], seed, bits)], 1u);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += KT)
        if (lh[b]) atomicAdd(&counts[b], lh[b]);
}

__global__ void __launch_bounds__(KT)
k_set_counts_global(const uint64_t* __restrict__ keys, uint64_t n, uint64_t seed, uint32_t bits,
                    uint32_t* __restrict__ counts) {
    const uint64_t stride = (uint64_t)gridDim.x * KT;
    for (uint64_t i = (uint64_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride)
        atomicAdd(&counts[set_of(keys[i], seed, bits)], 1u);
}

__global__ void __launch_bounds__(KT)
k_set_scatter(const uint64_t* __restrict__ keys, uint64_t n, uint64_t seed, uint32_t bits,
              unsigned long long* __restrict__ cursor, uint64_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * KT;
    for (uint64_t i = (uint64_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) {
        const uint64_t x = keys[i];
        out[atomicAdd(&cursor[set_of(x, seed, bits)], 1ull)] = x;
    }
}

__global__ void __launch_bounds__(KT)
k_set_ids(const uint64_t* __restrict__ keys, uint64_t n, uint64_t seed, uint32_t bits, uint64_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * KT;
    for (uint64_t i = (uint64_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride)
        out[i] = set_of(keys[i], seed, bits);
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

unsigned grid_of(uint64_t n) {
    uint64_t g = (n + 4 * KT - 1) / (4 * KT);
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_kmers(const uint64_t* seq, uint64_t npos, uint32_t k, uint64_t* out, hipStream_t s) {
    if (!npos) return hipSuccess;
    hipLaunchKernelGGL(k_kmers, dim3(grid_of(npos)), dim3(KT), 0, s, seq, npos, k, out);
    return hipGetLastError();
}

hipError_t launch_repeated(const uint64_t* sorted, uint64_t n, uint64_t* out, uint64_t cap,
                           unsigned long long* count, hipStream_t s) {
    if (n < 2) return hipSuccess;
    hipLaunchKernelGGL(k_repeated, dim3(grid_of(n)), dim3(KT), 0, s, sorted, n, out, cap, count);
    return hipGetLastError();
}

hipError_t launch_first_pos(const uint64_t* keys, uint64_t n, const uint64_t* rep, uint64_t nrep,
                            unsigned long long* first, hipStream_t s) {
    if (!n || !nrep) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_of(nrep)), dim3(KT), 0, s, first, nrep, ~0ull);
    hipLaunchKernelGGL(k_first_pos, dim3(grid_of(n)), dim3(KT), 0, s, keys, n, rep, nrep, first);
    return hipGetLastError();
}

hipError_t launch_later_pos(const uint64_t* keys, uint64_t n, const uint64_t* rep, uint64_t nrep,
                            const unsigned long long* first, uint64_t* out, uint64_t cap, unsigned long long* count,
                            hipStream_t s) {
    if (!n || !nrep) return hipSuccess;
    hipLaunchKernelGGL(k_later_pos, dim3(grid_of(n)), dim3(KT), 0, s, keys, n, rep, nrep, first, out, cap, count);
    return hipGetLastError();
}

hipError_t launch_drop_positions(const uint64_t* keys, uint64_t n, const uint64_t* removed, uint64_t nrem,
                                 uint64_t* out, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_drop_positions, dim3(grid_of(n)), dim3(KT), 0, s, keys, n, removed, nrem, out);
    return hipGetLastError();
}

hipError_t launch_set_partition(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t bits, uint32_t* counts,
                                uint64_t* offsets, unsigned long long* cursor, uint64_t* tiles, uint64_t* out,
                                hipStream_t s) {
    const uint32_t nb = 1u << bits;
    hipError_t e = launch_zero32(counts, nb + 1, s);
    if (e != hipSuccess) return e;
    if (n && nb <= 16384)
        hipLaunchKernelGGL(k_set_counts, dim3(grid_of(n)), dim3(KT), nb * 4, s, keys, n, seed, bits, counts);
    else if (n)
        hipLaunchKernelGGL(k_set_counts_global, dim3(grid_of(n)), dim3(KT), 0, s, keys, n, seed, bits, counts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_exclusive_scan(counts, offsets, nb + 1, tiles, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(cursor, offsets, 8ull * nb, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    if (n) hipLaunchKernelGGL(k_set_scatter, dim3(grid_of(n)), dim3(KT), 0, s, keys, n, seed, bits, cursor, out);
    return hipGetLastError();
}

hipError_t launch_set_ids(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t bits, uint64_t* out,
                          hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_set_ids, dim3(grid_of(n)), dim3(KT), 0, s, keys, n, seed, bits, out);
    return hipGetLastError();
}

}  // namespace mphfk
