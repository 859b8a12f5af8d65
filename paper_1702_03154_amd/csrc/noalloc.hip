// The hash-set partition of mphf_partition_sets without any device allocation, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// Its scratch (per-set counts, per-set cursors and the scan's tile sums) lives in `scratch`, a
// fixed device array of this library sized for 2^16 sets.  Host code never passes the array's name
// to a kernel or a copy: that name is a host-side stand-in, not a device address.  The address is
// taken once per device with hipGetSymbolAddress (the device current) and kept per device; every
// call on that device shares the array, so calls that overlap on one device race.
#include <mutex>

#include "api_internal.h"
#include "internal.h"
#include "mphf.h"

using namespace mphfk;

namespace {

constexpr uint32_t NOALLOC_MAX_BITS = 16;
constexpr uint64_t NB_MAX = 1ull << NOALLOC_MAX_BITS;
constexpr uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }
// counts: nb + 1 u32; cursors: nb u64; tiles: the scan's per-tile sums (u64)
constexpr uint64_t COUNTS_OFF = 0;
constexpr uint64_t CURSOR_OFF = COUNTS_OFF + align256(4 * (NB_MAX + 1));
constexpr uint64_t TILES_OFF = CURSOR_OFF + align256(8 * NB_MAX);
constexpr uint64_t TILES_WORDS = 64;
constexpr uint64_t SCRATCH_BYTES = TILES_OFF + 8 * TILES_WORDS;   // 787,200 bytes

}  // namespace

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

std::mutex g_mu;
unsigned char* g_scratch[64] = {};

// The device address of `scratch` on the current device (taken on the first call there).
mphf_status scratch_of_current_device(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return mphf_api::hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return mphf_api::set_error(MPHF_E_INVALID, "device index beyond 63");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return mphf_api::hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                              "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = (unsigned char*)p;
    }
    *out = g_scratch[dev];
    return MPHF_OK;
}

}  // namespace

extern "C" {

mphf_status mphf_partition_sets_noalloc(const uint64_t* keys, uint64_t n, uint32_t bits, uint64_t seed,
                                        uint64_t* out, uint64_t* offsets, void* stream) {
    if (bits < 1 || bits > NOALLOC_MAX_BITS)
        return mphf_api::set_error(MPHF_E_INVALID, "bits must be 1..16 (the fixed scratch holds 2^16 sets)");
    if (!offsets || !mphf_api::device_ptr(offsets) ||
        (n && (!keys || !out || !mphf_api::device_ptr(keys) || !mphf_api::device_ptr(out))))
        return mphf_api::set_error(MPHF_E_INVALID, "keys, out and offsets must be device memory");
    const uint64_t nb = 1ull << bits;
    if (scan_tmp_tiles(nb + 1) > TILES_WORDS)
        return mphf_api::set_error(MPHF_E_INVALID, "scan tiles exceed the fixed scratch");
    unsigned char* base = nullptr;
    mphf_status st = scratch_of_current_device(&base);
    if (st != MPHF_OK) return st;
    uint32_t* counts = (uint32_t*)(base + COUNTS_OFF);
    unsigned long long* cursor = (unsigned long long*)(base + CURSOR_OFF);
    uint64_t* tiles = (uint64_t*)(base + TILES_OFF);
    // counts are cleared by a kernel, the cursors copied from the offsets: nothing read from an
    // earlier call's contents
    hipError_t e = launch_set_partition(keys, n, seed, bits, counts, offsets, cursor, tiles, out, (hipStream_t)stream);
    if (e != hipSuccess) return mphf_api::hip_error(e, "partition");
    return MPHF_OK;
}

}  // extern "C"
