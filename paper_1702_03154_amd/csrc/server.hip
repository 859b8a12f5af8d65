// Serving loop: resident functions, lookup requests admitted by HBM budget and batched as they
// arrive (continuous batching).
//
// Requests wait in arrival order.  A dispatcher thread takes a free in-flight slot (its own stream,
// device memory and pinned staging), admits requests from the head of the queue while their keys
// and labels fit the slot, and enqueues the batch: one segmented lookup kernel labels every query
// against its own function (Algorithm 3).  Requests in pinned host memory are read and written by
// that kernel in place over PCIe; the others are copied into the slot's buffers and back.  A
// completer thread releases each batch's requests and slot as soon as the batch ends, in whatever
// order the batches end (a short batch does not hold its slot behind a long one launched before
// it).  With several slots, a batch formed while another runs overlaps it on the device; requests
// arriving in the meantime form the next batch.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_internal.h"

using namespace mphfk;
using mphf_api::set_error;

namespace {

constexpr int ST = 256;

// One request of a batch: its function and where its queries and labels are (the slot's device
// buffers, or the caller's pinned host arrays read and written directly over PCIe).
struct ReqDesc {
    SegDesc f;
    const uint64_t* q;
    uint64_t* out;
};

// Query i of the batch belongs to request r with seg_off[r] <= i < seg_off[r + 1]; it is the
// request's query i - seg_off[r].
__global__ void __launch_bounds__(ST)
k_lookup_segments(uint64_t n, const ReqDesc* __restrict__ segs, const uint64_t* __restrict__ seg_off,
                  uint32_t nseg) {
    const uint64_t stride = (uint64_t)gridDim.x * ST;
    uint32_t cur = 0;
    uint64_t end = 0;   // the request of the previous query covers [.., end)
    for (uint64_t i = (uint64_t)blockIdx.x * ST + threadIdx.x; i < n; i += stride) {
        if (i >= end) {   // queries of a thread only move forward: search to the right of cur
            uint32_t lo = cur, hi = nseg;   // seg_off[lo] <= i < seg_off[hi]
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (seg_off[mid] <= i) lo = mid; else hi = mid;
            }
            cur = lo;
            end = seg_off[lo + 1];
        }
        const ReqDesc d = segs[cur];
        const uint64_t j = i - seg_off[cur];
        d.out[j] = label_of(d.q[j], d.f.lev, d.f.nlev, d.f.sec, d.f.super, d.f.fbk, d.f.nfb, d.f.N);
    }
}

hipError_t launch_lookup_segments(uint64_t n, const ReqDesc* segs, const uint64_t* seg_off, uint32_t nseg,
                                  hipStream_t s) {
    if (!n || !nseg) return hipSuccess;
    uint64_t blocks = (n + 4 * ST - 1) / (4 * ST);   // four queries per thread, at most 2^24 - 1 blocks
    if (blocks > (1ull << 24) - 1) blocks = (1ull << 24) - 1;
    hipLaunchKernelGGL(k_lookup_segments, dim3((unsigned)blocks), dim3(ST), 0, s, n, segs, seg_off, nseg);
    return hipGetLastError();
}


struct Request {
    uint64_t ticket = 0;
    uint32_t fn = 0;
    const uint64_t* keys = nullptr;
    uint64_t n = 0;
    uint64_t* out = nullptr;
    const uint64_t* dkeys = nullptr;   // device aliases of pinned request arrays (else staged)
    uint64_t* dout = nullptr;
    bool done = false;
    mphf_status status = MPHF_OK;
    uint64_t batch = 0;
    uint32_t batch_requests = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint8_t* dev = nullptr;        // keys, labels, request offsets, descriptors
    uint8_t* host = nullptr;       // pinned staging of the offsets and descriptors
    bool busy = false;
    uint64_t keys = 0;
    std::vector<Request*> reqs;
};

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

}  // namespace

namespace mphf_api {

// The device-visible alias of a pinned host range [p, p + bytes), or null for other memory.
const void* pinned_alias(const void* p, uint64_t bytes) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
    hipPointerAttribute_t b;
    const void* last = (const char*)p + bytes - 1;
    if (hipPointerGetAttributes(&b, last) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (b.type != hipMemoryTypeHost || (const char*)b.devicePointer - (const char*)a.devicePointer != (ptrdiff_t)(bytes - 1))
        return nullptr;
    return a.devicePointer;
}

}  // namespace mphf_api

struct mphf_server {
    int device = 0;
    mphf_server_opts opts{};
    uint64_t slot_bytes = 0, slot_keys = 0, meta_bytes = 0;
    std::vector<SegDesc> fns;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, Request*> reqs;
    std::vector<Slot> slots;
    std::deque<int> inflight;   // slot indices of the batches on the device, in launch order
    uint64_t next_ticket = 1, next_batch = 0;
    bool stopping = false, completer_exit = false;
    mphf_server_stats stats{};
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::thread dispatcher, completer;

    double now_us() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    }
    int free_slot() const {
        for (size_t k = 0; k < slots.size(); ++k)
            if (!slots[k].busy) return (int)k;
        return -1;
    }
};

namespace {

// The batch's request offsets and descriptors in the slot's pinned staging (under the server lock:
// the function table may grow meanwhile).  A pinned request is read and written in place; any
// other request goes through the slot's device buffers at its offset.
void stage_batch(mphf_server* s, Slot& sl) {
    uint64_t* hoff = (uint64_t*)sl.host;
    ReqDesc* hdesc = (ReqDesc*)(sl.host + align256(8 * (s->opts.max_batch_requests + 1)));
    uint64_t* dkeys = (uint64_t*)sl.dev;
    uint64_t* dlab = (uint64_t*)(sl.dev + align256(8 * s->slot_keys));
    uint64_t acc = 0;
    for (size_t r = 0; r < sl.reqs.size(); ++r) {
        const Request* q = sl.reqs[r];
        hoff[r] = acc;
        hdesc[r].f = s->fns[q->fn];
        hdesc[r].q = q->dkeys ? q->dkeys : dkeys + acc;
        hdesc[r].out = q->dout ? q->dout : dlab + acc;
        acc += q->n;
    }
    hoff[sl.reqs.size()] = acc;
}

// Copies in (staged requests), one segmented lookup, copies out, completion event: all on the
// slot's stream.
hipError_t launch_batch(mphf_server* s, Slot& sl) {
    const uint32_t R = (uint32_t)sl.reqs.size();
    const uint64_t K = sl.keys;
    uint64_t* dkeys = (uint64_t*)sl.dev;
    uint64_t* dlab = (uint64_t*)(sl.dev + align256(8 * s->slot_keys));
    uint8_t* dmeta = sl.dev + 2 * align256(8 * s->slot_keys);
    const uint64_t* hoff = (const uint64_t*)sl.host;
    hipError_t e;
    for (uint32_t r = 0; r < R; ++r)
        if (!sl.reqs[r]->dkeys &&
            (e = hipMemcpyAsync(dkeys + hoff[r], sl.reqs[r]->keys, 8 * sl.reqs[r]->n, hipMemcpyHostToDevice,
                                sl.stream)) != hipSuccess)
            return e;
    if ((e = hipMemcpyAsync(dmeta, sl.host, s->meta_bytes, hipMemcpyHostToDevice, sl.stream)) != hipSuccess) return e;
    const uint64_t* doff = (const uint64_t*)dmeta;
    const ReqDesc* ddesc = (const ReqDesc*)(dmeta + align256(8 * (s->opts.max_batch_requests + 1)));
    if ((e = launch_lookup_segments(K, ddesc, doff, R, sl.stream)) != hipSuccess) return e;
    for (uint32_t r = 0; r < R; ++r)
        if (!sl.reqs[r]->dout &&
            (e = hipMemcpyAsync(sl.reqs[r]->out, dlab + hoff[r], 8 * sl.reqs[r]->n, hipMemcpyDeviceToHost,
                                sl.stream)) != hipSuccess)
            return e;
    return hipEventRecord(sl.done, sl.stream);
}

void dispatch_loop(mphf_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv.wait(lk, [&] { return (s->stopping && s->queue.empty()) || (!s->queue.empty() && s->free_slot() >= 0); });
        if (s->queue.empty()) break;
        const int k = s->free_slot();
        Slot& sl = s->slots[k];
        sl.reqs.clear();
        sl.keys = 0;
        // admit from the head of the queue while the requests fit the slot
        while (!s->queue.empty() && sl.reqs.size() < s->opts.max_batch_requests) {
            Request* r = s->queue.front();
            if (sl.keys + r->n > s->slot_keys) break;
            s->queue.pop_front();
            sl.reqs.push_back(r);
            sl.keys += r->n;
        }
        sl.busy = true;
        const uint64_t seq = s->next_batch++;
        const double t = s->now_us();
        for (Request* r : sl.reqs) {
            r->batch = seq;
            r->batch_requests = (uint32_t)sl.reqs.size();
            r->t_start = t;
        }
        uint64_t in_flight = 0;
        for (const Slot& o : s->slots)
            if (o.busy) in_flight += 16 * o.keys;
        if (in_flight > s->stats.peak_bytes_in_flight) s->stats.peak_bytes_in_flight = in_flight;
        if (sl.reqs.size() > s->stats.max_batch_requests_seen) s->stats.max_batch_requests_seen = sl.reqs.size();
        stage_batch(s, sl);
        lk.unlock();
        const hipError_t e = launch_batch(s, sl);
        lk.lock();
        if (e != hipSuccess) {
            (void)hipGetLastError();
            for (Request* r : sl.reqs) r->status = MPHF_E_DEVICE;
            (void)hipEventRecord(sl.done, sl.stream);   // completes after whatever was enqueued
        }
        s->inflight.push_back(k);
        s->cv.notify_all();
    }
}

void complete_loop(mphf_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    std::vector<int> fl;
    for (;;) {
        s->cv.wait(lk, [&] { return !s->inflight.empty() || s->completer_exit; });
        if (s->inflight.empty()) break;
        // the first batch on the device to end: its completion event, polled with the batches
        // launched meanwhile (the thread yields between rounds)
        int k = -1;
        hipError_t e = hipSuccess;
        while (k < 0) {
            fl.assign(s->inflight.begin(), s->inflight.end());
            lk.unlock();
            for (int j : fl) {
                const hipError_t q = hipEventQuery(s->slots[j].done);
                if (q != hipErrorNotReady) {
                    k = j;
                    e = q;
                    break;
                }
            }
            if (k < 0) std::this_thread::yield();
            lk.lock();
        }
        Slot& sl = s->slots[k];
        const double t = s->now_us();
        for (Request* r : sl.reqs) {
            if (e != hipSuccess) r->status = MPHF_E_DEVICE;
            r->t_done = t;
            r->done = true;
            s->stats.requests += 1;
            s->stats.keys += r->n;
        }
        s->stats.batches += 1;
        sl.reqs.clear();
        sl.keys = 0;
        sl.busy = false;
        for (auto it = s->inflight.begin(); it != s->inflight.end(); ++it)
            if (*it == k) {
                s->inflight.erase(it);
                break;
            }
        s->cv.notify_all();
    }
}

void free_server(mphf_server* s) {
    for (Slot& sl : s->slots) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
    }
    for (auto& kv : s->reqs) delete kv.second;
    delete s;
}

}  // namespace


extern "C" {

mphf_status mphf_server_default_opts(mphf_server_opts* o) {
    if (!o) return set_error(MPHF_E_INVALID, "opts is NULL");
    o->hbm_budget = 1ull << 30;
    o->max_inflight = 2;
    o->max_batch_requests = 1024;
    return MPHF_OK;
}

mphf_status mphf_server_create(const mphf_server_opts* opts, mphf_server_t** out) {
    if (!out) return set_error(MPHF_E_INVALID, "out is NULL");
    *out = nullptr;
    mphf_server_opts o;
    if (opts) o = *opts;
    else mphf_server_default_opts(&o);
    if (o.max_inflight < 1 || o.max_inflight > 8) return set_error(MPHF_E_INVALID, "max_inflight must be 1..8");
    if (o.max_batch_requests < 1 || o.max_batch_requests > 65536)
        return set_error(MPHF_E_INVALID, "max_batch_requests must be 1..65536");
    mphf_server* s = new mphf_server();
    s->opts = o;
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return mphf_api::hip_error(e, "hipGetDevice");
    }
    s->meta_bytes = align256(8 * (o.max_batch_requests + 1)) + align256(sizeof(ReqDesc) * o.max_batch_requests);
    s->slot_bytes = o.hbm_budget / o.max_inflight;
    if (s->slot_bytes < s->meta_bytes + 4096) {
        delete s;
        return set_error(MPHF_E_INVALID, "hbm_budget too small for the batch metadata");
    }
    s->slot_keys = (s->slot_bytes - s->meta_bytes - 512) / 16;
    s->slots.resize(o.max_inflight);
    for (Slot& sl : s->slots) {
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess ||
            (e = hipMalloc((void**)&sl.dev, 2 * align256(8 * s->slot_keys) + s->meta_bytes)) != hipSuccess ||
            (e = hipHostMalloc((void**)&sl.host, s->meta_bytes, hipHostMallocDefault)) != hipSuccess) {
            (void)hipGetLastError();
            free_server(s);
            return mphf_api::hip_error(e, "server setup");
        }
    }
    s->dispatcher = std::thread(dispatch_loop, s);
    s->completer = std::thread(complete_loop, s);
    *out = s;
    return MPHF_OK;
}

mphf_status mphf_server_register(mphf_server_t* s, const mphf_t* h, uint32_t* id) {
    if (!s || !h || !id) return set_error(MPHF_E_INVALID, "NULL argument");
    SegDesc d;
    int dev = 0;
    mphf_api::lookup_desc(h, &d, &dev);
    if (dev != s->device) return set_error(MPHF_E_INVALID, "the function lives on another device");
    std::lock_guard<std::mutex> g(s->mu);
    *id = (uint32_t)s->fns.size();
    s->fns.push_back(d);
    return MPHF_OK;
}

mphf_status mphf_server_submit(mphf_server_t* s, uint32_t id, const uint64_t* keys, uint64_t n, uint64_t* out,
                               uint64_t* ticket) {
    if (!s || !ticket) return set_error(MPHF_E_INVALID, "NULL argument");
    if (n && (!keys || !out)) return set_error(MPHF_E_INVALID, "keys or out is NULL");
    if (n && (mphf_api::device_ptr(keys) || mphf_api::device_ptr(out)))
        return set_error(MPHF_E_INVALID, "request arrays must be host memory");
    if (n > s->slot_keys)
        return set_error(MPHF_E_INVALID, "request larger than one batch's share of the HBM budget (" +
                                             std::to_string(s->slot_keys) + " keys)");
    std::lock_guard<std::mutex> g(s->mu);
    if (id >= s->fns.size()) return set_error(MPHF_E_INVALID, "unknown function id");
    if (s->stopping) return set_error(MPHF_E_INVALID, "the server is stopping");
    Request* r = new Request();
    r->ticket = s->next_ticket++;
    r->fn = id;
    r->keys = keys;
    r->n = n;
    r->out = out;
    if (n) {   // pinned arrays are read and written by the lookup kernel directly
        r->dkeys = (const uint64_t*)mphf_api::pinned_alias(keys, 8 * n);
        r->dout = (uint64_t*)mphf_api::pinned_alias(out, 8 * n);
    }
    r->t_submit = s->now_us();
    s->reqs[r->ticket] = r;
    if (n == 0) {   // nothing to copy or label: done at once
        r->done = true;
        r->t_start = r->t_done = r->t_submit;
        s->stats.requests += 1;
    } else {
        s->queue.push_back(r);
        s->cv.notify_all();
    }
    *ticket = r->ticket;
    return MPHF_OK;
}

mphf_status mphf_server_poll(mphf_server_t* s, uint64_t ticket, int wait, mphf_request_info* info) {
    if (!s) return set_error(MPHF_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(MPHF_E_INVALID, "unknown ticket");
    Request* r = it->second;
    if (wait) s->cv.wait(lk, [&] { return r->done; });
    if (info) {
        info->done = r->done ? 1u : 0u;
        info->batch_requests = r->batch_requests;
        info->batch = r->batch;
        info->submit_us = r->t_submit;
        info->start_us = r->t_start;
        info->done_us = r->t_done;
    }
    mphf_status st = MPHF_OK;
    if (r->done) {
        st = r->status;
        s->reqs.erase(it);
        delete r;
        if (st != MPHF_OK) return set_error(st, "the request's batch failed on the device");
    }
    return st;
}

mphf_status mphf_server_get_stats(const mphf_server_t* s, mphf_server_stats* st) {
    if (!s || !st) return set_error(MPHF_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> g(const_cast<mphf_server*>(s)->mu);
    *st = s->stats;
    return MPHF_OK;
}

void mphf_server_destroy(mphf_server_t* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stopping = true;
        s->cv.notify_all();
    }
    s->dispatcher.join();
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->completer_exit = true;
        s->cv.notify_all();
    }
    s->completer.join();
    free_server(s);
}

mphf_status mphf_host_alloc(uint64_t bytes, void** out) {
    if (!out) return set_error(MPHF_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!bytes) return MPHF_OK;
    const hipError_t e = hipHostMalloc(out, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return mphf_api::hip_error(e, "hipHostMalloc");
    }
    return MPHF_OK;
}

void mphf_host_free(void* p) {
    if (p) (void)hipHostFree(p);
}

}  // extern "C"
