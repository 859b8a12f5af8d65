// Pieces of the C-ABI runtime that the serving loop shares with the single-function entry points.
#pragma once

#include <string>

#include "internal.h"
#include "mphf.h"

namespace mphf_api {

// Records `msg` as this thread's last error and returns `st`.
mphf_status set_error(mphf_status st, const std::string& msg);
// Records a HIP failure (out of memory as MPHF_E_NOMEM, else MPHF_E_DEVICE).
mphf_status hip_error(hipError_t e, const char* what);
// True if p is device (or managed) memory of the current HIP context.
bool device_ptr(const void* p);
// The lookup descriptor of a built function (device pointers owned by the handle) and its device.
void lookup_desc(const mphf_t* h, mphfk::SegDesc* d, int* device);
// The device-visible alias of a pinned host range [p, p + bytes), or null for other memory.
const void* pinned_alias(const void* p, uint64_t bytes);

}  // namespace mphf_api
