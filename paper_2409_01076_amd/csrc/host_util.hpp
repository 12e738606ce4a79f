// host_util.hpp -- error reporting shared by the translation units of the
// library: every C entry point returns a status and leaves a message for
// smrt_last_error() in a thread-local string.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

namespace smrt_host {

// Largest lattice row, in bytes of stored values.  Inside a tile the kernels
// address HBM through 32-bit byte offsets from the tile's first row (a
// one-step tile spans at most 512 rows plus its halo), so 2 MiB rows keep
// every offset below 2^31.
constexpr long long kMaxRowBytes = 1LL << 21;

extern thread_local std::string g_error;

// Records a printf-style message and returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// SMRT_EDEVICE with the HIP error string.
int hip_fail(hipError_t e, const char* what);

// SMRT_EDEVICE if the last kernel launch on this thread failed.
int after_launch(const char* what);

} // namespace smrt_host

#define HIP_TRY(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return smrt_host::hip_fail(e_, #call);                               \
    } while (0)
