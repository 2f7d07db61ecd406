// Host-side helpers shared by the library's translation units: the
// thread-local last-error message, the HIP status check and a grow-only
// device buffer.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/dwos.h"

namespace dwos_host {

inline thread_local std::string g_last_error;

inline dwos_status fail(dwos_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

// grow-only device buffer
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { if (ptr) (void)hipFree(ptr); }
    hipError_t reserve(size_t b) {
        if (b <= bytes) return hipSuccess;
        if (ptr) { (void)hipFree(ptr); ptr = nullptr; bytes = 0; }
        hipError_t e = hipMalloc(&ptr, std::max<size_t>(b, 256));
        if (e == hipSuccess) bytes = std::max<size_t>(b, 256);
        return e;
    }
    template <class U> U* as() const { return static_cast<U*>(ptr); }
};

template <class U>
hipError_t upload(DevBuf& b, const U* host, size_t n, hipStream_t s) {
    hipError_t e = b.reserve(n * sizeof(U));
    if (e != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    e = hipMemcpyAsync(b.ptr, host, n * sizeof(U), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);   // host vectors may die after return
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace dwos_host

#define HIP_OK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::dwos_host::fail(e_ == hipErrorOutOfMemory ? DWOS_ENOMEM : DWOS_EDEVICE, \
                                     std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)
