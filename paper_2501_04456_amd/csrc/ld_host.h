// Host-side helpers shared by the C ABI files: error text, pointer kinds,
// parameter checks and the parameter tables handed to kernels.
#pragma once

#include <cstring>
#include <string>
#include <vector>

#include "ld_internal.h"

namespace ld {
namespace host {

extern thread_local std::string g_err;

// Record an error message and return the status.
ld_status fail(ld_status s, const char* fmt, ...);

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::ld::host::fail(LD_EHIP, "%s failed: %s", #expr,                    \
                                    hipGetErrorString(e_));                             \
    } while (0)

bool is_device_ptr(const void* p);
hipError_t copy_in(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t copy_out(void* dst, const void* src, size_t bytes, hipStream_t s);
ld_status check_params(const ld_params* p);
ld_status check_radius(const ld_radius* R);
void make_tables(const ld_params& p, const ld_radius& R, PairTable& tb, ExtParams& P);

// Read a caller array of `count` elements (host or device) into host memory.
template <class T>
ld_status read_host(std::vector<T>& v, const T* src, size_t count, hipStream_t s) {
    v.resize(count);
    if (is_device_ptr(src)) {
        HIP_TRY(hipMemcpyAsync(v.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        std::memcpy(v.data(), src, count * sizeof(T));
    }
    return LD_OK;
}

// Write a host array to a caller pointer (host or device); waits.
inline hipError_t put_out(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (!dst) return hipSuccess;
    if (is_device_ptr(dst)) {
        hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
        return e == hipSuccess ? hipStreamSynchronize(s) : e;
    }
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}

}  // namespace host
}  // namespace ld
