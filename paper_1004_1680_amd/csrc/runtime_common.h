// Host-side helpers shared by the single-grid and batched runtimes.
#pragma once
#include <hip/hip_runtime.h>

// Record a thread-local error message (mhd_last_error) and return code.
int mhd_fail(int code, const char* fmt, ...);

#define MHD_HIP_TRY(h, expr)                                                           \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (h)->failed = true;                                                        \
            return mhd_fail(MHD_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                       \
        }                                                                              \
    } while (0)
