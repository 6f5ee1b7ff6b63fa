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

// Internal accessors of a single-grid handle (used by the closure runtime).
struct mhd_ctx;
void* mhd_internal_state(mhd_ctx* h, int* all_in_first_buffer);  // buffer 0 base
int mhd_internal_gather_first(mhd_ctx* h);     // every field into buffer 0 (stream-ordered copies)
int mhd_internal_prec(const mhd_ctx* h);
void mhd_internal_dims(const mhd_ctx* h, int n[3]);
hipStream_t mhd_internal_stream(const mhd_ctx* h);
double mhd_internal_gamma(const mhd_ctx* h);
void mhd_internal_state_changed(mhd_ctx* h);   // the state was modified outside the operators
