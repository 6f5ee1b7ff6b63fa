// CFL time step of a caller's device state without any allocation: the
// entry point mhd_cfl_dt_noalloc (include/mhd.h).  It runs the kernels of
// mhd_cfl_dt (the FP64 max-reduction of the signal speed, section II.B; the
// CFL function of section IV.A) with their block partials, scalars and flag
// in a fixed device array of this file instead of a handle's buffers, so it
// can be called where hipMalloc cannot: under HIP graph capture, in tight
// serving loops, by harnesses that forbid allocation.
//
// The array lives in every device's global memory for the life of the
// process.  Its device address comes from hipGetSymbolAddress, once per
// device, on the first call made with that device current; host code only
// ever uses that address (the array's own name is a host-side stand-in).
// All calls on one device share the array: calls that overlap in time on
// one device (different streams, or threads) race and must be serialised by
// the caller.  Each call clears what has to start at zero with a kernel
// (no memset node, so a captured call replays correctly).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <mutex>

#include "../../include/mhd.h"
#include "mhd_kernels.h"
#include "runtime_common.h"

using namespace mhd;

namespace {

// the reduction's block count never exceeds this (cfl_blocks caps it)
constexpr int NOALLOC_BLOCKS = 4096;
// layout: partial maxima (doubles), partial flags (ints), scalar block
// (SCAL_COUNT doubles), flag block (FLAG_COUNT ints)
constexpr size_t OFF_PARTIAL = 0;
constexpr size_t OFF_BAD = OFF_PARTIAL + NOALLOC_BLOCKS * sizeof(double);
constexpr size_t OFF_SCAL = OFF_BAD + NOALLOC_BLOCKS * sizeof(int);
constexpr size_t OFF_FLAG = OFF_SCAL + SCAL_COUNT * sizeof(double);
constexpr size_t SCRATCH_BYTES = OFF_FLAG + FLAG_COUNT * sizeof(int);   // 49,200 bytes

constexpr int MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[MAX_DEVICES];     // device address of `scratch` per device

// the device address of `scratch` on the current device, looked up once
static int scratch_address(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return mhd_fail(MHD_EDEVICE, "no current HIP device");
    if (dev >= MAX_DEVICES) return mhd_fail(MHD_EDEVICE, "device %d above the %d this library tracks", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return mhd_fail(MHD_EDEVICE, "hipGetSymbolAddress of the CFL scratch array: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MHD_OK;
}

// clear the scalar and flag blocks before a reduction
__global__ void noalloc_clear_kernel(double* scal, int* flag)
{
    if (threadIdx.x < SCAL_COUNT) scal[threadIdx.x] = 0.0;
    if (threadIdx.x < FLAG_COUNT) flag[threadIdx.x] = 0;
}

// out = (dt, vmax, record) of the reduction just made
__global__ void noalloc_out_kernel(const double* scal, const int* flag, double* out)
{
    if (threadIdx.x == 0) {
        out[0] = scal[SCAL_DT];
        out[1] = scal[SCAL_VMAX];
        out[2] = (double)flag[0];
    }
}

template <typename T>
static int enqueue(const void* state, int nx, int ny, int nz, double gamma, double cfl, double* out,
                   unsigned char* base, hipStream_t s)
{
    const size_t N = (size_t)nx * ny * nz;
    const int nblk = cfl_blocks(N);
    if (nblk > NOALLOC_BLOCKS) return mhd_fail(MHD_EINVAL, "reduction of %d blocks above the scratch's %d", nblk, NOALLOC_BLOCKS);
    const T* f[8];
    for (int q = 0; q < 8; ++q) f[q] = static_cast<const T*>(state) + (size_t)q * N;
    double* partial = reinterpret_cast<double*>(base + OFF_PARTIAL);
    int* bad = reinterpret_cast<int*>(base + OFF_BAD);
    double* scal = reinterpret_cast<double*>(base + OFF_SCAL);
    int* flag = reinterpret_cast<int*>(base + OFF_FLAG);
    hipLaunchKernelGGL(noalloc_clear_kernel, dim3(1), dim3(64), 0, s, scal, flag);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_cfl<T>(f, nx, ny, nz, gamma, cfl, partial, bad, nblk, scal, flag, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(noalloc_out_kernel, dim3(1), dim3(64), 0, s, scal, flag, out);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return mhd_fail(MHD_EDEVICE, "CFL kernels: %s", hipGetErrorString(e));
    return MHD_OK;
}

extern "C" int mhd_cfl_dt_noalloc(const void* state_dev, int nx, int ny, int nz, int prec, double gamma,
                                  double cfl, double* out_dev, void* stream)
{
    if (!state_dev || !out_dev) return mhd_fail(MHD_EINVAL, "null device pointer");
    const int n[3] = { nx, ny, nz };
    for (int d = 0; d < 3; ++d)
        if (n[d] < 8 || n[d] % 4)
            return mhd_fail(MHD_EINVAL, "grid dimension %d = %d: must be >= 8 and a multiple of 4", d, n[d]);
    if (nx > 1024 || ny > 4096 || nz > 4096 || (long long)nx * ny * nz >= (1LL << 31))
        return mhd_fail(MHD_EINVAL, "grid above the limit (nx <= 1024, ny, nz <= 4096, < 2^31 cells)");
    if (prec != MHD_F32 && prec != MHD_F64) return mhd_fail(MHD_EINVAL, "precision must be MHD_F32 or MHD_F64");
    if (!(gamma > 1.0) || !isfinite(gamma)) return mhd_fail(MHD_EINVAL, "gamma must be > 1 (got %g)", gamma);
    if (!(cfl > 0.0) || !isfinite(cfl)) return mhd_fail(MHD_EINVAL, "cfl must be > 0 (got %g)", cfl);
    void* base = nullptr;
    int r = scratch_address(&base);
    if (r) return r;
    unsigned char* b = static_cast<unsigned char*>(base);
    return prec == MHD_F64 ? enqueue<double>(state_dev, nx, ny, nz, gamma, cfl, out_dev, b, (hipStream_t)stream)
                           : enqueue<float>(state_dev, nx, ny, nz, gamma, cfl, out_dev, b, (hipStream_t)stream);
}
