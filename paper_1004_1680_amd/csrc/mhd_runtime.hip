// Host runtime of the MHD library: handle lifetime, device buffers, argument
// checking and the enqueueing of the kernels behind the C ABI of mhd.h.
//
// Buffers.  Each handle owns two device allocations of 8 fields each.  Every
// operator reads the current copy of its inputs and writes the other copy
// of the fields it changes (never in place: neighbour pencils of one lane are
// another lane's output), then the per-field "current" index flips.
//
// Time step on the device.  Kernels read dt and the relaxation speed from a
// small device block; the host path writes it with a one-thread kernel
// (never hipMemsetAsync, so a HIP graph can capture a step), the device path
// writes it from the CFL reduction.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "../../include/mhd.h"
#include "mhd_kernels.h"
#include "runtime_common.h"

using namespace mhd;

static thread_local std::string g_last_error = "no error";

int mhd_fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
#define fail mhd_fail

struct mhd_ctx {
    int n[3];
    size_t N;
    double gamma;
    int prec;
    size_t esize;
    hipStream_t stream;
    int device;
    void* buf[2];
    bool own_buf;           // buf[] allocated here (false: the caller's, never freed here)
    int cur[8];
    double* scal;           // device SCAL_COUNT doubles
    int* flag;              // device FLAG_COUNT ints
    double* partial;        // reduction partials (max of cfl and diag needs)
    int* partial_bad;
    int nblk_cfl, nblk_diag;
    double* diag_out;       // device 9 doubles
    double* pinned;         // host pinned scratch (16 doubles)
    bool have_c;
    double c_host;
    bool scal_known;        // host knows what dt / c the device block holds
    // fused CFL: the last fluid operator of a step leaves the FP64 maximum
    // signal speed of the new state in cfl_acc; acc_valid while the state
    // is still the one it describes
    unsigned long long* cfl_acc;
    bool acc_valid;
    bool fuse_ok;           // grid shape allows the fused epilogue
    // reverse-half pairs M_d F_d: one fused launch each (true) or the two
    // operators in turn; same result bit for bit
    int rev_mode;           // 0 built-in choice, 1 fused, 2 the two operators
    // the middle of a step, M_z M_z F_z: one launch (1), or M_z and the fused
    // reverse pair (2); 0 the built-in choice
    int mid_mode;
    int limiter;            // slope limiter of the operators (MHD_LIMITER_*)
    int freeze;             // freezing speed of the fluid operator (MHD_FREEZE_*)
    double scal_dt, scal_c;
    bool failed;
    LaunchTuning tune;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

#define HIP_TRY MHD_HIP_TRY

static int check_handle(const mhd_ctx* h)
{
    if (!h) return fail(MHD_EINVAL, "null handle");
    if (h->failed) return fail(MHD_ESTATE, "handle failed earlier (HIP error); destroy it");
    return MHD_OK;
}

template <typename T>
static T* field_ptr(mhd_ctx* h, int f, int which)
{
    return reinterpret_cast<T*>(h->buf[which]) + (size_t)f * h->N;
}

template <typename T>
static void current_fields(mhd_ctx* h, const T* f[8])
{
    for (int q = 0; q < 8; ++q) f[q] = field_ptr<T>(h, q, h->cur[q]);
}

static int largest_chunk(int nd, long npencil, int waves_per_simd)
{
    // enough lanes to give every SIMD of the 256 CUs the waves it can hold,
    // with a chunk no shorter than 16 cells (the warm-up re-reads 6 cells)
    const long target = 256L * 4 * waves_per_simd * 64;
    int best = nd;
    for (int ch = nd; ch >= 16; --ch) {
        if (nd % ch) continue;
        best = ch;
        if (npencil * (nd / ch) >= target) break;
    }
    return best;
}

static void default_tuning(mhd_ctx* h)
{
    // the fused reverse-pair march holds two register windows: half the
    // waves per SIMD, so half the lanes fill the device
    h->tune.chunk[0] = h->tune.pair_chunk[0] = h->tune.triple_chunk[0] = 0;
    h->tune.wide = 0;
    h->tune.row_group = 0;
    for (int d = 1; d < 3; ++d) {
        const long npencil = (long)h->n[0] * h->n[3 - d];
        h->tune.chunk[d] = largest_chunk(h->n[d], npencil, 4);
        h->tune.pair_chunk[d] = largest_chunk(h->n[d], npencil, 2);
        h->tune.triple_chunk[d] = largest_chunk(h->n[d], npencil, 1);
    }
}

// built-in choice of fused reverse pairs: FP32 with van Leer's or minmod
// (measured faster at 256^3); not with MC or superbee, whose fused march
// kernels spill registers (2-3% and 34% slower than the two operators), nor
// in FP64 (the fused FP64 march runs 1 wave per SIMD)
static bool default_rev_fused(int prec, int limiter)
{
    return prec == MHD_F32 && (limiter == MHD_LIMITER_VANLEER || limiter == MHD_LIMITER_MINMOD);
}

static int sync_stream(mhd_ctx* h)
{
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return MHD_OK;
}

// ---------------------------------------------------------------------------
// lifetime
// ---------------------------------------------------------------------------

// a caller's state buffer: device memory of this device, 256-byte aligned,
// at least `bytes` long inside its allocation
static int check_user_buffer(const void* p, size_t bytes, int device, const char* name)
{
    if (reinterpret_cast<uintptr_t>(p) % 256)
        return fail(MHD_EINVAL, "%s: a state buffer must be 256-byte aligned", name);
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MHD_EINVAL, "%s: not memory known to HIP", name);
    }
    if (a.type != hipMemoryTypeDevice || a.isManaged)
        return fail(MHD_EINVAL, "%s: not device memory", name);
    if (a.device != device)
        return fail(MHD_EINVAL, "%s: memory of device %d, handle on device %d", name, a.device, device);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MHD_EINVAL, "%s: allocation range unknown", name);
    }
    if (static_cast<const char*>(p) + bytes > static_cast<const char*>(base) + size)
        return fail(MHD_EINVAL, "%s: allocation shorter than 8*nx*ny*nz elements", name);
    return MHD_OK;
}

extern "C" mhd_ctx* mhd_create_ex(int nx, int ny, int nz, double gamma, int prec, void* hip_stream,
                                   void* dev_buf_a, void* dev_buf_b)
{
    const int n[3] = { nx, ny, nz };
    for (int d = 0; d < 3; ++d)
        if (n[d] < 8 || n[d] % 4) {
            fail(MHD_EINVAL, "grid dimension %d = %d: must be >= 8 and a multiple of 4", d, n[d]);
            return nullptr;
        }
    if (nx > 1024 || ny > 4096 || nz > 4096 || (long long)nx * ny * nz >= (1LL << 31)) {
        fail(MHD_EINVAL, "grid above the limit (nx <= 1024, ny, nz <= 4096, < 2^31 cells)");
        return nullptr;
    }
    if (!(gamma > 1.0) || !isfinite(gamma)) {
        fail(MHD_EINVAL, "gamma must be > 1 (got %g)", gamma);
        return nullptr;
    }
    if (prec != MHD_F32 && prec != MHD_F64) {
        fail(MHD_EINVAL, "precision must be MHD_F32 or MHD_F64 (got %d)", prec);
        return nullptr;
    }
    if ((dev_buf_a == nullptr) != (dev_buf_b == nullptr)) {
        fail(MHD_EINVAL, "give both state buffers or neither");
        return nullptr;
    }
    mhd_ctx* h = new mhd_ctx();
    memset(h, 0, sizeof *h);
    h->n[0] = nx; h->n[1] = ny; h->n[2] = nz;
    h->N = (size_t)nx * ny * nz;
    h->gamma = gamma;
    h->prec = prec;
    h->esize = prec == MHD_F64 ? sizeof(double) : sizeof(float);
    h->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&h->device) != hipSuccess) {
        fail(MHD_EDEVICE, "no HIP device");
        delete h;
        return nullptr;
    }
    const size_t bytes = 8 * h->N * h->esize;
    h->nblk_cfl = cfl_blocks(h->N);
    h->nblk_diag = diag_blocks(h->N);
    const int npart = std::max(h->nblk_cfl, 10 * h->nblk_diag);
    if (dev_buf_a) {
        const char* a = static_cast<const char*>(dev_buf_a);
        const char* b = static_cast<const char*>(dev_buf_b);
        if (check_user_buffer(dev_buf_a, bytes, h->device, "dev_buf_a") ||
            check_user_buffer(dev_buf_b, bytes, h->device, "dev_buf_b")) {
            delete h;
            return nullptr;
        }
        if (a < b + bytes && b < a + bytes) {
            fail(MHD_EINVAL, "the two state buffers overlap");
            delete h;
            return nullptr;
        }
        h->buf[0] = dev_buf_a;
        h->buf[1] = dev_buf_b;
        h->own_buf = false;
    } else {
        h->own_buf = true;
        if (hipMalloc(&h->buf[0], bytes) != hipSuccess || hipMalloc(&h->buf[1], bytes) != hipSuccess) {
            (void)hipGetLastError();
            fail(MHD_ENOMEM, "device allocation of 2 x %zu bytes failed", bytes);
            mhd_destroy(h);
            return nullptr;
        }
    }
    bool ok = hipMalloc(&h->scal, SCAL_COUNT * sizeof(double)) == hipSuccess &&
              hipMalloc(&h->flag, FLAG_COUNT * sizeof(int)) == hipSuccess &&
              hipMalloc(&h->partial, npart * sizeof(double)) == hipSuccess &&
              hipMalloc(&h->partial_bad, h->nblk_cfl * sizeof(int)) == hipSuccess &&
              hipMalloc(&h->diag_out, 9 * sizeof(double)) == hipSuccess &&
              hipMalloc(&h->cfl_acc, (CFL_ACC_SLOTS + 1) * sizeof(unsigned long long)) == hipSuccess &&
              hipHostMalloc(&h->pinned, 16 * sizeof(double), hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        fail(MHD_ENOMEM, "device allocation of the handle's scratch failed");
        mhd_destroy(h);
        return nullptr;
    }
    ok = hipMemsetAsync(h->buf[0], 0, bytes, h->stream) == hipSuccess &&
         hipMemsetAsync(h->buf[1], 0, bytes, h->stream) == hipSuccess &&
         hipMemsetAsync(h->scal, 0, SCAL_COUNT * sizeof(double), h->stream) == hipSuccess &&
         hipMemsetAsync(h->flag, 0, FLAG_COUNT * sizeof(int), h->stream) == hipSuccess &&
         hipMemsetAsync(h->cfl_acc, 0, (CFL_ACC_SLOTS + 1) * sizeof(unsigned long long), h->stream) == hipSuccess &&
         hipStreamSynchronize(h->stream) == hipSuccess;
    if (!ok) {
        fail(MHD_EDEVICE, "device initialisation failed");
        mhd_destroy(h);
        return nullptr;
    }
    default_tuning(h);
    h->rev_mode = 0;
    h->fuse_ok = prec == MHD_F64 ? fused_cfl_possible<double>(nx) : fused_cfl_possible<float>(nx);
    h->acc_valid = false;
    return h;
}

extern "C" mhd_ctx* mhd_create(int nx, int ny, int nz, double gamma)
{
    return mhd_create_ex(nx, ny, nz, gamma, MHD_F32, nullptr, nullptr, nullptr);
}

extern "C" void mhd_destroy(mhd_ctx* h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->own_buf) {
        if (h->buf[0]) (void)hipFree(h->buf[0]);
        if (h->buf[1]) (void)hipFree(h->buf[1]);
    }
    if (h->scal) (void)hipFree(h->scal);
    if (h->flag) (void)hipFree(h->flag);
    if (h->partial) (void)hipFree(h->partial);
    if (h->partial_bad) (void)hipFree(h->partial_bad);
    if (h->diag_out) (void)hipFree(h->diag_out);
    if (h->cfl_acc) (void)hipFree(h->cfl_acc);
    if (h->pinned) (void)hipHostFree(h->pinned);
    delete h;
}

extern "C" int mhd_info(const mhd_ctx* h, int dims[3], int* prec)
{
    if (!h) return fail(MHD_EINVAL, "null handle");
    if (dims) { dims[0] = h->n[0]; dims[1] = h->n[1]; dims[2] = h->n[2]; }
    if (prec) *prec = h->prec;
    return MHD_OK;
}

// ---------------------------------------------------------------------------
// state transfer
// ---------------------------------------------------------------------------

static int reset_after_set(mhd_ctx* h)
{
    h->acc_valid = false;
    for (int q = 0; q < 8; ++q) h->cur[q] = 0;
    h->have_c = false;
    h->c_host = 0.0;
    h->scal_known = false;
    HIP_TRY(h, hipMemsetAsync(h->scal, 0, SCAL_COUNT * sizeof(double), h->stream));
    HIP_TRY(h, hipMemsetAsync(h->flag, 0, FLAG_COUNT * sizeof(int), h->stream));
    return MHD_OK;
}

extern "C" int mhd_set_state(mhd_ctx* h, const double* host, size_t n)
{
    int r = check_handle(h);
    if (r) return r;
    if (!host) return fail(MHD_EINVAL, "null host pointer");
    if (n != 8 * h->N) return fail(MHD_EINVAL, "state size %zu != 8*nx*ny*nz = %zu", n, 8 * h->N);
    HIP_TRY(h, hipSetDevice(h->device));
    if ((r = reset_after_set(h))) return r;
    if (h->prec == MHD_F64) {
        HIP_TRY(h, hipMemcpyAsync(h->buf[0], host, 8 * h->N * sizeof(double), hipMemcpyHostToDevice,
                                  h->stream));
    } else {
        double* stage = nullptr;
        if (hipMalloc(&stage, h->N * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MHD_ENOMEM, "staging allocation failed");
        }
        for (int q = 0; q < 8 && !r; ++q) {
            if (hipMemcpyAsync(stage, host + (size_t)q * h->N, h->N * sizeof(double),
                               hipMemcpyHostToDevice, h->stream) != hipSuccess ||
                launch_convert_in<float>(stage, field_ptr<float>(h, q, 0), h->N, h->stream) !=
                    hipSuccess)
                r = 1;
        }
        const hipError_t e = hipStreamSynchronize(h->stream);
        (void)hipFree(stage);
        if (r || e != hipSuccess) {
            h->failed = true;
            return fail(MHD_EDEVICE, "state upload failed");
        }
    }
    return sync_stream(h);
}

extern "C" int mhd_get_state(mhd_ctx* h, double* host, size_t n)
{
    int r = check_handle(h);
    if (r) return r;
    if (!host) return fail(MHD_EINVAL, "null host pointer");
    if (n != 8 * h->N) return fail(MHD_EINVAL, "state size %zu != 8*nx*ny*nz = %zu", n, 8 * h->N);
    HIP_TRY(h, hipSetDevice(h->device));
    if (h->prec == MHD_F64) {
        for (int q = 0; q < 8; ++q)
            HIP_TRY(h, hipMemcpyAsync(host + (size_t)q * h->N, field_ptr<double>(h, q, h->cur[q]),
                                      h->N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        return sync_stream(h);
    }
    double* stage = nullptr;
    if (hipMalloc(&stage, h->N * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MHD_ENOMEM, "staging allocation failed");
    }
    for (int q = 0; q < 8 && !r; ++q) {
        if (launch_convert_out<float>(field_ptr<float>(h, q, h->cur[q]), stage, h->N, h->stream) !=
                hipSuccess ||
            hipMemcpyAsync(host + (size_t)q * h->N, stage, h->N * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream) != hipSuccess)
            r = 1;
    }
    const hipError_t e = hipStreamSynchronize(h->stream);
    (void)hipFree(stage);
    if (r || e != hipSuccess) {
        h->failed = true;
        return fail(MHD_EDEVICE, "state download failed");
    }
    return MHD_OK;
}

extern "C" int mhd_set_state_device(mhd_ctx* h, const void* src, size_t n, int prec)
{
    int r = check_handle(h);
    if (r) return r;
    if (!src) return fail(MHD_EINVAL, "null device pointer");
    if (n != 8 * h->N) return fail(MHD_EINVAL, "state size %zu != 8*nx*ny*nz = %zu", n, 8 * h->N);
    if (prec != MHD_F32 && prec != MHD_F64) return fail(MHD_EINVAL, "bad precision %d", prec);
    HIP_TRY(h, hipSetDevice(h->device));
    if ((r = reset_after_set(h))) return r;
    const size_t n8 = 8 * h->N;
    hipError_t e;
    if (prec == h->prec)
        e = hipMemcpyAsync(h->buf[0], src, n8 * h->esize, hipMemcpyDeviceToDevice, h->stream);
    else if (prec == MHD_F64)
        e = launch_cast<double, float>((const double*)src, (float*)h->buf[0], n8, h->stream);
    else
        e = launch_cast<float, double>((const float*)src, (double*)h->buf[0], n8, h->stream);
    HIP_TRY(h, e);
    return MHD_OK;
}

extern "C" int mhd_get_state_device(mhd_ctx* h, void* dst, size_t n, int prec)
{
    int r = check_handle(h);
    if (r) return r;
    if (!dst) return fail(MHD_EINVAL, "null device pointer");
    if (n != 8 * h->N) return fail(MHD_EINVAL, "state size %zu != 8*nx*ny*nz = %zu", n, 8 * h->N);
    if (prec != MHD_F32 && prec != MHD_F64) return fail(MHD_EINVAL, "bad precision %d", prec);
    HIP_TRY(h, hipSetDevice(h->device));
    const size_t es = prec == MHD_F64 ? sizeof(double) : sizeof(float);
    for (int q = 0; q < 8; ++q) {
        char* d = (char*)dst + (size_t)q * h->N * es;
        hipError_t e;
        if (prec == h->prec)
            e = hipMemcpyAsync(d, (char*)h->buf[h->cur[q]] + (size_t)q * h->N * h->esize,
                               h->N * es, hipMemcpyDeviceToDevice, h->stream);
        else if (prec == MHD_F64)
            e = launch_cast<float, double>(field_ptr<float>(h, q, h->cur[q]), (double*)d, h->N,
                                           h->stream);
        else
            e = launch_cast<double, float>(field_ptr<double>(h, q, h->cur[q]), (float*)d, h->N,
                                           h->stream);
        HIP_TRY(h, e);
    }
    return MHD_OK;
}

// ---------------------------------------------------------------------------
// CFL and relaxation speed
// ---------------------------------------------------------------------------

template <typename T>
static hipError_t enqueue_cfl(mhd_ctx* h, double cfl, int* flag)
{
    const T* f[8];
    current_fields<T>(h, f);
    return launch_cfl<T>(f, h->n[0], h->n[1], h->n[2], h->gamma, cfl, h->partial, h->partial_bad,
                         h->nblk_cfl, h->scal, flag, h->stream);
}

extern "C" int mhd_cfl_dt(mhd_ctx* h, double cfl, double* dt_out)
{
    int r = check_handle(h);
    if (r) return r;
    if (!dt_out) return fail(MHD_EINVAL, "null dt pointer");
    if (!(cfl > 0.0) || !isfinite(cfl)) return fail(MHD_EINVAL, "cfl must be > 0 (got %g)", cfl);
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipMemsetAsync(h->flag + FLAG_SYNC, 0, sizeof(int), h->stream));
    h->scal_known = false;
    HIP_TRY(h, h->prec == MHD_F64 ? enqueue_cfl<double>(h, cfl, h->flag + FLAG_SYNC)
                                  : enqueue_cfl<float>(h, cfl, h->flag + FLAG_SYNC));
    HIP_TRY(h, hipMemcpyAsync(h->pinned, h->scal, SCAL_COUNT * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->pinned + 8, h->flag + FLAG_SYNC, sizeof(int),
                              hipMemcpyDeviceToHost, h->stream));
    if ((r = sync_stream(h))) return r;
    int bad;
    memcpy(&bad, h->pinned + 8, sizeof(int));
    if (bad == 1) {
        *dt_out = 0.0;
        return fail(MHD_ENONPHYS, "non-physical state: rho <= 0, p < 0 or non-finite value");
    }
    if (bad) {
        *dt_out = 0.0;
        return fail(MHD_EINVAL, "largest signal speed is zero: no CFL time step");
    }
    *dt_out = h->pinned[SCAL_DT];
    h->c_host = h->pinned[SCAL_VMAX];
    h->have_c = true;
    return MHD_OK;
}

extern "C" int mhd_set_relaxation_speed(mhd_ctx* h, double c)
{
    int r = check_handle(h);
    if (r) return r;
    if (!(c > 0.0) || !isfinite(c)) return fail(MHD_EINVAL, "relaxation speed must be > 0");
    h->c_host = c;
    h->have_c = true;
    return MHD_OK;
}

extern "C" int mhd_get_relaxation_speed(const mhd_ctx* hc, double* c)
{
    if (!hc || !c) return fail(MHD_EINVAL, "null argument");
    mhd_ctx* h = const_cast<mhd_ctx*>(hc);
    int r = check_handle(h);
    if (r) return r;
    if (!h->have_c) return fail(MHD_ESTATE, "relaxation speed not set (call mhd_cfl_dt)");
    if (h->c_host < 0.0) {      // set by a device-side CFL: read it back
        HIP_TRY(h, hipSetDevice(h->device));
        HIP_TRY(h, hipMemcpyAsync(h->pinned, h->scal + SCAL_C, sizeof(double),
                                  hipMemcpyDeviceToHost, h->stream));
        if ((r = sync_stream(h))) return r;
        h->c_host = h->pinned[0];
    }
    *c = h->c_host;
    return MHD_OK;
}

// ---------------------------------------------------------------------------
// operators
// ---------------------------------------------------------------------------

// op 0 = fluid, 1 = magnetic, 2 = magnetic then fluid in one launch, 3 =
// magnetic twice then fluid in one launch; flag (nullable): skip-and-copy
// switch
template <typename T>
static hipError_t enqueue_op(mhd_ctx* h, int op, int d, const int* flag, unsigned long long* acc)
{
    SweepParams<T> P;
    for (int q = 0; q < 8; ++q) {
        P.in[q] = field_ptr<T>(h, q, h->cur[q]);
        P.out[q] = field_ptr<T>(h, q, 1 - h->cur[q]);
    }
    P.nx = h->n[0]; P.ny = h->n[1]; P.nz = h->n[2];
    P.gamma = (T)h->gamma;
    P.scal = h->scal;
    P.flag = flag;
    P.cfl_acc = acc;
    P.gamma64 = h->gamma;
    P.limiter = h->limiter;
    P.freeze = h->freeze;
    hipError_t e = op == 0 ? launch_fluid<T>(P, d, h->tune, h->stream)
                 : op == 1 ? launch_magnetic<T>(P, d, h->tune, h->stream)
                 : op == 2 ? launch_magfluid<T>(P, d, h->tune, h->stream)
                           : launch_magmagfluid<T>(P, d, h->tune, h->stream);
    if (e == hipSuccess) {
        if (op != 1)
            for (int q = 0; q < 5; ++q) h->cur[q] = 1 - h->cur[q];
        if (op != 0)
            for (int q = 5; q < 8; ++q) h->cur[q] = 1 - h->cur[q];
    }
    return e;
}

// acc (nullable; fluid along x, alone or fused): fused CFL accumulator
static hipError_t op(mhd_ctx* h, int o, int d, const int* flag, unsigned long long* acc = nullptr)
{
    return h->prec == MHD_F64 ? enqueue_op<double>(h, o, d, flag, acc) : enqueue_op<float>(h, o, d, flag, acc);
}

static int check_dt(double dt)
{
    if (!(dt > 0.0) || !isfinite(dt)) return fail(MHD_EINVAL, "dt must be > 0 and finite (got %g)", dt);
    return MHD_OK;
}

static int prepare_host_dt(mhd_ctx* h, double dt, bool need_c)
{
    int r = check_handle(h);
    if (r) return r;
    if ((r = check_dt(dt))) return r;
    // the per-cell and per-pencil freezing speeds come from the state
    if (h->freeze != MHD_FREEZE_STEP) need_c = false;
    if (need_c && !h->have_c)
        return fail(MHD_ESTATE, "relaxation speed not set: call mhd_cfl_dt or mhd_set_relaxation_speed");
    HIP_TRY(h, hipSetDevice(h->device));
    // c_host < 0: the speed was set by a device-side CFL and stays there
    const double c = h->have_c ? h->c_host : 0.0;
    if (h->scal_known && h->scal_dt == dt && (c <= 0.0 || h->scal_c == c)) return MHD_OK;
    HIP_TRY(h, launch_set_scalars(h->scal, dt, c, h->flag, 0, h->stream));
    h->scal_known = c > 0.0;
    h->scal_dt = dt;
    h->scal_c = c;
    return MHD_OK;
}

extern "C" int mhd_fluid(mhd_ctx* h, int dim, double dt)
{
    if (dim < 0 || dim > 2) return fail(MHD_EINVAL, "dim must be 0, 1 or 2 (got %d)", dim);
    int r = prepare_host_dt(h, dt, true);
    if (r) return r;
    h->acc_valid = false;
    HIP_TRY(h, op(h, 0, dim, nullptr));
    return MHD_OK;
}

extern "C" int mhd_magnetic(mhd_ctx* h, int dim, double dt)
{
    if (dim < 0 || dim > 2) return fail(MHD_EINVAL, "dim must be 0, 1 or 2 (got %d)", dim);
    int r = prepare_host_dt(h, dt, false);
    if (r) return r;
    h->acc_valid = false;
    HIP_TRY(h, op(h, 1, dim, nullptr));
    return MHD_OK;
}

// the reverse pairs run as one fused launch each (the fused kernels take
// the step's freezing speed only)
static bool pairs_fused(const mhd_ctx* h)
{
    if (h->freeze != MHD_FREEZE_STEP) return false;
    return h->rev_mode == 1 || (h->rev_mode == 0 && default_rev_fused(h->prec, h->limiter));
}

static bool mid_fused(const mhd_ctx* h);

extern "C" int mhd_sweep(mhd_ctx* h, int dim, double dt)
{
    if (dim < 0 || dim > 7) return fail(MHD_EINVAL, "sweep code must be 0..7 (got %d)", dim);
    int r = prepare_host_dt(h, dt, true);
    if (r) return r;
    h->acc_valid = false;
    if (dim == 7) {
        // the middle of a step: M_z, then the reverse z pair
        if (mid_fused(h)) {
            HIP_TRY(h, op(h, 3, 2, nullptr));
        } else {
            HIP_TRY(h, op(h, 1, 2, nullptr));
            if (pairs_fused(h)) {
                HIP_TRY(h, op(h, 2, 2, nullptr));
            } else {
                HIP_TRY(h, op(h, 1, 2, nullptr));
                HIP_TRY(h, op(h, 0, 2, nullptr));
            }
        }
        return MHD_OK;
    }
    if (dim == 6) {
        // the reverse x pair with the fused CFL of its result
        unsigned long long* acc = h->fuse_ok ? h->cfl_acc : nullptr;
        if (acc) HIP_TRY(h, launch_clear_acc(acc, h->stream));
        if (pairs_fused(h)) {
            HIP_TRY(h, op(h, 2, 0, nullptr, acc));
        } else {
            HIP_TRY(h, op(h, 1, 0, nullptr));
            HIP_TRY(h, op(h, 0, 0, nullptr, acc));
        }
        h->acc_valid = h->fuse_ok;
        return MHD_OK;
    }
    const int d = dim % 3;
    if (dim < 3) {
        HIP_TRY(h, op(h, 0, d, nullptr));
        HIP_TRY(h, op(h, 1, d, nullptr));
    } else if (pairs_fused(h)) {
        HIP_TRY(h, op(h, 2, d, nullptr));
    } else {
        HIP_TRY(h, op(h, 1, d, nullptr));
        HIP_TRY(h, op(h, 0, d, nullptr));
    }
    return MHD_OK;
}

// M_z M_z F_z of a step in one launch: FP32 (the FP64 windows would not fit
// the register file), fused reverse pairs, van Leer's limiter, the step's
// freezing speed.  Built in: from 128^3 cells up (measured 4.5% faster per
// step at 256^3 and 5% at 512^3, equal at 96^3-128^3 and 1-2% slower below,
// where launch latency dominates and the 19-cell warm-up of the one wave per
// SIMD it runs is long against the pencils)
static bool mid_fused(const mhd_ctx* h)
{
    if (!pairs_fused(h) || h->limiter != MHD_LIMITER_VANLEER || h->prec != MHD_F32) return false;
    if (h->mid_mode == 0) return (long)h->n[0] * h->n[1] * h->n[2] >= 128L * 128 * 128;
    return h->mid_mode == 1;
}

// the 12 operators of a full step: x, y, z forward (fluid, magnetic), then
// z, y, x reverse (magnetic, fluid), each reverse pair in one launch when
// pairs_fused (9 launches), and M_z with the z pair in one when mid_fused
// (8 launches).  acc (nullable): the last operator (F_x) also accumulates
// the CFL maximum of the state it leaves.
static int enqueue_step_ops(mhd_ctx* h, const int* flag, unsigned long long* acc)
{
    const bool mid = mid_fused(h);
    for (int d = 0; d < 3; ++d) {
        HIP_TRY(h, op(h, 0, d, flag));
        if (d == 2 && mid) {
            HIP_TRY(h, op(h, 3, 2, flag));
            break;
        }
        HIP_TRY(h, op(h, 1, d, flag));
    }
    for (int d = mid ? 1 : 2; d >= 0; --d) {
        if (pairs_fused(h)) {
            HIP_TRY(h, op(h, 2, d, flag, d == 0 ? acc : nullptr));
        } else {
            HIP_TRY(h, op(h, 1, d, flag));
            HIP_TRY(h, op(h, 0, d, flag, d == 0 ? acc : nullptr));
        }
    }
    return MHD_OK;
}

extern "C" int mhd_set_limiter(mhd_ctx* h, int limiter)
{
    int r = check_handle(h);
    if (r) return r;
    if (limiter < MHD_LIMITER_VANLEER || limiter > MHD_LIMITER_SUPERBEE)
        return fail(MHD_EINVAL, "limiter must be 0..3 (got %d)", limiter);
    if (limiter != MHD_LIMITER_VANLEER && h->freeze != MHD_FREEZE_STEP)
        return fail(MHD_EINVAL, "the freezing-speed variants come with van Leer's limiter only");
    h->limiter = limiter;
    return MHD_OK;
}

extern "C" int mhd_set_freezing_speed(mhd_ctx* h, int mode)
{
    int r = check_handle(h);
    if (r) return r;
    if (mode < MHD_FREEZE_STEP || mode > MHD_FREEZE_PENCIL)
        return fail(MHD_EINVAL, "freezing-speed mode must be 0..2 (got %d)", mode);
    if (mode != MHD_FREEZE_STEP && h->limiter != MHD_LIMITER_VANLEER)
        return fail(MHD_EINVAL, "the freezing-speed variants come with van Leer's limiter only");
    h->freeze = mode;
    return MHD_OK;
}

extern "C" int mhd_get_freezing_speed(const mhd_ctx* h, int* mode)
{
    int r = check_handle(h);
    if (r) return r;
    if (!mode) return fail(MHD_EINVAL, "null output");
    *mode = h->freeze;
    return MHD_OK;
}

extern "C" int mhd_get_limiter(const mhd_ctx* h, int* limiter)
{
    int r = check_handle(h);
    if (r) return r;
    if (!limiter) return fail(MHD_EINVAL, "null output");
    *limiter = h->limiter;
    return MHD_OK;
}

extern "C" int mhd_step(mhd_ctx* h, double dt)
{
    int r = prepare_host_dt(h, dt, true);
    if (r) return r;
    h->acc_valid = false;
    if (h->fuse_ok) HIP_TRY(h, launch_clear_acc(h->cfl_acc, h->stream));
    if ((r = enqueue_step_ops(h, nullptr, h->fuse_ok ? h->cfl_acc : nullptr))) return r;
    HIP_TRY(h, launch_advance_time(h->scal, nullptr, nullptr, h->stream));
    h->acc_valid = h->fuse_ok;
    return MHD_OK;
}

extern "C" int mhd_step_auto(mhd_ctx* h, double cfl)
{
    int r = check_handle(h);
    if (r) return r;
    if (!(cfl > 0.0) || !isfinite(cfl)) return fail(MHD_EINVAL, "cfl must be > 0 (got %g)", cfl);
    HIP_TRY(h, hipSetDevice(h->device));
    h->scal_known = false;
    if (h->acc_valid) {
        // the previous step's last operator already found this state's
        // largest signal speed (same FP64 expression, same maximum)
        HIP_TRY(h, launch_cfl_from_acc(h->cfl_acc, h->n[0], cfl, h->scal, h->flag + FLAG_NONPHYS, h->stream));
    } else {
        HIP_TRY(h, h->prec == MHD_F64 ? enqueue_cfl<double>(h, cfl, h->flag + FLAG_NONPHYS)
                                      : enqueue_cfl<float>(h, cfl, h->flag + FLAG_NONPHYS));
        if (h->fuse_ok) HIP_TRY(h, launch_clear_acc(h->cfl_acc, h->stream));
    }
    h->acc_valid = false;
    if ((r = enqueue_step_ops(h, h->flag + FLAG_NONPHYS, h->fuse_ok ? h->cfl_acc : nullptr))) return r;
    h->acc_valid = h->fuse_ok;
    HIP_TRY(h, launch_advance_time(h->scal, h->flag + FLAG_NONPHYS, h->flag + FLAG_STEPS, h->stream));
    // the device CFL also set the relaxation speed; it stays on the device
    // (c_host < 0 marks that) until read back
    h->have_c = true;
    h->c_host = -1.0;
    return MHD_OK;
}

extern "C" int mhd_status(mhd_ctx* h, long long* steps_out)
{
    int r = check_handle(h);
    if (r) return r;
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipMemcpyAsync(h->pinned, h->flag, FLAG_COUNT * sizeof(int), hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->pinned + 4, h->scal, SCAL_COUNT * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
    if ((r = sync_stream(h))) return r;
    int fl[FLAG_COUNT];
    memcpy(fl, h->pinned, sizeof fl);
    if (steps_out) *steps_out = fl[FLAG_STEPS];
    if (fl[FLAG_NONPHYS]) {
        HIP_TRY(h, hipMemsetAsync(h->flag + FLAG_NONPHYS, 0, sizeof(int), h->stream));
        if ((r = sync_stream(h))) return r;
        return fl[FLAG_NONPHYS] == 1
                   ? fail(MHD_ENONPHYS, "non-physical state found by the device CFL; steps skipped")
                   : fail(MHD_EINVAL, "largest signal speed is zero; steps skipped");
    }
    return MHD_OK;
}

extern "C" int mhd_time(mhd_ctx* h, double* t)
{
    int r = check_handle(h);
    if (r) return r;
    if (!t) return fail(MHD_EINVAL, "null pointer");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipMemcpyAsync(h->pinned, h->scal + SCAL_TIME, sizeof(double), hipMemcpyDeviceToHost,
                              h->stream));
    if ((r = sync_stream(h))) return r;
    *t = h->pinned[0];
    return MHD_OK;
}

// ---------------------------------------------------------------------------
// diagnostics and restriction
// ---------------------------------------------------------------------------

template <typename T>
static hipError_t enqueue_diag(mhd_ctx* h)
{
    const T* f[8];
    current_fields<T>(h, f);
    return launch_diag<T>(f, h->n[0], h->n[1], h->n[2], h->partial, h->nblk_diag, h->diag_out,
                          h->stream);
}

extern "C" int mhd_diag(mhd_ctx* h, double out[9])
{
    int r = check_handle(h);
    if (r) return r;
    if (!out) return fail(MHD_EINVAL, "null output");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, h->prec == MHD_F64 ? enqueue_diag<double>(h) : enqueue_diag<float>(h));
    HIP_TRY(h, hipMemcpyAsync(h->pinned, h->diag_out, 9 * sizeof(double), hipMemcpyDeviceToHost,
                              h->stream));
    if ((r = sync_stream(h))) return r;
    memcpy(out, h->pinned, 9 * sizeof(double));
    return MHD_OK;
}

template <typename T>
static hipError_t enqueue_restrict(mhd_ctx* fine, mhd_ctx* coarse, int r)
{
    const T* f[8];
    T* c[8];
    current_fields<T>(fine, f);
    for (int q = 0; q < 8; ++q) c[q] = field_ptr<T>(coarse, q, 0);
    return launch_restrict<T>(f, c, fine->n[0], fine->n[1], fine->n[2], r, coarse->stream);
}

extern "C" int mhd_restrict(mhd_ctx* fine, mhd_ctx* coarse)
{
    int r = check_handle(fine);
    if (r) return r;
    if ((r = check_handle(coarse))) return r;
    if (fine == coarse) return fail(MHD_EINVAL, "fine and coarse handles must differ");
    if (fine->prec != coarse->prec) return fail(MHD_EINVAL, "precision tiers differ");
    if (fine->device != coarse->device) return fail(MHD_EINVAL, "handles on different devices");
    if (fine->n[0] % coarse->n[0]) return fail(MHD_EINVAL, "coarse nx does not divide fine nx");
    const int f = fine->n[0] / coarse->n[0];
    for (int d = 0; d < 3; ++d)
        if (coarse->n[d] * f != fine->n[d])
            return fail(MHD_EINVAL, "fine/coarse sizes are not one integer factor on every axis");
    HIP_TRY(fine, hipSetDevice(fine->device));
    HIP_TRY(fine, hipStreamSynchronize(fine->stream));
    if ((r = reset_after_set(coarse))) return r;
    HIP_TRY(coarse, fine->prec == MHD_F64 ? enqueue_restrict<double>(fine, coarse, f)
                                          : enqueue_restrict<float>(fine, coarse, f));
    return MHD_OK;
}

extern "C" int mhd_set_launch(mhd_ctx* h, int key, int value)
{
    int r = check_handle(h);
    if (r) return r;
    if (key == MHD_TUNE_REVERSE) {
        if (value < 0 || value > 2)
            return fail(MHD_EINVAL, "reverse-half choice must be 0, 1 or 2 (got %d)", value);
        h->rev_mode = value;
        return MHD_OK;
    }
    if (key == MHD_TUNE_WIDE_OFFSETS) {
        if (value < 0 || value > 1) return fail(MHD_EINVAL, "wide-offset switch must be 0 or 1 (got %d)", value);
        h->tune.wide = value;
        return MHD_OK;
    }
    if (key == MHD_TUNE_MIDDLE) {
        if (value < 0 || value > 2)
            return fail(MHD_EINVAL, "middle-of-step choice must be 0, 1 or 2 (got %d)", value);
        h->mid_mode = value;
        return MHD_OK;
    }
    if (key == MHD_TUNE_ROW_GROUP) {
        if (value < 0) return fail(MHD_EINVAL, "row group must be >= 0 (got %d)", value);
        h->tune.row_group = value;
        return MHD_OK;
    }
    const bool pair = key == MHD_TUNE_PAIR_CHUNK_Y || key == MHD_TUNE_PAIR_CHUNK_Z;
    const bool triple = key == MHD_TUNE_MIDDLE_CHUNK;
    if (key != MHD_TUNE_CHUNK_Y && key != MHD_TUNE_CHUNK_Z && !pair && !triple)
        return fail(MHD_EINVAL, "unknown launch key %d", key);
    const int d = triple ? 2 : pair ? key - MHD_TUNE_PAIR_CHUNK_Y + 1 : key;   // axis 1 (y) or 2 (z)
    int* slot = triple ? &h->tune.triple_chunk[d] : pair ? &h->tune.pair_chunk[d] : &h->tune.chunk[d];
    if (value == 0) {
        const LaunchTuning keep = h->tune;
        default_tuning(h);
        const int v = *slot;
        h->tune = keep;
        *slot = v;
        return MHD_OK;
    }
    if (value < 8 || h->n[d] % value)
        return fail(MHD_EINVAL, "chunk %d must be >= 8 and divide the axis length %d", value, h->n[d]);
    *slot = value;
    return MHD_OK;
}

extern "C" int mhd_get_launch(const mhd_ctx* h, int key, int* value)
{
    if (!h || !value) return fail(MHD_EINVAL, "null argument");
    if (key == MHD_TUNE_REVERSE) {
        *value = pairs_fused(h) ? 1 : 2;
        return MHD_OK;
    }
    if (key == MHD_TUNE_WIDE_OFFSETS) {
        *value = h->tune.wide;
        return MHD_OK;
    }
    if (key == MHD_TUNE_MIDDLE) {
        *value = mid_fused(h) ? 1 : 2;
        return MHD_OK;
    }
    if (key == MHD_TUNE_MIDDLE_CHUNK) {
        *value = h->tune.triple_chunk[2];
        return MHD_OK;
    }
    if (key == MHD_TUNE_ROW_GROUP) {
        const int rpw = x_rows_per_wg(h->n[0]);
        const int st = row_group_tiles(h->n[1], rpw, h->tune.row_group);
        *value = (st <= 0 || st * rpw >= h->n[1]) ? h->n[1] : st * rpw;
        return MHD_OK;
    }
    if (key == MHD_TUNE_PAIR_CHUNK_Y || key == MHD_TUNE_PAIR_CHUNK_Z) {
        *value = h->tune.pair_chunk[key - MHD_TUNE_PAIR_CHUNK_Y + 1];
        return MHD_OK;
    }
    if (key != MHD_TUNE_CHUNK_Y && key != MHD_TUNE_CHUNK_Z)
        return fail(MHD_EINVAL, "unknown launch key %d", key);
    *value = h->tune.chunk[key];
    return MHD_OK;
}

void* mhd_internal_state(mhd_ctx* h, int* all_in_first_buffer)
{
    int all = 1;
    for (int q = 0; q < 8; ++q) all = all && h->cur[q] == 0;
    *all_in_first_buffer = all;
    return h->buf[0];
}

// Bring every field into the first buffer (a device copy on the handle's
// stream for each field held in the second), so that the state is one
// contiguous array.  After a step the fields need not share a buffer: the
// fused middle of a step writes b once for two magnetic operators.
int mhd_internal_gather_first(mhd_ctx* h)
{
    for (int q = 0; q < 8; ++q) {
        if (h->cur[q] == 0) continue;
        HIP_TRY(h, hipMemcpyAsync((char*)h->buf[0] + (size_t)q * h->N * h->esize,
                                  (const char*)h->buf[1] + (size_t)q * h->N * h->esize, h->N * h->esize,
                                  hipMemcpyDeviceToDevice, h->stream));
        h->cur[q] = 0;
    }
    return MHD_OK;
}
int mhd_internal_prec(const mhd_ctx* h) { return h->prec; }
void mhd_internal_dims(const mhd_ctx* h, int n[3]) { n[0] = h->n[0]; n[1] = h->n[1]; n[2] = h->n[2]; }
hipStream_t mhd_internal_stream(const mhd_ctx* h) { return h->stream; }
void mhd_internal_state_changed(mhd_ctx* h)
{
    h->acc_valid = false;
}

double mhd_internal_gamma(const mhd_ctx* h) { return h->gamma; }

extern "C" int mhd_stream_copy(const void* src, void* dst, size_t bytes, void* stream)
{
    if (!src || !dst) return fail(MHD_EINVAL, "null device pointer");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(MHD_EINVAL, "the copy moves 16-byte words: size and both pointers must be multiples of 16");
    const char* a = static_cast<const char*>(src);
    const char* b = static_cast<const char*>(dst);
    if (a < b + bytes && b < a + bytes) return fail(MHD_EINVAL, "source and destination overlap");
    if (bytes == 0) return MHD_OK;
    const hipError_t e = launch_stream_copy(src, dst, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MHD_EDEVICE, "stream copy: %s", hipGetErrorString(e));
    return MHD_OK;
}

extern "C" const char* mhd_last_error(void)
{
    return g_last_error.c_str();
}
