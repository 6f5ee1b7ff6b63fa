// Reductions and data-movement kernels of the MHD library for gfx950:
//  * the CFL condition (section II.B; the CFL function of section IV.A) as
//    an FP64 max-reduction of the signal speed with wave64 shuffles;
//  * conserved totals and the divergence diagnostic (FP64, fixed order, so
//    the result is the same on every run);
//  * host <-> device precision conversion, the restriction operator and the
//    small scalar kernels that keep dt on the device.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mhd_device.h"
#include "mhd_kernels.h"

namespace mhd {

constexpr int RED_THREADS = 256;

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_or(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// CFL
// ---------------------------------------------------------------------------

int cfl_blocks(size_t ncell)
{
    size_t b = (ncell + RED_THREADS * 8 - 1) / (RED_THREADS * 8);
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

// Signal speed max_d |v_d| + sqrt((gamma p + |Bbar|^2)/rho) of cell c of an
// nx x ny x nz grid in FP64; folds it into vmax, or raises bad for a
// non-physical cell.
template <typename T>
__device__ __forceinline__ void cell_signal_speed(const T* const* f, size_t c, int nx, int ny,
                                                  int nz, double gamma, double& vmax, int& bad)
{
    const size_t sy = nx, sz = (size_t)nx * ny;
    const int i = (int)(c % nx);
    const int j = (int)((c / sy) % ny);
    const int k = (int)(c / sz);
    const size_t cx = i + 1 == nx ? c - (nx - 1) : c + 1;
    const size_t cy = j + 1 == ny ? c - (ny - 1) * sy : c + sy;
    const size_t cz = k + 1 == nz ? c - (size_t)(nz - 1) * sz : c + sz;
    signal_speed64((double)f[0][c], (double)f[1][c], (double)f[2][c], (double)f[3][c], (double)f[4][c],
                   (double)f[5][c], (double)f[5][cx], (double)f[6][c], (double)f[6][cy], (double)f[7][c],
                   (double)f[7][cz], gamma, vmax, bad);
}

// per-block maximum and non-physical flag of the signal speed
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) cfl_partial_kernel(
    const T* __restrict__ rho_, const T* __restrict__ mx_, const T* __restrict__ my_,
    const T* __restrict__ mz_, const T* __restrict__ e_, const T* __restrict__ bx_,
    const T* __restrict__ by_, const T* __restrict__ bz_, int nx, int ny, int nz, double gamma,
    double* partial, int* partial_bad)
{
    const size_t N = (size_t)nx * ny * nz;
    const T* f[8] = { rho_, mx_, my_, mz_, e_, bx_, by_, bz_ };
    double vmax = 0.0;
    int bad = 0;
    for (size_t c = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; c < N;
         c += (size_t)gridDim.x * RED_THREADS)
        cell_signal_speed(f, c, nx, ny, nz, gamma, vmax, bad);
    __shared__ double smax[RED_THREADS / 64];
    __shared__ int sbad[RED_THREADS / 64];
    vmax = wave_max(vmax);
    bad = wave_or(bad);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { smax[w] = vmax; sbad[w] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = smax[0];
        int b = sbad[0];
        for (int q = 1; q < RED_THREADS / 64; ++q) { m = fmax(m, smax[q]); b |= sbad[q]; }
        partial[blockIdx.x] = m;
        partial_bad[blockIdx.x] = b;
    }
}

// One block: final maximum; dt = cfl h / vmax.  A non-physical state
// raises *flag (never cleared here) and writes dt = 0 without touching the
// relaxation speed.
__global__ void __launch_bounds__(RED_THREADS) cfl_final_kernel(
    const double* partial, const int* partial_bad, int nblocks, int nx, double cfl, double* scal,
    int* flag)
{
    double m = 0.0;
    int bad = 0;
    for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) {
        m = fmax(m, partial[b]);
        bad |= partial_bad[b];
    }
    __shared__ double smax[RED_THREADS / 64];
    __shared__ int sbad[RED_THREADS / 64];
    m = wave_max(m);
    bad = wave_or(bad);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { smax[w] = m; sbad[w] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double vmax = smax[0];
        int b = sbad[0];
        for (int q = 1; q < RED_THREADS / 64; ++q) { vmax = fmax(vmax, smax[q]); b |= sbad[q]; }
        if (b || !(vmax > 0.0)) {
            scal[SCAL_DT] = 0.0;
            scal[SCAL_VMAX] = 0.0;
            flag[0] = b ? 1 : 2;
        } else {
            scal[SCAL_DT] = cfl * (1.0 / (double)nx) / vmax;
            scal[SCAL_VMAX] = vmax;
            scal[SCAL_C] = vmax;
        }
    }
}

template <typename T>
hipError_t launch_cfl(const T* const f[8], int nx, int ny, int nz, double gamma, double cfl,
                      double* partial, int* partial_bad, int nblocks, double* scal, int* flag,
                      hipStream_t s)
{
    hipLaunchKernelGGL(cfl_partial_kernel<T>, dim3(nblocks), dim3(RED_THREADS), 0, s, f[0], f[1],
                       f[2], f[3], f[4], f[5], f[6], f[7], nx, ny, nz, gamma, partial, partial_bad);
    hipLaunchKernelGGL(cfl_final_kernel, dim3(1), dim3(RED_THREADS), 0, s, partial, partial_bad,
                       nblocks, nx, cfl, scal, flag);
    return hipGetLastError();
}

template hipError_t launch_cfl<float>(const float* const[8], int, int, int, double, double,
                                      double*, int*, int, double*, int*, hipStream_t);
template hipError_t launch_cfl<double>(const double* const[8], int, int, int, double, double,
                                       double*, int*, int, double*, int*, hipStream_t);

// The CFL from the maximum that the fused epilogue of the previous step's
// last fluid operator accumulated (acc[0 .. CFL_ACC_SLOTS): bits of FP64
// maxima, acc[CFL_ACC_SLOTS]: non-physical flag); the same dt / relaxation
// speed / flag rules as cfl_final_kernel.  Clears acc for the next
// accumulation.  One block of CFL_ACC_SLOTS threads.
__global__ void __launch_bounds__(CFL_ACC_SLOTS) cfl_from_acc_kernel(unsigned long long* acc, int nx, double cfl,
                                                                     double* scal, int* flag)
{
    double m = __longlong_as_double((long long)acc[threadIdx.x]);
    m = wave_max(m);
    __shared__ double smax[CFL_ACC_SLOTS / 64];
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double vmax = smax[0];
        for (int q = 1; q < CFL_ACC_SLOTS / 64; ++q) vmax = fmax(vmax, smax[q]);
        // bit 0: a non-physical cell (or record); bit 1 alone: a step skipped
        // under a zero-speed record, whose state still has no signal speed
        const int b = (int)acc[CFL_ACC_SLOTS];
        if (b || !(vmax > 0.0)) {
            scal[SCAL_DT] = 0.0;
            scal[SCAL_VMAX] = 0.0;
            flag[0] = (b & 1) ? 1 : 2;
        } else {
            scal[SCAL_DT] = cfl * (1.0 / (double)nx) / vmax;
            scal[SCAL_VMAX] = vmax;
            scal[SCAL_C] = vmax;
        }
        acc[CFL_ACC_SLOTS] = 0;
    }
    acc[threadIdx.x] = 0;
}

hipError_t launch_cfl_from_acc(unsigned long long* acc, int nx, double cfl, double* scal, int* flag,
                               hipStream_t s)
{
    hipLaunchKernelGGL(cfl_from_acc_kernel, dim3(1), dim3(CFL_ACC_SLOTS), 0, s, acc, nx, cfl, scal, flag);
    return hipGetLastError();
}

__global__ void clear_acc_kernel(unsigned long long* acc)
{
    acc[threadIdx.x] = 0;
    if (threadIdx.x == 0) acc[CFL_ACC_SLOTS] = 0;
}

hipError_t launch_clear_acc(unsigned long long* acc, hipStream_t s)
{
    hipLaunchKernelGGL(clear_acc_kernel, dim3(1), dim3(CFL_ACC_SLOTS), 0, s, acc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-box CFL of a batched ensemble
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) batch_cfl_partial_kernel(
    BatchCflArgs<T> A, double gamma, double* partial, int* partial_bad)
{
    const int2 it = A.items[blockIdx.x];
    const BoxDesc bd = A.boxes[it.x];
    const T* f[8];
    for (int q = 0; q < 8; ++q) f[q] = A.base[q] + bd.off + (size_t)q * bd.ncell;
    double vmax = 0.0;
    int bad = 0;
    const size_t c0 = (size_t)it.y * CFL_CELLS;
    const size_t c1 = c0 + CFL_CELLS < bd.ncell ? c0 + CFL_CELLS : bd.ncell;
    for (size_t c = c0 + threadIdx.x; c < c1; c += RED_THREADS)
        cell_signal_speed(f, c, bd.n[0], bd.n[1], bd.n[2], gamma, vmax, bad);
    __shared__ double smax[RED_THREADS / 64];
    __shared__ int sbad[RED_THREADS / 64];
    vmax = wave_max(vmax);
    bad = wave_or(bad);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { smax[w] = vmax; sbad[w] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = smax[0];
        int b = sbad[0];
        for (int q = 1; q < RED_THREADS / 64; ++q) { m = fmax(m, smax[q]); b |= sbad[q]; }
        partial[blockIdx.x] = m;
        partial_bad[blockIdx.x] = b;
    }
}

// one workgroup per box: max over the box's items; dt and relaxation speed
// of the box, or its non-physical flag (then dt = 0)
__global__ void __launch_bounds__(RED_THREADS) batch_cfl_final_kernel(
    const double* partial, const int* partial_bad, const int* item_first, const BoxDesc* boxes,
    double cfl, double* scal, int* flag)
{
    const int b = blockIdx.x;
    double m = 0.0;
    int bad = 0;
    for (int i = item_first[b] + threadIdx.x; i < item_first[b + 1]; i += RED_THREADS) {
        m = fmax(m, partial[i]);
        bad |= partial_bad[i];
    }
    __shared__ double smax[RED_THREADS / 64];
    __shared__ int sbad[RED_THREADS / 64];
    m = wave_max(m);
    bad = wave_or(bad);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { smax[w] = m; sbad[w] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double vmax = smax[0];
        int bb = sbad[0];
        for (int q = 1; q < RED_THREADS / 64; ++q) { vmax = fmax(vmax, smax[q]); bb |= sbad[q]; }
        double* sc = scal + (size_t)b * SCAL_COUNT;
        if (bb || !(vmax > 0.0)) {
            sc[SCAL_DT] = 0.0;
            sc[SCAL_VMAX] = 0.0;
            flag[(size_t)b * FLAG_COUNT + FLAG_NONPHYS] = bb ? 1 : 2;
        } else {
            sc[SCAL_DT] = cfl * (1.0 / (double)boxes[b].n[0]) / vmax;
            sc[SCAL_VMAX] = vmax;
            sc[SCAL_C] = vmax;
        }
    }
}

template <typename T>
hipError_t launch_batch_cfl(const T* const base[8], const BoxDesc* boxes, const int2* items,
                            int nitems, const int* item_first, int nbox, double gamma,
                            double cfl, double* partial, int* partial_bad, double* scal,
                            int* flag, hipStream_t s)
{
    BatchCflArgs<T> A;
    for (int q = 0; q < 8; ++q) A.base[q] = base[q];
    A.boxes = boxes;
    A.items = items;
    hipLaunchKernelGGL(batch_cfl_partial_kernel<T>, dim3(nitems), dim3(RED_THREADS), 0, s, A,
                       gamma, partial, partial_bad);
    hipLaunchKernelGGL(batch_cfl_final_kernel, dim3(nbox), dim3(RED_THREADS), 0, s, partial,
                       partial_bad, item_first, boxes, cfl, scal, flag);
    return hipGetLastError();
}
template hipError_t launch_batch_cfl<float>(const float* const[8], const BoxDesc*, const int2*,
                                            int, const int*, int, double, double, double*, int*,
                                            double*, int*, hipStream_t);
template hipError_t launch_batch_cfl<double>(const double* const[8], const BoxDesc*, const int2*,
                                             int, const int*, int, double, double, double*, int*,
                                             double*, int*, hipStream_t);

// box b (one block of CFL_ACC_SLOTS threads per box): the rules of
// batch_cfl_final_kernel on the maxima the fused CFL accumulated; clears them
__global__ void __launch_bounds__(CFL_ACC_SLOTS) batch_cfl_from_acc_kernel(unsigned long long* acc,
                                                                           const BoxDesc* boxes, double cfl,
                                                                           double* scal, int* flag)
{
    const int b = blockIdx.x;
    unsigned long long* a = acc + (size_t)b * (CFL_ACC_SLOTS + 1);
    double m = __longlong_as_double((long long)a[threadIdx.x]);
    m = wave_max(m);
    __shared__ double smax[CFL_ACC_SLOTS / 64];
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double vmax = smax[0];
        for (int q = 1; q < CFL_ACC_SLOTS / 64; ++q) vmax = fmax(vmax, smax[q]);
        const int bb = (int)a[CFL_ACC_SLOTS];
        double* sc = scal + (size_t)b * SCAL_COUNT;
        if (bb || !(vmax > 0.0)) {
            sc[SCAL_DT] = 0.0;
            sc[SCAL_VMAX] = 0.0;
            flag[(size_t)b * FLAG_COUNT + FLAG_NONPHYS] = (bb & 1) ? 1 : 2;
        } else {
            sc[SCAL_DT] = cfl * (1.0 / (double)boxes[b].n[0]) / vmax;
            sc[SCAL_VMAX] = vmax;
            sc[SCAL_C] = vmax;
        }
        a[CFL_ACC_SLOTS] = 0;
    }
    a[threadIdx.x] = 0;
}

hipError_t launch_batch_cfl_from_acc(unsigned long long* acc, const BoxDesc* boxes, int nbox, double cfl,
                                     double* scal, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(batch_cfl_from_acc_kernel, dim3(nbox), dim3(CFL_ACC_SLOTS), 0, s, acc, boxes, cfl, scal, flag);
    return hipGetLastError();
}

__global__ void batch_clear_acc_kernel(unsigned long long* acc)
{
    unsigned long long* a = acc + (size_t)blockIdx.x * (CFL_ACC_SLOTS + 1);
    a[threadIdx.x] = 0;
    if (threadIdx.x == 0) a[CFL_ACC_SLOTS] = 0;
}

hipError_t launch_batch_clear_acc(unsigned long long* acc, int nbox, hipStream_t s)
{
    hipLaunchKernelGGL(batch_clear_acc_kernel, dim3(nbox), dim3(CFL_ACC_SLOTS), 0, s, acc);
    return hipGetLastError();
}

// per-box time advance (skipped for a box with a non-physical record)
__global__ void batch_advance_kernel(double* scal, int* flag, int nbox)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbox && flag[(size_t)b * FLAG_COUNT + FLAG_NONPHYS] == 0) {
        scal[(size_t)b * SCAL_COUNT + SCAL_TIME] += 2.0 * scal[(size_t)b * SCAL_COUNT + SCAL_DT];
        flag[(size_t)b * FLAG_COUNT + FLAG_STEPS] += 1;
    }
}

hipError_t launch_batch_advance(double* scal, int* flag, int nbox, hipStream_t s)
{
    hipLaunchKernelGGL(batch_advance_kernel, dim3((nbox + 63) / 64), dim3(64), 0, s, scal, flag, nbox);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagnostics
// ---------------------------------------------------------------------------

int diag_blocks(size_t ncell)
{
    size_t b = (ncell + RED_THREADS * 16 - 1) / (RED_THREADS * 16);
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int)b;
}

// partial[10 * block + q]: q < 8 field sums, 8 max |div b| (times h),
// 9 max |b|.  Fixed assignment of cells to threads and a fixed tree: the
// result does not depend on timing.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) diag_partial_kernel(
    const T* __restrict__ f0, const T* __restrict__ f1, const T* __restrict__ f2,
    const T* __restrict__ f3, const T* __restrict__ f4, const T* __restrict__ bx_,
    const T* __restrict__ by_, const T* __restrict__ bz_, int nx, int ny, int nz, double* partial)
{
    // a field has fewer than 2^31 cells (as in the sweep kernels): 32-bit
    // cell indices, whose divisions are far cheaper than 64-bit ones
    const unsigned N = (unsigned)nx * ny * nz;
    const unsigned sy = nx, sz = (unsigned)nx * ny;
    double acc[8] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    double dmax = 0.0, bmax = 0.0;
    for (unsigned c = blockIdx.x * RED_THREADS + threadIdx.x; c < N; c += gridDim.x * RED_THREADS) {
        const unsigned kj = c / sy;
        const int i = (int)(c - kj * sy);
        const int k = (int)(kj / ny);
        const int j = (int)(kj - (unsigned)k * ny);
        const unsigned cx = i + 1 == nx ? c - (nx - 1) : c + 1;
        const unsigned cy = j + 1 == ny ? c - (unsigned)(ny - 1) * sy : c + sy;
        const unsigned cz = k + 1 == nz ? c - (unsigned)(nz - 1) * sz : c + sz;
        const double bx = (double)bx_[c], by = (double)by_[c], bz = (double)bz_[c];
        acc[0] += (double)f0[c];
        acc[1] += (double)f1[c];
        acc[2] += (double)f2[c];
        acc[3] += (double)f3[c];
        acc[4] += (double)f4[c];
        acc[5] += bx;
        acc[6] += by;
        acc[7] += bz;
        const double dv = ((double)bx_[cx] - bx) + ((double)by_[cy] - by) + ((double)bz_[cz] - bz);
        dmax = fmax(dmax, fabs(dv));
        bmax = fmax(bmax, fmax(fabs(bx), fmax(fabs(by), fabs(bz))));
    }
    __shared__ double red[10][RED_THREADS / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) red[q][w] = v;
    }
    dmax = wave_max(dmax);
    bmax = wave_max(bmax);
    if (lane == 0) { red[8][w] = dmax; red[9][w] = bmax; }
    __syncthreads();
    if (threadIdx.x < 10) {
        const int q = threadIdx.x;
        double v = red[q][0];
        for (int ww = 1; ww < RED_THREADS / 64; ++ww)
            v = q < 8 ? v + red[q][ww] : fmax(v, red[q][ww]);
        partial[10 * blockIdx.x + q] = v;
    }
}

// One block: thread t folds the partials t, t + 256, ... in that order, then
// the wave and block combine in a fixed order (deterministic).
__global__ void __launch_bounds__(RED_THREADS) diag_final_kernel(const double* partial, int nblocks,
                                                                 double h3, double* out9)
{
    double v[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) v[q] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RED_THREADS)
#pragma unroll
        for (int q = 0; q < 10; ++q) v[q] = q < 8 ? v[q] + partial[10 * b + q] : fmax(v[q], partial[10 * b + q]);
    __shared__ double red[10][RED_THREADS / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        const double x = q < 8 ? wave_sum(v[q]) : wave_max(v[q]);
        if (lane == 0) red[q][w] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            r[q] = red[q][0];
            for (int ww = 1; ww < RED_THREADS / 64; ++ww) r[q] = q < 8 ? r[q] + red[q][ww] : fmax(r[q], red[q][ww]);
        }
        for (int q = 0; q < 8; ++q) out9[q] = r[q] * h3;
        out9[8] = r[9] > 0.0 ? r[8] / r[9] : 0.0;
    }
}

template <typename T>
hipError_t launch_diag(const T* const f[8], int nx, int ny, int nz, double* partial, int nblocks,
                       double* out9, hipStream_t s)
{
    const double h = 1.0 / (double)nx;
    hipLaunchKernelGGL(diag_partial_kernel<T>, dim3(nblocks), dim3(RED_THREADS), 0, s, f[0], f[1],
                       f[2], f[3], f[4], f[5], f[6], f[7], nx, ny, nz, partial);
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(RED_THREADS), 0, s, partial, nblocks, h * h * h, out9);
    return hipGetLastError();
}
template hipError_t launch_diag<float>(const float* const[8], int, int, int, double*, int, double*,
                                       hipStream_t);
template hipError_t launch_diag<double>(const double* const[8], int, int, int, double*, int,
                                        double*, hipStream_t);

// ---------------------------------------------------------------------------
// Conversions
// ---------------------------------------------------------------------------

template <typename S, typename T>
__global__ void cast_kernel(const S* __restrict__ src, T* __restrict__ dst, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (T)src[i];
}

template <typename S, typename T>
hipError_t launch_cast(const S* src, T* dst, size_t n, hipStream_t s)
{
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((cast_kernel<S, T>), dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}
template hipError_t launch_cast<double, float>(const double*, float*, size_t, hipStream_t);
template hipError_t launch_cast<float, double>(const float*, double*, size_t, hipStream_t);
template hipError_t launch_cast<float, float>(const float*, float*, size_t, hipStream_t);
template hipError_t launch_cast<double, double>(const double*, double*, size_t, hipStream_t);

// Plain streaming copy of 16-byte words, the bandwidth reference of the
// sweep kernels: each thread moves 4 words per round (a wave's 64 lanes read
// one contiguous KiB per word slot), all loads of a round before its stores;
// grid-stride over the buffer.
__global__ void __launch_bounds__(256) stream_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                          size_t n)
{
    const size_t stride = (size_t)gridDim.x * 256 * 4;
    for (size_t i = (size_t)blockIdx.x * 1024 + threadIdx.x; i < n; i += stride) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + (size_t)k * 256 < n) v[k] = src[i + (size_t)k * 256];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + (size_t)k * 256 < n) dst[i + (size_t)k * 256] = v[k];
    }
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    size_t grid = (n + 1023) / 1024;
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)grid), dim3(256), 0, s, static_cast<const uint4*>(src),
                       static_cast<uint4*>(dst), n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_convert_in(const double* src, T* dst, size_t n, hipStream_t s)
{
    return launch_cast<double, T>(src, dst, n, s);
}
template <typename T>
hipError_t launch_convert_out(const T* src, double* dst, size_t n, hipStream_t s)
{
    return launch_cast<T, double>(src, dst, n, s);
}
template hipError_t launch_convert_in<float>(const double*, float*, size_t, hipStream_t);
template hipError_t launch_convert_in<double>(const double*, double*, size_t, hipStream_t);
template hipError_t launch_convert_out<float>(const float*, double*, size_t, hipStream_t);
template hipError_t launch_convert_out<double>(const double*, double*, size_t, hipStream_t);

// ---------------------------------------------------------------------------
// Restriction
// ---------------------------------------------------------------------------
// One thread per coarse cell; consecutive threads take consecutive coarse x,
// so the r consecutive fine values each thread reads per fine row join into
// one contiguous run across the wave.  FP64 accumulation in a fixed order
// (fine z, then y, then x; faces: first transverse, then second).

template <typename T>
__global__ void __launch_bounds__(256) restrict_kernel(
    const T* f0, const T* f1, const T* f2, const T* f3, const T* f4, const T* g0, const T* g1,
    const T* g2, T* o0, T* o1, T* o2, T* o3, T* o4, T* p0, T* p1, T* p2, int nx, int ny, int nz,
    int r)
{
    const int cx = nx / r, cy = ny / r, cz = nz / r;
    const size_t Nc = (size_t)cx * cy * cz;
    const size_t C = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (C >= Nc) return;
    const int I = (int)(C % cx), J = (int)((C / cx) % cy), K = (int)(C / ((size_t)cx * cy));
    const T* fin[5] = { f0, f1, f2, f3, f4 };
    T* fout[5] = { o0, o1, o2, o3, o4 };
    const double rrr = (double)r * r * r;
    for (int f = 0; f < 5; ++f) {
        double acc = 0.0;
        for (int k = 0; k < r; ++k)
            for (int j = 0; j < r; ++j) {
                const T* row = fin[f] + (size_t)r * I +
                               (size_t)nx * ((size_t)(r * J + j) + (size_t)ny * (size_t)(r * K + k));
                for (int i = 0; i < r; ++i) acc += (double)row[i];
            }
        fout[f][C] = (T)(acc / rrr);
    }
    const T* gin[3] = { g0, g1, g2 };
    T* gout[3] = { p0, p1, p2 };
    const double rr = (double)r * r;
    for (int d = 0; d < 3; ++d) {
        const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        double acc = 0.0;
        for (int u = 0; u < r; ++u)
            for (int w = 0; w < r; ++w) {
                int pp[3] = { r * I, r * J, r * K };
                pp[t1] += u;
                pp[t2] += w;
                acc += (double)gin[d][(size_t)pp[0] + (size_t)nx * ((size_t)pp[1] + (size_t)ny * pp[2])];
            }
        gout[d][C] = (T)(acc / rr);
    }
}

// R consecutive values of a fine row with 16-byte (or, for R = 2 in FP32,
// 8-byte) loads; the row offset R * I keeps them aligned (rows start at
// multiples of 4 values)
template <typename T, int R>
__device__ __forceinline__ void load_run(const T* p, T (&v)[R])
{
    constexpr int W = 16 / (int)sizeof(T);             // values per 16 bytes
    if constexpr (R % W == 0) {
        typedef T V __attribute__((ext_vector_type(W)));
#pragma unroll
        for (int q = 0; q < R / W; ++q) {
            const V t = reinterpret_cast<const V*>(p)[q];
#pragma unroll
            for (int w = 0; w < W; ++w) v[q * W + w] = t[w];
        }
    } else {
        typedef T V __attribute__((ext_vector_type(R)));
        const V t = *reinterpret_cast<const V*>(p);
#pragma unroll
        for (int w = 0; w < R; ++w) v[w] = t[w];
    }
}

// Restriction by a fixed factor R (2, 4 or 8): one thread per (field,
// coarse cell), fields outermost so that a wave holds consecutive coarse
// cells of one field.  A cell field sums the R^3 fine values, issuing the
// R rows of one fine plane as vector loads before adding them; a face field
// sums the R^2 fine faces on the coarse face.  Same sums in the same order
// as restrict_kernel (k, then j, then i; FP64), so the same values.
struct RestrictArgs {
    const void* fine[8];
    void* coarse[8];
    int nx, ny, nz;
};

template <typename T, int R>
__global__ void __launch_bounds__(256) restrict_fixed_kernel(RestrictArgs a)
{
    const int nx = a.nx, ny = a.ny;
    const int cx = nx / R, cy = ny / R, cz = a.nz / R;
    const size_t Nc = (size_t)cx * cy * cz;
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 8 * Nc) return;
    const int f = (int)(g / Nc);
    const size_t C = g - (size_t)f * Nc;
    const int I = (int)(C % cx), J = (int)((C / cx) % cy), K = (int)(C / ((size_t)cx * cy));
    const T* in = reinterpret_cast<const T*>(a.fine[f]);
    T* out = reinterpret_cast<T*>(a.coarse[f]);
    double acc = 0.0;
    if (f < 5) {
        const T* base = in + (size_t)R * I + (size_t)nx * ((size_t)R * J + (size_t)ny * ((size_t)R * K));
        for (int k = 0; k < R; ++k) {
            T v[R][R];
#pragma unroll
            for (int j = 0; j < R; ++j) load_run<T, R>(base + (size_t)nx * ((size_t)j + (size_t)ny * k), v[j]);
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int i = 0; i < R; ++i) acc += (double)v[j][i];
        }
        out[C] = (T)(acc / ((double)R * R * R));
    } else {
        const int d = f - 5, t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        // strides of the two transverse axes
        const size_t st[3] = { 1, (size_t)nx, (size_t)nx * ny };
        const T* base = in + (size_t)R * I + st[1] * ((size_t)R * J) + st[2] * ((size_t)R * K);
        T v[R][R];
#pragma unroll
        for (int u = 0; u < R; ++u)
#pragma unroll
            for (int w = 0; w < R; ++w) v[u][w] = base[u * st[t1] + w * st[t2]];
#pragma unroll
        for (int u = 0; u < R; ++u)
#pragma unroll
            for (int w = 0; w < R; ++w) acc += (double)v[u][w];
        out[C] = (T)(acc / ((double)R * R));
    }
}

template <typename T>
hipError_t launch_restrict(const T* const fine[8], T* const coarse[8], int nx, int ny, int nz,
                           int r, hipStream_t s)
{
    const size_t Nc = (size_t)(nx / r) * (ny / r) * (nz / r);
    if (r == 2 || r == 4 || r == 8) {
        RestrictArgs a;
        for (int q = 0; q < 8; ++q) { a.fine[q] = fine[q]; a.coarse[q] = coarse[q]; }
        a.nx = nx; a.ny = ny; a.nz = nz;
        const unsigned blocks = (unsigned)((8 * Nc + 255) / 256);
        if (r == 2) hipLaunchKernelGGL((restrict_fixed_kernel<T, 2>), dim3(blocks), dim3(256), 0, s, a);
        else if (r == 4) hipLaunchKernelGGL((restrict_fixed_kernel<T, 4>), dim3(blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((restrict_fixed_kernel<T, 8>), dim3(blocks), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const unsigned blocks = (unsigned)((Nc + 255) / 256);
    hipLaunchKernelGGL(restrict_kernel<T>, dim3(blocks), dim3(256), 0, s, fine[0], fine[1], fine[2],
                       fine[3], fine[4], fine[5], fine[6], fine[7], coarse[0], coarse[1], coarse[2],
                       coarse[3], coarse[4], coarse[5], coarse[6], coarse[7], nx, ny, nz, r);
    return hipGetLastError();
}
template hipError_t launch_restrict<float>(const float* const[8], float* const[8], int, int, int,
                                           int, hipStream_t);
template hipError_t launch_restrict<double>(const double* const[8], double* const[8], int, int,
                                            int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Scalars
// ---------------------------------------------------------------------------

__global__ void set_scalars_kernel(double* scal, double dt, double c, int* flag, int clear_flag)
{
    if (threadIdx.x == 0) {
        scal[SCAL_DT] = dt;
        if (c > 0.0) scal[SCAL_C] = c;    // c <= 0: keep the device value
        if (clear_flag) flag[0] = 0;
    }
}

hipError_t launch_set_scalars(double* scal, double dt, double c, int* flag, int clear_flag,
                              hipStream_t s)
{
    hipLaunchKernelGGL(set_scalars_kernel, dim3(1), dim3(64), 0, s, scal, dt, c, flag, clear_flag);
    return hipGetLastError();
}

// Time advance of one full step (2 dt) unless a non-physical state was
// recorded (nonphys may be null); counts the steps that ran (steps may be
// null).
__global__ void advance_time_kernel(double* scal, const int* nonphys, int* steps)
{
    if (threadIdx.x == 0 && (nonphys == nullptr || *nonphys == 0)) {
        scal[SCAL_TIME] += 2.0 * scal[SCAL_DT];
        if (steps) *steps += 1;
    }
}

hipError_t launch_advance_time(double* scal, const int* nonphys, int* steps, hipStream_t s)
{
    hipLaunchKernelGGL(advance_time_kernel, dim3(1), dim3(64), 0, s, scal, nonphys, steps);
    return hipGetLastError();
}

}  // namespace mhd
