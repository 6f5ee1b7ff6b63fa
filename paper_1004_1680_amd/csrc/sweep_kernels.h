// Sweep kernels (templates) of the MHD update step for gfx950 (section II.B of Pang, Pen
// & Perrone, arXiv:1004.1680): the relaxing-TVD fluid operator F_d and the
// constrained-transport magnetic operator M_d along each axis d.
//
// Memory is structure of arrays with x fastest.  Two thread mappings keep
// every global access coalesced without a global transpose:
//  * x sweeps ("row" kernels): a row of the grid is contiguous; each thread
//    owns 4 consecutive cells of a row and loads them with one vector load
//    per field; stencil neighbours across threads go through LDS.  A
//    workgroup holds whole rows, so the periodic wrap stays inside it.
//  * y and z sweeps ("march" kernels): each lane owns one pencil along d;
//    the 64 lanes of a wave sit on consecutive x, so every load and store of
//    a wave is one contiguous run.  The lane walks along d keeping the
//    stencil in a register window (the two-stage scheme needs 3 cells of
//    look-ahead), so each input value is read once from memory.  A pencil
//    may be cut into chunks along d; each chunk re-reads a 6-cell warm-up.
// Neighbour pencils needed by the transverse field averages and by the
// edge velocities of constrained transport are read directly; they are the
// own data of adjacent lanes or adjacent workgroups and are served by the
// L1/L2 caches.  Workgroup indices are remapped so that consecutive tiles
// land on the same XCD (the hardware deals workgroups round-robin over the
// 8 XCDs, each with its own L2).
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mhd.h"
#include "mhd_device.h"
#include "mhd_kernels.h"

namespace mhd {

static_assert(LIM_VANLEER == MHD_LIMITER_VANLEER && LIM_MINMOD == MHD_LIMITER_MINMOD && LIM_MC == MHD_LIMITER_MC &&
                  LIM_SUPERBEE == MHD_LIMITER_SUPERBEE,
              "device limiter codes are the C ABI's");
static_assert(FRZ_STEP == MHD_FREEZE_STEP && FRZ_CELL == MHD_FREEZE_CELL && FRZ_PENCIL == MHD_FREEZE_PENCIL,
              "device freezing-speed codes are the C ABI's");

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Remap the hardware workgroup id so that XCD k (which receives ids
// k, k+8, k+16, ...) works on one contiguous range of logical tiles.
__device__ __forceinline__ int xcd_tile(int nblocks)
{
    const int b = blockIdx.x;
    const int per = nblocks >> 3;       // full rounds of 8
    if (b >= (per << 3)) return b;      // tail: identity
    return (b & 7) * per + (b >> 3);
}

template <typename T> struct vec4;
template <> struct vec4<float> {
    static __device__ __forceinline__ void load(const float* p, float o[4])
    {
        const float4 v = *reinterpret_cast<const float4*>(p);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
    static __device__ __forceinline__ void store(float* p, const float o[4])
    {
        *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
    }
};
template <> struct vec4<double> {
    static __device__ __forceinline__ void load(const double* p, double o[4])
    {
        const double2 a = reinterpret_cast<const double2*>(p)[0];
        const double2 b = reinterpret_cast<const double2*>(p)[1];
        o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    }
    static __device__ __forceinline__ void store(double* p, const double o[4])
    {
        reinterpret_cast<double2*>(p)[0] = make_double2(o[0], o[1]);
        reinterpret_cast<double2*>(p)[1] = make_double2(o[2], o[3]);
    }
};

template <typename T>
__device__ __forceinline__ void step_scalars(const SweepParams<T>& P, T& tau, T& halftau, T& c)
{
    const double dt = P.scal[SCAL_DT];
    tau = T(dt * (double)P.nx);          // dt / h with h = 1/nx
    halftau = T(0.5) * tau;
    c = T(P.scal[SCAL_C]);
}

// ---------------------------------------------------------------------------
// x sweeps: row kernels
// ---------------------------------------------------------------------------
// Launch: blockDim = rows_per_wg * tpr threads (tpr = nx/4 threads per row),
// grid = ceil(ny*nz / rows_per_wg) workgroups; dynamic LDS = 25 * blockDim
// values of T (fluid, and the fused magnetic-fluid pair) or 16 * blockDim
// (magnetic).

// Element offsets of the row kernels.  W32: every field of the grid fits in
// 4 GiB, offsets are 32-bit and an access is the field's (uniform) base
// plus one 32-bit byte offset per lane; otherwise 64-bit element offsets.
template <typename T, bool W32>
struct RowAddr {
    using off = std::conditional_t<W32, unsigned, size_t>;
    static __device__ __forceinline__ const T* at(const T* p, off e)
    {
        if constexpr (W32) return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + e * (unsigned)sizeof(T));
        else return p + e;
    }
    static __device__ __forceinline__ T* at(T* p, off e)
    {
        if constexpr (W32) return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + e * (unsigned)sizeof(T));
        else return p + e;
    }
    // offset of row (y, z)
    static __device__ __forceinline__ off row(int nx, int ny, int y, int z)
    {
        return (off)nx * ((off)y + (off)ny * (off)z);
    }
};

// Row geometry of one thread: row of the grid, position in it, neighbours
// in the row (for the LDS exchanges).  Idle threads (rloc >= rows_per_wg)
// exchange with themselves, so every LDS index stays below blockDim.x.
struct RowThread {
    int t, tprev, tnext, i0, y, z;
    int row0, tr, tpr;       // first thread of the row, position in it, threads per row
    bool active, inrow;
    __device__ __forceinline__ RowThread(int tile, int tpr_, int rows_per_wg, int ny, int nz)
    {
        t = threadIdx.x;
        tpr = tpr_;
        const int rloc = t / tpr;
        tr = t - rloc * tpr;
        const int row = tile * rows_per_wg + rloc;
        active = rloc < rows_per_wg && row < ny * nz;
        y = active ? row % ny : 0;
        z = active ? row / ny : 0;
        inrow = rloc < rows_per_wg;
        row0 = rloc * tpr;
        tprev = inrow ? rloc * tpr + (tr == 0 ? tpr - 1 : tr - 1) : t;
        tnext = inrow ? rloc * tpr + (tr == tpr - 1 ? 0 : tr + 1) : t;
        i0 = 4 * tr;
    }
};

// Freezing speed of the 4 cells of a row thread for one stage (state w,
// field bb): FRZ_STEP the step's c; FRZ_CELL |v_n| + c_fast of each cell;
// FRZ_PENCIL the largest of those along the row, an all-reduce over the
// row's threads by doubling windows in S (blockDim.x values of LDS, free
// on entry; free again on return).  Every thread of the workgroup calls it.
template <typename T, int FRZ>
__device__ __forceinline__ void row_stage_speeds(const T (&w)[4][5], const T (&bb)[4][3], T gamma, T c,
                                                 const RowThread& R, T* const S, T (&cs)[4])
{
    if constexpr (FRZ == FRZ_STEP) {
#pragma unroll
        for (int k = 0; k < 4; ++k) cs[k] = c;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) cs[k] = normal_speed(w[k], bb[k], gamma);
        if constexpr (FRZ == FRZ_PENCIL) {
            T v = fmax(fmax(cs[0], cs[1]), fmax(cs[2], cs[3]));
            // after the round with offset s each thread holds the maximum of
            // the 2s threads tr .. tr+2s-1 of its row (cyclically)
            for (int s = 1; s < R.tpr; s <<= 1) {
                S[R.t] = v;
                __syncthreads();
                const T o = S[R.inrow ? R.row0 + (R.tr + s) % R.tpr : R.t];
                __syncthreads();
                v = fmax(v, o);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) cs[k] = v;
        }
    }
}

// x fluid operator from given inputs: U of the thread's 4 cells, the frozen
// Bbar, and (CFL) the raw face values (own, next) of b_x, b_y, b_z for the
// fused CFL epilogue.  Stores the new U.  A: LDS of 25 values per thread.
// Every thread of the workgroup calls it (it holds barriers).
// CFL = true: the FP64 signal speed of every output cell, maximum per wave,
// atomic maximum into P.cfl_acc; needs full waves (blockDim.x a multiple of
// 64).
template <typename T, bool CFL, int LIM = LIM_VANLEER, int FRZ = FRZ_STEP, bool W32 = false>
__device__ __forceinline__ void fluid_x_core(const SweepParams<T>& P, const RowThread& R,
                                             typename RowAddr<T, W32>::off base,
                                             const T (&u)[4][5], const T (&bb)[4][3],
                                             const T (&fb)[CFL ? 4 : 1][6], T* const A)
{
    T* const B = A + 20 * blockDim.x;                       // A: 20, B: 5 values / thread
    const int nt = blockDim.x;
    const int t = R.t, tprev = R.tprev, tnext = R.tnext;
    T tau, halftau, c;
    step_scalars(P, tau, halftau, c);
    const T gamma = P.gamma;

    // stage 1: relaxed split and first-order upwind interface fluxes
    T fr[4][5], fl[4][5];
    T cs[4];
    row_stage_speeds<T, FRZ>(u, bb, gamma, c, R, A, cs);
#pragma unroll
    for (int k = 0; k < 4; ++k) relax_split(u[k], bb[k], gamma, cs[k], fr[k], fl[k]);
    // LDS regions alternate A, B, A, B between the four exchanges: a region
    // is rewritten only after the barrier that follows its last read.
    // exchange 1: F^L of the first cell goes to the previous thread
#pragma unroll
    for (int q = 0; q < 5; ++q) A[q * nt + t] = fl[0][q];
    __syncthreads();
    T f1[4][5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const T flnext = A[q * nt + tnext];
#pragma unroll
        for (int k = 0; k < 4; ++k) f1[k][q] = fr[k][q] - (k < 3 ? fl[k + 1][q] : flnext);
    }
    // exchange 2: interface flux of the last cell goes to the next thread
#pragma unroll
    for (int q = 0; q < 5; ++q) B[q * nt + t] = f1[3][q];
    __syncthreads();
    T uh[4][5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const T f1prev = B[q * nt + tprev];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            uh[k][q] = sub_scaled(u[k][q], halftau, f1[k][q] - (k > 0 ? f1[k - 1][q] : f1prev));
    }

    // stage 2: fluxes of the half-step state, van Leer limited (region A
    // was last read before the previous barrier)
    row_stage_speeds<T, FRZ>(uh, bb, gamma, c, R, A, cs);
#pragma unroll
    for (int k = 0; k < 4; ++k) relax_split(uh[k], bb[k], gamma, cs[k], fr[k], fl[k]);
    // exchange 3: edge values of the stage-2 parts
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        A[(0 + q) * nt + t] = fr[3][q];     // last F^R -> next thread
        A[(5 + q) * nt + t] = fr[0][q];     // first F^R -> previous thread
        A[(10 + q) * nt + t] = fl[0][q];    // first two F^L -> previous thread
        A[(15 + q) * nt + t] = fl[1][q];
    }
    __syncthreads();
    T phi[4][5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const T frprev = A[(0 + q) * nt + tprev];
        const T frnext = A[(5 + q) * nt + tnext];
        const T flnext0 = A[(10 + q) * nt + tnext];
        const T flnext1 = A[(15 + q) * nt + tnext];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T rm = k > 0 ? fr[k - 1][q] : frprev;
            const T rp = k < 3 ? fr[k + 1][q] : frnext;
            const T lp = k < 3 ? fl[k + 1][q] : flnext0;
            const T lpp = k < 2 ? fl[k + 2][q] : (k == 2 ? flnext0 : flnext1);
            phi[k][q] = limited_right<T, LIM>(rm, fr[k][q], rp) - limited_left<T, LIM>(fl[k][q], lp, lpp);
        }
    }
    // exchange 4: net flux of the last interface goes to the next thread
#pragma unroll
    for (int q = 0; q < 5; ++q) B[q * nt + t] = phi[3][q];
    __syncthreads();
    if constexpr (!CFL) {
        if (!R.active) return;
    }
    T onew[CFL ? 4 : 1][5] = {};
    if (R.active) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const T phiprev = B[q * nt + tprev];
            T o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] = sub_scaled(u[k][q], tau, phi[k][q] - (k > 0 ? phi[k - 1][q] : phiprev));
            vec4<T>::store(RowAddr<T, W32>::at(P.out[q], base + R.i0), o);
            if constexpr (CFL)
#pragma unroll
                for (int k = 0; k < 4; ++k) onew[k][q] = o[k];
        }
    }
    if constexpr (CFL) {
        // the CFL of the state this operator leaves (the last of a step),
        // from the values as stored; every lane of the wave takes part
        double vmax = 0.0;
        int bad = 0;
        const int slot = blockIdx.x & (CFL_ACC_SLOTS - 1);
        // FP32 tier: cells that surely cannot raise the maximum already in
        // this workgroup's slot (a speed found for this state, at most the
        // final maximum), nor exceed a cell of the wave that is evaluated,
        // skip the FP64 evaluation; every cell that is not surely physical
        // is evaluated, so the flag is exact too
        double tslot = 0.0, thr = 0.0;
        float ub[4];
        bool sure[4];
        if constexpr (sizeof(T) == 4) {
            tslot = __longlong_as_double((long long)__hip_atomic_load(P.cfl_acc + slot, __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_AGENT));
            // and a lower bound of a surely physical cell of the wave: the
            // largest over the wave of the lower bound of each lane's cell
            // with the largest upper bound (any cell's lower bound is a
            // speed the state reaches)
            float bub = -1.0f, bam = 0.0f, bxl = 0.0f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float am, xl;
                screen_upper32(onew[k][0], onew[k][1], onew[k][2], onew[k][3], onew[k][4], fb[k][0], fb[k][1],
                               fb[k][2], fb[k][3], fb[k][4], fb[k][5], (float)P.gamma, ub[k], am, xl, sure[k]);
                sure[k] = sure[k] && R.active;
                if (sure[k] && ub[k] > bub) { bub = ub[k]; bam = am; bxl = xl; }
            }
            float wlb = bub >= 0.0f ? screen_lower32(bam, bxl) : 0.0f;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) wlb = fmaxf(wlb, __shfl_xor(wlb, o, 64));
            thr = fmax(tslot, (double)wlb);
        }
        if constexpr (sizeof(T) == 4) {
            // the cells to evaluate are packed over the wave through LDS
            // (region A, free since the last barrier; 64 x 11 values per
            // wave) and evaluated 64 at a time, one per lane: the few cells
            // near a wave's maximum usually sit in one lane (4 consecutive
            // cells), whose 4 evaluations would otherwise run one after
            // the other with the rest of the wave idle
            const int lane = threadIdx.x & 63;
            const unsigned long long below = (1ull << lane) - 1ull;
            bool nd[4];
            int idx[4];
            int total = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                nd[k] = R.active && (!sure[k] || (double)ub[k] >= thr);
                const unsigned long long bal = __ballot(nd[k]);
                idx[k] = total + __popcll(bal & below);
                total += __popcll(bal);
            }
            float* const E = reinterpret_cast<float*>(A) + (threadIdx.x >> 6) * (64 * 11);
            for (int r = 0; r < total; r += 64) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (nd[k] && idx[k] >= r && idx[k] < r + 64) {
                        const int e = idx[k] - r;
#pragma unroll
                        for (int q = 0; q < 5; ++q) E[q * 64 + e] = onew[k][q];
#pragma unroll
                        for (int q = 0; q < 6; ++q) E[(5 + q) * 64 + e] = fb[k][q];
                    }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane < total - r) {
                    float c[11];
#pragma unroll
                    for (int q = 0; q < 11; ++q) c[q] = E[q * 64 + lane];
                    signal_speed64((double)c[0], (double)c[1], (double)c[2], (double)c[3], (double)c[4],
                                   (double)c[5], (double)c[6], (double)c[7], (double)c[8], (double)c[9],
                                   (double)c[10], P.gamma64, vmax, bad);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            // a persistent caller's next tile writes region A before its
            // first barrier
            __syncthreads();
        } else if (R.active) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                signal_speed64((double)onew[k][0], (double)onew[k][1], (double)onew[k][2], (double)onew[k][3],
                               (double)onew[k][4], (double)fb[k][0], (double)fb[k][1], (double)fb[k][2],
                               (double)fb[k][3], (double)fb[k][4], (double)fb[k][5], P.gamma64, vmax, bad);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            vmax = fmax(vmax, __shfl_xor(vmax, o, 64));
            bad |= __shfl_xor(bad, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            // a non-negative double orders like its bit pattern
            if (vmax > tslot)
                atomicMax(P.cfl_acc + slot, (unsigned long long)__double_as_longlong(vmax));
            if (bad) atomicOr(P.cfl_acc + CFL_ACC_SLOTS, 1ull);
        }
    }
}

// U of the thread's 4 cells (inactive threads: rho = 1, a harmless state)
template <typename T, bool W32 = false>
__device__ __forceinline__ void load_u4(const SweepParams<T>& P, const RowThread& R,
                                        typename RowAddr<T, W32>::off base, T (&u)[4][5])
{
    T tmp[4];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        if (R.active) vec4<T>::load(RowAddr<T, W32>::at(P.in[q], base + R.i0), tmp);
        else tmp[0] = tmp[1] = tmp[2] = tmp[3] = T(1);
#pragma unroll
        for (int k = 0; k < 4; ++k) u[k][q] = tmp[k];
    }
}

// One tile of rows_per_wg rows of one grid: fluid operator F_x.
template <typename T, bool CFL = false, int LIM = LIM_VANLEER, int FRZ = FRZ_STEP, bool W32 = false>
__device__ __forceinline__ void fluid_x_tile(const SweepParams<T>& P, int tile, int tpr,
                                             int rows_per_wg, T* const A)
{
    using RA = RowAddr<T, W32>;
    using off = typename RA::off;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const RowThread R(tile, tpr, rows_per_wg, ny, nz);
    const int y = R.y, z = R.z, i0 = R.i0;
    const bool active = R.active;
    const off base = RA::row(nx, ny, y, z);
    const off base_yp = RA::row(nx, ny, y + 1 == ny ? 0 : y + 1, z);
    const off base_zp = RA::row(nx, ny, y, z + 1 == nz ? 0 : z + 1);

    if (P.flag && *P.flag) {      // non-physical state recorded: keep the state
        if (active)
            for (int f = 0; f < 5; ++f) {
                T v[4];
                vec4<T>::load(RA::at(P.in[f], base + i0), v);
                vec4<T>::store(RA::at(P.out[f], base + i0), v);
            }
        // the record (1 non-physical, 2 zero signal speed) carries over to
        // the CFL that follows, as the separate reduction would find it
        if constexpr (CFL)
            if (threadIdx.x == 0) atomicOr(P.cfl_acc + CFL_ACC_SLOTS, (unsigned long long)*P.flag);
        return;
    }

    T u[4][5], bb[4][3];
    T fb[CFL ? 4 : 1][6];         // fused CFL: raw face values (own, next) of b_x, b_y, b_z
    load_u4<T, W32>(P, R, base, u);
    {
        T tmp[4], tmp2[4];
        // Bbar_x: faces i and i+1 along the row
        T bxn = T(0);
        if (active) {
            vec4<T>::load(RA::at(P.in[BX], base + i0), tmp);
            bxn = *RA::at(P.in[BX], base + (i0 + 4 == nx ? 0 : i0 + 4));
        } else tmp[0] = tmp[1] = tmp[2] = tmp[3] = T(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) bb[k][0] = T(0.5) * (tmp[k] + (k < 3 ? tmp[k + 1] : bxn));
        if constexpr (CFL)
#pragma unroll
            for (int k = 0; k < 4; ++k) { fb[k][0] = tmp[k]; fb[k][1] = k < 3 ? tmp[k + 1] : bxn; }
        // Bbar_y: faces at y and y+1; Bbar_z: faces at z and z+1
        if (active) { vec4<T>::load(RA::at(P.in[BY], base + i0), tmp); vec4<T>::load(RA::at(P.in[BY], base_yp + i0), tmp2); }
        else tmp[0] = tmp[1] = tmp[2] = tmp[3] = tmp2[0] = tmp2[1] = tmp2[2] = tmp2[3] = T(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) bb[k][1] = T(0.5) * (tmp[k] + tmp2[k]);
        if constexpr (CFL)
#pragma unroll
            for (int k = 0; k < 4; ++k) { fb[k][2] = tmp[k]; fb[k][3] = tmp2[k]; }
        if (active) { vec4<T>::load(RA::at(P.in[BZ], base + i0), tmp); vec4<T>::load(RA::at(P.in[BZ], base_zp + i0), tmp2); }
        else tmp[0] = tmp[1] = tmp[2] = tmp[3] = tmp2[0] = tmp2[1] = tmp2[2] = tmp2[3] = T(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) bb[k][2] = T(0.5) * (tmp[k] + tmp2[k]);
        if constexpr (CFL)
#pragma unroll
            for (int k = 0; k < 4; ++k) { fb[k][4] = tmp[k]; fb[k][5] = tmp2[k]; }
    }
    fluid_x_core<T, CFL, LIM, FRZ, W32>(P, R, base, u, bb, fb, A);
}

template <typename T, bool CFL, int LIM = LIM_VANLEER, int FRZ = FRZ_STEP, bool W32 = false>
__global__ void __launch_bounds__(256) fluid_x_kernel(SweepParams<T> P, int tpr, int rows_per_wg, int st)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tile = row_tile(xcd_tile(gridDim.x), st, P.ny / rows_per_wg, P.nz);
    fluid_x_tile<T, CFL, LIM, FRZ, W32>(P, tile, tpr, rows_per_wg, reinterpret_cast<T*>(smem_raw));
}

// Magnetic operator along x (e = y then z) of the thread's 4 cells.  For
// each e two edge-flux chains are evaluated: "own" (edges of this row,
// velocity from rows P and P-e) and "plus" (edges of row P+e, velocity from
// rows P+e and P), the latter for the constraint update of b_x; a plus
// chain is the own chain of the neighbour row, evaluated identically.
// Gives the new faces nb = (b_y of P, b_y of P+y, b_z of P, b_z of P+z, b_x
// of P) of the 4 cells; stores nothing.  own (optional): rho and m_x of
// the thread's 4 cells as loaded.  A: LDS of 16 values per thread.
// Every thread of the workgroup calls it (it holds barriers).
template <typename T, int LIM = LIM_VANLEER, bool W32 = false>
__device__ __forceinline__ void mag_x_core(const SweepParams<T>& P, const RowThread& R, T (&nb)[5][4],
                                           T* const A, T (*own)[4] = nullptr)
{
    using RA = RowAddr<T, W32>;
    using off = typename RA::off;
    T* const B = A + 12 * blockDim.x;                       // A: 12, B: 4 values / thread
    const int nt = blockDim.x;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int t = R.t, tprev = R.tprev, tnext = R.tnext, i0 = R.i0, y = R.y, z = R.z;
    const bool active = R.active;
    auto rbase = [&](int yy, int zz) -> off {
        return RA::row(nx, ny, wrapi(yy, ny), wrapi(zz, nz));
    };
    const off b0 = rbase(y, z);
    T tau, halftau, cdummy;
    step_scalars(P, tau, halftau, cdummy);

    // velocity v_x at 5 positions (i0..i0+4) of the rows P, P-y, P+y, P-z, P+z
    // rows index: 0 P, 1 P-y, 2 P+y, 3 P-z, 4 P+z
    T v[5][5];
    {
        const off rb[5] = { b0, rbase(y - 1, z), rbase(y + 1, z), rbase(y, z - 1), rbase(y, z + 1) };
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            T rho[4], m[4];
            if (active) {
                vec4<T>::load(RA::at(P.in[RHO], rb[r] + i0), rho);
                vec4<T>::load(RA::at(P.in[MX], rb[r] + i0), m);
            } else {
                rho[0] = rho[1] = rho[2] = rho[3] = T(1);
                m[0] = m[1] = m[2] = m[3] = T(0);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) v[r][k] = velocity(m[k], rho[k]);
            if (r == 0 && own) {                  // rho and m_x of the thread's own cells
#pragma unroll
                for (int k = 0; k < 4; ++k) { own[0][k] = rho[k]; own[1][k] = m[k]; }
            }
        }
    }
    // chains: 0 own-y, 1 plus-y, 2 own-z, 3 plus-z
    // velocity rows of each chain: (pencil, pencil - e)
    const int vr0[4] = { 0, 2, 0, 4 };
    const int vr1[4] = { 1, 0, 3, 0 };
    T q[4][5];
    {
        const off qb[4] = { b0, rbase(y + 1, z), b0, rbase(y, z + 1) };
        const int qf[4] = { BY, BY, BZ, BZ };
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            T tmp[4];
            if (active) vec4<T>::load(RA::at(P.in[qf[ch]], qb[ch] + i0), tmp);
            else tmp[0] = tmp[1] = tmp[2] = tmp[3] = T(0);
#pragma unroll
            for (int k = 0; k < 4; ++k) q[ch][k] = tmp[k];
        }
    }
    // exchange 0: the next cell's velocities and q (the next thread's first
    // cell; the row wraps) through LDS rather than loaded and divided again
#pragma unroll
    for (int r = 0; r < 5; ++r) A[r * nt + t] = v[r][0];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) A[(5 + ch) * nt + t] = q[ch][0];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 5; ++r) v[r][4] = A[r * nt + tnext];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) q[ch][4] = A[(5 + ch) * nt + tnext];
    T a[4][4], g[4][4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        T w[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) w[k] = face_avg(v[vr0[ch]][k], v[vr1[ch]][k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[ch][k] = edge_avg(w[k], w[k + 1]);
            g[ch][k] = upwind_flux1(a[ch][k], q[ch][k], q[ch][k + 1]);
        }
    }
    // exchange 1: last first-order flux -> next thread
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) B[ch * nt + t] = g[ch][3];
    __syncthreads();
    T qh[4][4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        const T gprev = B[ch * nt + tprev];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            qh[ch][k] = sub_scaled(q[ch][k], halftau, g[ch][k] - (k > 0 ? g[ch][k - 1] : gprev));
    }
    // exchange 2: half-step values at the thread edges
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        A[(0 + ch) * nt + t] = qh[ch][3];
        A[(4 + ch) * nt + t] = qh[ch][0];
        A[(8 + ch) * nt + t] = qh[ch][1];
    }
    __syncthreads();
    T f[4][4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        const T qm1 = A[(0 + ch) * nt + tprev];
        const T qp0 = A[(4 + ch) * nt + tnext];
        const T qp1 = A[(8 + ch) * nt + tnext];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T qm = k > 0 ? qh[ch][k - 1] : qm1;
            const T q1 = k < 3 ? qh[ch][k + 1] : qp0;
            const T q2 = k < 2 ? qh[ch][k + 2] : (k == 2 ? qp0 : qp1);
            f[ch][k] = upwind_flux2<T, LIM>(a[ch][k], qm, qh[ch][k], q1, q2);
        }
    }
    // exchange 3: last edge flux -> next thread (region B was last read
    // before the previous barrier)
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) B[ch * nt + t] = f[ch][3];
    __syncthreads();
    T fprev[4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) fprev[ch] = B[ch * nt + tprev];
    T bx[4];
    if (active) vec4<T>::load(RA::at(P.in[BX], b0 + i0), bx);
    else bx[0] = bx[1] = bx[2] = bx[3] = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T fo_y = k > 0 ? f[0][k - 1] : fprev[0];
        const T fp_y = k > 0 ? f[1][k - 1] : fprev[1];
        const T fo_z = k > 0 ? f[2][k - 1] : fprev[2];
        const T fp_z = k > 0 ? f[3][k - 1] : fprev[3];
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            const T fo = k > 0 ? f[ch][k - 1] : fprev[ch];
            nb[ch][k] = sub_scaled(q[ch][k], tau, f[ch][k] - fo);
        }
        const T b = add_scaled(bx[k], tau, fp_y - fo_y);
        nb[4][k] = add_scaled(b, tau, fp_z - fo_z);
    }
}

// One tile of rows_per_wg rows of one grid: magnetic operator M_x.
template <typename T, int LIM = LIM_VANLEER, bool W32 = false>
__device__ __forceinline__ void mag_x_tile(const SweepParams<T>& P, int tile, int tpr,
                                           int rows_per_wg, T* const A)
{
    using RA = RowAddr<T, W32>;
    const int nx = P.nx, ny = P.ny;
    const RowThread R(tile, tpr, rows_per_wg, ny, P.nz);
    const typename RA::off b0 = RA::row(nx, ny, R.y, R.z);
    if (P.flag && *P.flag) {
        if (R.active)
            for (int f = BX; f <= BZ; ++f) {
                T v[4];
                vec4<T>::load(RA::at(P.in[f], b0 + R.i0), v);
                vec4<T>::store(RA::at(P.out[f], b0 + R.i0), v);
            }
        return;
    }
    T nb[5][4];
    mag_x_core<T, LIM, W32>(P, R, nb, A);
    if (!R.active) return;
    vec4<T>::store(RA::at(P.out[BY], b0 + R.i0), nb[0]);
    vec4<T>::store(RA::at(P.out[BZ], b0 + R.i0), nb[2]);
    vec4<T>::store(RA::at(P.out[BX], b0 + R.i0), nb[4]);
}

template <typename T, int LIM = LIM_VANLEER, bool W32 = false>
__global__ void __launch_bounds__(256) mag_x_kernel(SweepParams<T> P, int tpr, int rows_per_wg, int st)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tile = row_tile(xcd_tile(gridDim.x), st, P.ny / rows_per_wg, P.nz);
    mag_x_tile<T, LIM, W32>(P, tile, tpr, rows_per_wg, reinterpret_cast<T*>(smem_raw));
}

// One tile of rows: the reverse-half pair M_x then F_x in one pass.  The new
// faces stay in registers: Bbar_y and Bbar_z take b_y, b_z of rows P+y, P+z
// from the plus chains, Bbar_x takes the next cell's new b_x through LDS.
// Same device functions in the same order as mag_x_tile followed by
// fluid_x_tile, so the result is bitwise that of the two operators.  A: LDS
// of 25 values per thread (the magnetic part uses the first 16; the b_x
// exchange uses values 20..21, which the fluid part first writes after a
// barrier that follows its last read).
template <typename T, bool CFL = false, int LIM = LIM_VANLEER, bool W32 = false>
__device__ __forceinline__ void magfluid_x_tile(const SweepParams<T>& P, int tile, int tpr,
                                                int rows_per_wg, T* const A)
{
    using RA = RowAddr<T, W32>;
    const int nx = P.nx, ny = P.ny;
    const RowThread R(tile, tpr, rows_per_wg, ny, P.nz);
    const typename RA::off base = RA::row(nx, ny, R.y, R.z);
    if (P.flag && *P.flag) {
        if (R.active)
            for (int f = 0; f < NFIELD; ++f) {
                T v[4];
                vec4<T>::load(RA::at(P.in[f], base + R.i0), v);
                vec4<T>::store(RA::at(P.out[f], base + R.i0), v);
            }
        // the record (1 non-physical, 2 zero signal speed) carries over to
        // the CFL that follows, as the separate reduction would find it
        if constexpr (CFL)
            if (threadIdx.x == 0) atomicOr(P.cfl_acc + CFL_ACC_SLOTS, (unsigned long long)*P.flag);
        return;
    }
    T nb[5][4];
    T own[2][4];
    mag_x_core<T, LIM, W32>(P, R, nb, A, own);
    // new b_x of the first cell -> previous thread
    T* const X = A + 20 * blockDim.x;
    X[R.t] = nb[4][0];
    __syncthreads();
    const T bxn = X[R.tnext];
    if (R.active) {
        vec4<T>::store(RA::at(P.out[BY], base + R.i0), nb[0]);
        vec4<T>::store(RA::at(P.out[BZ], base + R.i0), nb[2]);
        vec4<T>::store(RA::at(P.out[BX], base + R.i0), nb[4]);
    }
    T u[4][5], bb[4][3];
    T fb[CFL ? 4 : 1][6];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T bx1 = k < 3 ? nb[4][k + 1] : bxn;
        bb[k][0] = T(0.5) * (nb[4][k] + bx1);
        bb[k][1] = T(0.5) * (nb[0][k] + nb[1][k]);
        bb[k][2] = T(0.5) * (nb[2][k] + nb[3][k]);
        if constexpr (CFL) {
            fb[k][0] = nb[4][k]; fb[k][1] = bx1;
            fb[k][2] = nb[0][k]; fb[k][3] = nb[1][k];
            fb[k][4] = nb[2][k]; fb[k][5] = nb[3][k];
        }
    }
    // U: rho and m_x as the magnetic part loaded them (the same values; the
    // reciprocal of rho is then shared), m_y, m_z, e loaded here
    {
        T tmp[4];
#pragma unroll
        for (int q = 2; q < 5; ++q) {
            if (R.active) vec4<T>::load(RA::at(P.in[q], base + R.i0), tmp);
            else tmp[0] = tmp[1] = tmp[2] = tmp[3] = T(1);     // as load_u4
#pragma unroll
            for (int k = 0; k < 4; ++k) u[k][q] = tmp[k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) { u[k][0] = own[0][k]; u[k][1] = own[1][k]; }
    }
    fluid_x_core<T, CFL, LIM, FRZ_STEP, W32>(P, R, base, u, bb, fb, A);
}

template <typename T, bool CFL, int LIM = LIM_VANLEER, bool W32 = false>
__global__ void __launch_bounds__(256) magfluid_x_kernel(SweepParams<T> P, int tpr, int rows_per_wg, int st)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tile = row_tile(xcd_tile(gridDim.x), st, P.ny / rows_per_wg, P.nz);
    magfluid_x_tile<T, CFL, LIM, W32>(P, tile, tpr, rows_per_wg, reinterpret_cast<T*>(smem_raw));
}

// ---------------------------------------------------------------------------
// y and z sweeps: march kernels
// ---------------------------------------------------------------------------
// Lane -> pencil: p = x + nx * w over the transverse plane (w = z for a y
// sweep, w = y for a z sweep); global lane id = chunk * npencil + p.
// Launch: 256 threads, grid = ceil(npencil * nchunks / 256).  The state has
// fewer than 2^31 cells per field, so offsets are 32-bit.
//
// The march runs in groups of U positions whose body is unrolled, so the
// register window moves by renaming instead of copying; the start is moved
// back by up to U-1 extra warm-up positions to make the count a multiple of
// U (positions before the chunk produce no output).

template <int D> struct MarchGeom {
    int nd;              // pencil length
    unsigned sd;         // stride along d
    unsigned base;       // offset of (pencil, 0)
    unsigned b_t1p, b_t2p, b_t1m, b_t2m;   // bases of pencils P+t1, P+t2, P-t1, P-t2
    __device__ MarchGeom(int nx, int ny, int nz, int p)
    {
        const int x = p % nx, w = p / nx;
        const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
        if (D == 1) {           // n = y, t1 = z, t2 = x; w = z
            const unsigned sz = (unsigned)nx * ny;
            const int zp = w + 1 == nz ? 0 : w + 1, zm = w == 0 ? nz - 1 : w - 1;
            nd = ny; sd = nx;
            base = x + sz * w;
            b_t1p = x + sz * zp;  b_t1m = x + sz * zm;
            b_t2p = xp + sz * w;  b_t2m = xm + sz * w;
        } else {                // n = z, t1 = x, t2 = y; w = y
            const int yp = w + 1 == ny ? 0 : w + 1, ym = w == 0 ? ny - 1 : w - 1;
            nd = nz; sd = (unsigned)nx * ny;
            base = x + (unsigned)nx * w;
            b_t1p = xp + (unsigned)nx * w;  b_t1m = xm + (unsigned)nx * w;
            b_t2p = x + (unsigned)nx * yp;  b_t2m = x + (unsigned)nx * ym;
        }
    }
};

// positions unrolled per group: 4 in FP32; 2 in FP64, whose window takes
// twice the registers
template <typename T> constexpr int march_unroll() { return sizeof(T) == 4 ? 4 : 2; }

template <int U>
__device__ __forceinline__ int march_start(int j0, int chunk)
{
    const int total = chunk + 6;
    return j0 - 3 - ((U - (total % U)) % U);
}

// Register window of the fluid march (two-stage relaxing TVD along the
// pencil).  push() takes U and the frozen Bbar at the look-ahead position L
// and gives the new U of cell L-3; it needs U and Bbar at L-3 .. L+3, so
// pushes 6 positions before a chunk warm the window up (their results are
// not used).
template <typename T, int LIM = LIM_VANLEER, int FRZ = FRZ_STEP>
struct FluidWindow {
    T u3[5], u2[5], u1[5];            // U at L-3, L-2, L-1
    T bbm[3];                         // Bbar at L-1
    T frm[5];                         // stage-1 F^R at L-1
    T f1m[5];                         // stage-1 interface flux at L-3/2
    T r4[5], r3[5], r2[5];            // stage-2 F^R at L-4, L-3, L-2
    T l3[5], l2[5];                   // stage-2 F^L at L-3, L-2
    T phim[5];                        // net flux at interface (L-3)-1/2

    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            u3[q] = u2[q] = u1[q] = T(0);
            frm[q] = f1m[q] = r4[q] = r3[q] = r2[q] = l3[q] = l2[q] = phim[q] = T(0);
        }
        bbm[0] = bbm[1] = bbm[2] = T(0);
    }

    // c, c2: freezing speeds of stages 1 and 2 (the step's speed twice, or
    // the pencil's two maxima); FRZ_CELL takes each cell's own instead
    __device__ __forceinline__ void push(const T u0[5], const T bb0[3], T gamma, T c, T c2, T tau,
                                         T halftau, T unew[5])
    {
        // stage 1 at L: split, interface flux at L-1/2, half step at L-1
        T fr0[5], fl0[5], f1[5], uh[5];
        relax_split(u0, bb0, gamma, FRZ == FRZ_CELL ? normal_speed(u0, bb0, gamma) : c, fr0, fl0);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            f1[q] = frm[q] - fl0[q];
            uh[q] = sub_scaled(u1[q], halftau, f1[q] - f1m[q]);
        }
        // stage 2 at L-1
        T r1[5], l1[5];
        relax_split(uh, bbm, gamma, FRZ == FRZ_CELL ? normal_speed(uh, bbm, gamma) : c2, r1, l1);
        // net flux at interface (L-3)+1/2 and the update of cell L-3
        T phi[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            phi[q] = limited_right<T, LIM>(r4[q], r3[q], r2[q]) - limited_left<T, LIM>(l3[q], l2[q], l1[q]);
            unew[q] = sub_scaled(u3[q], tau, phi[q] - phim[q]);
        }
        // shift the window
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            phim[q] = phi[q];
            r4[q] = r3[q]; r3[q] = r2[q]; r2[q] = r1[q];
            l3[q] = l2[q]; l2[q] = l1[q];
            frm[q] = fr0[q]; f1m[q] = f1[q];
            u3[q] = u2[q]; u2[q] = u1[q]; u1[q] = u0[q];
        }
        bbm[0] = bb0[0]; bbm[1] = bb0[1]; bbm[2] = bb0[2];
    }
};

// Register window of the constrained-transport march.  Four edge-flux
// chains: 0 own-t1 (b_t1 of this pencil, velocity from P and P-t1), 1
// plus-t1 (b_t1 of pencil P+t1, velocity from P+t1 and P), 2 own-t2, 3
// plus-t2; a plus chain is the own chain of the neighbour pencil, evaluated
// identically, and feeds the constraint update of b_n.  push() takes the
// velocities v_n of the pencils (P, P-t1, P+t1, P-t2, P+t2), the chain
// fields and b_n at the look-ahead position L and gives the new faces at
// L-3: nb = (b_t1 of P, b_t1 of P+t1, b_t2 of P, b_t2 of P+t2, b_n of P).
// It needs inputs at L-3 .. L+3 (6 warm-up pushes, like the fluid window).
template <typename T, int LIM = LIM_VANLEER>
struct MagWindow {
    T wm[4];                 // face velocity at L-1
    T a3[4], a2[4];          // edge velocity at L-3, L-2
    T q3[4], q2[4], q1[4];   // q at L-3, L-2, L-1
    T gm[4];                 // first-order flux at L-2
    T h4[4], h3[4], h2[4];   // half-step q at L-4, L-3, L-2
    T fm[4];                 // edge flux at L-4
    T bnw[3];                // b_n at L-3, L-2, L-1

    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            wm[ch] = a3[ch] = a2[ch] = T(0);
            q3[ch] = q2[ch] = q1[ch] = gm[ch] = h4[ch] = h3[ch] = h2[ch] = fm[ch] = T(0);
        }
        bnw[0] = bnw[1] = bnw[2] = T(0);
    }

    __device__ __forceinline__ void push(const T v[5], const T q0[4], T bn0, T tau, T halftau, T nb[5])
    {
        // velocity pencils of each chain: (chain pencil, chain pencil - e)
        constexpr int vr0[4] = { 0, 2, 0, 4 };
        constexpr int vr1[4] = { 1, 0, 3, 0 };
        T a1[4];
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            const T w0 = face_avg(v[vr0[ch]], v[vr1[ch]]);       // w at L
            a1[ch] = edge_avg(wm[ch], w0);                       // a at L-1
            wm[ch] = w0;
        }
        push_edge(a1, q0, bn0, tau, halftau, nb);
    }

    // the same with the edge velocity a(L-1) of every chain given (a second
    // magnetic operator over the same velocity field reuses the first one's)
    __device__ __forceinline__ void push_edge(const T a1[4], const T q0[4], T bn0, T tau, T halftau, T nb[5])
    {
        T f[4];
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            const T g1 = upwind_flux1(a1[ch], q1[ch], q0[ch]);  // G1 at L-1
            const T hq1 = sub_scaled(q1[ch], halftau, g1 - gm[ch]);   // qh at L-1
            // edge flux at L-3 from a(L-3) and qh at L-4..L-1
            f[ch] = upwind_flux2<T, LIM>(a3[ch], h4[ch], h3[ch], h2[ch], hq1);
            a3[ch] = a2[ch]; a2[ch] = a1[ch];
            gm[ch] = g1;
            h4[ch] = h3[ch]; h3[ch] = h2[ch]; h2[ch] = hq1;
        }
        // advection of b_t1, b_t2 (own and plus pencils); constraint on b_n
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) nb[ch] = sub_scaled(q3[ch], tau, f[ch] - fm[ch]);
        const T b = add_scaled(bnw[0], tau, fm[1] - fm[0]);
        nb[4] = add_scaled(b, tau, fm[3] - fm[2]);
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            fm[ch] = f[ch];
            q3[ch] = q2[ch]; q2[ch] = q1[ch]; q1[ch] = q0[ch];
        }
        bnw[0] = bnw[1]; bnw[1] = bnw[2]; bnw[2] = bn0;
    }
};

// Lane -> (pencil p, chunk start j0) of a grid; false beyond the last lane.
template <int D>
__device__ __forceinline__ bool march_lane_of(int nx, int ny, int nz, long gid, int chunk, int& p, int& j0)
{
    const int npencil = nx * (D == 1 ? nz : ny);
    const int nchunk = (D == 1 ? ny : nz) / chunk;
    if (gid >= (long)npencil * nchunk) return false;
    p = (int)(gid % npencil);
    j0 = (int)(gid / npencil) * chunk;
    return true;
}

// Addressing of the march kernels.  W32: every byte offset of a field fits
// in 32 bits (FP32 grids up to 1024^3), so a load is the field's base (a
// wave-uniform register pair) plus a 32-bit per-lane byte offset, one add
// per pencil shared by all fields of that pencil; otherwise element offsets
// with 64-bit address arithmetic per access.  Offsets along the pencil
// advance by one stride per position instead of a multiply.
template <typename T, bool W32>
struct Addr {
    static constexpr unsigned scale = W32 ? (unsigned)sizeof(T) : 1u;
    static __device__ __forceinline__ T ld(const T* __restrict__ p, unsigned off)
    {
        if constexpr (W32) return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + off);
        else return p[off];
    }
    static __device__ __forceinline__ void st(T* p, unsigned off, T v)
    {
        if constexpr (W32) *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + off) = v;
        else p[off] = v;
    }
};

// a position along the pencil (periodic index j) and its scaled offset
struct MarchPos {
    int j;
    unsigned off;
    __device__ __forceinline__ void set(int jj, unsigned step)
    {
        j = jj;
        off = (unsigned)jj * step;
    }
    __device__ __forceinline__ void next(int nd, unsigned step)
    {
        if (++j == nd) { j = 0; off = 0u; }
        else off += step;
    }
};

// the periodic index of a (possibly negative) march position
__device__ __forceinline__ int wrap_pos(int j, int nd)
{
    int m = j % nd;
    return m < 0 ? m + nd : m;
}

// The two freezing speeds of the FRZ_PENCIL variant for one pencil: the
// largest |v_n| + c_fast of the old state (stage 1) and of the half-step
// state that stage 1 makes with it (stage 2), in two passes over the whole
// pencil with the march's own expressions (the same values as the row
// kernels find for an x pencil).  o_u: the five fluid fields of the pencil;
// bn, bt1, bt2 with bases gb (this pencil), gt1, gt2 (pencils P+t1, P+t2).
template <typename T, bool W32, typename UPtrs>
__device__ __forceinline__ void pencil_speeds(const UPtrs& in_u, const T* __restrict__ bn,
                                              const T* __restrict__ bt1, const T* __restrict__ bt2,
                                              unsigned gb, unsigned gt1, unsigned gt2, unsigned step, int nd,
                                              T gamma, T halftau, T& c1, T& c2)
{
    using A = Addr<T, W32>;
    auto load = [&](int j, T (&u)[5], T (&bb)[3]) {
        const int jn = j + 1 == nd ? 0 : j + 1;
        const unsigned o = (unsigned)j * step, on = (unsigned)jn * step;
#pragma unroll
        for (int q = 0; q < 5; ++q) u[q] = A::ld(in_u[q], gb + o);
        bb[0] = T(0.5) * (A::ld(bn, gb + o) + A::ld(bn, gb + on));
        bb[1] = T(0.5) * (A::ld(bt1, gb + o) + A::ld(bt1, gt1 + o));
        bb[2] = T(0.5) * (A::ld(bt2, gb + o) + A::ld(bt2, gt2 + o));
    };
    c1 = T(0);
    for (int j = 0; j < nd; ++j) {
        T u[5], bb[3];
        load(j, u, bb);
        c1 = fmax(c1, normal_speed(u, bb, gamma));
    }
    // stage 1 with c1 (as FluidWindow::push): at position L the split of L,
    // the interface flux at L-1/2 and the half-step state of cell L-1
    c2 = T(0);
    T frm[5] = {}, f1m[5] = {}, um[5] = {}, bbm[3] = {};
    for (int L = -1; L <= nd; ++L) {
        T u[5], bb[3], fr[5], fl[5];
        load(wrap_pos(L, nd), u, bb);
        relax_split(u, bb, gamma, c1, fr, fl);
        T f1[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) f1[q] = frm[q] - fl[q];
        if (L >= 1) {
            T uh[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) uh[q] = sub_scaled(um[q], halftau, f1[q] - f1m[q]);
            c2 = fmax(c2, normal_speed(uh, bbm, gamma));
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            frm[q] = fr[q];
            f1m[q] = f1[q];
            um[q] = u[q];
        }
        bbm[0] = bb[0]; bbm[1] = bb[1]; bbm[2] = bb[2];
    }
}

// One lane (pencil chunk gid) of a grid: fluid operator F_d.
template <typename T, int D, bool W32, int LIM = LIM_VANLEER, int FRZ = FRZ_STEP>
__device__ __forceinline__ void fluid_march_lane(const SweepParams<T>& P, long gid, int chunk)
{
    constexpr int N_ = D, T1 = (D + 1) % 3, T2 = (D + 2) % 3;
    using A = Addr<T, W32>;
    int p, j0;
    if (!march_lane_of<D>(P.nx, P.ny, P.nz, gid, chunk, p, j0)) return;
    const MarchGeom<D> G(P.nx, P.ny, P.nz, p);
    const int nd = G.nd;
    const T* __restrict__ in_u[5] = { P.in[RHO], P.in[MX + N_], P.in[MX + T1], P.in[MX + T2], P.in[EN] };
    T* out_u[5] = { P.out[RHO], P.out[MX + N_], P.out[MX + T1], P.out[MX + T2], P.out[EN] };
    const T* __restrict__ bn = P.in[BX + N_];
    const T* __restrict__ bt1 = P.in[BX + T1];
    const T* __restrict__ bt2 = P.in[BX + T2];

    if (P.flag && *P.flag) {
        for (int j = j0; j < j0 + chunk; ++j) {
            const unsigned o = G.base + G.sd * j;
            for (int q = 0; q < 5; ++q) out_u[q][o] = in_u[q][o];
        }
        return;
    }
    T tau, halftau, c;
    step_scalars(P, tau, halftau, c);
    const T gamma = P.gamma;
    const unsigned step = G.sd * A::scale;
    const unsigned gb = G.base * A::scale, gt1 = G.b_t1p * A::scale, gt2 = G.b_t2p * A::scale;
    T c2 = c;
    if constexpr (FRZ == FRZ_PENCIL) pencil_speeds<T, W32>(in_u, bn, bt1, bt2, gb, gt1, gt2, step, nd, gamma, halftau, c, c2);

    FluidWindow<T, LIM, FRZ> W;
    W.init();
    constexpr int U = march_unroll<T>();
    const int Lstart = march_start<U>(j0, chunk);
    // load position L and L + 1 (b_n of the next face)
    MarchPos pl, pn;
    pl.set(wrap_pos(Lstart, nd), step);
    pn = pl;
    pn.next(nd, step);
    T bn_cur = A::ld(bn, gb + pl.off);          // b_n at L
    // inputs of the next position, loaded one step ahead so that their
    // latency overlaps the arithmetic of the current step
    T nu[5], nbn, nt1a, nt1b, nt2a, nt2b;
    auto prefetch = [&]() {
        const unsigned o = gb + pl.off;
#pragma unroll
        for (int q = 0; q < 5; ++q) nu[q] = A::ld(in_u[q], o);
        nbn = A::ld(bn, gb + pn.off);
        nt1a = A::ld(bt1, o);
        nt1b = A::ld(bt1, gt1 + pl.off);
        nt2a = A::ld(bt2, o);
        nt2b = A::ld(bt2, gt2 + pl.off);
    };
    prefetch();
    // output offset of cell L - 3 (never wraps: outputs lie in the chunk)
    unsigned po = gb + (unsigned)(Lstart - 3) * step;
    for (int L0 = Lstart; L0 <= j0 + chunk + 2; L0 += U) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int L = L0 + k;
            T u0[5], bb0[3];
#pragma unroll
            for (int q = 0; q < 5; ++q) u0[q] = nu[q];
            const T bn_next = nbn;
            bb0[0] = T(0.5) * (bn_cur + bn_next);
            bb0[1] = T(0.5) * (nt1a + nt1b);
            bb0[2] = T(0.5) * (nt2a + nt2b);
            bn_cur = bn_next;
            pl = pn;
            pn.next(nd, step);
            prefetch();
            T unew[5];
            W.push(u0, bb0, gamma, c, c2, tau, halftau, unew);
            if (L - 3 >= j0) {
#pragma unroll
                for (int q = 0; q < 5; ++q) A::st(out_u[q], po, unew[q]);
            }
            po += step;
        }
    }
}

// at least 4 waves per SIMD for the FP32 magnetic march (<= 128 VGPRs), 2 for FP64
template <typename T> constexpr int march_waves() { return sizeof(T) == 4 ? 4 : 2; }

// the FP32 fluid window needs ~130 VGPRs: 3 waves per SIMD without spills
// (a 4-wave bound spills 3 registers per lane and made the z march 9% slower
// at 256^3, no faster at 512^3; the persistent ensemble kernel keeps 4 waves,
// where 3 made the ensemble step 12% slower)
template <typename T> constexpr int fluid_march_waves() { return sizeof(T) == 4 ? 3 : 2; }

template <typename T, int D, bool W32, int LIM = LIM_VANLEER, int FRZ = FRZ_STEP>
__global__ void __launch_bounds__(256, fluid_march_waves<T>()) fluid_march_kernel(SweepParams<T> P, int chunk)
{
    fluid_march_lane<T, D, W32, LIM, FRZ>(P, (long)xcd_tile(gridDim.x) * blockDim.x + threadIdx.x, chunk);
}

// Inputs of the magnetic window at one position: v_n of the 5 pencils, the
// 4 chain fields and b_n.
template <typename T>
struct MagBuf {
    T nrho[5], nm[5], nq[4], nbn;
    // hand the loaded values to the window (before the next load into it)
    __device__ __forceinline__ void take(T v[5], T q0[4], T& bn0) const
    {
#pragma unroll
        for (int r = 0; r < 5; ++r) v[r] = velocity(nm[r], nrho[r]);
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) q0[ch] = nq[ch];
        bn0 = nbn;
    }
};

// Prefetch depth of the CT and fused marches: inputs are loaded this many
// positions ahead of their use, in as many register buffers (2 instead of 1:
// 1-5% faster; the CT march stays at 4 waves per SIMD, 123 VGPRs, and the
// fused one at 2, 248 VGPRs)
constexpr int MARCH_PF = 2;

template <typename T, int D, bool W32>
struct MagLoads {
    using A = Addr<T, W32>;
    const T* __restrict__ rho;
    const T* __restrict__ mn;
    const T* __restrict__ bq1;
    const T* __restrict__ bq2;
    const T* __restrict__ bnin;
    unsigned pb[5];          // pencils: 0 P, 1 P-t1, 2 P+t1, 3 P-t2, 4 P+t2 (scaled)

    __device__ __forceinline__ MagLoads(const SweepParams<T>& P, const MarchGeom<D>& G)
    {
        constexpr int N_ = D, T1 = (D + 1) % 3, T2 = (D + 2) % 3;
        rho = P.in[RHO]; mn = P.in[MX + N_];
        bq1 = P.in[BX + T1]; bq2 = P.in[BX + T2]; bnin = P.in[BX + N_];
        pb[0] = G.base * A::scale; pb[1] = G.b_t1m * A::scale; pb[2] = G.b_t1p * A::scale;
        pb[3] = G.b_t2m * A::scale; pb[4] = G.b_t2p * A::scale;
    }
    // chain pencils: own-t1 P, plus-t1 P+t1, own-t2 P, plus-t2 P+t2
    __device__ __forceinline__ void load(MagBuf<T>& b, unsigned off) const
    {
        unsigned o[5];
#pragma unroll
        for (int r = 0; r < 5; ++r) o[r] = pb[r] + off;
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            b.nrho[r] = A::ld(rho, o[r]);
            b.nm[r] = A::ld(mn, o[r]);
        }
        b.nq[0] = A::ld(bq1, o[0]);
        b.nq[1] = A::ld(bq1, o[2]);
        b.nq[2] = A::ld(bq2, o[0]);
        b.nq[3] = A::ld(bq2, o[4]);
        b.nbn = A::ld(bnin, o[0]);
    }
};

// One lane of a grid: magnetic operator M_d.
template <typename T, int D, bool W32, int LIM = LIM_VANLEER>
__device__ __forceinline__ void mag_march_lane(const SweepParams<T>& P, long gid, int chunk)
{
    constexpr int N_ = D, T1 = (D + 1) % 3, T2 = (D + 2) % 3;
    using A = Addr<T, W32>;
    int p, j0;
    if (!march_lane_of<D>(P.nx, P.ny, P.nz, gid, chunk, p, j0)) return;
    const MarchGeom<D> G(P.nx, P.ny, P.nz, p);
    const int nd = G.nd;

    if (P.flag && *P.flag) {
        for (int j = j0; j < j0 + chunk; ++j) {
            const unsigned o = G.base + G.sd * j;
            P.out[BX][o] = P.in[BX][o];
            P.out[BY][o] = P.in[BY][o];
            P.out[BZ][o] = P.in[BZ][o];
        }
        return;
    }
    T tau, halftau, cdummy;
    step_scalars(P, tau, halftau, cdummy);
    const unsigned step = G.sd * A::scale;
    const unsigned gb = G.base * A::scale;

    MagWindow<T, LIM> W;
    W.init();
    const MagLoads<T, D, W32> in(P, G);
    constexpr int U = march_unroll<T>();
    constexpr int PF = MARCH_PF;
    static_assert(U % PF == 0, "the unrolled group cycles through the prefetch buffers");
    const int Lstart = march_start<U>(j0, chunk);
    // buffer b holds the inputs of position L with L = b (mod PF); pl is the
    // last position loaded
    MagBuf<T> buf[PF];
    MarchPos pl;
    pl.set(wrap_pos(Lstart, nd), step);
    in.load(buf[0], pl.off);
#pragma unroll
    for (int b = 1; b < PF; ++b) {
        pl.next(nd, step);
        in.load(buf[b], pl.off);
    }
    unsigned po = gb + (unsigned)(Lstart - 3) * step;
    for (int L0 = Lstart; L0 <= j0 + chunk + 2; L0 += U) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int L = L0 + k;
            T v[5], q0[4], bn0;
            buf[k % PF].take(v, q0, bn0);
            pl.next(nd, step);
            in.load(buf[k % PF], pl.off);
            T nb[5];
            W.push(v, q0, bn0, tau, halftau, nb);
            if (L - 3 >= j0) {
                A::st(P.out[BX + T1], po, nb[0]);
                A::st(P.out[BX + T2], po, nb[2]);
                A::st(P.out[BX + N_], po, nb[4]);
            }
            po += step;
        }
    }
}

template <typename T, int D, bool W32, int LIM = LIM_VANLEER>
__global__ void __launch_bounds__(256, march_waves<T>()) mag_march_kernel(SweepParams<T> P, int chunk)
{
    mag_march_lane<T, D, W32, LIM>(P, (long)xcd_tile(gridDim.x) * blockDim.x + threadIdx.x, chunk);
}

// positions unrolled per group, as in the single-operator marches
template <typename T> constexpr int magfluid_unroll() { return march_unroll<T>(); }

// the fused middle unrolls 6 positions in FP32: its windows are 1, 2 or 3
// positions deep, so over 6 positions every shift is a renaming of
// registers, where a group of 4 leaves moves at the loop's back edge
// (about 30 fewer VALU instructions per position; 2.11 against 2.19 ms at
// 512^3; the other marches gain nothing from it)
template <typename T> constexpr int triple_unroll() { return sizeof(T) == 4 ? 6 : 2; }

// One lane of a grid: the reverse-half pair M_d then F_d in one pass.  The
// magnetic window runs 4 positions ahead of the fluid window, whose frozen
// Bbar comes from the new faces in registers (b_t1, b_t2 of pencils P+t1,
// P+t2 from the plus chains) instead of from memory.  Same device functions
// in the same order as mag_march_lane followed by fluid_march_lane, so the
// result is bitwise that of the two operators, with the state read and
// written once.
//   magnetic look-ahead s: new faces at s-3;
//   fluid look-ahead s-4 (Bbar_n needs the new b_n at s-4 and s-3): new U
//   at s-7.
// Fluid outputs j0 .. j0+chunk-1 need new faces at j0-3 .. j0+chunk+3, which
// need magnetic inputs from j0-6: chunk + 13 positions.
template <typename T, int D, bool W32, int LIM = LIM_VANLEER>
__device__ __forceinline__ void magfluid_march_lane(const SweepParams<T>& P, long gid, int chunk)
{
    constexpr int N_ = D, T1 = (D + 1) % 3, T2 = (D + 2) % 3;
    using A = Addr<T, W32>;
    int p, j0;
    if (!march_lane_of<D>(P.nx, P.ny, P.nz, gid, chunk, p, j0)) return;
    const MarchGeom<D> G(P.nx, P.ny, P.nz, p);
    const int nd = G.nd;
    const T* __restrict__ in_u[5] = { P.in[RHO], P.in[MX + N_], P.in[MX + T1], P.in[MX + T2], P.in[EN] };
    T* out_u[5] = { P.out[RHO], P.out[MX + N_], P.out[MX + T1], P.out[MX + T2], P.out[EN] };

    if (P.flag && *P.flag) {
        for (int j = j0; j < j0 + chunk; ++j) {
            const unsigned o = G.base + G.sd * j;
            for (int q = 0; q < NFIELD; ++q) P.out[q][o] = P.in[q][o];
        }
        return;
    }
    T tau, halftau, c;
    step_scalars(P, tau, halftau, c);
    const T gamma = P.gamma;
    const unsigned step = G.sd * A::scale;
    const unsigned gb = G.base * A::scale;

    MagWindow<T, LIM> WM;
    WM.init();
    FluidWindow<T, LIM> WF;
    WF.init();
    const MagLoads<T, D, W32> in(P, G);
    constexpr int U = magfluid_unroll<T>();
    constexpr int PF = MARCH_PF;
    static_assert(U % PF == 0, "the unrolled group cycles through the prefetch buffers");
    const int total = chunk + 13;
    const int Sstart = j0 - 6 - ((U - (total % U)) % U);
    // load positions of the two windows (periodic); buffer b holds the
    // inputs of step s with s - Sstart = b (mod PF)
    MarchPos pm, pf;
    pm.set(wrap_pos(Sstart, nd), step);
    pf.set(wrap_pos(Sstart - 4, nd), step);
    MagBuf<T> buf[PF];
    T nu[PF][5];
    auto load_u = [&](T (&dst)[5]) {
        const unsigned o = gb + pf.off;
#pragma unroll
        for (int q = 0; q < 5; ++q) dst[q] = A::ld(in_u[q], o);
    };
    in.load(buf[0], pm.off);
    load_u(nu[0]);
#pragma unroll
    for (int b = 1; b < PF; ++b) {
        pm.next(nd, step);
        pf.next(nd, step);
        in.load(buf[b], pm.off);
        load_u(nu[b]);
    }
    // output offsets of the magnetic (s - 3) and fluid (s - 7) positions
    unsigned pmo = gb + (unsigned)(Sstart - 3) * step;
    unsigned pfo = gb + (unsigned)(Sstart - 7) * step;
    // new faces at the previous magnetic output position
    T pb_t1o = T(0), pb_t1p = T(0), pb_t2o = T(0), pb_t2p = T(0), pb_n = T(0);
    for (int S0 = Sstart; S0 <= j0 + chunk + 6; S0 += U) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int s = S0 + k;
            T v[5], q0[4], bn0, u0[5];
            buf[k % PF].take(v, q0, bn0);
#pragma unroll
            for (int q = 0; q < 5; ++q) u0[q] = nu[k % PF][q];
            pm.next(nd, step);
            pf.next(nd, step);
            in.load(buf[k % PF], pm.off);
            load_u(nu[k % PF]);

            T nb[5];
            WM.push(v, q0, bn0, tau, halftau, nb);
            const int jmo = s - 3;
            if (jmo >= j0 && jmo < j0 + chunk) {
                A::st(P.out[BX + T1], pmo, nb[0]);
                A::st(P.out[BX + T2], pmo, nb[2]);
                A::st(P.out[BX + N_], pmo, nb[4]);
            }
            pmo += step;
            // fluid at s-4: Bbar from the new faces of s-4 (and b_n of s-3)
            T bb0[3];
            bb0[0] = T(0.5) * (pb_n + nb[4]);
            bb0[1] = T(0.5) * (pb_t1o + pb_t1p);
            bb0[2] = T(0.5) * (pb_t2o + pb_t2p);
            pb_t1o = nb[0]; pb_t1p = nb[1]; pb_t2o = nb[2]; pb_t2p = nb[3]; pb_n = nb[4];
            T unew[5];
            WF.push(u0, bb0, gamma, c, c, tau, halftau, unew);
            if (s - 7 >= j0) {
#pragma unroll
                for (int q = 0; q < 5; ++q) A::st(out_u[q], pfo, unew[q]);
            }
            pfo += step;
        }
    }
}

// the fused lane holds both register windows (~220 VGPRs in FP32): 2 waves
// per SIMD without spills (3 waves spill ~100 VGPRs); FP64 takes 1
template <typename T> constexpr int magfluid_waves() { return sizeof(T) == 4 ? 2 : 1; }

template <typename T, int D, bool W32, int LIM = LIM_VANLEER>
__global__ void __launch_bounds__(256, magfluid_waves<T>()) magfluid_march_kernel(SweepParams<T> P, int chunk)
{
    magfluid_march_lane<T, D, W32, LIM>(P, (long)xcd_tile(gridDim.x) * blockDim.x + threadIdx.x, chunk);
}

// One lane of a grid: the middle of a step, M_d M_d F_d (the last forward
// magnetic operator and the first reverse pair), in one pass.  The second
// magnetic window runs 3 positions behind the first and takes its new faces
// as inputs (b_t1, b_t2 of pencils P, P+t1, P+t2 and b_n of P: all of what
// the second operator reads of b, since the plus chains are the neighbour
// pencils' own chains) and its edge velocities (the velocity field is the
// same for both); the fluid window runs behind the second as in the reverse
// pair.  Same device functions in the same order as mag_march_lane twice
// and fluid_march_lane, so the result is bitwise that of the three
// operators, with the state read and written once.
//   first magnetic look-ahead s: its new faces at s-3;
//   second magnetic look-ahead s-3 (edge velocity a(s-4)): new faces at s-6;
//   fluid look-ahead s-7: new U at s-10.
// Fluid outputs j0 .. j0+chunk-1 need second-operator faces at j0-3 ..
// j0+chunk+3, first-operator faces at j0-6 .. j0+chunk+6 and inputs from
// j0-9: chunk + 19 positions.
template <typename T, int D, bool W32, int LIM = LIM_VANLEER>
__device__ __forceinline__ void magmagfluid_march_lane(const SweepParams<T>& P, long gid, int chunk)
{
    constexpr int N_ = D, T1 = (D + 1) % 3, T2 = (D + 2) % 3;
    using A = Addr<T, W32>;
    int p, j0;
    if (!march_lane_of<D>(P.nx, P.ny, P.nz, gid, chunk, p, j0)) return;
    const MarchGeom<D> G(P.nx, P.ny, P.nz, p);
    const int nd = G.nd;
    const T* __restrict__ in_u[5] = { P.in[RHO], P.in[MX + N_], P.in[MX + T1], P.in[MX + T2], P.in[EN] };
    T* out_u[5] = { P.out[RHO], P.out[MX + N_], P.out[MX + T1], P.out[MX + T2], P.out[EN] };

    if (P.flag && *P.flag) {
        for (int j = j0; j < j0 + chunk; ++j) {
            const unsigned o = G.base + G.sd * j;
            for (int q = 0; q < NFIELD; ++q) P.out[q][o] = P.in[q][o];
        }
        return;
    }
    T tau, halftau, c;
    step_scalars(P, tau, halftau, c);
    const T gamma = P.gamma;
    const unsigned step = G.sd * A::scale;
    const unsigned gb = G.base * A::scale;

    MagWindow<T, LIM> WM1, WM2;
    WM1.init();
    WM2.init();
    FluidWindow<T, LIM> WF;
    WF.init();
    const MagLoads<T, D, W32> in(P, G);
    constexpr int U = triple_unroll<T>();
    constexpr int PF = MARCH_PF;
    static_assert(U % PF == 0, "the unrolled group cycles through the prefetch buffers");
    const int total = chunk + 19;
    const int Sstart = j0 - 9 - ((U - (total % U)) % U);
    MarchPos pm, pf;
    pm.set(wrap_pos(Sstart, nd), step);
    pf.set(wrap_pos(Sstart - 7, nd), step);
    MagBuf<T> buf[PF];
    T nu[PF][5];
    auto load_u = [&](T (&dst)[5]) {
        const unsigned o = gb + pf.off;
#pragma unroll
        for (int q = 0; q < 5; ++q) dst[q] = A::ld(in_u[q], o);
    };
    in.load(buf[0], pm.off);
    load_u(nu[0]);
#pragma unroll
    for (int b = 1; b < PF; ++b) {
        pm.next(nd, step);
        pf.next(nd, step);
        in.load(buf[b], pm.off);
        load_u(nu[b]);
    }
    // output offsets of the second magnetic (s - 6) and fluid (s - 10) positions
    unsigned pmo = gb + (unsigned)(Sstart - 6) * step;
    unsigned pfo = gb + (unsigned)(Sstart - 10) * step;
    // edge velocities a(s-4) for the second window: the first window's a(L-3)
    // as it stood before the previous push
    T a_prev[4] = { T(0), T(0), T(0), T(0) };
    // new faces of the second operator at its previous output position
    T pb_t1o = T(0), pb_t1p = T(0), pb_t2o = T(0), pb_t2p = T(0), pb_n = T(0);
    for (int S0 = Sstart; S0 <= j0 + chunk + 9; S0 += U) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int s = S0 + k;
            T v[5], q0[4], bn0, u0[5];
            buf[k % PF].take(v, q0, bn0);
#pragma unroll
            for (int q = 0; q < 5; ++q) u0[q] = nu[k % PF][q];
            pm.next(nd, step);
            pf.next(nd, step);
            in.load(buf[k % PF], pm.off);
            load_u(nu[k % PF]);

            T a_cur[4];
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) a_cur[ch] = WM1.a3[ch];     // a(s-3)
            T nb1[5];
            WM1.push(v, q0, bn0, tau, halftau, nb1);                 // faces at s-3
            T nb[5];
            WM2.push_edge(a_prev, nb1, nb1[4], tau, halftau, nb);     // faces at s-6
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) a_prev[ch] = a_cur[ch];
            const int jmo = s - 6;
            if (jmo >= j0 && jmo < j0 + chunk) {
                A::st(P.out[BX + T1], pmo, nb[0]);
                A::st(P.out[BX + T2], pmo, nb[2]);
                A::st(P.out[BX + N_], pmo, nb[4]);
            }
            pmo += step;
            // fluid at s-7: Bbar from the new faces of s-7 (and b_n of s-6)
            T bb0[3];
            bb0[0] = T(0.5) * (pb_n + nb[4]);
            bb0[1] = T(0.5) * (pb_t1o + pb_t1p);
            bb0[2] = T(0.5) * (pb_t2o + pb_t2p);
            pb_t1o = nb[0]; pb_t1p = nb[1]; pb_t2o = nb[2]; pb_t2p = nb[3]; pb_n = nb[4];
            T unew[5];
            WF.push(u0, bb0, gamma, c, c, tau, halftau, unew);
            if (s - 10 >= j0) {
#pragma unroll
                for (int q = 0; q < 5; ++q) A::st(out_u[q], pfo, unew[q]);
            }
            pfo += step;
        }
    }
}

// three register windows: one wave per SIMD (up to 512 registers, no spills)
template <typename T, int D, bool W32, int LIM = LIM_VANLEER>
__global__ void __launch_bounds__(256, 1) magmagfluid_march_kernel(SweepParams<T> P, int chunk)
{
    magmagfluid_march_lane<T, D, W32, LIM>(P, (long)xcd_tile(gridDim.x) * blockDim.x + threadIdx.x, chunk);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

template <typename T>
inline void row_shape(int nx, int& tpr, int& rows_per_wg, int& threads)
{
    tpr = nx / 4;
    rows_per_wg = x_rows_per_wg(nx);
    threads = rows_per_wg * tpr;
}

// the fused CFL epilogue needs the x fluid kernel's workgroups to be whole waves
template <typename T>
bool fused_cfl_possible(int nx)
{
    int tpr, rpw, threads;
    row_shape<T>(nx, tpr, rpw, threads);
    return threads % 64 == 0;
}

// every byte offset of a field fits in 32 bits (the march kernels' W32 path)
template <typename T>
inline bool offsets32(const SweepParams<T>& P, const LaunchTuning& tune)
{
    return !tune.wide && (unsigned long long)P.nx * P.ny * P.nz * sizeof(T) <= (1ull << 32);
}


template <typename T, int LIM, int FRZ = FRZ_STEP>
hipError_t launch_fluid_lim(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s)
{
    if (d == 0) {
        int tpr, rpw, threads;
        row_shape<T>(P.nx, tpr, rpw, threads);
        const int nrows = P.ny * P.nz;
        const int grid = (nrows + rpw - 1) / rpw;
        const size_t lds = sizeof(T) * 25 * threads;
        const int st = row_group_tiles(P.ny, rpw, tune.row_group);
        const bool fast = offsets32<T>(P, tune);
        if (P.cfl_acc) {
            if (threads % 64) return hipErrorInvalidValue;      // fused CFL needs full waves
            if (fast)
                hipLaunchKernelGGL((fluid_x_kernel<T, true, LIM, FRZ, true>), dim3(grid), dim3(threads), lds, s, P,
                                   tpr, rpw, st);
            else
                hipLaunchKernelGGL((fluid_x_kernel<T, true, LIM, FRZ>), dim3(grid), dim3(threads), lds, s, P, tpr, rpw, st);
        } else {
            if (fast)
                hipLaunchKernelGGL((fluid_x_kernel<T, false, LIM, FRZ, true>), dim3(grid), dim3(threads), lds, s, P,
                                   tpr, rpw, st);
            else
                hipLaunchKernelGGL((fluid_x_kernel<T, false, LIM, FRZ>), dim3(grid), dim3(threads), lds, s, P, tpr, rpw, st);
        }
    } else {
        const int nd = d == 1 ? P.ny : P.nz;
        const int npencil = P.nx * (d == 1 ? P.nz : P.ny);
        int chunk = tune.chunk[d];
        // the pencil variant reads its whole pencil twice before marching:
        // one chunk per pencil
        if (chunk <= 0 || nd % chunk || FRZ == FRZ_PENCIL) chunk = nd;
        const long lanes = (long)npencil * (nd / chunk);
        const int grid = (int)((lanes + 255) / 256);
        if (offsets32<T>(P, tune)) {
            if (d == 1) hipLaunchKernelGGL((fluid_march_kernel<T, 1, true, LIM, FRZ>), dim3(grid), dim3(256), 0, s, P, chunk);
            else hipLaunchKernelGGL((fluid_march_kernel<T, 2, true, LIM, FRZ>), dim3(grid), dim3(256), 0, s, P, chunk);
        } else {
            if (d == 1) hipLaunchKernelGGL((fluid_march_kernel<T, 1, false, LIM, FRZ>), dim3(grid), dim3(256), 0, s, P, chunk);
            else hipLaunchKernelGGL((fluid_march_kernel<T, 2, false, LIM, FRZ>), dim3(grid), dim3(256), 0, s, P, chunk);
        }
    }
    return hipGetLastError();
}

template <typename T, int LIM>
hipError_t launch_magnetic_lim(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s)
{
    if (d == 0) {
        int tpr, rpw, threads;
        row_shape<T>(P.nx, tpr, rpw, threads);
        const int nrows = P.ny * P.nz;
        const int grid = (nrows + rpw - 1) / rpw;
        const size_t lds = sizeof(T) * 16 * threads;
        const int st = row_group_tiles(P.ny, rpw, tune.row_group);
        if (offsets32<T>(P, tune))
            hipLaunchKernelGGL((mag_x_kernel<T, LIM, true>), dim3(grid), dim3(threads), lds, s, P, tpr, rpw, st);
        else
            hipLaunchKernelGGL((mag_x_kernel<T, LIM>), dim3(grid), dim3(threads), lds, s, P, tpr, rpw, st);
    } else {
        const int nd = d == 1 ? P.ny : P.nz;
        const int npencil = P.nx * (d == 1 ? P.nz : P.ny);
        int chunk = tune.chunk[d];
        if (chunk <= 0 || nd % chunk) chunk = nd;
        const long lanes = (long)npencil * (nd / chunk);
        const int grid = (int)((lanes + 255) / 256);
        if (offsets32<T>(P, tune)) {
            if (d == 1) hipLaunchKernelGGL((mag_march_kernel<T, 1, true, LIM>), dim3(grid), dim3(256), 0, s, P, chunk);
            else hipLaunchKernelGGL((mag_march_kernel<T, 2, true, LIM>), dim3(grid), dim3(256), 0, s, P, chunk);
        } else {
            if (d == 1) hipLaunchKernelGGL((mag_march_kernel<T, 1, false, LIM>), dim3(grid), dim3(256), 0, s, P, chunk);
            else hipLaunchKernelGGL((mag_march_kernel<T, 2, false, LIM>), dim3(grid), dim3(256), 0, s, P, chunk);
        }
    }
    return hipGetLastError();
}

// the single operators with the limiter P.limiter; the fluid operator's
// freezing-speed variants (P.freeze) come with van Leer's limiter only
template <typename T>
hipError_t launch_fluid(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s)
{
    if (P.freeze != FRZ_STEP) {
        if (P.limiter != LIM_VANLEER) return hipErrorInvalidValue;
        if (P.freeze == FRZ_CELL) return launch_fluid_lim<T, LIM_VANLEER, FRZ_CELL>(P, d, tune, s);
        if (P.freeze == FRZ_PENCIL) return launch_fluid_lim<T, LIM_VANLEER, FRZ_PENCIL>(P, d, tune, s);
        return hipErrorInvalidValue;
    }
    switch (P.limiter) {
    case LIM_VANLEER: return launch_fluid_lim<T, LIM_VANLEER>(P, d, tune, s);
    case LIM_MINMOD: return launch_fluid_lim<T, LIM_MINMOD>(P, d, tune, s);
    case LIM_MC: return launch_fluid_lim<T, LIM_MC>(P, d, tune, s);
    case LIM_SUPERBEE: return launch_fluid_lim<T, LIM_SUPERBEE>(P, d, tune, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_magnetic(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s)
{
    switch (P.limiter) {
    case LIM_VANLEER: return launch_magnetic_lim<T, LIM_VANLEER>(P, d, tune, s);
    case LIM_MINMOD: return launch_magnetic_lim<T, LIM_MINMOD>(P, d, tune, s);
    case LIM_MC: return launch_magnetic_lim<T, LIM_MC>(P, d, tune, s);
    case LIM_SUPERBEE: return launch_magnetic_lim<T, LIM_SUPERBEE>(P, d, tune, s);
    default: return hipErrorInvalidValue;
    }
}

// the reverse-half pair M_d then F_d in one launch; P.cfl_acc (x only)
// adds the fused CFL epilogue
template <typename T, int LIM>
hipError_t launch_magfluid_lim(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s)
{
    if (d == 0) {
        int tpr, rpw, threads;
        row_shape<T>(P.nx, tpr, rpw, threads);
        const int nrows = P.ny * P.nz;
        const int grid = (nrows + rpw - 1) / rpw;
        const size_t lds = sizeof(T) * 25 * threads;
        const int st = row_group_tiles(P.ny, rpw, tune.row_group);
        const bool fast = offsets32<T>(P, tune);
        if (P.cfl_acc) {
            if (threads % 64) return hipErrorInvalidValue;      // fused CFL needs full waves
            if (fast)
                hipLaunchKernelGGL((magfluid_x_kernel<T, true, LIM, true>), dim3(grid), dim3(threads), lds, s, P,
                                   tpr, rpw, st);
            else
                hipLaunchKernelGGL((magfluid_x_kernel<T, true, LIM>), dim3(grid), dim3(threads), lds, s, P, tpr, rpw, st);
        } else {
            if (fast)
                hipLaunchKernelGGL((magfluid_x_kernel<T, false, LIM, true>), dim3(grid), dim3(threads), lds, s, P,
                                   tpr, rpw, st);
            else
                hipLaunchKernelGGL((magfluid_x_kernel<T, false, LIM>), dim3(grid), dim3(threads), lds, s, P, tpr, rpw, st);
        }
    } else {
        if (P.cfl_acc) return hipErrorInvalidValue;
        const int nd = d == 1 ? P.ny : P.nz;
        const int npencil = P.nx * (d == 1 ? P.nz : P.ny);
        int chunk = tune.pair_chunk[d];
        if (chunk <= 0 || nd % chunk) chunk = nd;
        const long lanes = (long)npencil * (nd / chunk);
        const int grid = (int)((lanes + 255) / 256);
        if (offsets32<T>(P, tune)) {
            if (d == 1) hipLaunchKernelGGL((magfluid_march_kernel<T, 1, true, LIM>), dim3(grid), dim3(256), 0, s, P, chunk);
            else hipLaunchKernelGGL((magfluid_march_kernel<T, 2, true, LIM>), dim3(grid), dim3(256), 0, s, P, chunk);
        } else {
            if (d == 1) hipLaunchKernelGGL((magfluid_march_kernel<T, 1, false, LIM>), dim3(grid), dim3(256), 0, s, P, chunk);
            else hipLaunchKernelGGL((magfluid_march_kernel<T, 2, false, LIM>), dim3(grid), dim3(256), 0, s, P, chunk);
        }
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_magfluid(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s)
{
    switch (P.limiter) {
    case LIM_VANLEER: return launch_magfluid_lim<T, LIM_VANLEER>(P, d, tune, s);
    case LIM_MINMOD: return launch_magfluid_lim<T, LIM_MINMOD>(P, d, tune, s);
    case LIM_MC: return launch_magfluid_lim<T, LIM_MC>(P, d, tune, s);
    case LIM_SUPERBEE: return launch_magfluid_lim<T, LIM_SUPERBEE>(P, d, tune, s);
    default: return hipErrorInvalidValue;
    }
}

// M_d M_d F_d in one launch (march axes; van Leer's limiter)
template <typename T>
hipError_t launch_magmagfluid(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s)
{
    if (d == 0 || P.cfl_acc || P.limiter != LIM_VANLEER) return hipErrorInvalidValue;
    const int nd = d == 1 ? P.ny : P.nz;
    const int npencil = P.nx * (d == 1 ? P.nz : P.ny);
    int chunk = tune.triple_chunk[d];
    if (chunk <= 0 || nd % chunk) chunk = nd;
    const long lanes = (long)npencil * (nd / chunk);
    const int grid = (int)((lanes + 255) / 256);
    if (offsets32<T>(P, tune)) {
        if (d == 1) hipLaunchKernelGGL((magmagfluid_march_kernel<T, 1, true>), dim3(grid), dim3(256), 0, s, P, chunk);
        else hipLaunchKernelGGL((magmagfluid_march_kernel<T, 2, true>), dim3(grid), dim3(256), 0, s, P, chunk);
    } else {
        if (d == 1) hipLaunchKernelGGL((magmagfluid_march_kernel<T, 1, false>), dim3(grid), dim3(256), 0, s, P, chunk);
        else hipLaunchKernelGGL((magmagfluid_march_kernel<T, 2, false>), dim3(grid), dim3(256), 0, s, P, chunk);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched ensembles: persistent kernels over (box, tile) work items
// ---------------------------------------------------------------------------
// The grid is a multiple of 8 workgroups.  XCD k (hardware workgroups k,
// k+8, ...) takes the k-th eighth of the item list, whose items belong to
// few boxes, so neighbour pencils of one box meet in one L2.  Each item runs
// the same tile / lane function as the single-grid kernels, so a box of an
// ensemble evolves bit for bit like the same box on its own.

template <typename T>
__device__ __forceinline__ SweepParams<T> box_params(const BatchParams<T>& B, int box,
                                                     const BoxDesc& bd)
{
    SweepParams<T> P;
#pragma unroll
    for (int f = 0; f < 8; ++f) {
        P.in[f] = B.in_base[f] + bd.off + (size_t)f * bd.ncell;
        P.out[f] = B.out_base[f] + bd.off + (size_t)f * bd.ncell;
    }
    P.nx = bd.n[0]; P.ny = bd.n[1]; P.nz = bd.n[2];
    P.gamma = B.gamma;
    P.scal = B.scal + (size_t)box * SCAL_COUNT;
    P.flag = B.flag ? B.flag + (size_t)box * FLAG_COUNT : nullptr;
    P.cfl_acc = B.cfl_acc ? B.cfl_acc + (size_t)box * (CFL_ACC_SLOTS + 1) : nullptr;
    P.gamma64 = B.gamma64;
    P.limiter = 0;
    P.freeze = FRZ_STEP;
    return P;
}

// op 0 fluid, 1 magnetic, 2 the fused reverse-half pair (magnetic then
// fluid), 3 the middle of a step M_z M_z F_z (z only, one wave per SIMD)
template <typename T, int OP>
constexpr int batch_waves(int d)
{
    return d == 0 ? 1 : (OP == 3 ? 1 : OP == 2 ? magfluid_waves<T>() : march_waves<T>());
}

// W32: every box's fields have 32-bit byte offsets (see Addr)
// CFL (x fluid operator or x pair only): also accumulate each box's CFL
// maximum of the result (B.cfl_acc)
template <typename T, int OP, int D, bool W32, int LIM = LIM_VANLEER, bool CFL = false>
__global__ void __launch_bounds__(256, (batch_waves<T, OP>(D))) batch_sweep_kernel(BatchParams<T> B)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int g8 = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7, r = blockIdx.x >> 3;
    const int per = (B.nitems + 7) >> 3;
    const int i0 = xcd * per;
    const int i1 = min(B.nitems, i0 + per);
    for (int i = i0 + r; i < i1; i += g8) {
        const int2 it = B.items[i];
        const BoxDesc bd = B.boxes[it.x];
        const SweepParams<T> P = box_params(B, it.x, bd);
        if constexpr (D == 0) {
            if constexpr (OP == 0)
                fluid_x_tile<T, CFL, LIM>(P, it.y, bd.tpr, bd.rpw, reinterpret_cast<T*>(smem_raw));
            else if constexpr (OP == 1)
                mag_x_tile<T, LIM>(P, it.y, bd.tpr, bd.rpw, reinterpret_cast<T*>(smem_raw));
            else
                magfluid_x_tile<T, CFL, LIM>(P, it.y, bd.tpr, bd.rpw, reinterpret_cast<T*>(smem_raw));
        } else {
            const long gid = (long)it.y * blockDim.x + threadIdx.x;
            if constexpr (OP == 0)
                fluid_march_lane<T, D, W32, LIM>(P, gid, bd.chunk[D]);
            else if constexpr (OP == 1)
                mag_march_lane<T, D, W32, LIM>(P, gid, bd.chunk[D]);
            else if constexpr (OP == 2)
                magfluid_march_lane<T, D, W32, LIM>(P, gid, bd.pchunk[D]);
            else
                magmagfluid_march_lane<T, D, W32, LIM>(P, gid, bd.pchunk[D]);   // the pairs' work list
        }
    }
}

template <typename T, int OP, int LIM>
static void launch_batch_op_dir(const BatchParams<T>& B, int d, int grid, size_t lds, hipStream_t s)
{
    // x tiles have no march addressing: one instantiation (two for the
    // operators that can end a step: with and without the fused CFL)
    if (d == 0) {
        if constexpr (OP != 1) {
            if (B.cfl_acc) {
                hipLaunchKernelGGL((batch_sweep_kernel<T, OP, 0, true, LIM, true>), dim3(grid), dim3(256), lds, s, B);
                return;
            }
        }
        hipLaunchKernelGGL((batch_sweep_kernel<T, OP, 0, true, LIM>), dim3(grid), dim3(256), lds, s, B);
    } else if (B.offsets32) {
        if (d == 1) hipLaunchKernelGGL((batch_sweep_kernel<T, OP, 1, true, LIM>), dim3(grid), dim3(256), lds, s, B);
        else hipLaunchKernelGGL((batch_sweep_kernel<T, OP, 2, true, LIM>), dim3(grid), dim3(256), lds, s, B);
    } else {
        if (d == 1) hipLaunchKernelGGL((batch_sweep_kernel<T, OP, 1, false, LIM>), dim3(grid), dim3(256), lds, s, B);
        else hipLaunchKernelGGL((batch_sweep_kernel<T, OP, 2, false, LIM>), dim3(grid), dim3(256), lds, s, B);
    }
}

template <typename T, int LIM>
static void launch_batch_op_lim(const BatchParams<T>& B, int op, int d, int grid, size_t lds, hipStream_t s)
{
    if (op == 0) launch_batch_op_dir<T, 0, LIM>(B, d, grid, lds, s);
    else if (op == 1) launch_batch_op_dir<T, 1, LIM>(B, d, grid, lds, s);
    else if (op == 2) launch_batch_op_dir<T, 2, LIM>(B, d, grid, lds, s);
    else if constexpr (sizeof(T) == 4 && LIM == LIM_VANLEER) {
        // the middle: z only, FP32, van Leer's limiter (the single grid's rules)
        if (B.offsets32) hipLaunchKernelGGL((batch_sweep_kernel<T, 3, 2, true, LIM>), dim3(grid), dim3(256), 0, s, B);
        else hipLaunchKernelGGL((batch_sweep_kernel<T, 3, 2, false, LIM>), dim3(grid), dim3(256), 0, s, B);
    }
}

template <typename T>
hipError_t launch_batch_op(const BatchParams<T>& B, int op, int d, int grid, hipStream_t s)
{
    if (B.cfl_acc && (d != 0 || op == 1)) return hipErrorInvalidValue;   // only x fluid / x pair
    if (op == 3 && (d != 2 || sizeof(T) != 4 || B.limiter != LIM_VANLEER)) return hipErrorInvalidValue;
    const size_t lds = d == 0 ? sizeof(T) * (op == 1 ? 16 : 25) * 256 : 0;
    switch (B.limiter) {
    case LIM_VANLEER: launch_batch_op_lim<T, LIM_VANLEER>(B, op, d, grid, lds, s); break;
    case LIM_MINMOD: launch_batch_op_lim<T, LIM_MINMOD>(B, op, d, grid, lds, s); break;
    case LIM_MC: launch_batch_op_lim<T, LIM_MC>(B, op, d, grid, lds, s); break;
    case LIM_SUPERBEE: launch_batch_op_lim<T, LIM_SUPERBEE>(B, op, d, grid, lds, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mhd
