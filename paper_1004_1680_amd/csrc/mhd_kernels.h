// Kernel parameter blocks and launcher declarations of the MHD library.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace mhd {

// Device scalar block of a handle (FP64): time step of the current step,
// relaxation speed, simulated time; and the step counters.
enum { SCAL_DT = 0, SCAL_C = 1, SCAL_TIME = 2, SCAL_VMAX = 3, SCAL_COUNT = 4 };
// Device flag block: [0] non-physical state recorded by the device-side
// CFL of mhd_step_auto, [1] number of such steps that ran, [2] result of the
// synchronous CFL.
enum { FLAG_NONPHYS = 0, FLAG_STEPS = 1, FLAG_SYNC = 2, FLAG_COUNT = 4 };

template <typename T>
struct SweepParams {
    const T* in[8];          // current fields (rho, m_x, m_y, m_z, e, b_x, b_y, b_z)
    T* out[8];               // destination fields (only those the operator writes)
    int nx, ny, nz;
    T gamma;
    const double* scal;      // device scalar block (dt, relaxation speed)
    const int* flag;         // if *flag != 0 the operator copies in -> out
};

// Launch shape choices of the march kernels: chunk length along y and z
// (0 = whole pencil).  Index 0 is unused (x sweeps hold whole rows).
struct LaunchTuning {
    int chunk[3];
};

template <typename T>
hipError_t launch_fluid(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s);
template <typename T>
hipError_t launch_magnetic(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s);

// CFL: per-block maxima of the signal speed into partial[], then a final
// reduction writes scal[SCAL_VMAX], scal[SCAL_C] = vmax, scal[SCAL_DT] =
// cfl h / vmax (or, if dt_cap > 0, min(that, dt_cap)), and flags
// non-physical cells in flag[FLAG_NONPHYS].
template <typename T>
hipError_t launch_cfl(const T* const f[8], int nx, int ny, int nz, double gamma, double cfl,
                      double* partial, int* partial_bad, int nblocks, double* scal, int* flag,
                      hipStream_t s);
int cfl_blocks(size_t ncell);

// Diagnostics: 8 field sums (FP64, fixed order), max |div b|, max |b|.
template <typename T>
hipError_t launch_diag(const T* const f[8], int nx, int ny, int nz, double* partial,
                       int nblocks, double* out9, hipStream_t s);
int diag_blocks(size_t ncell);

// Host double <-> device T conversion of one field.
template <typename T>
hipError_t launch_convert_in(const double* src, T* dst, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_convert_out(const T* src, double* dst, size_t n, hipStream_t s);
template <typename S, typename T>
hipError_t launch_cast(const S* src, T* dst, size_t n, hipStream_t s);

// Restriction by factor r of all 8 fields.
template <typename T>
hipError_t launch_restrict(const T* const fine[8], T* const coarse[8], int nx, int ny, int nz,
                           int r, hipStream_t s);

// Small scalar kernels (graph-capturable replacements of host writes).
hipError_t launch_set_scalars(double* scal, double dt, double c, int* flag, int clear_flag,
                              hipStream_t s);
hipError_t launch_advance_time(double* scal, const int* nonphys, int* steps, hipStream_t s);

}  // namespace mhd
