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
constexpr int CFL_ACC_SLOTS = 256;     // fused-CFL maximum slots (+1 word for the flag)

template <typename T>
struct SweepParams {
    const T* in[8];          // current fields (rho, m_x, m_y, m_z, e, b_x, b_y, b_z)
    T* out[8];               // destination fields (only those the operator writes)
    int nx, ny, nz;
    T gamma;
    const double* scal;      // device scalar block (dt, relaxation speed)
    const int* flag;         // if *flag != 0 the operator copies in -> out
    // fused CFL (x fluid operator, alone or fused; null: off): the FP64 signal-speed
    // maximum of the operator's output is accumulated in cfl_acc[0 ..
    // CFL_ACC_SLOTS) (bits of the double, atomic max into the slot of the
    // workgroup, spreading the atomics); cfl_acc[CFL_ACC_SLOTS] gets bit 0
    // for a non-physical cell, and an operator skipped under a record ORs
    // that record (1 non-physical, 2 zero signal speed) into it
    unsigned long long* cfl_acc;
    double gamma64;          // gamma in FP64 for that speed
    int limiter;             // slope limiter of the single operators (LIM_*; 0: van Leer)
    int freeze;              // freezing speed of the fluid operator (FRZ_*; 0: the step's c)
};

// Launch shape choices of the march kernels: chunk length along y and z
// (0 = whole pencil) of the single operators and of the fused reverse-half
// pairs.  Index 0 is unused (x sweeps hold whole rows).
struct LaunchTuning {
    int chunk[3];
    int pair_chunk[3];
    int triple_chunk[3];     // the same for M_d M_d F_d in one launch
    int wide;                // 1: 64-bit addressing in the marches even where 32-bit offsets fit
    int row_group;           // x sweeps: most rows (along y) in one group of the tile order (0: built-in)
};

// rows of one x-sweep workgroup: 4 cells per thread, up to 256 threads
inline int x_rows_per_wg(int nx)
{
    const int r = 256 / (nx / 4);
    return r < 1 ? 1 : r;
}

// tiles per group of the x sweeps' visit order (row_tile): the largest
// divisor st of ny / rows_per_wg with st * rows_per_wg <= max_rows (64 rows
// when max_rows is 0); 0 (linear order) when rows_per_wg does not divide ny
inline int row_group_tiles(int ny, int rows_per_wg, int max_rows)
{
    if (max_rows <= 0) max_rows = 64;
    if (ny % rows_per_wg) return 0;
    const int ty = ny / rows_per_wg;
    int st = 0;
    for (int c = 1; c <= ty && c * rows_per_wg <= max_rows; ++c)
        if (ty % c == 0) st = c;
    return st;
}

// Visit order of the row tiles of an x sweep (the single-grid kernels and
// the ensembles' work lists).  A tile holds rows_per_wg
// consecutive rows along y at one z; tile L covers rows L * rows_per_wg ..
// of the flattened (z, y) index, ty = ny / rows_per_wg tiles per y line.
// Visit o goes to groups of st tiles along y, one group per z in turn, so
// the rows z - 1 and z + 1 that a tile reads belong to tiles st positions
// before and after it, which the same XCD (consecutive visits share one,
// see xcd_tile) holds in its L2; in the linear order they are a whole y
// line of tiles away.  Rows y +- 1 at a group's edge are read twice.  A
// bijection of [0, ty * nz) when st divides ty; st <= 0 or st >= ty keeps
// the linear order.
__host__ __device__ inline int row_tile(int o, int st, int ty, int nz)
{
    if (st <= 0 || st >= ty) return o;
    const int per_col = st * nz;
    const int c = o / per_col;
    const int rem = o - c * per_col;
    const int z = rem / st;
    return z * ty + c * st + (rem - z * st);
}


// ---------------------------------------------------------------------------
// Batched ensembles: boxes of different sizes in one pair of buffers.  Box b
// holds its 8 fields contiguously (field-major, x fastest) at element
// offset off in each buffer.  Work items (box, tile) of one sweep direction
// are processed by a persistent grid of workgroups.
// ---------------------------------------------------------------------------
struct BoxDesc {
    int n[3];
    int chunk[3];                 // march chunk along y (1) and z (2)
    int pchunk[3];                // the same for the fused reverse-half pairs
    int tpr, rpw;                 // row-kernel shape (threads per row, rows per tile)
    int ntile[3];                 // tiles per direction
    unsigned ncell;
    unsigned long long off;       // element offset of the box in each buffer
};

template <typename T>
struct BatchParams {
    const T* in_base[8];          // buffer holding the current copy of each field
    T* out_base[8];               // the other buffer
    const BoxDesc* boxes;
    const int2* items;            // (box, tile)
    int nitems;
    T gamma;
    const double* scal;           // per box: SCAL_COUNT doubles
    const int* flag;              // per box: FLAG_COUNT ints (null: never skip)
    bool offsets32;               // every box's fields have 32-bit byte offsets
    int limiter;                  // slope limiter (LIM_*; 0: van Leer)
    // fused CFL of the x operator that ends a step (null: off): box b's FP64
    // maximum signal speed accumulates in cfl_acc[b * (CFL_ACC_SLOTS + 1) ..],
    // as for a single grid
    unsigned long long* cfl_acc;
    double gamma64;
};

// op 0 fluid, 1 magnetic, 2 magnetic then fluid in one pass (the reverse-half
// pair); d = sweep axis; grid = persistent workgroups (x8)
template <typename T>
hipError_t launch_batch_op(const BatchParams<T>& B, int op, int d, int grid, hipStream_t s);

template <typename T>
struct BatchCflArgs {
    const T* base[8];             // buffer holding the current copy of each field
    const BoxDesc* boxes;
    const int2* items;
};

// per-box CFL: items (box, block of CFL_CELLS cells); item_first[b] ..
// item_first[b+1]-1 are box b's items
constexpr int CFL_CELLS = 2048;
// per box, dt / relaxation speed / non-physical flag from the maxima the
// fused CFL accumulated (the rules of batch_cfl_final), then clears them
hipError_t launch_batch_cfl_from_acc(unsigned long long* acc, const BoxDesc* boxes, int nbox, double cfl,
                                     double* scal, int* flag, hipStream_t s);
hipError_t launch_batch_clear_acc(unsigned long long* acc, int nbox, hipStream_t s);

template <typename T>
hipError_t launch_batch_cfl(const T* const base[8], const BoxDesc* boxes, const int2* items,
                            int nitems, const int* item_first, int nbox, double gamma,
                            double cfl, double* partial, int* partial_bad, double* scal,
                            int* flag, hipStream_t s);
hipError_t launch_batch_advance(double* scal, int* flag, int nbox, hipStream_t s);

template <typename T>
hipError_t launch_fluid(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s);
template <typename T>
bool fused_cfl_possible(int nx);
template <typename T>
hipError_t launch_magnetic(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s);
// M_d then F_d in one pass, bitwise the two operators in turn; P.cfl_acc
// (d = 0 only) adds the fused CFL epilogue of launch_fluid
template <typename T>
hipError_t launch_magfluid(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s);
// M_d M_d F_d in one pass along a march axis (the middle of a step, d = 2),
// bitwise the three operators in turn; van Leer's limiter
template <typename T>
hipError_t launch_magmagfluid(const SweepParams<T>& P, int d, const LaunchTuning& tune, hipStream_t s);

// CFL: per-block maxima of the signal speed into partial[], then a final
// reduction writes scal[SCAL_VMAX], scal[SCAL_C] = vmax, scal[SCAL_DT] =
// cfl h / vmax (or, if dt_cap > 0, min(that, dt_cap)), and flags
// non-physical cells in flag[FLAG_NONPHYS].
template <typename T>
hipError_t launch_cfl(const T* const f[8], int nx, int ny, int nz, double gamma, double cfl,
                      double* partial, int* partial_bad, int nblocks, double* scal, int* flag,
                      hipStream_t s);
int cfl_blocks(size_t ncell);
// CFL from the maximum accumulated by the fused epilogue (then cleared), and
// clearing the accumulator
hipError_t launch_cfl_from_acc(unsigned long long* acc, int nx, double cfl, double* scal, int* flag,
                               hipStream_t s);
hipError_t launch_clear_acc(unsigned long long* acc, hipStream_t s);

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

// Plain device copy of `bytes` (a multiple of 16; 16-byte aligned pointers).
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

// Restriction by factor r of all 8 fields.
template <typename T>
hipError_t launch_restrict(const T* const fine[8], T* const coarse[8], int nx, int ny, int nz,
                           int r, hipStream_t s);

// Small scalar kernels (graph-capturable replacements of host writes).
hipError_t launch_set_scalars(double* scal, double dt, double c, int* flag, int clear_flag,
                              hipStream_t s);
hipError_t launch_advance_time(double* scal, const int* nonphys, int* steps, hipStream_t s);

}  // namespace mhd
