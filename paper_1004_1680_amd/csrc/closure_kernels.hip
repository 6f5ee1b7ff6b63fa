// Kernels of the learned closure for gfx950: periodic 3x3x3 convolutions on
// BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulate) and the small
// elementwise / reduction kernels around them.
//
// Convolution as an implicit GEMM, D[co][cell] = sum_K A[co][K] B[K][cell],
// K = (offset o, input channel ci) flattened as o * CIN + ci, 32 per MFMA.
// MFMA 16x16x32 operand layout (wave64): lane l holds A[l%16][8(l/16)+e],
// B[8(l/16)+e][l%16] (e = 0..7) and D[4(l/16)+e][l%16] (e = 0..3).
//  * A: weights, repacked once per weight update into exactly that layout
//    (one 16-byte load per lane per K step);
//  * B: activations, channel-last x[cell][CIN]: the 8 K values of a lane are
//    8 consecutive channels of one shifted cell (one 16-byte load);
//  * D: 4 consecutive output channels of one cell per lane.
// A workgroup computes a 16 x 4 x 4 tile of cells x all output channels from
// an LDS copy of its input halo; each wave one z plane (4 rows of 16 cells).  dgrad is the same kernel on the gradient with the weights
// flipped (o -> 26 - o) and transposed (ci <-> co), with the ReLU mask of
// the forward activation fused in the epilogue.
//
// wgrad, dW[o][ci][co] = sum_cell x[cell + d(o)][ci] dy[cell][co], has K =
// cells: it reads channel-major copies xT[ci][cell], dyT[co][cell] written
// by the producing kernels, so a lane's 8 K values are 8 consecutive cells
// of one channel; the x shift of an offset is built from two aligned
// 16-byte loads.  Each workgroup accumulates a slab of rows for all 27
// offsets (wave w takes offsets w, w+4, ...) and writes partial sums; a
// second kernel adds the partials in a fixed order (deterministic).
//
// Requirements: nx, ny, nz multiples of 32 (nx for the 32-cell K steps of
// wgrad), fewer than 2^31 cells.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "closure_kernels.h"

namespace mhd {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);          // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

__device__ __forceinline__ bf16x8 as_bf8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ uint4 ld16(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }

__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ---------------------------------------------------------------------------
// weight packing
// ---------------------------------------------------------------------------
// Wp[s][m][lane][e] = W'[o][ci][co] with K = 32 s + 8 (lane/16) + e,
// o = K / cin, ci = K % cin, co = 16 m + lane % 16; zero outside.  flip:
// W'[o][ci][co] = W[26 - o][co][ci] (dgrad of a layer with weights W[27][co][ci]).
__global__ void pack_weights_kernel(const float* __restrict__ w, int cin, int cout, int flip,
                                    uint16_t* __restrict__ wp)
{
    const int ks = (27 * cin + 31) / 32, mb = (cout + 15) / 16;
    const int total = ks * mb * 64 * 8;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        const int e = t & 7, lane = (t >> 3) & 63, m = (t >> 9) % mb, s = (t >> 9) / mb;
        const int K = 32 * s + 8 * (lane >> 4) + e;
        const int o = K / cin, ci = K % cin, co = 16 * m + (lane & 15);
        float v = 0.0f;
        if (o < 27 && co < cout)
            v = flip ? w[((size_t)(26 - o) * cout + co) * cin + ci] : w[((size_t)o * cin + ci) * cout + co];
        wp[t] = f2bf(v);
    }
}

hipError_t launch_pack_weights(const float* w, int cin, int cout, int flip, uint16_t* wp, hipStream_t s)
{
    hipLaunchKernelGGL(pack_weights_kernel, dim3(64), dim3(256), 0, s, w, cin, cout, flip, wp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// forward / dgrad convolution
// ---------------------------------------------------------------------------

// Output tile of a workgroup: 16 (x) x 4 (y) x 4 (z) cells; wave w takes
// the z plane w, its 4 MFMA column blocks the 4 rows y, lane r the cell x.
// The input halo (18 x 6 x 6 cells, periodic) is staged once in LDS with a
// cell stride of CIN + 8 bf16 for CIN = 32 (80 bytes: the 16-byte reads of
// 16 consecutive cells then spread over all banks), and every one of the 27
// offsets reads its B fragments from there.
constexpr int CT_X = 16, CT_Y = 4, CT_Z = 4;
constexpr int CH_X = CT_X + 2, CH_Y = CT_Y + 2, CH_Z = CT_Z + 2, CH_CELLS = CH_X * CH_Y * CH_Z;

template <int CIN>
__host__ __device__ constexpr int conv_cell_stride() { return CIN == 8 ? 8 : CIN + 8; }

template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(256) conv3d_kernel(ConvArgs A)
{
    constexpr int KS = (27 * CIN + 31) / 32;
    constexpr int MB = (COUT + 15) / 16;
    constexpr int NB = CT_Y;
    constexpr int CS = conv_cell_stride<CIN>();
    constexpr int PARTS = CIN / 8;                         // 16-byte pieces per cell
    __shared__ __align__(16) uint16_t tile[CH_CELLS * CS];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
    const long N = (long)nx * ny * nz;
    const int tx = nx / CT_X, ty = ny / CT_Y;
    const int b = blockIdx.x;
    const int x0 = (b % tx) * CT_X, y0 = ((b / tx) % ty) * CT_Y, z0 = (b / (tx * ty)) * CT_Z;
    const uint16_t* __restrict__ x = A.x;
    const uint4* __restrict__ wp = reinterpret_cast<const uint4*>(A.wp);

    // stage the halo: piece q of halo cell h, consecutive threads on
    // consecutive pieces (contiguous along x in global memory)
    for (int t = threadIdx.x; t < CH_CELLS * PARTS; t += 256) {
        const int h = t / PARTS, q = t % PARTS;
        const int hx = h % CH_X, hy = (h / CH_X) % CH_Y, hz = h / (CH_X * CH_Y);
        const unsigned src = (unsigned)wrap1(x0 - 1 + hx, nx) +
                             (unsigned)nx * ((unsigned)wrap1(y0 - 1 + hy, ny) +
                                             (unsigned)ny * (unsigned)wrap1(z0 - 1 + hz, nz));
        *reinterpret_cast<uint4*>(tile + h * CS + 8 * q) = ld16(x + (size_t)src * CIN + 8 * q);
    }
    __syncthreads();

    f4 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f4{ 0.f, 0.f, 0.f, 0.f };

#pragma unroll 3
    for (int s = 0; s < KS; ++s) {
        const int K = 32 * s + 8 * g;
        const int o = K / CIN, c0 = K % CIN;
        const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
        bf16x8 bf[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            uint4 v = make_uint4(0, 0, 0, 0);
            if (o < 27) {
                const int h = (wave + 1 + dz) * (CH_X * CH_Y) + (nb + 1 + dy) * CH_X + (r + 1 + dx);
                v = *reinterpret_cast<const uint4*>(tile + h * CS + c0);
            }
            bf[nb] = as_bf8(v);
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const bf16x8 af = as_bf8(wp[((size_t)s * MB + m) * 64 + lane]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[nb], acc[m][nb], 0, 0, 0);
        }
    }

    // epilogue: lane holds channels co = 16 m + 4 g + e of cell (x0 + r, y0 + nb, z0 + wave)
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        const int co0 = 16 * m + 4 * g;
        if (co0 >= COUT) continue;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const long c = (long)(x0 + r) + (long)nx * ((long)(y0 + nb) + (long)ny * (z0 + wave));
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                v[e] = acc[m][nb][e];
                if (EPI == EPI_BIAS_RELU || EPI == EPI_BIAS_F32) v[e] += A.bias[co0 + e];
                if (EPI == EPI_BIAS_RELU) v[e] = fmaxf(v[e], 0.0f);
            }
            if (EPI == EPI_MASK) {
                const uint2 mk = *reinterpret_cast<const uint2*>(A.mask + (size_t)c * COUT + co0);
                const uint16_t mm[4] = { (uint16_t)(mk.x & 0xffff), (uint16_t)(mk.x >> 16),
                                         (uint16_t)(mk.y & 0xffff), (uint16_t)(mk.y >> 16) };
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (!(bf2f(mm[e]) > 0.0f)) v[e] = 0.0f;
            }
            if (EPI == EPI_BIAS_F32 || EPI == EPI_F32) {
                *reinterpret_cast<float4*>(A.yf + (size_t)c * COUT + co0) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
                uint16_t bb[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) bb[e] = f2bf(v[e]);
                *reinterpret_cast<uint2*>(A.yb + (size_t)c * COUT + co0) =
                    make_uint2((uint32_t)bb[0] | ((uint32_t)bb[1] << 16), (uint32_t)bb[2] | ((uint32_t)bb[3] << 16));
                if (A.ybT)
#pragma unroll
                    for (int e = 0; e < 4; ++e) A.ybT[(size_t)(co0 + e) * N + c] = bb[e];
            }
        }
    }
}

template <int CIN, int COUT>
static hipError_t conv_dispatch_epi(const ConvArgs& A, int epi, hipStream_t s)
{
    const unsigned grid = (unsigned)((A.n[0] / CT_X) * (A.n[1] / CT_Y) * (A.n[2] / CT_Z));
    switch (epi) {
    case EPI_BIAS_RELU: hipLaunchKernelGGL((conv3d_kernel<CIN, COUT, EPI_BIAS_RELU>), dim3(grid), dim3(256), 0, s, A); break;
    case EPI_BIAS_F32: hipLaunchKernelGGL((conv3d_kernel<CIN, COUT, EPI_BIAS_F32>), dim3(grid), dim3(256), 0, s, A); break;
    case EPI_MASK: hipLaunchKernelGGL((conv3d_kernel<CIN, COUT, EPI_MASK>), dim3(grid), dim3(256), 0, s, A); break;
    case EPI_F32: hipLaunchKernelGGL((conv3d_kernel<CIN, COUT, EPI_F32>), dim3(grid), dim3(256), 0, s, A); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_conv3d(const ConvArgs& A, int cin, int cout, int epi, hipStream_t s)
{
    if (cin == 8 && cout == 32) return conv_dispatch_epi<8, 32>(A, epi, s);
    if (cin == 32 && cout == 32) return conv_dispatch_epi<32, 32>(A, epi, s);
    if (cin == 32 && cout == 8) return conv_dispatch_epi<32, 8>(A, epi, s);
    if (cin == 8 && cout == 8) return conv_dispatch_epi<8, 8>(A, epi, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// wgrad
// ---------------------------------------------------------------------------

// 8 consecutive values of a row starting at xs + dx (periodic), xs a
// multiple of 8, from aligned 16-byte loads
__device__ __forceinline__ uint4 shifted8(const uint16_t* row, int xs, int dx, int nx)
{
    if (dx == 0) return ld16(row + xs);
    if (dx > 0) {
        const uint4 a = ld16(row + xs);
        const uint4 b = ld16(row + (xs + 8 == nx ? 0 : xs + 8));
        return make_uint4((a.x >> 16) | (a.y << 16), (a.y >> 16) | (a.z << 16),
                          (a.z >> 16) | (a.w << 16), (a.w >> 16) | (b.x << 16));
    }
    const uint4 a = ld16(row + (xs == 0 ? nx - 8 : xs - 8));
    const uint4 b = ld16(row + xs);
    return make_uint4((a.w >> 16) | (b.x << 16), (b.x >> 16) | (b.y << 16),
                      (b.y >> 16) | (b.z << 16), (b.z >> 16) | (b.w << 16));
}

template <int CI, int CO>
__global__ void __launch_bounds__(256) conv3d_wgrad_kernel(WgradArgs A)
{
    constexpr int MB = (CO + 15) / 16, NBI = (CI + 15) / 16, NT = 7;   // offsets w + 4t
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
    const size_t N = (size_t)nx * ny * nz;
    const int nrows = ny * nz;
    const int row0 = blockIdx.x * A.rows_per_wg;
    const int row1 = min(nrows, row0 + A.rows_per_wg);

    f4 acc[NT][MB][NBI];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int q = 0; q < NBI; ++q) acc[t][m][q] = f4{ 0.f, 0.f, 0.f, 0.f };

    for (int row = row0; row < row1; ++row) {
        const int j = row % ny, k = row / ny;
        for (int x0 = 0; x0 < nx; x0 += 32) {
            const int xs = x0 + 8 * g;
            bf16x8 af[MB];
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int co = 16 * m + r;
                af[m] = as_bf8(co < CO ? ld16(A.dyT + (size_t)co * N + (size_t)row * nx + xs)
                                       : make_uint4(0, 0, 0, 0));
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int o = wave + 4 * t;
                if (o >= 27) continue;
                const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
                const size_t srow = (size_t)nx * ((size_t)wrap1(j + dy, ny) + (size_t)ny * wrap1(k + dz, nz));
#pragma unroll
                for (int q = 0; q < NBI; ++q) {
                    const int ci = 16 * q + r;
                    const bf16x8 bf = as_bf8(ci < CI ? shifted8(A.xT + (size_t)ci * N + srow, xs, dx, nx)
                                                     : make_uint4(0, 0, 0, 0));
#pragma unroll
                    for (int m = 0; m < MB; ++m)
                        acc[t][m][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[m], bf, acc[t][m][q], 0, 0, 0);
                }
            }
        }
    }
    // D[co][ci] of offset o: lane holds co = 16 m + 4 g + e, ci = 16 q + r
    float* out = A.partial + (size_t)blockIdx.x * 27 * CI * CO;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int o = wave + 4 * t;
        if (o >= 27) continue;
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int q = 0; q < NBI; ++q) {
                const int ci = 16 * q + r;
                if (ci >= CI) continue;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int co = 16 * m + 4 * g + e;
                    if (co < CO) out[((size_t)o * CI + ci) * CO + co] = acc[t][m][q][e];
                }
            }
    }
}

// dw[i] = sum over workgroups of partial[wg][i], in workgroup order
__global__ void wgrad_reduce_kernel(const float* __restrict__ partial, int nwg, int count, float* __restrict__ dw)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float acc = 0.0f;
    for (int w = 0; w < nwg; ++w) acc += partial[(size_t)w * count + i];
    dw[i] = acc;
}

// dbias[co] = sum_cell dyT[co][cell]: BG_BLOCKS workgroups per channel
// (blockIdx.y = channel) write FP64 partials, a final pass adds them in
// block order (deterministic)
__global__ void __launch_bounds__(256) bias_grad_partial_kernel(const uint16_t* __restrict__ dyT, size_t N,
                                                                double* __restrict__ partial)
{
    const int co = blockIdx.y;
    const uint16_t* row = dyT + (size_t)co * N;
    double acc = 0.0;
    // 8 values per thread per iteration (one 16-byte load; N is a multiple of 8)
    for (size_t c = ((size_t)blockIdx.x * 256 + threadIdx.x) * 8; c < N; c += (size_t)gridDim.x * 256 * 8) {
        const uint4 v = ld16(row + c);
        const uint32_t w[4] = { v.x, v.y, v.z, v.w };
        float part = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) part += bf2f((uint16_t)(w[q] & 0xffff)) + bf2f((uint16_t)(w[q] >> 16));
        acc += (double)part;
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)co * gridDim.x + blockIdx.x] = sh[0];
}

__global__ void bias_grad_final_kernel(const double* __restrict__ partial, int nblk, int cout, float* dbias)
{
    const int co = threadIdx.x;
    if (co >= cout) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += partial[(size_t)co * nblk + b];
    dbias[co] = (float)acc;
}

int wgrad_blocks(const int n[3], int& rows_per_wg)
{
    const int nrows = n[1] * n[2];
    rows_per_wg = (nrows + 511) / 512;
    return (nrows + rows_per_wg - 1) / rows_per_wg;
}

hipError_t launch_conv3d_wgrad(const WgradArgs& A, int cin, int cout, float* dw, hipStream_t s)
{
    const int nwg = (A.n[1] * A.n[2] + A.rows_per_wg - 1) / A.rows_per_wg;
    if (cin == 8 && cout == 32)
        hipLaunchKernelGGL((conv3d_wgrad_kernel<8, 32>), dim3(nwg), dim3(256), 0, s, A);
    else if (cin == 32 && cout == 32)
        hipLaunchKernelGGL((conv3d_wgrad_kernel<32, 32>), dim3(nwg), dim3(256), 0, s, A);
    else if (cin == 32 && cout == 8)
        hipLaunchKernelGGL((conv3d_wgrad_kernel<32, 8>), dim3(nwg), dim3(256), 0, s, A);
    else if (cin == 8 && cout == 8)
        hipLaunchKernelGGL((conv3d_wgrad_kernel<8, 8>), dim3(nwg), dim3(256), 0, s, A);
    else
        return hipErrorInvalidValue;
    const int count = 27 * cin * cout;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((count + 255) / 256), dim3(256), 0, s, A.partial, nwg, count, dw);
    return hipGetLastError();
}

hipError_t launch_bias_grad(const uint16_t* dyT, size_t N, int cout, float* dbias, double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(bias_grad_partial_kernel, dim3(BG_BLOCKS, cout), dim3(256), 0, s, dyT, N, partial);
    hipLaunchKernelGGL(bias_grad_final_kernel, dim3(1), dim3(64), 0, s, partial, BG_BLOCKS, cout, dbias);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------

// float [cell][c] -> bf16 [cell][c] and (if dstT) bf16 [c][cell]
__global__ void to_bf16_kernel(const float* __restrict__ src, size_t N, int c, uint16_t* dst, uint16_t* dstT)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N * c; t += (size_t)gridDim.x * blockDim.x) {
        const uint16_t b = f2bf(src[t]);
        if (dst) dst[t] = b;
        if (dstT) dstT[(t % c) * N + t / c] = b;
    }
}

hipError_t launch_to_bf16(const float* src, size_t N, int c, uint16_t* dst, uint16_t* dstT, hipStream_t s)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3(2048), dim3(256), 0, s, src, N, c, dst, dstT);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// closure elementwise and reduction kernels
// ---------------------------------------------------------------------------
// States are FP32 field-major u[f][cell]; the network sees x[cell][8] =
// (u - mean) / std in bf16 (and its channel-major copy for wgrad).

__global__ void normalize_kernel(const float* __restrict__ u, size_t N, ClosureScales sc,
                                 uint16_t* __restrict__ x, uint16_t* __restrict__ xT)
{
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        uint16_t b[8];
#pragma unroll
        for (int f = 0; f < 8; ++f) {
            b[f] = f2bf((u[(size_t)f * N + c] - sc.in_mean[f]) / sc.in_std[f]);
            xT[(size_t)f * N + c] = b[f];
        }
        uint4 v;
        v.x = (uint32_t)b[0] | ((uint32_t)b[1] << 16);
        v.y = (uint32_t)b[2] | ((uint32_t)b[3] << 16);
        v.z = (uint32_t)b[4] | ((uint32_t)b[5] << 16);
        v.w = (uint32_t)b[6] | ((uint32_t)b[7] << 16);
        *reinterpret_cast<uint4*>(x + c * 8) = v;
    }
}

hipError_t launch_normalize(const float* u, size_t N, const ClosureScales& sc, uint16_t* x, uint16_t* xT, hipStream_t s)
{
    hipLaunchKernelGGL(normalize_kernel, dim3(2048), dim3(256), 0, s, u, N, sc, x, xT);
    return hipGetLastError();
}

// Deterministic channel sums: a[c * cstride + f * fstride] over cells c for
// channels f < nch; per-block partials then one final block.
__global__ void __launch_bounds__(256) chsum_partial_kernel(const float* __restrict__ a, size_t N, size_t cstride,
                                                            size_t fstride, int nch, double* partial)
{
    double acc[8] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < N; c += (size_t)gridDim.x * 256)
        for (int f = 0; f < nch; ++f) acc[f] += (double)a[c * cstride + (size_t)f * fstride];
    __shared__ double sh[8][256];
    for (int f = 0; f < nch; ++f) sh[f][threadIdx.x] = acc[f];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int f = 0; f < nch; ++f) sh[f][threadIdx.x] += sh[f][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < nch) partial[(size_t)blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void chsum_final_kernel(const double* partial, int nblk, int nch, double scale, double* out)
{
    const int f = threadIdx.x;
    if (f >= nch) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += partial[(size_t)b * 8 + f];
    out[f] = acc * scale;
}

hipError_t launch_chsum(const float* a, size_t N, size_t cstride, size_t fstride, int nch, double scale,
                        double* partial, double* out, hipStream_t s)
{
    const int nblk = CHSUM_BLOCKS;
    hipLaunchKernelGGL(chsum_partial_kernel, dim3(nblk), dim3(256), 0, s, a, N, cstride, fstride, nch, partial);
    hipLaunchKernelGGL(chsum_final_kernel, dim3(1), dim3(64), 0, s, partial, nblk, nch, scale, out);
    return hipGetLastError();
}

// delta[f][c] = s_f (o[c][f] - mean_f) (f < 5); delta_b = curl of A = s (o5, o6, o7)
__global__ void project_kernel(const float* __restrict__ o, const double* __restrict__ mean, int nx, int ny, int nz,
                               ClosureScales sc, float* __restrict__ delta)
{
    const size_t N = (size_t)nx * ny * nz;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
        for (int f = 0; f < 5; ++f) delta[(size_t)f * N + c] = sc.out_scale[f] * (float)((double)o[c * 8 + f] - mean[f]);
        const size_t cxp = (size_t)wrap1(i + 1, nx) + (size_t)nx * (j + (size_t)ny * k);
        const size_t cyp = (size_t)i + (size_t)nx * (wrap1(j + 1, ny) + (size_t)ny * k);
        const size_t czp = (size_t)i + (size_t)nx * (j + (size_t)ny * wrap1(k + 1, nz));
        const float s5 = sc.out_scale[5], s6 = sc.out_scale[6], s7 = sc.out_scale[7];
        const float ax = s5 * o[c * 8 + 5], ay = s6 * o[c * 8 + 6], az = s7 * o[c * 8 + 7];
        delta[5 * N + c] = (s7 * o[cyp * 8 + 7] - az) - (s6 * o[czp * 8 + 6] - ay);
        delta[6 * N + c] = (s5 * o[czp * 8 + 5] - ax) - (s7 * o[cxp * 8 + 7] - az);
        delta[7 * N + c] = (s6 * o[cxp * 8 + 6] - ay) - (s5 * o[cyp * 8 + 5] - ax);
    }
}

hipError_t launch_project(const float* o, const double* mean, const int n[3], const ClosureScales& sc, float* delta,
                          hipStream_t s)
{
    hipLaunchKernelGGL(project_kernel, dim3(2048), dim3(256), 0, s, o, mean, n[0], n[1], n[2], sc, delta);
    return hipGetLastError();
}

// adjoint of the projection: g[f][c] -> go[c][8]
__global__ void project_T_kernel(const float* __restrict__ g, const double* __restrict__ gmean, int nx, int ny,
                                 int nz, ClosureScales sc, float* __restrict__ go)
{
    const size_t N = (size_t)nx * ny * nz;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
        for (int f = 0; f < 5; ++f) go[c * 8 + f] = sc.out_scale[f] * (float)((double)g[(size_t)f * N + c] - gmean[f]);
        const size_t cxm = (size_t)wrap1(i - 1, nx) + (size_t)nx * (j + (size_t)ny * k);
        const size_t cym = (size_t)i + (size_t)nx * (wrap1(j - 1, ny) + (size_t)ny * k);
        const size_t czm = (size_t)i + (size_t)nx * (j + (size_t)ny * wrap1(k - 1, nz));
        const float* gx = g + 5 * N;
        const float* gy = g + 6 * N;
        const float* gz = g + 7 * N;
        go[c * 8 + 7] = sc.out_scale[7] * ((gx[cym] - gx[c]) - (gy[cxm] - gy[c]));
        go[c * 8 + 6] = sc.out_scale[6] * ((gz[cxm] - gz[c]) - (gx[czm] - gx[c]));
        go[c * 8 + 5] = sc.out_scale[5] * ((gy[czm] - gy[c]) - (gz[cym] - gz[c]));
    }
}

hipError_t launch_project_T(const float* g, const double* gmean, const int n[3], const ClosureScales& sc, float* go,
                            hipStream_t s)
{
    hipLaunchKernelGGL(project_T_kernel, dim3(2048), dim3(256), 0, s, g, gmean, n[0], n[1], n[2], sc, go);
    return hipGetLastError();
}

// r = (delta - target) / t_f; g = 2 r / t_f / (8 N); per-block sums of r^2
__global__ void __launch_bounds__(256) loss_kernel(const float* __restrict__ delta, const float* __restrict__ target,
                                                   size_t N, ClosureScales sc, float* __restrict__ g, double* partial)
{
    double acc = 0.0;
    const double inv = 1.0 / (8.0 * (double)N);
    for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < 8 * N; t += (size_t)gridDim.x * 256) {
        const int f = (int)(t / N);
        const float r = (delta[t] - target[t]) / sc.target_scale[f];
        acc += (double)r * (double)r;
        g[t] = (float)(2.0 * (double)r / (double)sc.target_scale[f] * inv);
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x * 8] = sh[0];
}

hipError_t launch_loss(const float* delta, const float* target, size_t N, const ClosureScales& sc, float* g,
                       double* partial, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(loss_kernel, dim3(CHSUM_BLOCKS), dim3(256), 0, s, delta, target, N, sc, g, partial);
    hipLaunchKernelGGL(chsum_final_kernel, dim3(1), dim3(64), 0, s, partial, CHSUM_BLOCKS, 1,
                       1.0 / (8.0 * (double)N), out);
    return hipGetLastError();
}

// Guard of the corrected state u + theta delta for theta = 2^-k, k = 0..3:
// bit k of *bad is raised if some cell has rho <= 0, p < 0 or a non-finite
// value at that theta (pressure from the cell-centred field, the mean of
// the two faces).
__global__ void guard_levels_kernel(const float* __restrict__ u, const float* __restrict__ delta, int nx, int ny,
                                    int nz, float gamma, int* bad)
{
    const size_t N = (size_t)nx * ny * nz;
    int b = 0;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
        const size_t cn[3] = { (size_t)wrap1(i + 1, nx) + (size_t)nx * (j + (size_t)ny * k),
                               (size_t)i + (size_t)nx * (wrap1(j + 1, ny) + (size_t)ny * k),
                               (size_t)i + (size_t)nx * (j + (size_t)ny * wrap1(k + 1, nz)) };
        float u0[8], d0[8], u1[3], d1[3];
        for (int f = 0; f < 8; ++f) {
            u0[f] = u[(size_t)f * N + c];
            d0[f] = delta[(size_t)f * N + c];
        }
        for (int a = 0; a < 3; ++a) {
            u1[a] = u[(size_t)(5 + a) * N + cn[a]];
            d1[a] = delta[(size_t)(5 + a) * N + cn[a]];
        }
        for (int lev = 0; lev < GUARD_LEVELS; ++lev) {
            const float th = ldexpf(1.0f, -lev);
            float v[8];
            bool ok = true;
            for (int f = 0; f < 8; ++f) {
                v[f] = u0[f] + th * d0[f];
                ok = ok && isfinite(v[f]);
            }
            float b2 = 0.0f;
            for (int a = 0; a < 3; ++a) {
                const float bc = 0.5f * (v[5 + a] + (u1[a] + th * d1[a]));
                b2 += bc * bc;
            }
            const float p = (gamma - 1.0f) * (v[4] - 0.5f * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / v[0] -
                                               0.5f * b2);
            ok = ok && v[0] > 0.0f && p >= 0.0f;
            if (!ok) b |= 1 << lev;
        }
    }
    if (b) atomicOr(bad, b);
}

hipError_t launch_guard_levels(const float* u, const float* delta, const int n[3], float gamma, int* bad,
                               hipStream_t s)
{
    hipLaunchKernelGGL(guard_levels_kernel, dim3(2048), dim3(256), 0, s, u, delta, n[0], n[1], n[2], gamma, bad);
    return hipGetLastError();
}

// u += theta delta with the largest theta = 2^-k whose guard bit is clear;
// none clear: u stays (the plain step).  counts[0] counts dropped
// corrections, counts[1] reduced ones (theta < 1).
__global__ void apply_level_kernel(float* __restrict__ u, const float* __restrict__ delta, size_t n, const int* bad,
                                   int* counts)
{
    const int mask = *bad;
    int lev = 0;
    while (lev < GUARD_LEVELS && (mask >> lev) & 1) ++lev;
    if (blockIdx.x == 0 && threadIdx.x == 0 && counts) {
        if (lev == GUARD_LEVELS) counts[0] += 1;
        else if (lev > 0) counts[1] += 1;
    }
    if (lev == GUARD_LEVELS) return;
    const float th = ldexpf(1.0f, -lev);
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        u[t] = u[t] + th * delta[t];
}

hipError_t launch_apply_level(float* u, const float* delta, size_t n, const int* bad, int* counts, hipStream_t s)
{
    hipLaunchKernelGGL(apply_level_kernel, dim3(2048), dim3(256), 0, s, u, delta, n, bad, counts);
    return hipGetLastError();
}

__global__ void zero_int_kernel(int* p) { if (threadIdx.x == 0) *p = 0; }
hipError_t launch_zero_int(int* p, hipStream_t s)
{
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

// Adam (Kingma & Ba) on FP32 master parameters
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// target = u_ref - u_plain, elementwise over 8N values
__global__ void residual_kernel(const float* __restrict__ ref, const float* __restrict__ plain, size_t n,
                                float* __restrict__ out)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        out[t] = ref[t] - plain[t];
}

hipError_t launch_residual(const float* ref, const float* plain, size_t n, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(residual_kernel, dim3(2048), dim3(256), 0, s, ref, plain, n, out);
    return hipGetLastError();
}

// Per-field sums of a field-major pair (u, t), blockIdx.y = field:
// partial[(b * 8 + f) * 5 + q], q = sum u, sum u^2, sum |u|, sum |t|, and
// sum of the roughness r = sum over axes |u(c+a) - 2 u(c) + u(c-a)|
__global__ void __launch_bounds__(256) stats_partial_kernel(const float* __restrict__ u,
                                                            const float* __restrict__ t, int nx, int ny, int nz,
                                                            double* __restrict__ partial)
{
    const size_t N = (size_t)nx * ny * nz;
    const int f = blockIdx.y;
    const float* uf = u + (size_t)f * N;
    const float* tf = t + (size_t)f * N;
    double a[5] = { 0.0, 0.0, 0.0, 0.0, 0.0 };
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < N; c += (size_t)gridDim.x * 256) {
        const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
        const double x = uf[c];
        a[0] += x;
        a[1] += x * x;
        a[2] += fabs(x);
        a[3] += fabs((double)tf[c]);
        const size_t row = (size_t)nx * (j + (size_t)ny * k);
        const double xp = uf[row + wrap1(i + 1, nx)], xm = uf[row + wrap1(i - 1, nx)];
        const double yp = uf[(size_t)i + (size_t)nx * (wrap1(j + 1, ny) + (size_t)ny * k)];
        const double ym = uf[(size_t)i + (size_t)nx * (wrap1(j - 1, ny) + (size_t)ny * k)];
        const double zp = uf[(size_t)i + (size_t)nx * (j + (size_t)ny * wrap1(k + 1, nz))];
        const double zm = uf[(size_t)i + (size_t)nx * (j + (size_t)ny * wrap1(k - 1, nz))];
        a[4] += fabs(xp - 2.0 * x + xm) + fabs(yp - 2.0 * x + ym) + fabs(zp - 2.0 * x + zm);
    }
    __shared__ double sh[5][256];
    for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 5) partial[((size_t)blockIdx.x * 8 + f) * 5 + threadIdx.x] = sh[threadIdx.x][0];
}

// out[q * 8 + f] = sum over blocks of partial[(b * 8 + f) * 5 + q]
__global__ void stats_final_kernel(const double* __restrict__ partial, int nblk, double* __restrict__ out)
{
    const int k = threadIdx.x;
    if (k >= 40) return;
    const int q = k / 8, f = k % 8;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += partial[((size_t)b * 8 + f) * 5 + q];
    out[k] = acc;
}

hipError_t launch_stats(const float* u, const float* t, const int n[3], double* partial, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(stats_partial_kernel, dim3(STATS_BLOCKS, 8), dim3(256), 0, s, u, t, n[0], n[1], n[2], partial);
    hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(64), 0, s, partial, STATS_BLOCKS, out);
    return hipGetLastError();
}

// Roughness gate: g0(c) = (1/8) sum_f inv_R[f] * sum over axes
// |u_f(c+a) - 2 u_f(c) + u_f(c-a)| (u field-major FP32)
__global__ void __launch_bounds__(256) gate_rough_kernel(const float* __restrict__ u, int nx, int ny, int nz,
                                                         GateScales gs, float* __restrict__ g0)
{
    const size_t N = (size_t)nx * ny * nz;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
        const size_t row = (size_t)nx * (j + (size_t)ny * k);
        const size_t nb[6] = { row + wrap1(i + 1, nx), row + wrap1(i - 1, nx),
                               (size_t)i + (size_t)nx * (wrap1(j + 1, ny) + (size_t)ny * k),
                               (size_t)i + (size_t)nx * (wrap1(j - 1, ny) + (size_t)ny * k),
                               (size_t)i + (size_t)nx * (j + (size_t)ny * wrap1(k + 1, nz)),
                               (size_t)i + (size_t)nx * (j + (size_t)ny * wrap1(k - 1, nz)) };
        float acc = 0.0f;
        for (int f = 0; f < 8; ++f) {
            const float* uf = u + (size_t)f * N;
            const float x2 = 2.0f * uf[c];
            float r = 0.0f;
            for (int a = 0; a < 3; ++a) r += fabsf((uf[nb[2 * a]] - x2) + uf[nb[2 * a + 1]]);
            acc += r * gs.inv_r[f];
        }
        g0[c] = 0.125f * acc;
    }
}

// g(c) = max of g0 over c and its six face neighbours
__global__ void __launch_bounds__(256) gate_max_kernel(const float* __restrict__ g0, int nx, int ny, int nz,
                                                       float* __restrict__ g)
{
    const size_t N = (size_t)nx * ny * nz;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
        const size_t row = (size_t)nx * (j + (size_t)ny * k);
        float m = g0[c];
        m = fmaxf(m, g0[row + wrap1(i + 1, nx)]);
        m = fmaxf(m, g0[row + wrap1(i - 1, nx)]);
        m = fmaxf(m, g0[(size_t)i + (size_t)nx * (wrap1(j + 1, ny) + (size_t)ny * k)]);
        m = fmaxf(m, g0[(size_t)i + (size_t)nx * (wrap1(j - 1, ny) + (size_t)ny * k)]);
        m = fmaxf(m, g0[(size_t)i + (size_t)nx * (j + (size_t)ny * wrap1(k + 1, nz))]);
        m = fmaxf(m, g0[(size_t)i + (size_t)nx * (j + (size_t)ny * wrap1(k - 1, nz))]);
        g[c] = m;
    }
}

hipError_t launch_gate(const float* u, const int n[3], const GateScales& gs, float* g0, float* g, hipStream_t s)
{
    hipLaunchKernelGGL(gate_rough_kernel, dim3(2048), dim3(256), 0, s, u, n[0], n[1], n[2], gs, g0);
    hipLaunchKernelGGL(gate_max_kernel, dim3(2048), dim3(256), 0, s, g0, n[0], n[1], n[2], g);
    return hipGetLastError();
}

// a[c][f] *= g[c], channel-last rows of 8
__global__ void row_scale_kernel(float* __restrict__ a, const float* __restrict__ g, size_t N)
{
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const float s = g[c];
        float4* p = reinterpret_cast<float4*>(a + c * 8);
        float4 v0 = p[0], v1 = p[1];
        v0.x *= s; v0.y *= s; v0.z *= s; v0.w *= s;
        v1.x *= s; v1.y *= s; v1.z *= s; v1.w *= s;
        p[0] = v0;
        p[1] = v1;
    }
}

hipError_t launch_row_scale(float* a, const float* g, size_t N, hipStream_t s)
{
    hipLaunchKernelGGL(row_scale_kernel, dim3(2048), dim3(256), 0, s, a, g, N);
    return hipGetLastError();
}

}  // namespace mhd
