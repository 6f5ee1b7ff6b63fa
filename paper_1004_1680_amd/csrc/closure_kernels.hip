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
// of one channel.  A workgroup stages a tile of x with its halo in LDS; each
// of its 9 waves owns one (dy, dz) pair and builds the dx = -1, 0, +1
// fragments from three aligned 16-byte reads.  Persistent workgroups write
// partial sums, which two passes add in a fixed order (deterministic).
//
// Requirements: nx, ny, nz multiples of 32 (the tiles: 16 x 4 x 4 cells for
// forward / dgrad, 32 x 4 x 2 for wgrad), fewer than 2^31 cells.
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

// (i, j, k) of cell c = i + nx (j + ny k), 32-bit arithmetic (fewer than 2^31 cells)
__device__ __forceinline__ void cell_ijk(unsigned c, int nx, int ny, int& i, int& j, int& k)
{
    const unsigned q = c / (unsigned)nx;
    i = (int)(c - q * (unsigned)nx);
    const unsigned k_ = q / (unsigned)ny;
    j = (int)(q - k_ * (unsigned)ny);
    k = (int)k_;
}

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
// The input halo (18 x 6 x 6 cells, periodic) is staged once in LDS and
// every one of the 27 offsets reads its B fragments from there.  A B read
// has 16 lanes on 16 consecutive cells reading the same 16-byte chunk; with
// 64-byte cells (CIN = 32) the chunks of cells h and h + 4 would share
// banks, so chunk q of cell h is stored at position q ^ 2 ((h >> 2) & 1):
// any 8 consecutive cells then fall on distinct bank groups (measured on
// gfx950: a lane stride that is an odd multiple of 32 bytes modulo 256, or
// this swizzle, is conflict-free; 64 or 80 bytes costs two passes).
constexpr int CT_X = 16, CT_Y = 4, CT_Z = 4;
constexpr int CH_X = CT_X + 2, CH_Y = CT_Y + 2, CH_Z = CT_Z + 2, CH_CELLS = CH_X * CH_Y * CH_Z;

template <int CIN>
__host__ __device__ constexpr int conv_cell_stride() { return CIN; }
// position (in 8-bf16 chunks) of chunk q of halo cell h
template <int CIN>
__device__ __forceinline__ int conv_chunk(int h, int q) { return CIN == 32 ? (q ^ (((h >> 2) & 1) << 1)) : q; }

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
    // consecutive pieces (contiguous along x in global memory); all loads
    // of a thread are issued before its LDS writes
    constexpr int FILL = (CH_CELLS * PARTS + 255) / 256;
    uint4 fv[FILL];
#pragma unroll
    for (int f = 0; f < FILL; ++f) {
        const int t = threadIdx.x + 256 * f;
        fv[f] = make_uint4(0, 0, 0, 0);
        if (t < CH_CELLS * PARTS) {
            const int h = t / PARTS, q = t % PARTS;
            const int hx = h % CH_X, hy = (h / CH_X) % CH_Y, hz = h / (CH_X * CH_Y);
            const unsigned src = (unsigned)wrap1(x0 - 1 + hx, nx) +
                                 (unsigned)nx * ((unsigned)wrap1(y0 - 1 + hy, ny) +
                                                 (unsigned)ny * (unsigned)wrap1(z0 - 1 + hz, nz));
            fv[f] = ld16(x + (size_t)src * CIN + 8 * q);
        }
    }
#pragma unroll
    for (int f = 0; f < FILL; ++f) {
        const int t = threadIdx.x + 256 * f;
        if (t < CH_CELLS * PARTS) {
            const int h = t / PARTS, q = t % PARTS;
            *reinterpret_cast<uint4*>(tile + h * CS + 8 * conv_chunk<CIN>(h, q)) = fv[f];
        }
    }
    __syncthreads();

    f4 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f4{ 0.f, 0.f, 0.f, 0.f };

    // K step s: weight fragments from global memory (L2), activation
    // fragments from the LDS halo; the loop is unrolled and the fragments of
    // step s + 1 are loaded while the MFMAs of step s run
    const int hbase = (wave + 1) * (CH_X * CH_Y) + CH_X + (r + 1);
    auto load_a = [&](int s, bf16x8* a) {
#pragma unroll
        for (int m = 0; m < MB; ++m) a[m] = as_bf8(wp[((size_t)s * MB + m) * 64 + lane]);
    };
    auto load_b = [&](int s, bf16x8* bv) {
        const int K = 32 * s + 8 * g;
        const int o = K / CIN, c0 = K % CIN;
        const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
        const int h0 = hbase + dz * (CH_X * CH_Y) + dy * CH_X + dx;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            uint4 v = make_uint4(0, 0, 0, 0);
            const int h = h0 + nb * CH_X;
            if (o < 27) v = *reinterpret_cast<const uint4*>(tile + h * CS + 8 * conv_chunk<CIN>(h, c0 / 8));
            bv[nb] = as_bf8(v);
        }
    };
    bf16x8 a_cur[MB], b_cur[NB];
    load_a(0, a_cur);
    load_b(0, b_cur);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        bf16x8 a_nxt[MB], b_nxt[NB];
        if (s + 1 < KS) {
            load_a(s + 1, a_nxt);
            load_b(s + 1, b_nxt);
        }
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_cur[m], b_cur[nb], acc[m][nb], 0, 0, 0);
        if (s + 1 < KS) {
#pragma unroll
            for (int m = 0; m < MB; ++m) a_cur[m] = a_nxt[m];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) b_cur[nb] = b_nxt[nb];
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

// 8 consecutive bf16 starting one element after (dx = +1) or before
// (dx = -1) the aligned group c, from the aligned groups around it
__device__ __forceinline__ uint4 shift_right1(uint4 c, uint4 n)    // elements c[1..7], n[0]
{
    return make_uint4((c.x >> 16) | (c.y << 16), (c.y >> 16) | (c.z << 16), (c.z >> 16) | (c.w << 16),
                      (c.w >> 16) | (n.x << 16));
}
__device__ __forceinline__ uint4 shift_left1(uint4 p, uint4 c)     // elements p[7], c[0..6]
{
    return make_uint4((p.w >> 16) | (c.x << 16), (c.x >> 16) | (c.y << 16), (c.y >> 16) | (c.z << 16),
                      (c.z >> 16) | (c.w << 16));
}

// Tile of wgrad: 32 (x) x 4 (y) x 2 (z) cells = 8 K steps of 32 cells (one
// row segment each).
constexpr int WT_X = 32, WT_Y = 4, WT_Z = 2;
constexpr int WL_Y = WT_Y + 2, WL_Z = WT_Z + 2;          // x rows with their y / z halo

// wgrad: dW[o][ci][co] = sum_c x[c + d(o)][ci] dy[c][co]
//                     = sum_c dy[c - dx][co] x[c + (0, dy, dz)][ci]
// (the x offset moved onto dy), with M = co (A = dy shifted along x), N = ci
// (B = x rows, aligned: no shifting), K = cells.  Three waves per
// workgroup; wave w owns the offsets with dz = w - 1 and all nine (dx, dy),
// so an A fragment feeds 3 x NBI and a B fragment 3 x MB products.  LDS:
// x without an x halo, [ci][hz][hy][32], and dy with one, [co][ks][48],
// channel strides padded by 16 bf16 (75 KB for 32 -> 32 channels).  The
// elements one before and after a lane's 8 dy values come from the lanes
// 16 below and above (ds_bpermute) or, at the segment's ends, from the
// halo.  With 8 channels on one side a 16-row (16-column) block carries two
// offsets.  Persistent over tiles; each workgroup writes its partial sums,
// wgrad_reduce adds them in a fixed order.  (A first form shifted x and ran
// nine waves of three offsets each: it read x with halo in all three axes
// and the dword reads of each shifted fragment's edge elements conflicted
// in the LDS banks; 315, 271 and 130 us against 236, 110 and 100 us for
// 32 -> 32, 32 -> 8 and 8 -> 32 channels at 128^3.)
constexpr int WG_WAVES = 3;

template <int CI, int CO>
__global__ void __launch_bounds__(64 * WG_WAVES, (CI * CO > 256 ? 1 : 2)) conv3d_wgrad_kernel(WgradArgs A)
{
    constexpr int MB = (CO + 15) / 16, NBI = (CI + 15) / 16;
    constexpr int KSTEPS = WT_Y * WT_Z;
    constexpr int XROWS = WL_Z * WL_Y;                       // 4 x 6 rows of x per tile
    constexpr int XCS = XROWS * WT_X + 16;                   // channel strides, padded as above
    constexpr int DX = WT_X + 16;                            // dy row with 8 halo cells each side
    constexpr int DYS = KSTEPS * DX + 16;
    constexpr int NT = 64 * WG_WAVES;
    __shared__ __align__(16) uint16_t xs[CI * XCS];
    __shared__ __align__(16) uint16_t dys[CO * DYS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int ddz = wave - 1;
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
    const size_t N = (size_t)nx * ny * nz;
    const int tx = nx / WT_X, ty = ny / WT_Y, ntiles = tx * ty * (nz / WT_Z);

    // 8 channels of dy (x) fill only half of an MFMA block's rows (columns):
    // there the rows (columns) carry (channel, dx) ((channel, dy)) pairs,
    // 8 channels x 2 offsets per block, two blocks for the three offsets
    constexpr bool FM = CO == 8 && CI > 8, FN = CI == 8 && CO > 8;
    constexpr int AN = FM ? 2 : 3, BN = FN ? 2 : 3;
    f4 acc[AN][BN][MB][NBI];                                // [dx + 1][dy + 1], or the folded blocks
#pragma unroll
    for (int a = 0; a < AN; ++a)
#pragma unroll
        for (int b = 0; b < BN; ++b)
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int q = 0; q < NBI; ++q) acc[a][b][m][q] = f4{ 0.f, 0.f, 0.f, 0.f };

    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int x0 = (t % tx) * WT_X, y0 = ((t / tx) % ty) * WT_Y, z0 = (t / (tx * ty)) * WT_Z;
        // fill: x rows (ci, hz, hy) of 32 cells = 4 loads of 16 bytes, dy rows
        // (co, ks) of 48 cells (x0 - 8 .. x0 + 40, periodic) = 6 loads
        constexpr int XI = CI * XROWS * (WT_X / 8), DI = CO * KSTEPS * (DX / 8), ITEMS = XI + DI;
        // as many of a thread's loads in flight at once as the registers
        // allow (the fill waits for one round trip per batch): 24 (all) with
        // 32 -> 32 channels at one wave per SIMD, 12 at two
        constexpr int FMAX = CI * CO > 256 ? 24 : 12;
        constexpr int FILL = (ITEMS + NT - 1) / NT, FB = FILL < FMAX ? FILL : FMAX;
        __syncthreads();                                   // previous tile's reads are done
#pragma unroll
        for (int f0 = 0; f0 < FILL; f0 += FB) {
            uint4 fv[FB];
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                const int it = threadIdx.x + NT * (f0 + f);
                fv[f] = make_uint4(0, 0, 0, 0);
                if (f0 + f < FILL && it < XI) {
                    const int gx = it % (WT_X / 8), row = (it / (WT_X / 8)) % XROWS, ci = it / (WT_X / 8 * XROWS);
                    const int hy = row % WL_Y, hz = row / WL_Y;
                    const size_t src = (size_t)ci * N + (size_t)(x0 + 8 * gx) +
                                       (size_t)nx * ((size_t)wrap1(y0 - 1 + hy, ny) + (size_t)ny * wrap1(z0 - 1 + hz, nz));
                    fv[f] = ld16(A.xT + src);
                } else if (f0 + f < FILL && it < ITEMS) {
                    const int d = it - XI, gx = d % (DX / 8), ks = (d / (DX / 8)) % KSTEPS;
                    const int co = d / (DX / 8 * KSTEPS);
                    const int sx = x0 - 8 + 8 * gx, gxs = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
                    const size_t src = (size_t)co * N + (size_t)gxs +
                                       (size_t)nx * ((size_t)(y0 + ks % WT_Y) + (size_t)ny * (z0 + ks / WT_Y));
                    fv[f] = ld16(A.dyT + src);
                }
            }
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                const int it = threadIdx.x + NT * (f0 + f);
                if (f0 + f < FILL && it < XI) {
                    const int gx = it % (WT_X / 8), row = (it / (WT_X / 8)) % XROWS, ci = it / (WT_X / 8 * XROWS);
                    *reinterpret_cast<uint4*>(xs + ci * XCS + row * WT_X + 8 * gx) = fv[f];
                } else if (f0 + f < FILL && it < ITEMS) {
                    const int d = it - XI, gx = d % (DX / 8), ks = (d / (DX / 8)) % KSTEPS;
                    const int co = d / (DX / 8 * KSTEPS);
                    *reinterpret_cast<uint4*>(dys + co * DYS + ks * DX + 8 * gx) = fv[f];
                }
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int ks = 0; ks < KSTEPS; ++ks) {
            const int ky = ks % WT_Y, kz = ks / WT_Y;
            // A: dy of channel co = 16 m + r (FM: r mod 8), cells 8 g .. 8 g + 7
            // of the row, shifted by -dx
            bf16x8 af[AN][MB];
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int co = FM ? (r & 7) : 16 * m + r;
                const uint16_t* row = dys + (co < CO ? co : 0) * DYS + ks * DX;
                uint4 mid = *reinterpret_cast<const uint4*>(row + 8 + 8 * g);
                // the row's halo element before (g = 0: cell -1) or after
                // (g = 3: cell 32) the lane's segment
                const uint32_t halo = *reinterpret_cast<const uint32_t*>(row + (g == 3 ? 40 : 6));
                const uint32_t pw = (uint32_t)__shfl((int)mid.w, lane - 16, 64);
                const uint32_t nw = (uint32_t)__shfl((int)mid.x, lane + 16, 64);
                const uint32_t prev = g == 0 ? halo : pw;       // its high half: cell 8 g - 1
                const uint32_t next = g == 3 ? halo : nw;       // its low half: cell 8 g + 8
                if (co >= CO) mid = make_uint4(0, 0, 0, 0);
                const uint32_t prevv = co < CO ? prev : 0u, nextv = co < CO ? next : 0u;
                const uint4 sm1 = shift_right1(mid, make_uint4(nextv, 0, 0, 0));   // dx = -1: dy at c + 1
                const uint4 sp1 = shift_left1(make_uint4(0, 0, 0, prevv), mid);    // dx = +1: dy at c - 1
                if constexpr (FM) {
                    // rows r < 8: dx = -1 | +1, rows r >= 8: dx = 0 | none
                    af[0][m] = as_bf8(r < 8 ? sm1 : mid);
                    af[1][m] = as_bf8(r < 8 ? sp1 : make_uint4(0, 0, 0, 0));
                } else {
                    af[0][m] = as_bf8(sm1);
                    af[1][m] = as_bf8(mid);
                    af[2][m] = as_bf8(sp1);
                }
            }
            if constexpr (FN) {
                // columns r < 8: dy = -1 | +1, columns r >= 8: dy = 0 | none
                bf16x8 bf[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int b = 2 * j + (r >> 3), ci = r & 7;
                    bf[j] = as_bf8(b < 3 ? *reinterpret_cast<const uint4*>(
                                               xs + ci * XCS + ((kz + 1 + ddz) * WL_Y + ky + b) * WT_X + 8 * g)
                                         : make_uint4(0, 0, 0, 0));
                }
#pragma unroll
                for (int a = 0; a < AN; ++a)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int m = 0; m < MB; ++m)
                            acc[a][j][m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a][m], bf[j], acc[a][j][m][0],
                                                                                      0, 0, 0);
            } else {
#pragma unroll
                for (int b = 0; b < 3; ++b) {              // dy = b - 1
                    bf16x8 bf[NBI];
#pragma unroll
                    for (int q = 0; q < NBI; ++q) {
                        const int ci = 16 * q + r;
                        bf[q] = as_bf8(ci < CI ? *reinterpret_cast<const uint4*>(
                                                     xs + ci * XCS + ((kz + 1 + ddz) * WL_Y + ky + b) * WT_X + 8 * g)
                                               : make_uint4(0, 0, 0, 0));
                    }
#pragma unroll
                    for (int a = 0; a < AN; ++a)
#pragma unroll
                        for (int m = 0; m < MB; ++m)
#pragma unroll
                            for (int q = 0; q < NBI; ++q)
                                acc[a][b][m][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a][m], bf[q],
                                                                                          acc[a][b][m][q], 0, 0, 0);
                }
            }
        }
    }
    // D of an MFMA block: lane holds rows 4 g + e (e = 0..3), column r;
    // unfolded, row = co - 16 m and column = ci - 16 q
    float* out = A.partial + (size_t)blockIdx.x * 27 * CI * CO;
#pragma unroll
    for (int a = 0; a < AN; ++a)
#pragma unroll
        for (int b = 0; b < BN; ++b)
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
                for (int q = 0; q < NBI; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = 4 * g + e;
                        const int co = FM ? (row & 7) : 16 * m + row;
                        const int dxi = FM ? 2 * a + (row >> 3) : a;            // dx + 1
                        const int ci = FN ? (r & 7) : 16 * q + r;
                        const int dyi = FN ? 2 * b + (r >> 3) : b;              // dy + 1
                        if (co >= CO || ci >= CI || dxi > 2 || dyi > 2) continue;
                        const int o = (ddz + 1) * 9 + dyi * 3 + dxi;
                        out[((size_t)o * CI + ci) * CO + co] = acc[a][b][m][q][e];
                    }
}

// dw[i] = sum over workgroups of partial[wg][i] in workgroup order: pass 1
// sums WR_GROUPS contiguous ranges of workgroups, pass 2 the ranges
constexpr int WR_GROUPS = 16;
__global__ void wgrad_reduce1_kernel(const float* __restrict__ partial, int nwg, int count, float* __restrict__ mid)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int grp = blockIdx.y;
    if (i >= count) return;
    const int per = (nwg + WR_GROUPS - 1) / WR_GROUPS;
    const int w0 = grp * per, w1 = min(nwg, w0 + per);
    float acc = 0.0f;
    for (int w = w0; w < w1; ++w) acc += partial[(size_t)w * count + i];
    mid[(size_t)grp * count + i] = acc;
}

__global__ void wgrad_reduce2_kernel(const float* __restrict__ mid, int count, float* __restrict__ dw)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float acc = 0.0f;
    for (int k = 0; k < WR_GROUPS; ++k) acc += mid[(size_t)k * count + i];
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

int wgrad_blocks(const int n[3], int& tiles_per_wg)
{
    const int ntiles = (n[0] / WT_X) * (n[1] / WT_Y) * (n[2] / WT_Z);
    const int nwg = ntiles < WGRAD_MAX_WG ? ntiles : WGRAD_MAX_WG;
    tiles_per_wg = (ntiles + nwg - 1) / nwg;
    return nwg;
}

hipError_t launch_conv3d_wgrad(const WgradArgs& A, int cin, int cout, float* dw, hipStream_t s)
{
    int tpw = 0;
    const int nwg = wgrad_blocks(A.n, tpw);
    constexpr int T2 = 64 * WG_WAVES;
    if (cin == 8 && cout == 32)
        hipLaunchKernelGGL((conv3d_wgrad_kernel<8, 32>), dim3(nwg), dim3(T2), 0, s, A);
    else if (cin == 32 && cout == 32)
        hipLaunchKernelGGL((conv3d_wgrad_kernel<32, 32>), dim3(nwg), dim3(T2), 0, s, A);
    else if (cin == 32 && cout == 8)
        hipLaunchKernelGGL((conv3d_wgrad_kernel<32, 8>), dim3(nwg), dim3(T2), 0, s, A);
    else if (cin == 8 && cout == 8)
        hipLaunchKernelGGL((conv3d_wgrad_kernel<8, 8>), dim3(nwg), dim3(T2), 0, s, A);
    else
        return hipErrorInvalidValue;
    const int count = 27 * cin * cout;
    float* mid = A.partial + (size_t)nwg * count;
    hipLaunchKernelGGL(wgrad_reduce1_kernel, dim3((count + 255) / 256, WR_GROUPS), dim3(256), 0, s, A.partial, nwg,
                       count, mid);
    hipLaunchKernelGGL(wgrad_reduce2_kernel, dim3((count + 255) / 256), dim3(256), 0, s, mid, count, dw);
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
            if (xT) xT[(size_t)f * N + c] = b[f];
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

// out[f] = scale * sum over blocks of partial[b * 8 + f]: 256 threads, each a
// fixed stride of blocks, then a fixed tree (deterministic)
__global__ void __launch_bounds__(256) chsum_final_kernel(const double* partial, int nblk, int nch, double scale,
                                                          double* out)
{
    __shared__ double sh[8][256];
    for (int f = 0; f < nch; ++f) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) acc += partial[(size_t)b * 8 + f];
        sh[f][threadIdx.x] = acc;
    }
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int f = 0; f < nch; ++f) sh[f][threadIdx.x] += sh[f][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < nch) out[threadIdx.x] = sh[threadIdx.x][0] * scale;
}

hipError_t launch_chsum(const float* a, size_t N, size_t cstride, size_t fstride, int nch, double scale,
                        double* partial, double* out, hipStream_t s)
{
    const int nblk = CHSUM_BLOCKS;
    hipLaunchKernelGGL(chsum_partial_kernel, dim3(nblk), dim3(256), 0, s, a, N, cstride, fstride, nch, partial);
    hipLaunchKernelGGL(chsum_final_kernel, dim3(1), dim3(256), 0, s, partial, nblk, nch, scale, out);
    return hipGetLastError();
}

// delta[f][c] = s_f (o[c][f] - mean_f) (f < 5); delta_b = curl of A = s (o5, o6, o7)
__global__ void project_kernel(const float* __restrict__ o, const double* __restrict__ mean, int nx, int ny, int nz,
                               ClosureScales sc, float* __restrict__ delta)
{
    const size_t N = (size_t)nx * ny * nz;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_ijk((unsigned)c, nx, ny, i, j, k);
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
        int i, j, k;
        cell_ijk((unsigned)c, nx, ny, i, j, k);
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
    const int f = blockIdx.y;
    const float ts = sc.target_scale[f];
    const double gsc = 2.0 / (double)ts / (8.0 * (double)N);
    const size_t off = (size_t)f * N;
    double acc = 0.0;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < N; c += (size_t)gridDim.x * 256) {
        const float r = (delta[off + c] - target[off + c]) / ts;
        acc += (double)r * (double)r;
        g[off + c] = (float)((double)r * gsc);
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)f * gridDim.x + blockIdx.x] = sh[0];
}

// out = scale * sum of partial[0 .. n), 256 threads at fixed strides, then a
// fixed tree (deterministic)
__global__ void __launch_bounds__(256) sum_final_kernel(const double* __restrict__ partial, int n, double scale,
                                                        double* out)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < n; b += 256) acc += partial[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0] * scale;
}

hipError_t launch_loss(const float* delta, const float* target, size_t N, const ClosureScales& sc, float* g,
                       double* partial, double* out, hipStream_t s)
{
    // LOSS_BLOCKS per field, 8 * LOSS_BLOCKS dense partials (fits the CHSUM_BLOCKS * 8 scratch)
    constexpr int LOSS_BLOCKS = CHSUM_BLOCKS / 2;
    hipLaunchKernelGGL(loss_kernel, dim3(LOSS_BLOCKS, 8), dim3(256), 0, s, delta, target, N, sc, g, partial);
    hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(256), 0, s, partial, 8 * LOSS_BLOCKS, 1.0 / (8.0 * (double)N),
                       out);
    return hipGetLastError();
}

// Guard of the corrected state u + theta delta for theta = 2^-k, k = 0..3:
// bit k of *bad is raised if some cell has rho <= 0, p < 0 or a non-finite
// value at that theta (pressure from the cell-centred field, the mean of
// the two faces; tested without a division as 2 rho (e - |B|^2/2) >= |m|^2).
__global__ void __launch_bounds__(256) guard_levels_kernel(const float* __restrict__ u,
                                                          const float* __restrict__ delta, int nx, int ny, int nz,
                                                          int* bad)
{
    // 4 consecutive x cells per thread (nx is a multiple of 4)
    const unsigned N = (unsigned)nx * ny * nz, N4 = N / 4;
    int b = 0;
    for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < N4; t += gridDim.x * blockDim.x) {
        const unsigned c = 4 * t;
        int i, j, k;
        cell_ijk(c, nx, ny, i, j, k);
        const unsigned xp = c - i + wrap1(i + 4, nx);
        const unsigned cyp = (unsigned)i + (unsigned)nx * ((unsigned)wrap1(j + 1, ny) + (unsigned)ny * k);
        const unsigned czp = (unsigned)i + (unsigned)nx * ((unsigned)j + (unsigned)ny * wrap1(k + 1, nz));
        float u0[8][4], d0[8][4], u1[3][4], d1[3][4];
        for (int f = 0; f < 8; ++f) {
            const float4 a4 = *reinterpret_cast<const float4*>(u + (size_t)f * N + c);
            const float4 b4 = *reinterpret_cast<const float4*>(delta + (size_t)f * N + c);
            u0[f][0] = a4.x; u0[f][1] = a4.y; u0[f][2] = a4.z; u0[f][3] = a4.w;
            d0[f][0] = b4.x; d0[f][1] = b4.y; d0[f][2] = b4.z; d0[f][3] = b4.w;
        }
        // upper faces: b_x of the next cell along x, b_y / b_z of the next row / plane
        for (int q = 0; q < 3; ++q) { u1[0][q] = u0[5][q + 1]; d1[0][q] = d0[5][q + 1]; }
        u1[0][3] = u[(size_t)5 * N + xp];
        d1[0][3] = delta[(size_t)5 * N + xp];
        {
            const float4 a4 = *reinterpret_cast<const float4*>(u + (size_t)6 * N + cyp);
            const float4 b4 = *reinterpret_cast<const float4*>(delta + (size_t)6 * N + cyp);
            const float4 c4 = *reinterpret_cast<const float4*>(u + (size_t)7 * N + czp);
            const float4 e4 = *reinterpret_cast<const float4*>(delta + (size_t)7 * N + czp);
            u1[1][0] = a4.x; u1[1][1] = a4.y; u1[1][2] = a4.z; u1[1][3] = a4.w;
            d1[1][0] = b4.x; d1[1][1] = b4.y; d1[1][2] = b4.z; d1[1][3] = b4.w;
            u1[2][0] = c4.x; u1[2][1] = c4.y; u1[2][2] = c4.z; u1[2][3] = c4.w;
            d1[2][0] = e4.x; d1[2][1] = e4.y; d1[2][2] = e4.z; d1[2][3] = e4.w;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int lev = 0; lev < GUARD_LEVELS; ++lev) {
                const float th = ldexpf(1.0f, -lev);
                float v[8];
                bool ok = true;
                for (int f = 0; f < 8; ++f) {
                    v[f] = u0[f][q] + th * d0[f][q];
                    ok = ok && isfinite(v[f]);
                }
                float b2 = 0.0f;
                for (int a = 0; a < 3; ++a) {
                    const float bc = 0.5f * (v[5 + a] + (u1[a][q] + th * d1[a][q]));
                    b2 += bc * bc;
                }
                // p >= 0 with rho > 0  <=>  2 rho (e - |B|^2 / 2) >= |m|^2 (gamma > 1)
                const float lhs = 2.0f * v[0] * (v[4] - 0.5f * b2);
                const float m2 = v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
                ok = ok && v[0] > 0.0f && lhs >= m2;
                if (!ok) b |= 1 << lev;
            }
    }
    // one atomic per wave: OR of the level bits over its lanes
    int wb = 0;
#pragma unroll
    for (int lev = 0; lev < GUARD_LEVELS; ++lev)
        if (__ballot((b >> lev) & 1)) wb |= 1 << lev;
    if ((threadIdx.x & 63) == 0 && wb) atomicOr(bad, wb);
}

hipError_t launch_guard_levels(const float* u, const float* delta, const int n[3], float gamma, int* bad,
                               hipStream_t s)
{
    (void)gamma;                      // the sign of p does not depend on gamma > 1
    hipLaunchKernelGGL(guard_levels_kernel, dim3(2048), dim3(256), 0, s, u, delta, n[0], n[1], n[2], bad);
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
        int i, j, k;
        cell_ijk((unsigned)c, nx, ny, i, j, k);
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

// out[q * 8 + f] = sum over blocks of partial[(b * 8 + f) * 5 + q]: 256
// threads over the blocks, then a fixed tree per output
__global__ void __launch_bounds__(256) stats_final_kernel(const double* __restrict__ partial, int nblk,
                                                          double* __restrict__ out)
{
    __shared__ double sh[256];
    for (int k = 0; k < 40; ++k) {
        const int q = k / 8, f = k % 8;
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) acc += partial[((size_t)b * 8 + f) * 5 + q];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = sh[0];
        __syncthreads();
    }
}

hipError_t launch_stats(const float* u, const float* t, const int n[3], double* partial, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(stats_partial_kernel, dim3(STATS_BLOCKS, 8), dim3(256), 0, s, u, t, n[0], n[1], n[2], partial);
    hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(256), 0, s, partial, STATS_BLOCKS, out);
    return hipGetLastError();
}

// Roughness gate: g0(c) = (1/8) sum_f inv_R[f] * sum over axes
// |u_f(c+a) - 2 u_f(c) + u_f(c-a)| (u field-major FP32).  A thread takes 4
// consecutive x cells (nx is a multiple of 4): one 16-byte load per field
// for the cells and for each y / z neighbour row, two scalars for x.
__global__ void __launch_bounds__(256) gate_rough_kernel(const float* __restrict__ u, int nx, int ny, int nz,
                                                         GateScales gs, float* __restrict__ g0)
{
    const unsigned N = (unsigned)nx * ny * nz, N4 = N / 4;
    for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < N4; t += gridDim.x * blockDim.x) {
        const unsigned c = 4 * t;
        int i, j, k;
        cell_ijk(c, nx, ny, i, j, k);
        const unsigned row = c - i;
        const unsigned cyp = (unsigned)i + (unsigned)nx * ((unsigned)wrap1(j + 1, ny) + (unsigned)ny * k);
        const unsigned cym = (unsigned)i + (unsigned)nx * ((unsigned)wrap1(j - 1, ny) + (unsigned)ny * k);
        const unsigned czp = (unsigned)i + (unsigned)nx * ((unsigned)j + (unsigned)ny * wrap1(k + 1, nz));
        const unsigned czm = (unsigned)i + (unsigned)nx * ((unsigned)j + (unsigned)ny * wrap1(k - 1, nz));
        const unsigned xm = row + wrap1(i - 1, nx), xp = row + wrap1(i + 4, nx);
        float acc[4] = { 0.f, 0.f, 0.f, 0.f };
        for (int f = 0; f < 8; ++f) {
            const float* uf = u + (size_t)f * N;
            const float4 v = *reinterpret_cast<const float4*>(uf + c);
            const float4 vyp = *reinterpret_cast<const float4*>(uf + cyp);
            const float4 vym = *reinterpret_cast<const float4*>(uf + cym);
            const float4 vzp = *reinterpret_cast<const float4*>(uf + czp);
            const float4 vzm = *reinterpret_cast<const float4*>(uf + czm);
            const float a[6] = { uf[xm], v.x, v.y, v.z, v.w, uf[xp] };
            const float yp[4] = { vyp.x, vyp.y, vyp.z, vyp.w }, ym[4] = { vym.x, vym.y, vym.z, vym.w };
            const float zp[4] = { vzp.x, vzp.y, vzp.z, vzp.w }, zm[4] = { vzm.x, vzm.y, vzm.z, vzm.w };
            const float w = gs.inv_r[f];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float x2 = 2.0f * a[q + 1];
                const float r = fabsf((a[q + 2] - x2) + a[q]) + fabsf((yp[q] - x2) + ym[q]) + fabsf((zp[q] - x2) + zm[q]);
                acc[q] += r * w;
            }
        }
        *reinterpret_cast<float4*>(g0 + c) = make_float4(0.125f * acc[0], 0.125f * acc[1], 0.125f * acc[2], 0.125f * acc[3]);
    }
}

// g(c) = max of g0 over c and its six face neighbours
__global__ void __launch_bounds__(256) gate_max_kernel(const float* __restrict__ g0, int nx, int ny, int nz,
                                                       float* __restrict__ g)
{
    const size_t N = (size_t)nx * ny * nz;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_ijk((unsigned)c, nx, ny, i, j, k);
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
