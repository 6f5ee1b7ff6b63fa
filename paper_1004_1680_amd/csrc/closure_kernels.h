// Learned-closure kernels: BF16 MFMA convolutions and helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mhd {

enum {
    EPI_BIAS_RELU = 0,   // y = relu(acc + bias) -> bf16 (+ channel-major copy)
    EPI_BIAS_F32 = 1,    // y = acc + bias -> fp32
    EPI_MASK = 2,        // y = acc * (mask > 0) -> bf16 (+ channel-major copy)
    EPI_F32 = 3          // y = acc -> fp32
};

struct ConvArgs {
    int n[3];
    const uint16_t* x;      // bf16 [cell][cin]
    const uint16_t* wp;     // packed weights
    const float* bias;      // [cout] (bias epilogues)
    const uint16_t* mask;   // bf16 [cell][cout] (EPI_MASK)
    float* yf;              // fp32 [cell][cout]
    uint16_t* yb;           // bf16 [cell][cout]
    uint16_t* ybT;          // bf16 [cout][cell] or null
};

struct WgradArgs {
    int n[3];
    const uint16_t* xT;     // bf16 [cin][cell]
    const uint16_t* dyT;    // bf16 [cout][cell]
    float* partial;         // [workgroups + 16][27][cin][cout] (partial sums, then the reduction's)
    int tiles_per_wg;
};
constexpr int WGRAD_MAX_WG = 512;   // persistent workgroups of wgrad (bounds the partial sums)

// packed size (bf16 elements) of a layer's weights
inline size_t packed_weight_elems(int cin, int cout)
{
    return (size_t)((27 * cin + 31) / 32) * ((cout + 15) / 16) * 64 * 8;
}

hipError_t launch_pack_weights(const float* w, int cin, int cout, int flip, uint16_t* wp, hipStream_t s);
hipError_t launch_conv3d(const ConvArgs& A, int cin, int cout, int epi, hipStream_t s);
int wgrad_blocks(const int n[3], int& tiles_per_wg);   // workgroups of a wgrad launch
hipError_t launch_conv3d_wgrad(const WgradArgs& A, int cin, int cout, float* dw, hipStream_t s);
constexpr int BG_BLOCKS = 64;      // partial sums per channel of the bias gradient (needs BG_BLOCKS * cout doubles)
hipError_t launch_bias_grad(const uint16_t* dyT, size_t N, int cout, float* dbias, double* partial, hipStream_t s);
hipError_t launch_to_bf16(const float* src, size_t N, int c, uint16_t* dst, uint16_t* dstT, hipStream_t s);

// per-channel input normalisation, output and target scales of the closure
struct ClosureScales {
    float in_mean[8], in_std[8], out_scale[8], target_scale[8];
};
constexpr int CHSUM_BLOCKS = 512;

hipError_t launch_normalize(const float* u, size_t N, const ClosureScales& sc, uint16_t* x, uint16_t* xT, hipStream_t s);
hipError_t launch_chsum(const float* a, size_t N, size_t cstride, size_t fstride, int nch, double scale,
                        double* partial, double* out, hipStream_t s);
hipError_t launch_project(const float* o, const double* mean, const int n[3], const ClosureScales& sc, float* delta,
                          hipStream_t s);
hipError_t launch_project_T(const float* g, const double* gmean, const int n[3], const ClosureScales& sc, float* go,
                            hipStream_t s);
hipError_t launch_loss(const float* delta, const float* target, size_t N, const ClosureScales& sc, float* g,
                       double* partial, double* out, hipStream_t s);
constexpr int GUARD_LEVELS = 4;     // theta = 1, 1/2, 1/4, 1/8
hipError_t launch_guard_levels(const float* u, const float* delta, const int n[3], float gamma, int* bad,
                               hipStream_t s);
hipError_t launch_apply_level(float* u, const float* delta, size_t n, const int* bad, int* counts, hipStream_t s);
hipError_t launch_zero_int(int* p, hipStream_t s);
constexpr int STATS_BLOCKS = 256;
hipError_t launch_residual(const float* ref, const float* plain, size_t n, float* out, hipStream_t s);
hipError_t launch_stats(const float* u, const float* t, const int n[3], double* partial, double* out, hipStream_t s);
struct GateScales {
    float inv_r[8];     // 1 / (training-set mean roughness) per field
};
hipError_t launch_gate(const float* u, const int n[3], const GateScales& gs, float* g0, float* g, hipStream_t s);
hipError_t launch_row_scale(float* a, const float* g, size_t N, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);

}  // namespace mhd
