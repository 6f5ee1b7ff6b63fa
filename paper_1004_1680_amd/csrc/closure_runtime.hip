// Learned closure of a coarse grid (C ABI part of mhd.h): a 3-layer
// periodic 3x3x3 conv net, 8 -> 32 -> 32 -> 8 channels, BF16 weights and
// activations with FP32 accumulation on MFMA, predicts the correction that
// takes one plain coarse step toward the restricted fine solution.  The
// output is projected so that the correction changes no conserved total and
// no cell's div b (mean-free fluid corrections, discrete curl of an edge
// potential); a correction that would leave the physical range is scaled
// by the largest of 1, 1/2, 1/4, 1/8 that keeps every cell physical, or
// dropped (the plain step is kept).  Training: MSE loss, backward pass on the same
// MFMA kernels, Adam on FP32 master weights.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <vector>

#include "../../include/mhd.h"
#include "closure_kernels.h"
#include "runtime_common.h"

using namespace mhd;
#define HIP_TRY MHD_HIP_TRY

static const int LCIN[3] = { 8, 32, 32 }, LCOUT[3] = { 32, 32, 8 };
static const size_t NPARAM = 27 * 8 * 32 + 32 + 27 * 32 * 32 + 32 + 27 * 32 * 8 + 8;

static size_t woff(int l)      // offset of layer l's weights in the flat parameter vector
{
    size_t o = 0;
    for (int k = 0; k < l; ++k) o += (size_t)27 * LCIN[k] * LCOUT[k] + LCOUT[k];
    return o;
}
static size_t boff(int l) { return woff(l) + (size_t)27 * LCIN[l] * LCOUT[l]; }

struct mhd_closure {
    int n[3];
    size_t N;
    hipStream_t stream;
    bool failed;
    ClosureScales sc;
    float *params, *grads, *adam_m, *adam_v;
    int adam_step;
    uint16_t* wp[3];       // packed forward weights
    uint16_t* wpT[3];      // packed dgrad weights (layers 2, 3)
    bool packed;
    uint16_t *x0, *x0T, *a1, *a1T, *a2, *a2T, *gob, *gobT, *g2, *g2T, *g1, *g1T;
    float *o, *delta, *g, *go;
    float* wpart;          // wgrad partials
    double *chpart, *chout, *loss, *stpart, *stout;
    bool gate_on;           // roughness gate of the output (mhd_closure_set_gate)
    GateScales gs;
    float *gate0, *gate;
    int *bad, *fallbacks;
    int tiles_per_wg, nwg;
};

static int check_cl(const mhd_closure* c)
{
    if (!c) return mhd_fail(MHD_EINVAL, "null closure handle");
    if (c->failed) return mhd_fail(MHD_ESTATE, "closure handle failed earlier (HIP error)");
    return MHD_OK;
}

extern "C" void mhd_closure_destroy(mhd_closure* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    void* ptrs[] = { c->params, c->grads, c->adam_m, c->adam_v, c->wp[0], c->wp[1], c->wp[2], c->wpT[0],
                     c->wpT[1], c->wpT[2], c->x0, c->x0T, c->a1, c->a1T, c->a2, c->a2T, c->gob, c->gobT,
                     c->g2, c->g2T, c->g1, c->g1T, c->o, c->delta, c->g, c->go, c->wpart,
                     c->chpart, c->chout, c->loss, c->stpart, c->stout, c->bad, c->fallbacks,
                     c->gate0, c->gate };
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete c;
}

extern "C" mhd_closure* mhd_closure_create(int nx, int ny, int nz, void* hip_stream)
{
    if (nx < 32 || ny < 32 || nz < 32 || nx % 32 || ny % 32 || nz % 32 ||
        (long long)nx * ny * nz >= (1LL << 31)) {
        mhd_fail(MHD_EINVAL, "closure grid must have dimensions that are multiples of 32");
        return nullptr;
    }
    mhd_closure* c = new mhd_closure();
    memset(c, 0, sizeof *c);
    c->n[0] = nx; c->n[1] = ny; c->n[2] = nz;
    c->N = (size_t)nx * ny * nz;
    c->stream = (hipStream_t)hip_stream;
    for (int f = 0; f < 8; ++f) {
        c->sc.in_mean[f] = 0.0f; c->sc.in_std[f] = 1.0f;
        c->sc.out_scale[f] = 1.0f; c->sc.target_scale[f] = 1.0f;
    }
    const size_t N = c->N;
    c->nwg = wgrad_blocks(c->n, c->tiles_per_wg);
    bool ok = true;
    auto A = [&](void** p, size_t bytes) { if (ok && hipMalloc(p, bytes) != hipSuccess) ok = false; };
    A((void**)&c->params, NPARAM * 4); A((void**)&c->grads, NPARAM * 4);
    A((void**)&c->adam_m, NPARAM * 4); A((void**)&c->adam_v, NPARAM * 4);
    for (int l = 0; l < 3; ++l) {
        A((void**)&c->wp[l], packed_weight_elems(LCIN[l], LCOUT[l]) * 2);
        A((void**)&c->wpT[l], packed_weight_elems(LCOUT[l], LCIN[l]) * 2);
    }
    A((void**)&c->x0, N * 8 * 2); A((void**)&c->x0T, N * 8 * 2);
    A((void**)&c->a1, N * 32 * 2); A((void**)&c->a1T, N * 32 * 2);
    A((void**)&c->a2, N * 32 * 2); A((void**)&c->a2T, N * 32 * 2);
    A((void**)&c->gob, N * 8 * 2); A((void**)&c->gobT, N * 8 * 2);
    A((void**)&c->g2, N * 32 * 2); A((void**)&c->g2T, N * 32 * 2);
    A((void**)&c->g1, N * 32 * 2); A((void**)&c->g1T, N * 32 * 2);
    A((void**)&c->o, N * 8 * 4); A((void**)&c->delta, N * 8 * 4); A((void**)&c->g, N * 8 * 4);
    A((void**)&c->go, N * 8 * 4);
    A((void**)&c->wpart, (size_t)(c->nwg + 16) * 27 * 32 * 32 * 4);
    A((void**)&c->chpart, (size_t)CHSUM_BLOCKS * 8 * 8); A((void**)&c->chout, 16 * 8);
    A((void**)&c->loss, 8); A((void**)&c->bad, 4); A((void**)&c->fallbacks, 8);
    A((void**)&c->stpart, (size_t)STATS_BLOCKS * 8 * 5 * 8); A((void**)&c->stout, 40 * 8);
    A((void**)&c->gate0, N * 4); A((void**)&c->gate, N * 4);
    if (!ok) {
        (void)hipGetLastError();
        mhd_fail(MHD_ENOMEM, "closure allocation failed");
        mhd_closure_destroy(c);
        return nullptr;
    }
    ok = hipMemset(c->params, 0, NPARAM * 4) == hipSuccess && hipMemset(c->adam_m, 0, NPARAM * 4) == hipSuccess &&
         hipMemset(c->adam_v, 0, NPARAM * 4) == hipSuccess && hipMemset(c->fallbacks, 0, 8) == hipSuccess &&
         hipMemset(c->bad, 0, 4) == hipSuccess;
    if (!ok) {
        mhd_fail(MHD_EDEVICE, "closure initialisation failed");
        mhd_closure_destroy(c);
        return nullptr;
    }
    return c;
}

extern "C" int mhd_closure_set_params(mhd_closure* c, const float* params, size_t n)
{
    int r = check_cl(c);
    if (r) return r;
    if (!params || n != NPARAM) return mhd_fail(MHD_EINVAL, "expected %zu parameters", NPARAM);
    HIP_TRY(c, hipMemcpyAsync(c->params, params, NPARAM * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->adam_m, 0, NPARAM * 4, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->adam_v, 0, NPARAM * 4, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->adam_step = 0;
    c->packed = false;
    return MHD_OK;
}

extern "C" int mhd_closure_get_params(mhd_closure* c, float* params, size_t n)
{
    int r = check_cl(c);
    if (r) return r;
    if (!params || n != NPARAM) return mhd_fail(MHD_EINVAL, "expected %zu parameters", NPARAM);
    HIP_TRY(c, hipMemcpyAsync(params, c->params, NPARAM * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MHD_OK;
}

extern "C" int mhd_closure_set_scales(mhd_closure* c, const float* in_mean, const float* in_std,
                                      const float* out_scale, const float* target_scale)
{
    int r = check_cl(c);
    if (r) return r;
    if (!in_mean || !in_std || !out_scale || !target_scale) return mhd_fail(MHD_EINVAL, "null scales");
    for (int f = 0; f < 8; ++f) {
        if (!(in_std[f] > 0.0f) || !(target_scale[f] > 0.0f))
            return mhd_fail(MHD_EINVAL, "scales must be positive");
        c->sc.in_mean[f] = in_mean[f]; c->sc.in_std[f] = in_std[f];
        c->sc.out_scale[f] = out_scale[f]; c->sc.target_scale[f] = target_scale[f];
    }
    return MHD_OK;
}

extern "C" int mhd_closure_set_gate(mhd_closure* c, const float* mean_roughness)
{
    int r = check_cl(c);
    if (r) return r;
    if (!mean_roughness) {
        c->gate_on = false;
        return MHD_OK;
    }
    for (int f = 0; f < 8; ++f)
        if (!(mean_roughness[f] > 0.0f) || !isfinite(mean_roughness[f]))
            return mhd_fail(MHD_EINVAL, "mean roughness must be positive and finite");
    for (int f = 0; f < 8; ++f) c->gs.inv_r[f] = 1.0f / mean_roughness[f];
    c->gate_on = true;
    return MHD_OK;
}

extern "C" int mhd_closure_get_gate(mhd_closure* c, float* gate_dev)
{
    int r = check_cl(c);
    if (r) return r;
    if (!gate_dev) return mhd_fail(MHD_EINVAL, "null device pointer");
    if (!c->gate_on) return mhd_fail(MHD_ESTATE, "no gate set");
    HIP_TRY(c, hipMemcpyAsync(gate_dev, c->gate, c->N * 4, hipMemcpyDeviceToDevice, c->stream));
    return MHD_OK;
}

static int pack_all(mhd_closure* c)
{
    if (c->packed) return MHD_OK;
    for (int l = 0; l < 3; ++l) {
        HIP_TRY(c, launch_pack_weights(c->params + woff(l), LCIN[l], LCOUT[l], 0, c->wp[l], c->stream));
        if (l > 0)
            HIP_TRY(c, launch_pack_weights(c->params + woff(l), LCOUT[l], LCIN[l], 1, c->wpT[l], c->stream));
    }
    c->packed = true;
    return MHD_OK;
}

// u: FP32 field-major [8][cell] -> delta [8][cell]; with `train` the
// channel-major activation copies that wgrad reads are written too
static int forward(mhd_closure* c, const float* u, bool train)
{
    int r = pack_all(c);
    if (r) return r;
    HIP_TRY(c, launch_normalize(u, c->N, c->sc, c->x0, train ? c->x0T : nullptr, c->stream));
    ConvArgs A;
    memset(&A, 0, sizeof A);
    A.n[0] = c->n[0]; A.n[1] = c->n[1]; A.n[2] = c->n[2];
    A.x = c->x0; A.wp = c->wp[0]; A.bias = c->params + boff(0); A.yb = c->a1; A.ybT = train ? c->a1T : nullptr;
    HIP_TRY(c, launch_conv3d(A, 8, 32, EPI_BIAS_RELU, c->stream));
    A.x = c->a1; A.wp = c->wp[1]; A.bias = c->params + boff(1); A.yb = c->a2; A.ybT = train ? c->a2T : nullptr;
    HIP_TRY(c, launch_conv3d(A, 32, 32, EPI_BIAS_RELU, c->stream));
    A.x = c->a2; A.wp = c->wp[2]; A.bias = c->params + boff(2); A.yb = nullptr; A.ybT = nullptr; A.yf = c->o;
    HIP_TRY(c, launch_conv3d(A, 32, 8, EPI_BIAS_F32, c->stream));
    if (c->gate_on) {
        HIP_TRY(c, launch_gate(u, c->n, c->gs, c->gate0, c->gate, c->stream));
        HIP_TRY(c, launch_row_scale(c->o, c->gate, c->N, c->stream));
    }
    // projection: means of the 5 fluid outputs over the box
    HIP_TRY(c, launch_chsum(c->o, c->N, 8, 1, 5, 1.0 / (double)c->N, c->chpart, c->chout, c->stream));
    HIP_TRY(c, launch_project(c->o, c->chout, c->n, c->sc, c->delta, c->stream));
    return MHD_OK;
}

// loss of the last forward against target, and every parameter gradient
static int backward(mhd_closure* c, const float* target)
{
    const size_t N = c->N;
    HIP_TRY(c, launch_loss(c->delta, target, N, c->sc, c->g, c->chpart, c->loss, c->stream));
    HIP_TRY(c, launch_chsum(c->g, N, 1, N, 5, 1.0 / (double)N, c->chpart, c->chout + 8, c->stream));
    HIP_TRY(c, launch_project_T(c->g, c->chout + 8, c->n, c->sc, c->go, c->stream));
    if (c->gate_on) HIP_TRY(c, launch_row_scale(c->go, c->gate, N, c->stream));
    HIP_TRY(c, launch_to_bf16(c->go, N, 8, c->gob, c->gobT, c->stream));
    WgradArgs W;
    W.n[0] = c->n[0]; W.n[1] = c->n[1]; W.n[2] = c->n[2];
    W.partial = c->wpart;
    W.tiles_per_wg = c->tiles_per_wg;
    // layer 3
    W.xT = c->a2T; W.dyT = c->gobT;
    HIP_TRY(c, launch_conv3d_wgrad(W, 32, 8, c->grads + woff(2), c->stream));
    HIP_TRY(c, launch_bias_grad(c->gobT, N, 8, c->grads + boff(2), c->chpart, c->stream));
    ConvArgs A;
    memset(&A, 0, sizeof A);
    A.n[0] = c->n[0]; A.n[1] = c->n[1]; A.n[2] = c->n[2];
    A.x = c->gob; A.wp = c->wpT[2]; A.mask = c->a2; A.yb = c->g2; A.ybT = c->g2T;
    HIP_TRY(c, launch_conv3d(A, 8, 32, EPI_MASK, c->stream));
    // layer 2
    W.xT = c->a1T; W.dyT = c->g2T;
    HIP_TRY(c, launch_conv3d_wgrad(W, 32, 32, c->grads + woff(1), c->stream));
    HIP_TRY(c, launch_bias_grad(c->g2T, N, 32, c->grads + boff(1), c->chpart, c->stream));
    A.x = c->g2; A.wp = c->wpT[1]; A.mask = c->a1; A.yb = c->g1; A.ybT = c->g1T;
    HIP_TRY(c, launch_conv3d(A, 32, 32, EPI_MASK, c->stream));
    // layer 1
    W.xT = c->x0T; W.dyT = c->g1T;
    HIP_TRY(c, launch_conv3d_wgrad(W, 8, 32, c->grads + woff(0), c->stream));
    HIP_TRY(c, launch_bias_grad(c->g1T, N, 32, c->grads + boff(0), c->chpart, c->stream));
    return MHD_OK;
}

extern "C" int mhd_closure_forward(mhd_closure* c, const float* u_dev, float* delta_dev)
{
    int r = check_cl(c);
    if (r) return r;
    if (!u_dev || !delta_dev) return mhd_fail(MHD_EINVAL, "null device pointer");
    if ((r = forward(c, u_dev, false))) return r;
    HIP_TRY(c, hipMemcpyAsync(delta_dev, c->delta, c->N * 8 * 4, hipMemcpyDeviceToDevice, c->stream));
    return MHD_OK;
}

extern "C" int mhd_closure_grad(mhd_closure* c, const float* u_dev, const float* target_dev, double* loss,
                                float* grad_host, size_t n)
{
    int r = check_cl(c);
    if (r) return r;
    if (!u_dev || !target_dev) return mhd_fail(MHD_EINVAL, "null device pointer");
    if (grad_host && n != NPARAM) return mhd_fail(MHD_EINVAL, "expected %zu gradient entries", NPARAM);
    if ((r = forward(c, u_dev, true))) return r;
    if ((r = backward(c, target_dev))) return r;
    if (loss) HIP_TRY(c, hipMemcpyAsync(loss, c->loss, 8, hipMemcpyDeviceToHost, c->stream));
    if (grad_host) HIP_TRY(c, hipMemcpyAsync(grad_host, c->grads, NPARAM * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MHD_OK;
}

extern "C" int mhd_closure_train_step(mhd_closure* c, const float* u_dev, const float* target_dev, float lr,
                                      double* loss)
{
    int r = check_cl(c);
    if (r) return r;
    if (!u_dev || !target_dev) return mhd_fail(MHD_EINVAL, "null device pointer");
    if (!(lr > 0.0f)) return mhd_fail(MHD_EINVAL, "learning rate must be > 0");
    if ((r = forward(c, u_dev, true))) return r;
    if ((r = backward(c, target_dev))) return r;
    c->adam_step += 1;
    HIP_TRY(c, launch_adam(c->params, c->grads, c->adam_m, c->adam_v, (int)NPARAM, lr, 0.9f, 0.999f, 1e-8f,
                           c->adam_step, c->stream));
    c->packed = false;
    if (loss) {
        HIP_TRY(c, hipMemcpyAsync(loss, c->loss, 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return MHD_OK;
}

extern "C" int mhd_closure_step(mhd_closure* c, mhd_ctx* coarse, double cfl)
{
    int r = check_cl(c);
    if (r) return r;
    if (!coarse) return mhd_fail(MHD_EINVAL, "null coarse handle");
    int n[3];
    mhd_internal_dims(coarse, n);
    if (n[0] != c->n[0] || n[1] != c->n[1] || n[2] != c->n[2])
        return mhd_fail(MHD_EINVAL, "coarse grid and closure grid differ");
    if (mhd_internal_prec(coarse) != MHD_F32) return mhd_fail(MHD_EINVAL, "the closure runs on an FP32 handle");
    if (mhd_internal_stream(coarse) != c->stream)
        return mhd_fail(MHD_EINVAL, "closure and coarse handle must share a stream");
    if ((r = mhd_step_auto(coarse, cfl))) return r;
    if ((r = mhd_internal_gather_first(coarse))) return r;
    int all0 = 0;
    float* u = (float*)mhd_internal_state(coarse, &all0);
    if (!all0) return mhd_fail(MHD_ESTATE, "coarse state not in its first buffer");
    if ((r = forward(c, u, false))) return r;
    HIP_TRY(c, launch_zero_int(c->bad, c->stream));
    HIP_TRY(c, launch_guard_levels(u, c->delta, c->n, (float)mhd_internal_gamma(coarse), c->bad, c->stream));
    HIP_TRY(c, launch_apply_level(u, c->delta, c->N * 8, c->bad, c->fallbacks, c->stream));
    mhd_internal_state_changed(coarse);   // the fused CFL of the plain step no longer applies
    return MHD_OK;
}

extern "C" int mhd_closure_residual(mhd_closure* c, const float* u_ref_dev, const float* u_plain_dev,
                                    float* target_dev)
{
    int r = check_cl(c);
    if (r) return r;
    if (!u_ref_dev || !u_plain_dev || !target_dev) return mhd_fail(MHD_EINVAL, "null device pointer");
    HIP_TRY(c, launch_residual(u_ref_dev, u_plain_dev, c->N * 8, target_dev, c->stream));
    return MHD_OK;
}

extern "C" int mhd_closure_stats(mhd_closure* c, const float* u_dev, const float* target_dev, double* out)
{
    int r = check_cl(c);
    if (r) return r;
    if (!u_dev || !target_dev || !out) return mhd_fail(MHD_EINVAL, "null pointer");
    HIP_TRY(c, launch_stats(u_dev, target_dev, c->n, c->stpart, c->stout, c->stream));
    HIP_TRY(c, hipMemcpyAsync(out, c->stout, 40 * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MHD_OK;
}

extern "C" int mhd_closure_fallbacks(mhd_closure* c, int* count)
{
    int r = check_cl(c);
    if (r) return r;
    if (!count) return mhd_fail(MHD_EINVAL, "null output");
    HIP_TRY(c, hipMemcpyAsync(count, c->fallbacks, 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MHD_OK;
}

extern "C" int mhd_closure_reduced(mhd_closure* c, int* count)
{
    int r = check_cl(c);
    if (r) return r;
    if (!count) return mhd_fail(MHD_EINVAL, "null output");
    HIP_TRY(c, hipMemcpyAsync(count, c->fallbacks + 1, 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MHD_OK;
}

// ---------------------------------------------------------------------------
// single layers (parity tests of the MFMA kernels)
// ---------------------------------------------------------------------------

struct scratch_ctx { bool failed; };

static int layer_shape_ok(const int* n, int cin, int cout)
{
    if (!n || n[0] % 32 || n[1] % 32 || n[2] % 32 || n[0] < 32 || n[1] < 32 || n[2] < 32)
        return mhd_fail(MHD_EINVAL, "grid dimensions must be multiples of 32");
    if (!((cin == 8 && cout == 32) || (cin == 32 && cout == 32) || (cin == 32 && cout == 8) || (cin == 8 && cout == 8)))
        return mhd_fail(MHD_EINVAL, "channel pair %d -> %d not supported", cin, cout);
    return MHD_OK;
}

extern "C" int mhd_conv3d_forward(const int* n, int cin, int cout, const void* x, const float* w_host,
                                  const float* bias_host, float* y, void* stream)
{
    int r = layer_shape_ok(n, cin, cout);
    if (r) return r;
    if (!x || !w_host || !y) return mhd_fail(MHD_EINVAL, "null pointer");
    scratch_ctx h{ false };
    hipStream_t s = (hipStream_t)stream;
    float *w = nullptr, *b = nullptr;
    uint16_t* wp = nullptr;
    const size_t nw = (size_t)27 * cin * cout;
    HIP_TRY(&h, hipMalloc(&w, nw * 4));
    HIP_TRY(&h, hipMalloc(&b, cout * 4));
    HIP_TRY(&h, hipMalloc(&wp, packed_weight_elems(cin, cout) * 2));
    HIP_TRY(&h, hipMemcpyAsync(w, w_host, nw * 4, hipMemcpyHostToDevice, s));
    std::vector<float> zb(cout, 0.0f);
    HIP_TRY(&h, hipMemcpyAsync(b, bias_host ? bias_host : zb.data(), cout * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(&h, launch_pack_weights(w, cin, cout, 0, wp, s));
    ConvArgs A;
    memset(&A, 0, sizeof A);
    A.n[0] = n[0]; A.n[1] = n[1]; A.n[2] = n[2];
    A.x = (const uint16_t*)x; A.wp = wp; A.bias = b; A.yf = y;
    HIP_TRY(&h, launch_conv3d(A, cin, cout, EPI_BIAS_F32, s));
    HIP_TRY(&h, hipStreamSynchronize(s));
    (void)hipFree(w); (void)hipFree(b); (void)hipFree(wp);
    return MHD_OK;
}

extern "C" int mhd_conv3d_dgrad(const int* n, int cin, int cout, const void* dy, const float* w_host, float* dx,
                                void* stream)
{
    int r = layer_shape_ok(n, cin, cout);
    if (r) return r;
    if (!dy || !w_host || !dx) return mhd_fail(MHD_EINVAL, "null pointer");
    scratch_ctx h{ false };
    hipStream_t s = (hipStream_t)stream;
    float* w = nullptr;
    uint16_t* wp = nullptr;
    const size_t nw = (size_t)27 * cin * cout;
    HIP_TRY(&h, hipMalloc(&w, nw * 4));
    HIP_TRY(&h, hipMalloc(&wp, packed_weight_elems(cout, cin) * 2));
    HIP_TRY(&h, hipMemcpyAsync(w, w_host, nw * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(&h, launch_pack_weights(w, cout, cin, 1, wp, s));
    ConvArgs A;
    memset(&A, 0, sizeof A);
    A.n[0] = n[0]; A.n[1] = n[1]; A.n[2] = n[2];
    A.x = (const uint16_t*)dy; A.wp = wp; A.yf = dx;
    HIP_TRY(&h, launch_conv3d(A, cout, cin, EPI_F32, s));
    HIP_TRY(&h, hipStreamSynchronize(s));
    (void)hipFree(w); (void)hipFree(wp);
    return MHD_OK;
}

extern "C" int mhd_conv3d_wgrad(const int* n, int cin, int cout, const void* xT, const void* dyT, float* dw_host,
                                float* dbias_host, void* stream)
{
    int r = layer_shape_ok(n, cin, cout);
    if (r) return r;
    if (!xT || !dyT || !dw_host) return mhd_fail(MHD_EINVAL, "null pointer");
    scratch_ctx h{ false };
    hipStream_t s = (hipStream_t)stream;
    WgradArgs W;
    W.n[0] = n[0]; W.n[1] = n[1]; W.n[2] = n[2];
    W.xT = (const uint16_t*)xT; W.dyT = (const uint16_t*)dyT;
    const int nwg = wgrad_blocks(W.n, W.tiles_per_wg);
    float *part = nullptr, *dw = nullptr, *db = nullptr;
    const size_t nw = (size_t)27 * cin * cout;
    HIP_TRY(&h, hipMalloc(&part, (size_t)(nwg + 16) * nw * 4));
    HIP_TRY(&h, hipMalloc(&dw, nw * 4));
    HIP_TRY(&h, hipMalloc(&db, cout * 4));
    W.partial = part;
    HIP_TRY(&h, launch_conv3d_wgrad(W, cin, cout, dw, s));
    // the wgrad partials are consumed by then (same stream): reuse them
    HIP_TRY(&h, launch_bias_grad((const uint16_t*)dyT, (size_t)n[0] * n[1] * n[2], cout, db, (double*)part, s));
    HIP_TRY(&h, hipMemcpyAsync(dw_host, dw, nw * 4, hipMemcpyDeviceToHost, s));
    if (dbias_host) HIP_TRY(&h, hipMemcpyAsync(dbias_host, db, cout * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(&h, hipStreamSynchronize(s));
    (void)hipFree(part); (void)hipFree(dw); (void)hipFree(db);
    return MHD_OK;
}
