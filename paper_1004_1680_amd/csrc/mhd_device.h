// Device arithmetic of the MHD update step (Pang, Pen & Perrone,
// arXiv:1004.1680, section II), shared by all sweep kernels so that the x,
// y and z sweeps evaluate every formula with the same expression tree (the
// scheme is then exactly symmetric under a cyclic relabelling of the axes).
//
// Conventions:
//  * sweep-local axes (n, t1, t2) = (d, d+1, d+2) taken cyclically;
//  * u = (rho, m_n, m_t1, m_t2, e), bb = cell-centred field (Bbar_n, Bbar_t1,
//    Bbar_t2), Bbar_d = (b_d[c] + b_d[c+d]) / 2;
//  * every product and sum is rounded as written (built with
//    -ffp-contract=off; no fused multiply-add is formed).
#pragma once
#include <hip/hip_runtime.h>

namespace mhd {

enum { RHO = 0, MX = 1, MY = 2, MZ = 3, EN = 4, BX = 5, BY = 6, BZ = 7 };
constexpr int NFIELD = 8;

// Division policy of the two precision tiers.  FP64 divides with IEEE
// rounding everywhere (the same rounding as a plain evaluation of each
// formula).  FP32 multiplies by the hardware reciprocal (v_rcp_f32, within
// 1 ulp), and takes one reciprocal of rho per cell: an FP32 IEEE division is
// a ~10-instruction sequence and the sweeps would otherwise spend most of
// their instructions on the 18 divisions per cell.
template <typename T> struct Arith;
template <> struct Arith<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float by_rho(float m, float rho, float inv) { return m * inv; }
};
template <> struct Arith<double> {
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double by_rho(double m, double rho, double) { return m / rho; }
};

// u - s d and u + s d: plain in FP64; one fused multiply-add in FP32.
template <typename T>
__device__ __forceinline__ T sub_scaled(T u, T s, T d)
{
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(-s, d, u);
    else return u - s * d;
}
template <typename T>
__device__ __forceinline__ T add_scaled(T u, T s, T d)
{
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(s, d, u);
    else return u + s * d;
}

// Flux of equations (1)-(3) along the sweep axis with b frozen:
// (m_n, m_n v_n + P* - Bn^2, m_t1 v_n - Bn Bt1, m_t2 v_n - Bn Bt2,
//  (e + P*) v_n - Bn (B.v)), P* = p + b^2/2 (section II.A).
template <typename T>
__device__ __forceinline__ void fluid_flux(const T u[5], const T bb[3], T gamma, T f[5])
{
    const T rho = u[0], mn = u[1], mt1 = u[2], mt2 = u[3], e = u[4];
    if constexpr (sizeof(T) == 4) {
        // FP32: one reciprocal of rho; sums of products as fused multiply-adds
        const float inv = Arith<float>::rcp(rho);
        const float vn = mn * inv, vt1 = mt1 * inv, vt2 = mt2 * inv;
        const float b2 = __builtin_fmaf(bb[2], bb[2], __builtin_fmaf(bb[1], bb[1], bb[0] * bb[0]));
        const float ke = 0.5f * __builtin_fmaf(mt2, vt2, __builtin_fmaf(mt1, vt1, mn * vn));
        const float p = (gamma - 1.0f) * (e - ke - 0.5f * b2);
        const float ptot = __builtin_fmaf(0.5f, b2, p);
        const float bv = __builtin_fmaf(bb[2], vt2, __builtin_fmaf(bb[1], vt1, bb[0] * vn));
        f[0] = mn;
        f[1] = __builtin_fmaf(mn, vn, ptot) - bb[0] * bb[0];
        f[2] = __builtin_fmaf(mt1, vn, -bb[0] * bb[1]);
        f[3] = __builtin_fmaf(mt2, vn, -bb[0] * bb[2]);
        f[4] = __builtin_fmaf(e + ptot, vn, -bb[0] * bv);
    } else {
        const T vn = mn / rho;
        const T vt1 = mt1 / rho;
        const T vt2 = mt2 / rho;
        const T b2 = bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2];
        const T mm = mn * mn + mt1 * mt1 + mt2 * mt2;
        const T p = (gamma - T(1)) * (e - T(0.5) * mm / rho - T(0.5) * b2);
        const T ptot = p + T(0.5) * b2;
        const T bv = bb[0] * vn + bb[1] * vt1 + bb[2] * vt2;
        f[0] = mn;
        f[1] = mn * vn + ptot - bb[0] * bb[0];
        f[2] = mt1 * vn - bb[0] * bb[1];
        f[3] = mt2 * vn - bb[0] * bb[2];
        f[4] = (e + ptot) * vn - bb[0] * bv;
    }
}

// Relaxed split of the flux into right- and left-moving parts with the
// relaxation speed c (Jin & Xin relaxation, section II.B):
// F^R = (c u + F)/2, F^L = (c u - F)/2.
// The FP32 tier folds the factor 1/2 into c and F (exact scalings) so that
// each part is one fused multiply-add.
template <typename T>
__device__ __forceinline__ void relax_split(const T u[5], const T bb[3], T gamma, T c,
                                            T fr[5], T fl[5])
{
    T f[5];
    fluid_flux(u, bb, gamma, f);
    if constexpr (sizeof(T) == 4) {
        const T hc = T(0.5) * c;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const T hf = T(0.5) * f[q];
            fr[q] = __builtin_fmaf(hc, u[q], hf);
            fl[q] = __builtin_fmaf(hc, u[q], -hf);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            fr[q] = T(0.5) * (c * u[q] + f[q]);
            fl[q] = T(0.5) * (c * u[q] - f[q]);
        }
    }
}

// Freezing (relaxation) speed of the fluid operator.  The method's reading
// is one number per step (the CFL speed, FRZ_STEP); two variants take it
// from the state of each stage: FRZ_CELL uses |v_n| + c_fast of each cell,
// FRZ_PENCIL the largest such value along the pencil (section II.B asks
// only that it exceed the characteristic speeds of the flux).
enum { FRZ_STEP = 0, FRZ_CELL = 1, FRZ_PENCIL = 2 };

// |v_n| + sqrt((gamma p + |Bbar|^2)/rho) of one cell with the pressure of
// fluid_flux (the variants' freezing speed).  FP64: every operation as
// written, IEEE division and square root; FP32: one reciprocal of rho.
template <typename T>
__device__ __forceinline__ T normal_speed(const T u[5], const T bb[3], T gamma)
{
    const T rho = u[0], mn = u[1], mt1 = u[2], mt2 = u[3], e = u[4];
    if constexpr (sizeof(T) == 4) {
        const float inv = Arith<float>::rcp(rho);
        const float vn = mn * inv, vt1 = mt1 * inv, vt2 = mt2 * inv;
        const float b2 = __builtin_fmaf(bb[2], bb[2], __builtin_fmaf(bb[1], bb[1], bb[0] * bb[0]));
        const float ke = 0.5f * __builtin_fmaf(mt2, vt2, __builtin_fmaf(mt1, vt1, mn * vn));
        const float p = (gamma - 1.0f) * (e - ke - 0.5f * b2);
        return fabsf(vn) + sqrtf(__builtin_fmaf(gamma, p, b2) * inv);
    } else {
        const T vn = mn / rho;
        const T b2 = bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2];
        const T mm = mn * mn + mt1 * mt1 + mt2 * mt2;
        const T p = (gamma - T(1)) * (e - T(0.5) * mm / rho - T(0.5) * b2);
        return fabs(vn) + sqrt((gamma * p + b2) / rho);
    }
}

// van Leer limiter (section II.B): 2ab/(a+b) if ab > 0, else 0.
template <typename T>
__device__ __forceinline__ T van_leer(T a, T b)
{
    const T ab = a * b;
    return ab > T(0) ? Arith<T>::div(T(2) * ab, a + b) : T(0);
}

// velocity m / rho
template <typename T>
__device__ __forceinline__ T velocity(T m, T rho)
{
    return Arith<T>::div(m, rho);
}

// van Leer correction from two one-sided differences d1, d2 (not halved):
// vl(d1/2, d2/2) = d1 d2 / (d1 + d2) when d1 d2 > 0.  The FP32 tier uses
// this reduced form (3 fewer multiplications); the FP64 tier keeps the
// halved differences of the plain formula.
template <typename T>
__device__ __forceinline__ T vl_half(T d1, T d2)
{
    if constexpr (sizeof(T) == 4) {
        const T p = d1 * d2;
        return p > T(0) ? p * Arith<T>::rcp(d1 + d2) : T(0);
    } else {
        return van_leer(T(0.5) * d1, T(0.5) * d2);
    }
}

// x + vl_half(d1, d2), the correction added in one fused operation in FP32
template <typename T>
__device__ __forceinline__ T plus_vl_half(T x, T d1, T d2)
{
    if constexpr (sizeof(T) == 4) {
        const T p = d1 * d2;
        return p > T(0) ? __builtin_fmaf(p, Arith<T>::rcp(d1 + d2), x) : x;
    } else {
        return x + van_leer(T(0.5) * d1, T(0.5) * d2);
    }
}

// Other slope limiters, a method variant (the paper uses van Leer's): with
// a, b the halved one-sided differences and a b > 0, sign(a) times
//   minmod:   min(|a|, |b|)
//   MC:       min(2|a|, 2|b|, |a + b| / 2)   (monotonised central)
//   superbee: max(min(2|a|, |b|), min(|a|, 2|b|))
// and 0 otherwise.  Every step but the final sum is exact, in either tier.
enum { LIM_VANLEER = 0, LIM_MINMOD = 1, LIM_MC = 2, LIM_SUPERBEE = 3 };

template <typename T, int LIM>
__device__ __forceinline__ T slope_limiter(T a, T b)
{
    if (!(a * b > T(0))) return T(0);
    const T fa = fabs(a), fb = fabs(b);
    T m;
    if constexpr (LIM == LIM_MINMOD) m = fmin(fa, fb);
    else if constexpr (LIM == LIM_MC) m = fmin(fmin(T(2) * fa, T(2) * fb), T(0.5) * fabs(a + b));
    else m = fmax(fmin(T(2) * fa, fb), fmin(fa, T(2) * fb));
    return copysign(m, a);
}

// x + phi(d1/2, d2/2) with the limiter LIM
template <typename T, int LIM>
__device__ __forceinline__ T plus_limited_half(T x, T d1, T d2)
{
    if constexpr (LIM == LIM_VANLEER) return plus_vl_half(x, d1, d2);
    else return x + slope_limiter<T, LIM>(T(0.5) * d1, T(0.5) * d2);
}

// Second-order right-moving part at interface i+1/2 from F^R at i-1, i, i+1.
template <typename T, int LIM = LIM_VANLEER>
__device__ __forceinline__ T limited_right(T rm, T r0, T rp)
{
    return plus_limited_half<T, LIM>(r0, r0 - rm, rp - r0);
}

// Second-order left-moving part at interface i+1/2 from F^L at i, i+1, i+2.
template <typename T, int LIM = LIM_VANLEER>
__device__ __forceinline__ T limited_left(T l0, T lp, T lpp)
{
    return plus_limited_half<T, LIM>(lp, l0 - lp, lp - lpp);
}

// Constrained transport (section II.B): edge velocity of v_d on the edge at
// c + d/2 - e/2 from the face averages w(c) = (v(c) + v(c-e))/2 and
// w(c+d); first-order upwind edge flux of q = b_e; second-order upwind edge
// flux of the half-step q with the van Leer limiter.
template <typename T>
__device__ __forceinline__ T face_avg(T v, T v_minus_e) { return T(0.5) * (v + v_minus_e); }

template <typename T>
__device__ __forceinline__ T edge_avg(T w, T w_plus_d) { return T(0.5) * (w + w_plus_d); }

template <typename T>
__device__ __forceinline__ T upwind_flux1(T a, T q0, T q1)
{
    return a > T(0) ? a * q0 : a * q1;
}

// qm = q(c-d), q0 = q(c), q1 = q(c+d), q2 = q(c+2d) of the half-step field.
// Upwind cell c (a > 0): q0 + vl(q0 - qm, q1 - q0); upwind cell c+d
// (a < 0): q1 + vl(q1 - q2, q0 - q1); times a.  The operands are selected
// first (no divergent branch); a = 0 gives a signed zero.
template <typename T, int LIM = LIM_VANLEER>
__device__ __forceinline__ T upwind_flux2(T a, T qm, T q0, T q1, T q2)
{
    const bool right = a > T(0);
    const T up = right ? q0 : q1;
    const T d1 = right ? q0 - qm : q1 - q2;
    const T d2 = right ? q1 - q0 : q0 - q1;
    return a * plus_limited_half<T, LIM>(up, d1, d2);
}

// Index helpers for a periodic [nz][ny][nx] grid.
__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Signal speed max_d |v_d| + sqrt((gamma p + |Bbar|^2) / rho) of one cell in
// FP64 (the CFL condition, section II.B), the cell-centred field the mean of
// the two faces of each axis (b*0: own low face, b*1: the next cell's).
// Folds it into vmax, or raises bad for rho <= 0, p < 0 or a non-finite
// value.  The CFL reduction and the fused epilogue of the last fluid
// operator both call it, so they find the same maximum bit for bit.
__device__ __forceinline__ void signal_speed64(double rho, double mx, double my, double mz, double e,
                                               double bx0, double bx1, double by0, double by1, double bz0,
                                               double bz1, double gamma, double& vmax, int& bad)
{
    const double bx = 0.5 * (bx0 + bx1);
    const double by = 0.5 * (by0 + by1);
    const double bz = 0.5 * (bz0 + bz1);
    const double b2 = bx * bx + by * by + bz * bz;
    const double mm = mx * mx + my * my + mz * mz;
    const double p = (gamma - 1.0) * (e - 0.5 * mm / rho - 0.5 * b2);
    // max_d |m_d / rho| as one division: for rho > 0 a correctly rounded
    // division is odd and monotonic in the numerator, so this is the same
    // value as the largest of the three quotients (rho <= 0 is flagged)
    const double ax = fabs(mx), ay = fabs(my), az = fabs(mz);
    double am = ax > ay ? ax : ay;
    am = am > az ? am : az;
    const double vm = am / rho;
    const double sp = vm + sqrt((gamma * p + b2) / rho);
    if (!(rho > 0.0) || !(p >= 0.0) || !isfinite(sp) || !isfinite(e) || !isfinite(mm) || !isfinite(b2))
        bad = 1;
    else if (sp > vmax)
        vmax = sp;
}

// FP32 screen of one cell for the fused CFL of the FP32 tier: bounds
// lb <= speed <= ub of the FP64 signal speed that signal_speed64 finds for
// the same (float) inputs, and whether the cell is surely physical there
// (rho > 0, p > 0, everything finite; the bounds are meaningful only then).
// Margins: the pressure of the cell may differ from its FP64 value by
// dp = 1e-4 (gamma - 1)(|e| + m^2/(2 rho) + |B|^2/2), about 100 times what
// the FP32 rounding of this expression can do (a few units of 2^-24 of the
// largest term it cancels), and the other factors by 1e-5 relative (each
// FP32 operation, the hardware reciprocal and square root included, is
// within 2^-23; square roots of arguments below 2^-96 are not taken, the
// bounds use 2^-48 above and 0 below instead).  A
// cell that is surely physical and whose upper bound is below a speed
// already found, or below the lower bound of another such cell, cannot be
// the maximum.  A non-finite e, m^2 or |B|^2 makes p > dp fail (an infinite
// or undefined p or dp), so the test p > dp with a finite ub covers every
// way signal_speed64 can flag the cell.  The upper bound and the two terms
// of the lower one (am = max |m_d| / rho, xl = the lower speed^2 bound) come
// from screen_upper32; screen_lower32 finishes the lower bound, which is
// needed for one cell per lane only.
__device__ __forceinline__ float sqrt_above32(float y)
{
    return y < 0x1p-96f ? 0x1p-48f : __builtin_amdgcn_sqrtf(y);
}
__device__ __forceinline__ float sqrt_below32(float y)
{
    return y < 0x1p-96f ? 0.0f : __builtin_amdgcn_sqrtf(y);
}

__device__ __forceinline__ void screen_upper32(float rho, float mx, float my, float mz, float e,
                                               float bx0, float bx1, float by0, float by1, float bz0,
                                               float bz1, float gamma, float& ub, float& am, float& xl,
                                               bool& sure)
{
    const float bx = 0.5f * (bx0 + bx1);
    const float by = 0.5f * (by0 + by1);
    const float bz = 0.5f * (bz0 + bz1);
    const float b2 = bx * bx + by * by + bz * bz;
    const float mm = mx * mx + my * my + mz * mz;
    const float inv = __builtin_amdgcn_rcpf(rho);
    const float ke = 0.5f * mm * inv, me = 0.5f * b2;
    const float p = (gamma - 1.0f) * (e - ke - me);
    const float dp = 1e-4f * (gamma - 1.0f) * (fabsf(e) + ke + me);
    am = fmaxf(fabsf(mx), fmaxf(fabsf(my), fabsf(mz))) * inv;
    // p > dp for a surely physical cell: no clamping at zero needed
    const float x = gamma * (p + dp) + b2;
    xl = (gamma * (p - dp) + b2) * inv;
    ub = (am + sqrt_above32(x * inv)) * 1.00001f;
    sure = rho > 0.0f && p > dp && isfinite(ub);
}

__device__ __forceinline__ float screen_lower32(float am, float xl)
{
    return (am + sqrt_below32(xl)) * 0.99999f;
}

}  // namespace mhd
