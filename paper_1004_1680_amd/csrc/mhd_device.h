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

// Flux of equations (1)-(3) along the sweep axis with b frozen:
// (m_n, m_n v_n + P* - Bn^2, m_t1 v_n - Bn Bt1, m_t2 v_n - Bn Bt2,
//  (e + P*) v_n - Bn (B.v)), P* = p + b^2/2 (section II.A).
template <typename T>
__device__ __forceinline__ void fluid_flux(const T u[5], const T bb[3], T gamma, T f[5])
{
    const T rho = u[0], mn = u[1], mt1 = u[2], mt2 = u[3], e = u[4];
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

// Relaxed split of the flux into right- and left-moving parts with the
// relaxation speed c (Jin & Xin relaxation, section II.B):
// F^R = (c u + F)/2, F^L = (c u - F)/2.
template <typename T>
__device__ __forceinline__ void relax_split(const T u[5], const T bb[3], T gamma, T c,
                                            T fr[5], T fl[5])
{
    T f[5];
    fluid_flux(u, bb, gamma, f);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        fr[q] = T(0.5) * (c * u[q] + f[q]);
        fl[q] = T(0.5) * (c * u[q] - f[q]);
    }
}

// van Leer limiter (section II.B): 2ab/(a+b) if ab > 0, else 0.
template <typename T>
__device__ __forceinline__ T van_leer(T a, T b)
{
    const T ab = a * b;
    return ab > T(0) ? T(2) * ab / (a + b) : T(0);
}

// Second-order right-moving part at interface i+1/2 from F^R at i-1, i, i+1.
template <typename T>
__device__ __forceinline__ T limited_right(T rm, T r0, T rp)
{
    return r0 + van_leer(T(0.5) * (r0 - rm), T(0.5) * (rp - r0));
}

// Second-order left-moving part at interface i+1/2 from F^L at i, i+1, i+2.
template <typename T>
__device__ __forceinline__ T limited_left(T l0, T lp, T lpp)
{
    return lp + van_leer(T(0.5) * (l0 - lp), T(0.5) * (lp - lpp));
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
template <typename T>
__device__ __forceinline__ T upwind_flux2(T a, T qm, T q0, T q1, T q2)
{
    if (a > T(0))
        return a * (q0 + van_leer(T(0.5) * (q0 - qm), T(0.5) * (q1 - q0)));
    if (a < T(0))
        return a * (q1 + van_leer(T(0.5) * (q1 - q2), T(0.5) * (q0 - q1)));
    return T(0);
}

// Index helpers for a periodic [nz][ny][nx] grid.
__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

}  // namespace mhd
