/*
 * FP64 CPU oracle for the ideal-MHD update step of Pang, Pen & Perrone,
 * "Magnetohydrodynamics on Heterogeneous architectures: a performance
 * comparison" (arXiv:1004.1680).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * HIP path.
 *
 * It is written to be read against the paper, not to be fast: every operator
 * works on whole arrays, one formula per loop, in the order the method states
 * it.  The only parallelism is an OpenMP loop over independent pencils or
 * planes, which does not change any arithmetic.
 *
 * Storage (paper section III, the Cell and ATI data layouts; section IV.A
 * read counts): structure of arrays, 8 fields, each [nz][ny][nx] with x
 * fastest:
 *   0 rho, 1 m_x, 2 m_y, 3 m_z, 4 e (total energy incl. b^2/2) at cell centres;
 *   5 b_x, 6 b_y, 7 b_z, where b_d[c] is the flux through the LOW d-face of
 *   cell c (constrained transport, section II.B).
 * The grid is periodic on every axis, spacing h = 1/nx on all three axes.
 *
 * Readings of points the paper leaves open (each taken once, here):
 *   - cell-centred field  Bbar_d(c) = (b_d[c] + b_d[c+d]) / 2;
 *   - the relaxation (freezing) speed c of the fluid sweeps is one number
 *     per full step: the largest signal speed max_d |v_d| + c_fast found by
 *     the CFL function at the start of the step (a constant relaxation speed
 *     as in Jin & Xin; no square root is taken inside the sweeps); per-cell
 *     and per-pencil speeds are selectable method variants
 *     (oracle_set_freeze);
 *   - two-stage step: first-order upwind half step, then a van-Leer-limited
 *     full step from the old state with fluxes of the half-step state;
 *   - every operator of a full step uses the same dt; a step advances 2 dt;
 *   - forward half: fluid then magnetic per axis; reverse half: magnetic
 *     then fluid;
 *   - the magnetic sweep along d advects b_e (e the two other axes, in the
 *     cyclic order d+1, d+2) with the edge-averaged velocity v_d and applies
 *     the same edge flux to b_d, so that div b is unchanged;
 *   - all sums inside a formula are written in sweep-local axis order
 *     (normal, first transverse, second transverse), with the transverse
 *     axes taken cyclically, so that the method is exactly symmetric under
 *     a cyclic relabelling of the axes.
 *
 * Compile with -ffp-contract=off: no fused multiply-add is formed, every
 * product and sum is rounded as written.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#include "mhd_oracle.h"

#define NF 8
enum { RHO = 0, MX = 1, MY = 2, MZ = 3, EN = 4, BX = 5, BY = 6, BZ = 7 };

/* ------------------------------------------------------------------------- */
/* small helpers                                                             */
/* ------------------------------------------------------------------------- */

static int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* linear index of cell (i,j,k) with periodic wrap */
static size_t cell(const int n[3], int i, int j, int k)
{
    return (size_t)wrap(i, n[0]) + (size_t)n[0] *
           ((size_t)wrap(j, n[1]) + (size_t)n[1] * (size_t)wrap(k, n[2]));
}

/* cell index offset by s cells along axis a from (i,j,k) */
static size_t cell_shift(const int n[3], int i, int j, int k, int a, int s)
{
    int p[3] = { i, j, k };
    p[a] += s;
    return cell(n, p[0], p[1], p[2]);
}

/* Slope limiter phi(a, b) of two halved one-sided differences, zero unless
 * they have the same sign.  Section II.B uses van Leer's, the harmonic mean
 * 2ab/(a+b); the others are method variants: minmod (the smaller
 * magnitude), MC (the central value (a+b)/2 limited to twice either one)
 * and superbee (the larger of min(2|a|, |b|) and min(|a|, 2|b|)).  The
 * choice is process-wide (oracle_set_limiter), van Leer's by default. */
enum { LIMITER_VANLEER = 0, LIMITER_MINMOD = 1, LIMITER_MC = 2, LIMITER_SUPERBEE = 3 };
static int g_limiter = LIMITER_VANLEER;

static double van_leer(double a, double b)
{
    double ab = a * b;
    if (g_limiter == LIMITER_VANLEER) {
        if (ab > 0.0)
            return 2.0 * ab / (a + b);
        return 0.0;
    }
    if (!(ab > 0.0))
        return 0.0;
    double m;
    if (g_limiter == LIMITER_MINMOD) {
        m = fmin(fabs(a), fabs(b));
    } else if (g_limiter == LIMITER_MC) {
        double central = 0.5 * fabs(a + b);
        m = fmin(fmin(2.0 * fabs(a), 2.0 * fabs(b)), central);
    } else {
        m = fmax(fmin(2.0 * fabs(a), fabs(b)), fmin(fabs(a), 2.0 * fabs(b)));
    }
    return copysign(m, a);
}

int oracle_set_limiter(int kind)
{
    if (kind < LIMITER_VANLEER || kind > LIMITER_SUPERBEE) return -1;
    g_limiter = kind;
    return 0;
}

/* Relaxation (freezing) speed of the fluid sweeps.  The reading taken for
 * the paper's method is one number per step, the CFL speed passed in as c
 * (FREEZE_GRID).  The paper does not fix this choice (section II.B only
 * asks the speed to exceed the flux's characteristic speeds); two method
 * variants take it from the state of each stage instead:
 *   FREEZE_CELL:   c_i = |v_n| + c_fast of cell i (local Lax-Friedrichs-like);
 *   FREEZE_PENCIL: c = the largest |v_n| + c_fast along the pencil,
 * with c_fast = sqrt((gamma p + |Bbar|^2)/rho), stage 1 from the old state
 * and stage 2 from the half-step state.  Process-wide, FREEZE_GRID by
 * default (oracle_set_freeze). */
enum { FREEZE_GRID = 0, FREEZE_CELL = 1, FREEZE_PENCIL = 2 };
static int g_freeze = FREEZE_GRID;

int oracle_set_freeze(int mode)
{
    if (mode < FREEZE_GRID || mode > FREEZE_PENCIL) return -1;
    g_freeze = mode;
    return 0;
}

/* phi(a, b) with limiter `kind` (for tests of the formulas themselves) */
double oracle_limiter_value(int kind, double a, double b)
{
    int saved = g_limiter;
    double r;
    g_limiter = kind;
    r = van_leer(a, b);
    g_limiter = saved;
    return r;
}

/* ------------------------------------------------------------------------- */
/* Fluid flux along a sweep axis, equations (1)-(3) with b frozen            */
/* ------------------------------------------------------------------------- */

/* u = (rho, m_n, m_t1, m_t2, e) and bb = (Bbar_n, Bbar_t1, Bbar_t2) in
 * sweep-local order.  Returns the flux of equations (1)-(3) along n. */
static void fluid_flux(const double u[5], const double bb[3], double gamma,
                       double f[5])
{
    double rho = u[0], mn = u[1], mt1 = u[2], mt2 = u[3], e = u[4];
    double vn = mn / rho;
    double vt1 = mt1 / rho;
    double vt2 = mt2 / rho;
    /* magnetic pressure b^2/2 and kinetic energy rho v^2/2 = m.m/(2 rho) */
    double b2 = bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2];
    double mm = mn * mn + mt1 * mt1 + mt2 * mt2;
    double p = (gamma - 1.0) * (e - 0.5 * mm / rho - 0.5 * b2);
    double ptot = p + 0.5 * b2;                      /* P_* = p + b^2/2 */
    double bv = bb[0] * vn + bb[1] * vt1 + bb[2] * vt2;
    f[0] = mn;                                       /* eq. (1) */
    f[1] = mn * vn + ptot - bb[0] * bb[0];           /* eq. (2), normal */
    f[2] = mt1 * vn - bb[0] * bb[1];                 /* eq. (2), transverse */
    f[3] = mt2 * vn - bb[0] * bb[2];
    f[4] = (e + ptot) * vn - bb[0] * bv;             /* eq. (3) */
}

/* |v_n| + c_fast of one cell (the variants' freezing speed), with the same
 * pressure as fluid_flux: c_fast = sqrt((gamma p + |Bbar|^2)/rho). */
static double normal_speed(const double u[5], const double bb[3], double gamma)
{
    double rho = u[0], mn = u[1], mt1 = u[2], mt2 = u[3], e = u[4];
    double vn = mn / rho;
    double b2 = bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2];
    double mm = mn * mn + mt1 * mt1 + mt2 * mt2;
    double p = (gamma - 1.0) * (e - 0.5 * mm / rho - 0.5 * b2);
    return fabs(vn) + sqrt((gamma * p + b2) / rho);
}

/* freezing speed of every cell of a pencil for one stage (state w) */
static void stage_speeds(int n, const double *w, const double *bb, double gamma,
                         double c, double *cc)
{
    int i, q;
    double cmax = 0.0;
    for (i = 0; i < n; i++) {
        double uc[5], b[3];
        if (g_freeze == FREEZE_GRID) {
            cc[i] = c;
            continue;
        }
        for (q = 0; q < 5; q++) uc[q] = w[q * n + i];
        for (q = 0; q < 3; q++) b[q] = bb[q * n + i];
        cc[i] = normal_speed(uc, b, gamma);
        if (cc[i] > cmax) cmax = cc[i];
    }
    if (g_freeze == FREEZE_PENCIL)
        for (i = 0; i < n; i++) cc[i] = cmax;
}

/* ------------------------------------------------------------------------- */
/* One-dimensional relaxing-TVD update of one pencil (section II.B, eq. (6)) */
/* ------------------------------------------------------------------------- */

/* u[q*n + i]: the 5 local conserved fields along the pencil (updated in
 * place); bb[q*n + i]: the 3 local components of Bbar, held fixed.
 * tau = dt / h; c = relaxation speed (at least the largest signal speed). */
static void fluid_pencil(int n, double *u, const double *bb, double gamma,
                         double tau, double c)
{
    double *fr = malloc(sizeof(double) * 5 * n);
    double *fl = malloc(sizeof(double) * 5 * n);
    double *fi = malloc(sizeof(double) * 5 * n);   /* interface fluxes i+1/2 */
    double *uh = malloc(sizeof(double) * 5 * n);
    double *cc = malloc(sizeof(double) * n);       /* freezing speed per cell */
    double halftau = 0.5 * tau;
    int i, q;

    /* stage 1: split each cell's flux into right- and left-moving parts,
     * F^R = (cU + F)/2, F^L = (cU - F)/2, and take first-order upwind
     * interface fluxes F_{i+1/2} = F^R_i - F^L_{i+1}. */
    stage_speeds(n, u, bb, gamma, c, cc);
    for (i = 0; i < n; i++) {
        double uc[5], b[3], f[5];
        for (q = 0; q < 5; q++) uc[q] = u[q * n + i];
        for (q = 0; q < 3; q++) b[q] = bb[q * n + i];
        fluid_flux(uc, b, gamma, f);
        for (q = 0; q < 5; q++) {
            fr[q * n + i] = 0.5 * (cc[i] * uc[q] + f[q]);
            fl[q * n + i] = 0.5 * (cc[i] * uc[q] - f[q]);
        }
    }
    for (i = 0; i < n; i++)
        for (q = 0; q < 5; q++)
            fi[q * n + i] = fr[q * n + i] - fl[q * n + wrap(i + 1, n)];
    /* half step in time */
    for (i = 0; i < n; i++)
        for (q = 0; q < 5; q++)
            uh[q * n + i] = u[q * n + i] -
                            halftau * (fi[q * n + i] - fi[q * n + wrap(i - 1, n)]);

    /* stage 2: fluxes of the half-step state, second-order TVD correction
     * with the van Leer limiter on each moving part */
    stage_speeds(n, uh, bb, gamma, c, cc);
    for (i = 0; i < n; i++) {
        double uc[5], b[3], f[5];
        for (q = 0; q < 5; q++) uc[q] = uh[q * n + i];
        for (q = 0; q < 3; q++) b[q] = bb[q * n + i];
        fluid_flux(uc, b, gamma, f);
        for (q = 0; q < 5; q++) {
            fr[q * n + i] = 0.5 * (cc[i] * uc[q] + f[q]);
            fl[q * n + i] = 0.5 * (cc[i] * uc[q] - f[q]);
        }
    }
    for (i = 0; i < n; i++) {
        int im = wrap(i - 1, n), ip = wrap(i + 1, n), ipp = wrap(i + 2, n);
        for (q = 0; q < 5; q++) {
            const double *R = fr + q * n, *L = fl + q * n;
            /* right-moving part: upwind cell i */
            double fR = R[i] + van_leer(0.5 * (R[i] - R[im]), 0.5 * (R[ip] - R[i]));
            /* left-moving part: upwind cell i+1 */
            double fL = L[ip] + van_leer(0.5 * (L[i] - L[ip]), 0.5 * (L[ip] - L[ipp]));
            fi[q * n + i] = fR - fL;
        }
    }
    /* full step from the old state */
    for (i = 0; i < n; i++)
        for (q = 0; q < 5; q++)
            u[q * n + i] = u[q * n + i] -
                           tau * (fi[q * n + i] - fi[q * n + wrap(i - 1, n)]);

    free(fr); free(fl); free(fi); free(uh); free(cc);
}

int oracle_fluid_sweep(int nx, int ny, int nz, double gamma,
                       const double *in, double *out, int d, double dt,
                       double c)
{
    int n[3] = { nx, ny, nz };
    size_t N = (size_t)nx * ny * nz;
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    int len = n[d];
    int np1 = n[t1], np2 = n[t2];
    double tau = dt * (double)nx;    /* dt / h with h = 1/nx */
    long pp;

    if (d < 0 || d > 2 || nx < 1 || ny < 1 || nz < 1) return -1;
    if (out != in) memcpy(out, in, sizeof(double) * NF * N);

    #pragma omp parallel for schedule(static)
    for (pp = 0; pp < (long)np1 * np2; pp++) {
        int a = (int)(pp % np1), b = (int)(pp / np1);
        double *u = malloc(sizeof(double) * 5 * len);
        double *bb = malloc(sizeof(double) * 3 * len);
        int s, q;
        for (s = 0; s < len; s++) {
            int p[3];
            size_t c, cn, c1, c2;
            p[d] = s; p[t1] = a; p[t2] = b;
            c = cell(n, p[0], p[1], p[2]);
            cn = cell_shift(n, p[0], p[1], p[2], d, 1);
            c1 = cell_shift(n, p[0], p[1], p[2], t1, 1);
            c2 = cell_shift(n, p[0], p[1], p[2], t2, 1);
            u[0 * len + s] = in[RHO * N + c];
            u[1 * len + s] = in[(MX + d) * N + c];
            u[2 * len + s] = in[(MX + t1) * N + c];
            u[3 * len + s] = in[(MX + t2) * N + c];
            u[4 * len + s] = in[EN * N + c];
            bb[0 * len + s] = 0.5 * (in[(BX + d) * N + c] + in[(BX + d) * N + cn]);
            bb[1 * len + s] = 0.5 * (in[(BX + t1) * N + c] + in[(BX + t1) * N + c1]);
            bb[2 * len + s] = 0.5 * (in[(BX + t2) * N + c] + in[(BX + t2) * N + c2]);
        }
        fluid_pencil(len, u, bb, gamma, tau, c);
        for (s = 0; s < len; s++) {
            int p[3];
            size_t c;
            p[d] = s; p[t1] = a; p[t2] = b;
            c = cell(n, p[0], p[1], p[2]);
            out[RHO * N + c] = u[0 * len + s];
            out[(MX + d) * N + c] = u[1 * len + s];
            out[(MX + t1) * N + c] = u[2 * len + s];
            out[(MX + t2) * N + c] = u[3 * len + s];
            out[EN * N + c] = u[4 * len + s];
        }
        (void)q;
        free(u); free(bb);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Magnetic advection-constraint sweep (section II.B, constrained transport) */
/* ------------------------------------------------------------------------- */

/* Along axis d with velocity v_d frozen: for each other axis e (order d+1,
 * d+2), the term v_d b_e of the EMF advects b_e along d and, through the
 * constraint, changes b_d by the e-derivative of the same edge flux
 * (equation (4)).  The edge flux f sits on the edge at c + d/2 - e/2. */
int oracle_mag_sweep(int nx, int ny, int nz, double gamma,
                     const double *in, double *out, int d, double dt)
{
    int n[3] = { nx, ny, nz };
    size_t N = (size_t)nx * ny * nz;
    double tau = dt * (double)nx;
    double halftau = 0.5 * tau;
    double *v, *a, *g, *qh, *f;
    int ei;
    (void)gamma;

    if (d < 0 || d > 2 || nx < 1 || ny < 1 || nz < 1) return -1;
    if (out != in) memcpy(out, in, sizeof(double) * NF * N);

    v = malloc(sizeof(double) * N);
    a = malloc(sizeof(double) * N);
    g = malloc(sizeof(double) * N);
    qh = malloc(sizeof(double) * N);
    f = malloc(sizeof(double) * N);

    /* frozen velocity along the sweep */
    for (size_t c = 0; c < N; c++)
        v[c] = in[(MX + d) * N + c] / in[RHO * N + c];

    for (ei = 1; ei <= 2; ei++) {
        int e = (d + ei) % 3;
        const double *q = out + (BX + e) * N;   /* current b_e */
        int k;

        /* edge velocity: average of v_d over the two cells sharing the
         * e-face (face velocity), then over the two faces sharing the edge */
        #pragma omp parallel for schedule(static)
        for (k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    size_t c = cell(n, i, j, k);
                    size_t cme = cell_shift(n, i, j, k, e, -1);
                    size_t cpd = cell_shift(n, i, j, k, d, 1);
                    int pd[3] = { i, j, k };
                    size_t cpdme;
                    double w0, w1;
                    pd[d] += 1;
                    cpdme = cell_shift(n, pd[0], pd[1], pd[2], e, -1);
                    w0 = 0.5 * (v[c] + v[cme]);
                    w1 = 0.5 * (v[cpd] + v[cpdme]);
                    a[c] = 0.5 * (w0 + w1);
                }

        /* stage 1: first-order upwind edge flux and half step of b_e */
        #pragma omp parallel for schedule(static)
        for (k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    size_t c = cell(n, i, j, k);
                    size_t cpd = cell_shift(n, i, j, k, d, 1);
                    if (a[c] > 0.0)
                        g[c] = a[c] * q[c];
                    else
                        g[c] = a[c] * q[cpd];
                }
        #pragma omp parallel for schedule(static)
        for (k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    size_t c = cell(n, i, j, k);
                    size_t cmd = cell_shift(n, i, j, k, d, -1);
                    qh[c] = q[c] - halftau * (g[c] - g[cmd]);
                }

        /* stage 2: van-Leer-limited upwind edge value of the half-step b_e */
        #pragma omp parallel for schedule(static)
        for (k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    size_t c = cell(n, i, j, k);
                    size_t cmd = cell_shift(n, i, j, k, d, -1);
                    size_t cpd = cell_shift(n, i, j, k, d, 1);
                    size_t cp2 = cell_shift(n, i, j, k, d, 2);
                    double ac = a[c];
                    if (ac > 0.0)
                        f[c] = ac * (qh[c] + van_leer(0.5 * (qh[c] - qh[cmd]),
                                                      0.5 * (qh[cpd] - qh[c])));
                    else if (ac < 0.0)
                        f[c] = ac * (qh[cpd] + van_leer(0.5 * (qh[cpd] - qh[cp2]),
                                                        0.5 * (qh[c] - qh[cpd])));
                    else
                        f[c] = 0.0;
                }

        /* apply the edge flux: advection of b_e along d, and the constraint
         * update of b_d along e (same flux, so div b does not change) */
        #pragma omp parallel for schedule(static)
        for (k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    size_t c = cell(n, i, j, k);
                    size_t cmd = cell_shift(n, i, j, k, d, -1);
                    int pm[3] = { i, j, k };
                    size_t cmdpe;
                    pm[d] -= 1;
                    cmdpe = cell_shift(n, pm[0], pm[1], pm[2], e, 1);
                    out[(BX + e) * N + c] = q[c] - tau * (f[c] - f[cmd]);
                    out[(BX + d) * N + c] = out[(BX + d) * N + c] +
                                            tau * (f[cmdpe] - f[cmd]);
                }
    }
    free(v); free(a); free(g); free(qh); free(f);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sweeps and the Strang-ordered full step (section II.B; section IV.A)      */
/* ------------------------------------------------------------------------- */

int oracle_sweep(int nx, int ny, int nz, double gamma, double *s, int code,
                 double dt, double c)
{
    size_t N = (size_t)nx * ny * nz;
    double *tmp;
    int d = code % 3, r;
    if (code < 0 || code > 5) return -1;
    tmp = malloc(sizeof(double) * NF * N);
    if (code < 3) {          /* forward half: fluid, then magnetic */
        r = oracle_fluid_sweep(nx, ny, nz, gamma, s, tmp, d, dt, c);
        if (!r) r = oracle_mag_sweep(nx, ny, nz, gamma, tmp, s, d, dt);
    } else {                 /* reverse half: magnetic, then fluid */
        r = oracle_mag_sweep(nx, ny, nz, gamma, s, tmp, d, dt);
        if (!r) r = oracle_fluid_sweep(nx, ny, nz, gamma, tmp, s, d, dt, c);
    }
    free(tmp);
    return r;
}

int oracle_step(int nx, int ny, int nz, double gamma, double *s, double dt,
                double c)
{
    /* x, y, z, then z, y, x; every operator uses dt, the step covers 2 dt */
    static const int order[6] = { 0, 1, 2, 5, 4, 3 };
    int r = 0;
    for (int o = 0; o < 6 && !r; o++)
        r = oracle_sweep(nx, ny, nz, gamma, s, order[o], dt, c);
    return r;
}

/* ------------------------------------------------------------------------- */
/* CFL time step (section II.B; the CFL function of section IV.A)            */
/* ------------------------------------------------------------------------- */

/* vmax = max over cells of (max_d |v_d| + c_fast), with
 * c_fast = sqrt((gamma p + |Bbar|^2)/rho) the largest magnetosonic speed;
 * dt = cfl * h / vmax.  vmax is also the relaxation speed of the step.
 * Returns -4 (dt = vmax = 0) if any cell has rho <= 0, p < 0 or a
 * non-finite value. */
int oracle_cfl(int nx, int ny, int nz, double gamma, const double *s,
               double cfl, double *dt, double *vmax_out)
{
    int n[3] = { nx, ny, nz };
    size_t N = (size_t)nx * ny * nz;
    double vmax = 0.0;
    int bad = 0;
    long k;

    #pragma omp parallel for reduction(max:vmax) reduction(|:bad) schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cell(n, i, j, (int)k);
                double rho = s[RHO * N + c];
                double mx = s[MX * N + c], my = s[MY * N + c], mz = s[MZ * N + c];
                double e = s[EN * N + c];
                double bx = 0.5 * (s[BX * N + c] + s[BX * N + cell_shift(n, i, j, (int)k, 0, 1)]);
                double by = 0.5 * (s[BY * N + c] + s[BY * N + cell_shift(n, i, j, (int)k, 1, 1)]);
                double bz = 0.5 * (s[BZ * N + c] + s[BZ * N + cell_shift(n, i, j, (int)k, 2, 1)]);
                double b2 = bx * bx + by * by + bz * bz;
                double mm = mx * mx + my * my + mz * mz;
                double p = (gamma - 1.0) * (e - 0.5 * mm / rho - 0.5 * b2);
                double vx = fabs(mx / rho), vy = fabs(my / rho), vz = fabs(mz / rho);
                double vm = vx > vy ? vx : vy;
                double sp;
                vm = vm > vz ? vm : vz;
                sp = vm + sqrt((gamma * p + b2) / rho);
                if (!(rho > 0.0) || !(p >= 0.0) || !isfinite(sp) ||
                    !isfinite(e) || !isfinite(mm) || !isfinite(b2))
                    bad = 1;
                else if (sp > vmax)
                    vmax = sp;
            }
    if (bad || !(vmax > 0.0)) {
        *dt = 0.0;
        *vmax_out = 0.0;
        return bad ? -4 : -1;
    }
    *dt = cfl * (1.0 / (double)nx) / vmax;
    *vmax_out = vmax;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Diagnostics: conserved totals and the divergence of b                     */
/* ------------------------------------------------------------------------- */

/* out[0..7] = h^3 * sum over cells of each field (plain loop order k,j,i);
 * out[8] = max_c |sum_d (b_d[c+d] - b_d[c])| / max |b| (= max|div b| h/max|b|) */
void oracle_diag(int nx, int ny, int nz, const double *s, double out[9])
{
    int n[3] = { nx, ny, nz };
    size_t N = (size_t)nx * ny * nz;
    double h = 1.0 / (double)nx;
    double h3 = h * h * h;
    double dmax = 0.0, bmax = 0.0;
    for (int f = 0; f < NF; f++) {
        double acc = 0.0;
        for (size_t c = 0; c < N; c++) acc += s[f * N + c];
        out[f] = acc * h3;
    }
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cell(n, i, j, k);
                double dv = (s[BX * N + cell_shift(n, i, j, k, 0, 1)] - s[BX * N + c]) +
                            (s[BY * N + cell_shift(n, i, j, k, 1, 1)] - s[BY * N + c]) +
                            (s[BZ * N + cell_shift(n, i, j, k, 2, 1)] - s[BZ * N + c]);
                if (fabs(dv) > dmax) dmax = fabs(dv);
                for (int f = BX; f <= BZ; f++)
                    if (fabs(s[f * N + c]) > bmax) bmax = fabs(s[f * N + c]);
            }
    out[8] = bmax > 0.0 ? dmax / bmax : 0.0;
}

/* ------------------------------------------------------------------------- */
/* Restriction by an integer factor r                                        */
/* ------------------------------------------------------------------------- */

/* Coarse cell-centred fields are the mean over the r^3 fine cells of the
 * block; a coarse face value b_d is the mean of the r^2 fine face values that
 * tile that coarse face (fine index r*I_d along d).  Totals are kept and the
 * coarse div b is the block mean of the fine div b. */
int oracle_restrict(int nx, int ny, int nz, int r, const double *fine,
                    double *coarse)
{
    int cx, cy, cz;
    size_t Nf = (size_t)nx * ny * nz, Nc;
    if (r < 1 || nx % r || ny % r || nz % r) return -1;
    cx = nx / r; cy = ny / r; cz = nz / r;
    Nc = (size_t)cx * cy * cz;
    for (int K = 0; K < cz; K++)
        for (int J = 0; J < cy; J++)
            for (int I = 0; I < cx; I++) {
                size_t C = (size_t)I + (size_t)cx * ((size_t)J + (size_t)cy * K);
                for (int f = 0; f < 5; f++) {
                    double acc = 0.0;
                    for (int k = 0; k < r; k++)
                        for (int j = 0; j < r; j++)
                            for (int i = 0; i < r; i++)
                                acc += fine[f * Nf + (size_t)(r * I + i) +
                                            (size_t)nx * ((size_t)(r * J + j) + (size_t)ny * (size_t)(r * K + k))];
                    coarse[f * Nc + C] = acc / ((double)r * r * r);
                }
                for (int d = 0; d < 3; d++) {
                    double acc = 0.0;
                    for (int u = 0; u < r; u++)
                        for (int w = 0; w < r; w++) {
                            int p[3] = { r * I, r * J, r * K };
                            /* the two transverse offsets span the coarse face */
                            p[(d + 1) % 3] += u;
                            p[(d + 2) % 3] += w;
                            acc += fine[(BX + d) * Nf + (size_t)p[0] +
                                        (size_t)nx * ((size_t)p[1] + (size_t)ny * (size_t)p[2])];
                        }
                    coarse[(BX + d) * Nc + C] = acc / ((double)r * r);
                }
            }
    return 0;
}
