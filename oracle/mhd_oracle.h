/*
 * FP64 CPU oracle of the ideal-MHD update step (Pang, Pen & Perrone,
 * arXiv:1004.1680, section II).  TEST INFRASTRUCTURE ONLY: used by the tests,
 * the smoke check and the CPU-baseline leg of the benchmark, never by the
 * product library.  Shares no code with the HIP path.
 *
 * State arrays hold 8 fields, field-major [f][k][j][i] with x fastest:
 * rho, m_x, m_y, m_z, e, b_x, b_y, b_z (b_d on the low d-face of each cell).
 * Grid spacing h = 1/nx on every axis; periodic boundaries.
 * Return codes: 0 ok, -1 bad argument, -4 non-physical state.
 */
#ifndef MHD_ORACLE_H
#define MHD_ORACLE_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* c: relaxation speed of the fluid sweep (the step's CFL speed) */
int oracle_fluid_sweep(int nx, int ny, int nz, double gamma,
                       const double *in, double *out, int d, double dt,
                       double c);
int oracle_mag_sweep(int nx, int ny, int nz, double gamma,
                     const double *in, double *out, int d, double dt);
/* code 0..2: fluid then magnetic along code; 3..5: magnetic then fluid
 * along code-3; in place on s */
int oracle_sweep(int nx, int ny, int nz, double gamma, double *s, int code,
                 double dt, double c);
/* xyz then zyx, each of the 12 operators with dt; in place */
int oracle_step(int nx, int ny, int nz, double gamma, double *s, double dt,
                double c);
/* dt = cfl h / vmax and vmax = max signal speed (the relaxation speed) */
int oracle_cfl(int nx, int ny, int nz, double gamma, const double *s,
               double cfl, double *dt, double *vmax);
void oracle_diag(int nx, int ny, int nz, const double *s, double out[9]);
/* process-wide slope limiter: 0 van Leer (default), 1 minmod, 2 MC,
 * 3 superbee; -1 for another value */
int oracle_set_limiter(int kind);
double oracle_limiter_value(int kind, double a, double b);
/* process-wide freezing speed of the fluid sweeps: 0 the c argument (one
 * number per step, default), 1 |v_n| + c_fast per cell, 2 its largest value
 * along the pencil; both variants per stage; -1 for another value */
int oracle_set_freeze(int mode);
int oracle_restrict(int nx, int ny, int nz, int r, const double *fine,
                    double *coarse);

#ifdef __cplusplus
}
#endif
#endif
