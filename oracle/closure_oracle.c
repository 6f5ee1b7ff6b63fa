/*
 * FP64 CPU oracle of the learned-closure pieces (test infrastructure only;
 * shares no code with the HIP path).
 *
 * Periodic 3x3x3 convolution, stride 1, on an nx x ny x nz grid with
 * channel-last activations x[cell][c] (cell = i + nx*(j + ny*k)):
 *   y[cell][co] = bias[co] + sum_{o, ci} w[o][ci][co] * x[cell + d(o)][ci]
 * with offset o = (dz+1)*9 + (dy+1)*3 + (dx+1), dx, dy, dz in {-1, 0, 1}.
 * Backward: dx[cell][ci] = sum_{o, co} w[o][ci][co] dy[cell - d(o)][co];
 *           dw[o][ci][co] = sum_cell x[cell + d(o)][ci] dy[cell][co];
 *           dbias[co]     = sum_cell dy[cell][co].
 *
 * Conservative projection of the network output o[cell][8] into a state
 * correction delta[f][cell] (field-major, the state layout):
 *   fluid f < 5: delta_f = s_f (o_f - mean_cells o_f)   (totals unchanged);
 *   field:       (A_x, A_y, A_z) = s_b (o_5, o_6, o_7) on the x-, y-, z-edges
 *                and delta_b = discrete curl of A, e.g.
 *                delta_bx[c] = (A_z[c+y] - A_z[c]) - (A_y[c+z] - A_y[c]),
 *                so the discrete div of delta_b vanishes in every cell.
 * project_T applies the adjoint map (gradient of a scalar through the
 * projection).
 *
 * Roughness gate (optional): with R[8] > 0 (training-set means),
 *   r_f(c) = sum over the three axes a of |u_f(c+a) - 2 u_f(c) + u_f(c-a)|,
 *   g0(c)  = (1/8) sum_f r_f(c) / R_f,
 *   g(c)   = max of g0 over c and its six face neighbours,
 * and the projection acts on g(c) o(c) instead of o(c): corrections vanish
 * where the state is locally linear, whatever the network outputs.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static int wrapc(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

static size_t cidx(int nx, int ny, int nz, int i, int j, int k)
{
    return (size_t)wrapc(i, nx) + (size_t)nx * ((size_t)wrapc(j, ny) + (size_t)ny * (size_t)wrapc(k, nz));
}

void oracle_conv3d(int nx, int ny, int nz, int cin, int cout, const double *x,
                   const double *w, const double *bias, double *y)
{
    long k;
    #pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cidx(nx, ny, nz, i, j, (int)k);
                for (int co = 0; co < cout; co++) {
                    double acc = bias ? bias[co] : 0.0;
                    for (int o = 0; o < 27; o++) {
                        int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
                        size_t s = cidx(nx, ny, nz, i + dx, j + dy, (int)k + dz);
                        for (int ci = 0; ci < cin; ci++)
                            acc += w[((size_t)o * cin + ci) * cout + co] * x[s * cin + ci];
                    }
                    y[c * cout + co] = acc;
                }
            }
}

void oracle_conv3d_dgrad(int nx, int ny, int nz, int cin, int cout, const double *dy,
                         const double *w, double *dx_out)
{
    long k;
    #pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cidx(nx, ny, nz, i, j, (int)k);
                for (int ci = 0; ci < cin; ci++) {
                    double acc = 0.0;
                    for (int o = 0; o < 27; o++) {
                        int dx = o % 3 - 1, ddy = (o / 3) % 3 - 1, dz = o / 9 - 1;
                        size_t s = cidx(nx, ny, nz, i - dx, j - ddy, (int)k - dz);
                        for (int co = 0; co < cout; co++)
                            acc += w[((size_t)o * cin + ci) * cout + co] * dy[s * cout + co];
                    }
                    dx_out[c * cin + ci] = acc;
                }
            }
}

void oracle_conv3d_wgrad(int nx, int ny, int nz, int cin, int cout, const double *x,
                         const double *dy, double *dw, double *dbias)
{
    int o;
    size_t N = (size_t)nx * ny * nz;
    #pragma omp parallel for schedule(static)
    for (o = 0; o < 27; o++) {
        int dx = o % 3 - 1, ddy = (o / 3) % 3 - 1, dz = o / 9 - 1;
        for (int ci = 0; ci < cin; ci++)
            for (int co = 0; co < cout; co++) {
                double acc = 0.0;
                for (int k = 0; k < nz; k++)
                    for (int j = 0; j < ny; j++)
                        for (int i = 0; i < nx; i++) {
                            size_t c = cidx(nx, ny, nz, i, j, k);
                            size_t s = cidx(nx, ny, nz, i + dx, j + ddy, k + dz);
                            acc += x[s * cin + ci] * dy[c * cout + co];
                        }
                dw[((size_t)o * cin + ci) * cout + co] = acc;
            }
    }
    if (dbias)
        for (int co = 0; co < cout; co++) {
            double acc = 0.0;
            for (size_t c = 0; c < N; c++) acc += dy[c * cout + co];
            dbias[co] = acc;
        }
}

void oracle_closure_project(int nx, int ny, int nz, const double *o, const double *scale,
                            double *delta)
{
    size_t N = (size_t)nx * ny * nz;
    for (int f = 0; f < 5; f++) {
        double mean = 0.0;
        for (size_t c = 0; c < N; c++) mean += o[c * 8 + f];
        mean /= (double)N;
        for (size_t c = 0; c < N; c++) delta[f * N + c] = scale[f] * (o[c * 8 + f] - mean);
    }
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cidx(nx, ny, nz, i, j, k);
                size_t cxp = cidx(nx, ny, nz, i + 1, j, k);
                size_t cyp = cidx(nx, ny, nz, i, j + 1, k);
                size_t czp = cidx(nx, ny, nz, i, j, k + 1);
                double ax = scale[5] * o[c * 8 + 5], ay = scale[6] * o[c * 8 + 6], az = scale[7] * o[c * 8 + 7];
                double az_yp = scale[7] * o[cyp * 8 + 7], ay_zp = scale[6] * o[czp * 8 + 6];
                double ax_zp = scale[5] * o[czp * 8 + 5], az_xp = scale[7] * o[cxp * 8 + 7];
                double ay_xp = scale[6] * o[cxp * 8 + 6], ax_yp = scale[5] * o[cyp * 8 + 5];
                delta[5 * N + c] = (az_yp - az) - (ay_zp - ay);
                delta[6 * N + c] = (ax_zp - ax) - (az_xp - az);
                delta[7 * N + c] = (ay_xp - ay) - (ax_yp - ax);
            }
}

/* g[f][cell]: gradient with respect to delta; go[cell][8]: gradient with
 * respect to the network output o */
void oracle_closure_project_T(int nx, int ny, int nz, const double *g, const double *scale,
                              double *go)
{
    size_t N = (size_t)nx * ny * nz;
    for (int f = 0; f < 5; f++) {
        double mean = 0.0;
        for (size_t c = 0; c < N; c++) mean += g[f * N + c];
        mean /= (double)N;
        for (size_t c = 0; c < N; c++) go[c * 8 + f] = scale[f] * (g[f * N + c] - mean);
    }
    for (size_t c = 0; c < N; c++) go[c * 8 + 5] = go[c * 8 + 6] = go[c * 8 + 7] = 0.0;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cidx(nx, ny, nz, i, j, k);
                size_t cxm = cidx(nx, ny, nz, i - 1, j, k);
                size_t cym = cidx(nx, ny, nz, i, j - 1, k);
                size_t czm = cidx(nx, ny, nz, i, j, k - 1);
                /* A_z enters bx[c - y] (+), bx[c] (-), by[c - x] (-), by[c] (+) */
                go[c * 8 + 7] += scale[7] * ((g[5 * N + cym] - g[5 * N + c]) - (g[6 * N + cxm] - g[6 * N + c]));
                /* A_y enters bx[c - z] (-), bx[c] (+), bz[c - x] (+), bz[c] (-) */
                go[c * 8 + 6] += scale[6] * ((g[7 * N + cxm] - g[7 * N + c]) - (g[5 * N + czm] - g[5 * N + c]));
                /* A_x enters by[c - z] (+), by[c] (-), bz[c - y] (-), bz[c] (+) */
                go[c * 8 + 5] += scale[5] * ((g[6 * N + czm] - g[6 * N + c]) - (g[7 * N + cym] - g[7 * N + c]));
            }
}

/* u[f][cell] (field-major) -> g[cell] */
void oracle_closure_gate(int nx, int ny, int nz, const double *u, const double *R, double *g)
{
    size_t N = (size_t)nx * ny * nz;
    double *g0 = (double *)malloc(N * sizeof(double));
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cidx(nx, ny, nz, i, j, k);
                size_t nb[6] = { cidx(nx, ny, nz, i + 1, j, k), cidx(nx, ny, nz, i - 1, j, k),
                                 cidx(nx, ny, nz, i, j + 1, k), cidx(nx, ny, nz, i, j - 1, k),
                                 cidx(nx, ny, nz, i, j, k + 1), cidx(nx, ny, nz, i, j, k - 1) };
                double acc = 0.0;
                for (int f = 0; f < 8; f++) {
                    const double *uf = u + (size_t)f * N;
                    double r = 0.0;
                    for (int a = 0; a < 3; a++)
                        r += fabs(uf[nb[2 * a]] - 2.0 * uf[c] + uf[nb[2 * a + 1]]);
                    acc += r / R[f];
                }
                g0[c] = acc / 8.0;
            }
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cidx(nx, ny, nz, i, j, k);
                double m = g0[c];
                size_t nb[6] = { cidx(nx, ny, nz, i + 1, j, k), cidx(nx, ny, nz, i - 1, j, k),
                                 cidx(nx, ny, nz, i, j + 1, k), cidx(nx, ny, nz, i, j - 1, k),
                                 cidx(nx, ny, nz, i, j, k + 1), cidx(nx, ny, nz, i, j, k - 1) };
                for (int q = 0; q < 6; q++)
                    if (g0[nb[q]] > m) m = g0[nb[q]];
                g[c] = m;
            }
    free(g0);
}
