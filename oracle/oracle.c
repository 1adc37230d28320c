/*
 * oracle.c -- plain, slow, FP64 CPU reference for one micromagnetic time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no source with the GPU path.
 *
 * What it computes (Zhu, "Grace", arXiv:1411.2565):
 *   - the effective field of Sec. 2, eq. (2): exchange + uniaxial anisotropy +
 *     demagnetisation + external (Zeeman) field, with the energy density of
 *     eq. (1);
 *   - the demagnetisation field as the plain O(N^2) direct sum over all source
 *     cells (Sec. 1 and Sec. 3 name this brute-force evaluation; the FFT route of
 *     Sec. 3 is an exact re-evaluation of the same zero-padded linear
 *     convolution, so the definition is what is written here), using the
 *     cell-averaged Newell tensor for rectangular cells;
 *   - the six-neighbour exchange field (Sec. 3), free (Neumann) boundaries;
 *   - the Landau-Lifshitz form of the LLG equation, eq. (3), integrated with
 *     the explicit Euler method (Sec. 3), optionally renormalising |m| = 1;
 *   - the total energy of eq. (1) summed over cells, and the exact discrete
 *     adjoint of the Euler rollout for an L2 loss on the final state.
 *
 * Readings where the paper is silent or garbled (each one is listed in the
 * design notes of the repository):
 *   - eq. (1)'s exchange term repeats the x component; it is read as the sum
 *     over the three components of |grad m_c|^2;
 *   - eq. (2) is read as H = -(1/mu0) dE/dM so that H is in A/m;
 *   - gamma*mu0 is one constant gamma0 in m/(A s);
 *   - the anisotropy field is (2 Ku/(mu0 Ms)) (m.u) u, energy Ku (1 - (m.u)^2);
 *   - mu0 = 4 pi 1e-7 exactly.
 *
 * Units are SI.  Vector fields are stored structure-of-arrays
 * [3][nz][ny][nx] with x fastest; scalar maps are [nz][ny][nx].
 * The tensor table covers the non-negative octant of cell offsets and is
 * stored [6][nz][ny][nx] in the component order xx, yy, zz, xy, xz, yz.
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORC_MU0 (4.0e-7 * M_PI)

enum { ORC_T_EXCH = 1, ORC_T_DEMAG = 2, ORC_T_ANIS = 4, ORC_T_ZEEMAN = 8 };

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    double A;       /* exchange stiffness, J/m */
    double Ku;      /* uniaxial anisotropy constant, J/m^3 */
    double u[3];    /* easy axis (unit) */
    double alpha;   /* damping */
    double gamma0;  /* gamma*mu0, m/(A s) */
    const double *Ms;    /* [N] saturation magnetisation, A/m */
    const double *hext;  /* [3][N] external field, A/m */
    const double *tab;   /* [6][nz][ny][nx] octant tensor table */
    int terms;           /* ORC_T_* mask */
    int renorm;          /* 1: m <- m/|m| after each Euler step */
} orc_problem;

/* ------------------------------------------------------------------------ */
/* Newell, Williams & Dunlop (1993) cell-averaged demagnetising tensor.       */
/* f and g are the auxiliary functions whose second differences over the     */
/* 27-point stencil give N_xx and N_xy between two identical rectangular     */
/* cells.  A term whose polynomial prefactor vanishes is dropped (0*inf).    */
/* ------------------------------------------------------------------------ */

static double newell_f(double x, double y, double z)
{
    x = fabs(x); y = fabs(y); z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    if (R == 0.0) return 0.0;
    double r = (2.0 * x2 - y2 - z2) * R / 6.0;
    double p = 0.5 * y * (z2 - x2);
    if (p != 0.0) r += p * asinh(y / sqrt(x2 + z2));
    p = 0.5 * z * (y2 - x2);
    if (p != 0.0) r += p * asinh(z / sqrt(x2 + y2));
    p = x * y * z;
    if (p != 0.0) r -= p * atan(y * z / (x * R));
    return r;
}

static double newell_g(double x, double y, double z)
{
    const double sgn = ((x < 0.0) ? -1.0 : 1.0) * ((y < 0.0) ? -1.0 : 1.0);
    x = fabs(x); y = fabs(y); z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    if (R == 0.0) return 0.0;
    double r = -x * y * R / 3.0;
    double p = x * y * z;
    if (p != 0.0) r += p * asinh(z / sqrt(x2 + y2));
    p = y * (3.0 * z2 - y2) / 6.0;
    if (p != 0.0) r += p * asinh(x / sqrt(y2 + z2));
    p = x * (3.0 * z2 - x2) / 6.0;
    if (p != 0.0) r += p * asinh(y / sqrt(x2 + z2));
    p = z * z2 / 6.0;
    if (p != 0.0) r -= p * atan(x * y / (z * R));
    p = 0.5 * z * y2;
    if (p != 0.0) r -= p * atan(x * z / (y * R));
    p = 0.5 * z * x2;
    if (p != 0.0) r -= p * atan(y * z / (x * R));
    return sgn * r;
}

/* Second difference in all three directions: weights 2 at the centre and -1
 * at +-1 cell along each axis, multiplied over axes, divided by 4 pi V. */
static double newell_stencil(double (*fn)(double, double, double),
                             double X, double Y, double Z,
                             double dx, double dy, double dz)
{
    static const double w[3] = {-1.0, 2.0, -1.0};
    double s = 0.0;
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c)
                s += w[a + 1] * w[b + 1] * w[c + 1] *
                     fn(X + a * dx, Y + b * dy, Z + c * dz);
    return s / (4.0 * M_PI * dx * dy * dz);
}

/* Six components at offset (X,Y,Z) [m] with the Newell formulas; the yy, zz,
 * xz and yz components come from xx and xy by permuting axes. */
static void tensor_newell(double X, double Y, double Z,
                          double dx, double dy, double dz, double out[6])
{
    out[0] = newell_stencil(newell_f, X, Y, Z, dx, dy, dz);
    out[1] = newell_stencil(newell_f, Y, X, Z, dy, dx, dz);
    out[2] = newell_stencil(newell_f, Z, Y, X, dz, dy, dx);
    out[3] = newell_stencil(newell_g, X, Y, Z, dx, dy, dz);
    out[4] = newell_stencil(newell_g, X, Z, Y, dx, dz, dy);
    out[5] = newell_stencil(newell_g, Y, Z, X, dy, dz, dx);
}

/* Gauss-Legendre nodes and weights on [0,1] by Newton iteration on P_n. */
static void gauss_legendre01(int n, double *t, double *w)
{
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = pk;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = pk;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        t[i] = 0.5 * (1.0 - x);
        w[i] = 1.0 / ((1.0 - x * x) * dp * dp); /* 2/((1-x^2)P'^2), halved for [0,1] */
    }
}

/* Far field: the cell-pair average is the point-dipole kernel
 *   K(r) = (1/4 pi) (I/|r|^3 - 3 r r^T/|r|^5)
 * integrated over the separation s in [-d, d]^3 with the triangular weight
 * prod_a (d_a - |s_a|), divided by the cell volume.  Each axis is split at
 * s = 0 (kink of the weight) and integrated with n-point Gauss-Legendre. */
static void tensor_quadrature(double X, double Y, double Z,
                              double dx, double dy, double dz, int n, double out[6])
{
    double t[32], w[32];
    if (n > 32) n = 32;
    gauss_legendre01(n, t, w);
    const double d[3] = {dx, dy, dz};
    double sx[64], sy[64], sz[64], wx[64], wy[64], wz[64];
    double *sa[3] = {sx, sy, sz}, *wa[3] = {wx, wy, wz};
    for (int a = 0; a < 3; ++a)
        for (int h = 0; h < 2; ++h)
            for (int q = 0; q < n; ++q) {
                sa[a][h * n + q] = (h ? -1.0 : 1.0) * d[a] * t[q];
                wa[a][h * n + q] = w[q] * (1.0 - t[q]);
            }
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 2 * n; ++i)
        for (int j = 0; j < 2 * n; ++j)
            for (int k = 0; k < 2 * n; ++k) {
                const double x = X + sx[i], y = Y + sy[j], z = Z + sz[k];
                const double r2 = x * x + y * y + z * z;
                const double r = sqrt(r2);
                const double ir5 = 1.0 / (r2 * r2 * r);
                const double ww = wx[i] * wy[j] * wz[k];
                acc[0] += ww * (r2 - 3.0 * x * x) * ir5;
                acc[1] += ww * (r2 - 3.0 * y * y) * ir5;
                acc[2] += ww * (r2 - 3.0 * z * z) * ir5;
                acc[3] += ww * (-3.0 * x * y) * ir5;
                acc[4] += ww * (-3.0 * x * z) * ir5;
                acc[5] += ww * (-3.0 * y * z) * ir5;
            }
    const double V = dx * dy * dz;
    for (int c = 0; c < 6; ++c) out[c] = acc[c] * V / (4.0 * M_PI);
}

/* Oracle's own near/far split: Newell for max |offset| <= 12 cells along
 * every axis, 6-point tent quadrature beyond. */
#define ORC_NEAR_CELLS 12
#define ORC_QUAD_NODES 6

/* method: 0 = split as above, 1 = Newell only, 2 = quadrature only. */
void orc_tensor_at(double X, double Y, double Z, double dx, double dy, double dz,
                   int method, int nodes, double out[6])
{
    if (nodes <= 0) nodes = ORC_QUAD_NODES;
    if (method == 1) { tensor_newell(X, Y, Z, dx, dy, dz, out); return; }
    if (method == 2) { tensor_quadrature(X, Y, Z, dx, dy, dz, nodes, out); return; }
    const double ox = fabs(X) / dx, oy = fabs(Y) / dy, oz = fabs(Z) / dz;
    double mx = ox > oy ? ox : oy;
    mx = mx > oz ? mx : oz;
    if (mx <= ORC_NEAR_CELLS + 0.5)
        tensor_newell(X, Y, Z, dx, dy, dz, out);
    else
        tensor_quadrature(X, Y, Z, dx, dy, dz, nodes, out);
}

/* Octant table: tab[c][oz][oy][ox] for 0 <= o_a < n_a. */
void orc_tensor_table(int nx, int ny, int nz, double dx, double dy, double dz, double *tab)
{
    const size_t N = (size_t)nx * ny * nz;
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int oz = 0; oz < nz; ++oz)
        for (int oy = 0; oy < ny; ++oy)
            for (int ox = 0; ox < nx; ++ox) {
                double v[6];
                orc_tensor_at(ox * dx, oy * dy, oz * dz, dx, dy, dz, 0, 0, v);
                const size_t i = ((size_t)oz * ny + oy) * nx + ox;
                for (int c = 0; c < 6; ++c) tab[c * N + i] = v[c];
            }
}

/* ------------------------------------------------------------------------ */
/* Demagnetising field by direct summation:                                  */
/*   H_i = - sum_j N(r_i - r_j) M_j,  M_j = Ms_j m_j,  self term included.   */
/* N(o) is even in every axis for xx, yy, zz and odd in the two named axes   */
/* for xy, xz, yz, which fixes the sign when a table entry is read at |o|.   */
/* A cell is magnetic when its Ms > 0; Ms = 0 marks vacuum (see orc_heff). */
static inline int magnetic(const orc_problem *p, size_t i) { return p->Ms[i] > 0.0; }

/* ------------------------------------------------------------------------ */

/* Apply the convolution to an arbitrary vector field v ([3][N]):
 * out_i = sum_j N(r_i - r_j) v_j   (no minus sign, no Ms). */
void orc_conv(int nx, int ny, int nz, const double *tab, const double *v, double *out)
{
    const size_t N = (size_t)nx * ny * nz;
    const double *T[6];
    for (int c = 0; c < 6; ++c) T[c] = tab + c * N;
    const double *vx = v, *vy = v + N, *vz = v + 2 * N;
#pragma omp parallel
    {
        double *row = (double *)malloc(sizeof(double) * 6 * (2 * nx - 1));
        double *acc = (double *)malloc(sizeof(double) * 3 * nx);
#pragma omp for collapse(2) schedule(static)
        for (int iz = 0; iz < nz; ++iz)
            for (int iy = 0; iy < ny; ++iy) {
                memset(acc, 0, sizeof(double) * 3 * nx);
                for (int jz = 0; jz < nz; ++jz)
                    for (int jy = 0; jy < ny; ++jy) {
                        const int oz = iz - jz, oy = iy - jy;
                        const int az = abs(oz), ay = abs(oy);
                        const double sy = oy < 0 ? -1.0 : 1.0, sz = oz < 0 ? -1.0 : 1.0;
                        /* signed tensor row for ox in [-(nx-1), nx-1] */
                        for (int ox = -(nx - 1); ox <= nx - 1; ++ox) {
                            const int ax = abs(ox);
                            const double sx = ox < 0 ? -1.0 : 1.0;
                            const size_t t = ((size_t)az * ny + ay) * nx + ax;
                            double *r6 = row + 6 * (ox + nx - 1);
                            r6[0] = T[0][t]; r6[1] = T[1][t]; r6[2] = T[2][t];
                            r6[3] = sx * sy * T[3][t];
                            r6[4] = sx * sz * T[4][t];
                            r6[5] = sy * sz * T[5][t];
                        }
                        const size_t js = ((size_t)jz * ny + jy) * nx;
                        for (int ix = 0; ix < nx; ++ix) {
                            double hx = 0.0, hy = 0.0, hz = 0.0;
                            const double *rr = row + 6 * (ix + nx - 1); /* ox = ix - jx, jx = 0 */
                            for (int jx = 0; jx < nx; ++jx) {
                                const double *r6 = rr - 6 * jx;
                                const double mx = vx[js + jx], my = vy[js + jx], mz = vz[js + jx];
                                hx += r6[0] * mx + r6[3] * my + r6[4] * mz;
                                hy += r6[3] * mx + r6[1] * my + r6[5] * mz;
                                hz += r6[4] * mx + r6[5] * my + r6[2] * mz;
                            }
                            acc[ix] += hx; acc[nx + ix] += hy; acc[2 * nx + ix] += hz;
                        }
                    }
                const size_t is = ((size_t)iz * ny + iy) * nx;
                for (int ix = 0; ix < nx; ++ix) {
                    out[is + ix] = acc[ix];
                    out[N + is + ix] = acc[nx + ix];
                    out[2 * N + is + ix] = acc[2 * nx + ix];
                }
            }
        free(row);
        free(acc);
    }
}

/* H_demag at all cells. */
void orc_demag(const orc_problem *p, const double *m, double *H)
{
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    double *M = (double *)calloc(3 * N, sizeof(double));
    for (int c = 0; c < 3; ++c)
        for (size_t i = 0; i < N; ++i) M[c * N + i] = p->Ms[i] * m[c * N + i];
    orc_conv(p->nx, p->ny, p->nz, p->tab, M, H);
    for (size_t i = 0; i < 3 * N; ++i) H[i] = -H[i];
    free(M);
}

/* H_demag at a list of observer cells only (linear cell indices), against
 * every source cell: out[3][nobs]. */
void orc_demag_observers(const orc_problem *p, const double *m,
                         const int64_t *obs, int64_t nobs, double *out)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t N = (size_t)nx * ny * nz;
    const double *T[6];
    for (int c = 0; c < 6; ++c) T[c] = p->tab + c * N;
#pragma omp parallel for schedule(dynamic)
    for (int64_t q = 0; q < nobs; ++q) {
        const int64_t i = obs[q];
        const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((int64_t)nx * ny));
        double hx = 0.0, hy = 0.0, hz = 0.0;
        for (int jz = 0; jz < nz; ++jz)
            for (int jy = 0; jy < ny; ++jy) {
                const int oz = iz - jz, oy = iy - jy;
                const double sy = oy < 0 ? -1.0 : 1.0, sz = oz < 0 ? -1.0 : 1.0;
                const size_t tb = ((size_t)abs(oz) * ny + abs(oy)) * nx;
                const size_t js = ((size_t)jz * ny + jy) * nx;
                for (int jx = 0; jx < nx; ++jx) {
                    const int ox = ix - jx;
                    const double sx = ox < 0 ? -1.0 : 1.0;
                    const size_t t = tb + (size_t)abs(ox);
                    const double Mx = p->Ms[js + jx] * m[js + jx];
                    const double My = p->Ms[js + jx] * m[N + js + jx];
                    const double Mz = p->Ms[js + jx] * m[2 * N + js + jx];
                    const double nxy = sx * sy * T[3][t], nxz = sx * sz * T[4][t], nyz = sy * sz * T[5][t];
                    hx += T[0][t] * Mx + nxy * My + nxz * Mz;
                    hy += nxy * Mx + T[1][t] * My + nyz * Mz;
                    hz += nxz * Mx + nyz * My + T[2][t] * Mz;
                }
            }
        out[q] = -hx; out[nobs + q] = -hy; out[2 * nobs + q] = -hz;
    }
}

/* ------------------------------------------------------------------------ */
/* One Euler step evaluated at a list of cells only (every source still      */
/* enters the demag sum): out[3][nobs] is the updated m at those cells.      */
/* Used to time the oracle on a bounded sample of a large workload.          */
/* ------------------------------------------------------------------------ */
static void cross3(const double a[3], const double b[3], double c[3]);

void orc_step_cells(const orc_problem *p, const double *m, const int64_t *obs, int64_t nobs,
                    double dt, double *out)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t N = (size_t)nx * ny * nz;
    double *Hd = (double *)calloc(3 * (size_t)nobs, sizeof(double));
    if (p->terms & ORC_T_DEMAG) orc_demag_observers(p, m, obs, nobs, Hd);
    const double c1 = -p->gamma0 / (1.0 + p->alpha * p->alpha), c2 = p->alpha * c1;
    const double cd[3] = {1.0 / (p->dx * p->dx), 1.0 / (p->dy * p->dy), 1.0 / (p->dz * p->dz)};
    for (int64_t q = 0; q < nobs; ++q) {
        const int64_t i = obs[q];
        const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((int64_t)nx * ny));
        const double mi[3] = {m[i], m[N + i], m[2 * N + i]};
        if (!magnetic(p, (size_t)i)) {  /* vacuum: unchanged */
            for (int c = 0; c < 3; ++c) out[c * nobs + q] = mi[c];
            continue;
        }
        double h[3] = {Hd[q], Hd[nobs + q], Hd[2 * nobs + q]};
        if (p->terms & ORC_T_EXCH) {
            const int coord[3] = {ix, iy, iz}, n[3] = {nx, ny, nz};
            const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
            const double k = 2.0 * p->A / (ORC_MU0 * p->Ms[i]);
            for (int a = 0; a < 3; ++a)
                for (int s = -1; s <= 1; s += 2) {
                    const int cc = coord[a] + s;
                    if (cc < 0 || cc >= n[a]) continue;
                    const int64_t j = i + s * stride[a];
                    if (!magnetic(p, (size_t)j)) continue;
                    for (int c = 0; c < 3; ++c) h[c] += k * cd[a] * (m[c * N + j] - mi[c]);
                }
        }
        if (p->terms & ORC_T_ANIS) {
            const double mu = mi[0] * p->u[0] + mi[1] * p->u[1] + mi[2] * p->u[2];
            for (int c = 0; c < 3; ++c) h[c] += 2.0 * p->Ku / (ORC_MU0 * p->Ms[i]) * mu * p->u[c];
        }
        if (p->terms & ORC_T_ZEEMAN)
            for (int c = 0; c < 3; ++c) h[c] += p->hext[c * N + i];
        double mxh[3], mxmxh[3], v[3];
        cross3(mi, h, mxh);
        cross3(mi, mxh, mxmxh);
        for (int c = 0; c < 3; ++c) v[c] = mi[c] + dt * (c1 * mxh[c] + c2 * mxmxh[c]);
        double nrm = 1.0;
        if (p->renorm) nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int c = 0; c < 3; ++c) out[c * nobs + q] = v[c] / nrm;
    }
    free(Hd);
}

/* number of OpenMP threads the oracle runs with */
int orc_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Local field terms.                                                        */
/* ------------------------------------------------------------------------ */

/* Neumann six-neighbour Laplacian: (L v)_i = sum_d sum_{s=+-1, inside}
 * (v_{i+s e_d} - v_i) / d_d^2, applied per component. */
void orc_laplacian(int nx, int ny, int nz, double dx, double dy, double dz,
                   const double *v, double *out)
{
    const size_t N = (size_t)nx * ny * nz;
    const double cx = 1.0 / (dx * dx), cy = 1.0 / (dy * dy), cz = 1.0 / (dz * dz);
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < 3; ++c)
        for (int iz = 0; iz < nz; ++iz)
            for (int iy = 0; iy < ny; ++iy)
                for (int ix = 0; ix < nx; ++ix) {
                    const size_t i = c * N + ((size_t)iz * ny + iy) * nx + ix;
                    const double vi = v[i];
                    double s = 0.0;
                    if (ix > 0) s += cx * (v[i - 1] - vi);
                    if (ix < nx - 1) s += cx * (v[i + 1] - vi);
                    if (iy > 0) s += cy * (v[i - nx] - vi);
                    if (iy < ny - 1) s += cy * (v[i + nx] - vi);
                    if (iz > 0) s += cz * (v[i - (size_t)nx * ny] - vi);
                    if (iz < nz - 1) s += cz * (v[i + (size_t)nx * ny] - vi);
                    out[i] = s;
                }
}

/* Non-regular geometry (named as future work in Sec. 6): a cell with      */
/* Ms = 0 is vacuum.  It is no demag source (M = Ms m = 0); exchange omits   */
/* vacuum neighbours, a free surface like the sample boundary; exchange and  */
/* anisotropy fields are zero in vacuum (demag and Zeeman fields exist       */
/* there); its m is never updated; energies skip it.                         */

/* Six-neighbour Laplacian over magnetic cells: missing and vacuum          */
/* neighbours are omitted; zero at vacuum cells.  Equals orc_laplacian when   */
/* every cell is magnetic.                                                   */
static void laplacian_magnetic(const orc_problem *p, const double *v, double *out)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t N = (size_t)nx * ny * nz, sy = (size_t)nx, sz = (size_t)nx * ny;
    const double cx = 1.0 / (p->dx * p->dx), cy = 1.0 / (p->dy * p->dy), cz = 1.0 / (p->dz * p->dz);
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < 3; ++c)
        for (int iz = 0; iz < nz; ++iz)
            for (int iy = 0; iy < ny; ++iy)
                for (int ix = 0; ix < nx; ++ix) {
                    const size_t j = ((size_t)iz * ny + iy) * nx + ix, i = c * N + j;
                    double s = 0.0;
                    if (magnetic(p, j)) {
                        const double vi = v[i];
                        if (ix > 0 && magnetic(p, j - 1)) s += cx * (v[i - 1] - vi);
                        if (ix < nx - 1 && magnetic(p, j + 1)) s += cx * (v[i + 1] - vi);
                        if (iy > 0 && magnetic(p, j - sy)) s += cy * (v[i - sy] - vi);
                        if (iy < ny - 1 && magnetic(p, j + sy)) s += cy * (v[i + sy] - vi);
                        if (iz > 0 && magnetic(p, j - sz)) s += cz * (v[i - sz] - vi);
                        if (iz < nz - 1 && magnetic(p, j + sz)) s += cz * (v[i + sz] - vi);
                    }
                    out[i] = s;
                }
}

/* Effective field of eq. (2) restricted to the terms in the mask. */
void orc_heff(const orc_problem *p, const double *m, int terms, double *H)
{
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    memset(H, 0, sizeof(double) * 3 * N);
    if (terms & ORC_T_DEMAG) orc_demag(p, m, H);
    if (terms & ORC_T_EXCH) {
        double *L = (double *)malloc(sizeof(double) * 3 * N);
        laplacian_magnetic(p, m, L);
        for (int c = 0; c < 3; ++c)
            for (size_t i = 0; i < N; ++i)
                if (magnetic(p, i)) H[c * N + i] += 2.0 * p->A / (ORC_MU0 * p->Ms[i]) * L[c * N + i];
        free(L);
    }
    if (terms & ORC_T_ANIS) {
        for (size_t i = 0; i < N; ++i) {
            if (!magnetic(p, i)) continue;
            const double mu = m[i] * p->u[0] + m[N + i] * p->u[1] + m[2 * N + i] * p->u[2];
            const double k = 2.0 * p->Ku / (ORC_MU0 * p->Ms[i]) * mu;
            for (int c = 0; c < 3; ++c) H[c * N + i] += k * p->u[c];
        }
    }
    if (terms & ORC_T_ZEEMAN)
        for (size_t i = 0; i < 3 * N; ++i) H[i] += p->hext[i];
}

/* ------------------------------------------------------------------------ */
/* LLG, eq. (3), Landau-Lifshitz form for the unit vector m:                 */
/*   dm/dt = -gamma0/(1+alpha^2) [ m x H + alpha m x (m x H) ]               */
/* Explicit Euler with every term at time level n.                           */
/* ------------------------------------------------------------------------ */

static inline void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void cross3(const double a[3], const double b[3], double c[3]) { cross(a, b, c); }

void orc_llg_rhs(const orc_problem *p, const double *m, const double *H, double *f)
{
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    const double c1 = -p->gamma0 / (1.0 + p->alpha * p->alpha);
    const double c2 = p->alpha * c1;
    for (size_t i = 0; i < N; ++i) {
        if (!magnetic(p, i)) {  /* vacuum: m does not move */
            for (int c = 0; c < 3; ++c) f[c * N + i] = 0.0;
            continue;
        }
        const double mi[3] = {m[i], m[N + i], m[2 * N + i]};
        const double hi[3] = {H[i], H[N + i], H[2 * N + i]};
        double mxh[3], mxmxh[3];
        cross(mi, hi, mxh);
        cross(mi, mxh, mxmxh);
        for (int c = 0; c < 3; ++c) f[c * N + i] = c1 * mxh[c] + c2 * mxmxh[c];
    }
}

/* One Euler step in place; H (if non-NULL) receives the field used. */
void orc_step(const orc_problem *p, double *m, double dt, double *Hout)
{
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    double *H = Hout ? Hout : (double *)malloc(sizeof(double) * 3 * N);
    double *f = (double *)malloc(sizeof(double) * 3 * N);
    orc_heff(p, m, p->terms, H);
    orc_llg_rhs(p, m, H, f);
    for (size_t i = 0; i < 3 * N; ++i) m[i] += dt * f[i];
    if (p->renorm)
        for (size_t i = 0; i < N; ++i) {
            if (!magnetic(p, i)) continue;
            const double n = sqrt(m[i] * m[i] + m[N + i] * m[N + i] + m[2 * N + i] * m[2 * N + i]);
            m[i] /= n; m[N + i] /= n; m[2 * N + i] /= n;
        }
    free(f);
    if (!Hout) free(H);
}

/* nsteps Euler steps starting from m (in place). traj, if non-NULL, receives
 * the nsteps+1 states [nsteps+1][3][N]. */
void orc_run(const orc_problem *p, double *m, int64_t nsteps, double dt, double *traj)
{
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    if (traj) memcpy(traj, m, sizeof(double) * 3 * N);
    for (int64_t s = 0; s < nsteps; ++s) {
        orc_step(p, m, dt, NULL);
        if (traj) memcpy(traj + (size_t)(s + 1) * 3 * N, m, sizeof(double) * 3 * N);
    }
}

/* ------------------------------------------------------------------------ */
/* Time-dependent external field.  The paper's input file (Sec. 5) gives the  */
/* field as Hx Hy Hz with a startTime, a decayTime and a stopTime and does    */
/* not define the profile between them.  Read here as: off before startTime, */
/* full strength from startTime to decayTime, a linear decay to zero between */
/* decayTime and stopTime, off from stopTime on.  The profile multiplies the */
/* whole external field (uniform or per cell).  Times are absolute, in       */
/* seconds; step n of an Euler run evaluates its field at t_n, with          */
/* t_{n+1} = t_n + dt accumulated in FP64.                                   */
/* ------------------------------------------------------------------------ */
double orc_field_scale(double t, double t_start, double t_decay, double t_stop)
{
    if (t < t_start) return 0.0;
    if (t <= t_decay) return 1.0;
    if (t >= t_stop) return 0.0;
    return (t_stop - t) / (t_stop - t_decay);
}

/* nsteps Euler steps from m (in place) with the external field of p scaled
 * by the profile above at each step's start time; t0 is the time of the
 * first step.  Returns the time after the last step. */
double orc_run_scheduled(const orc_problem *p, double *m, int64_t nsteps, double dt, double t0,
                         double t_start, double t_decay, double t_stop)
{
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    double *h = (double *)malloc(sizeof(double) * 3 * N);
    orc_problem q = *p;
    q.hext = h;
    double t = t0;
    for (int64_t s = 0; s < nsteps; ++s) {
        const double sc = orc_field_scale(t, t_start, t_decay, t_stop);
        for (size_t i = 0; i < 3 * N; ++i) h[i] = sc * p->hext[i];
        orc_step(&q, m, dt, NULL);
        t += dt;
    }
    free(h);
    return t;
}

/* Loss of a final state against a target: 1/2 sum over all 3N components of
 * (m - t)^2 (the mismatch the gradient of the rollout is taken for). */
double orc_loss(const double *m, const double *t, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double d = m[i] - t[i];
        s += d * d;
    }
    return 0.5 * s;
}

/* ------------------------------------------------------------------------ */
/* Explicit Runge-Kutta steps of the same right-hand side f (fixed-step     */
/* members of the Runge-Kutta family that adaptive time steps, named as      */
/* future work in Sec. 6, build on).  With the Butcher tableau (A, b) of s   */
/* stages:                                                                   */
/*   m_1 = m,   m_i = P(m + dt sum_{j<i} A[i][j] k_j),   k_i = f(m_i, H(m_i))  */
/*   m'  = P(m + dt sum_i b[i] k_i)                                          */
/* P renormalises every cell when renorm is on, the identity otherwise: the  */
/* stage states are unit vectors like the step result.                       */
/*   method 1, Heun (explicit trapezoidal rule, order 2):                    */
/*     A[1][0] = 1;  b = (1/2, 1/2)                                          */
/*   method 2, classic fourth-order Runge-Kutta:                             */
/*     A[1][0] = 1/2, A[2][1] = 1/2, A[3][2] = 1;  b = (1/6, 1/3, 1/3, 1/6)  */
/*   method 0 is the Euler step above.                                       */
/* ------------------------------------------------------------------------ */
static void renormalise(const orc_problem *p, double *m, size_t N)
{
    if (!p->renorm) return;
    for (size_t i = 0; i < N; ++i) {
        if (!magnetic(p, i)) continue;
        const double n = sqrt(m[i] * m[i] + m[N + i] * m[N + i] + m[2 * N + i] * m[2 * N + i]);
        m[i] /= n; m[N + i] /= n; m[2 * N + i] /= n;
    }
}

int orc_step_rk(const orc_problem *p, double *m, double dt, int method)
{
    if (method == 0) {
        orc_step(p, m, dt, NULL);
        return 0;
    }
    double A[4][4] = {{0}}, b[4] = {0};
    int s;
    if (method == 1) {
        s = 2;
        A[1][0] = 1.0;
        b[0] = 0.5; b[1] = 0.5;
    } else if (method == 2) {
        s = 4;
        A[1][0] = 0.5; A[2][1] = 0.5; A[3][2] = 1.0;
        b[0] = 1.0 / 6.0; b[1] = 1.0 / 3.0; b[2] = 1.0 / 3.0; b[3] = 1.0 / 6.0;
    } else {
        return -1;
    }
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    double *k = (double *)malloc(sizeof(double) * 3 * N * s);
    double *mi = (double *)malloc(sizeof(double) * 3 * N);
    double *H = (double *)malloc(sizeof(double) * 3 * N);
    for (int i = 0; i < s; ++i) {
        for (size_t e = 0; e < 3 * N; ++e) {
            double acc = 0.0;
            for (int j = 0; j < i; ++j) acc += A[i][j] * k[(size_t)j * 3 * N + e];
            mi[e] = m[e] + dt * acc;
        }
        if (i > 0) renormalise(p, mi, N);
        orc_heff(p, mi, p->terms, H);
        orc_llg_rhs(p, mi, H, k + (size_t)i * 3 * N);
    }
    for (size_t e = 0; e < 3 * N; ++e) {
        double acc = 0.0;
        for (int i = 0; i < s; ++i) acc += b[i] * k[(size_t)i * 3 * N + e];
        m[e] += dt * acc;
    }
    renormalise(p, m, N);
    free(k);
    free(mi);
    free(H);
    return 0;
}

/* nsteps steps of the given method (0 Euler, 1 Heun, 2 RK4) from m, in place. */
int orc_run_rk(const orc_problem *p, double *m, int64_t nsteps, double dt, int method)
{
    for (int64_t s = 0; s < nsteps; ++s)
        if (orc_step_rk(p, m, dt, method)) return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adaptive time steps (named as future work in Sec. 6) with an embedded     */
/* Runge-Kutta pair: the step advances with the higher-order result          */
/*   m' = P(m + dt sum_i b[i] k_i)                                           */
/* and estimates its local error from the lower-order one,                    */
/*   err = max over cells of | dt sum_i (b[i] - bh[i]) k_i |                  */
/* (unprojected sums; for pair 2 the last k is f at m', so b has 0 there).   */
/* A step is accepted when err <= tol.  Accepted or not, the next step is    */
/*   dt <- dt min(5, max(0.2, 0.9 (tol/err)^(1/(q+1))))   (5 when err = 0),  */
/* q the order of the lower method, and the step that would pass t_end is    */
/* shortened to end there.                                                   */
/*   pair 1, Heun with embedded Euler, order 2(1):                           */
/*     A[1][0] = 1;  b = (1/2, 1/2);  bh = (1, 0)                            */
/*   pair 2, Bogacki-Shampine, order 3(2):                                   */
/*     A[1][0] = 1/2, A[2][1] = 3/4;  b = (2/9, 1/3, 4/9, 0);                */
/*     bh = (7/24, 1/4, 1/3, 1/8), the fourth stage evaluated at m'          */
/*   pair 3, Dormand-Prince, order 5(4), seven stages, the seventh at m'     */
/*     (the published 1980 tableau, written out below).                      */
/* Returns 0, or -1 for an unknown pair, -2 when max_steps attempts do not   */
/* reach t_end.                                                              */
/* ------------------------------------------------------------------------ */
int orc_run_adaptive(const orc_problem *p, double *m, double t_end, double *dt_io, double tol, int pair,
                     int64_t max_steps, int64_t *accepted, int64_t *rejected)
{
    double A[7][7] = {{0}}, b[7] = {0}, bh[7] = {0};
    int s, q;
    if (pair == 1) {
        s = 2; q = 1;
        A[1][0] = 1.0;
        b[0] = 0.5; b[1] = 0.5;
        bh[0] = 1.0;
    } else if (pair == 2) {
        s = 4; q = 2;
        A[1][0] = 0.5; A[2][1] = 0.75;
        b[0] = 2.0 / 9.0; b[1] = 1.0 / 3.0; b[2] = 4.0 / 9.0;
        bh[0] = 7.0 / 24.0; bh[1] = 0.25; bh[2] = 1.0 / 3.0; bh[3] = 0.125;
    } else if (pair == 3) {
        s = 7; q = 4;
        A[1][0] = 1.0 / 5.0;
        A[2][0] = 3.0 / 40.0; A[2][1] = 9.0 / 40.0;
        A[3][0] = 44.0 / 45.0; A[3][1] = -56.0 / 15.0; A[3][2] = 32.0 / 9.0;
        A[4][0] = 19372.0 / 6561.0; A[4][1] = -25360.0 / 2187.0; A[4][2] = 64448.0 / 6561.0;
        A[4][3] = -212.0 / 729.0;
        A[5][0] = 9017.0 / 3168.0; A[5][1] = -355.0 / 33.0; A[5][2] = 46732.0 / 5247.0;
        A[5][3] = 49.0 / 176.0; A[5][4] = -5103.0 / 18656.0;
        b[0] = 35.0 / 384.0; b[2] = 500.0 / 1113.0; b[3] = 125.0 / 192.0;
        b[4] = -2187.0 / 6784.0; b[5] = 11.0 / 84.0;
        bh[0] = 5179.0 / 57600.0; bh[2] = 7571.0 / 16695.0; bh[3] = 393.0 / 640.0;
        bh[4] = -92097.0 / 339200.0; bh[5] = 187.0 / 2100.0; bh[6] = 1.0 / 40.0;
    } else {
        return -1;
    }
    /* pairs 2 and 3: the stages before the last build m', the last is f(m') */
    const int sres = pair >= 2 ? s - 1 : s;
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    double *k = (double *)malloc(sizeof(double) * 3 * N * s);
    double *mi = (double *)malloc(sizeof(double) * 3 * N);
    double *mn = (double *)malloc(sizeof(double) * 3 * N);
    double *H = (double *)malloc(sizeof(double) * 3 * N);
    double t = 0.0, dt = *dt_io;
    int64_t acc = 0, rej = 0;
    int status = 0;
    while (t < t_end) {
        if (acc + rej >= max_steps) { status = -2; break; }
        const double h = (t + dt > t_end) ? t_end - t : dt;
        for (int i = 0; i < sres; ++i) {
            for (size_t e = 0; e < 3 * N; ++e) {
                double a = 0.0;
                for (int j = 0; j < i; ++j) a += A[i][j] * k[(size_t)j * 3 * N + e];
                mi[e] = m[e] + h * a;
            }
            if (i > 0) renormalise(p, mi, N);
            orc_heff(p, mi, p->terms, H);
            orc_llg_rhs(p, mi, H, k + (size_t)i * 3 * N);
        }
        for (size_t e = 0; e < 3 * N; ++e) {
            double a = 0.0;
            for (int i = 0; i < sres; ++i) a += b[i] * k[(size_t)i * 3 * N + e];
            mn[e] = m[e] + h * a;
        }
        renormalise(p, mn, N);
        if (pair >= 2) {
            orc_heff(p, mn, p->terms, H);
            orc_llg_rhs(p, mn, H, k + (size_t)(s - 1) * 3 * N);
        }
        double err = 0.0;
        for (size_t i = 0; i < N; ++i) {
            double e2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                double a = 0.0;
                for (int j = 0; j < s; ++j) a += (b[j] - bh[j]) * k[(size_t)j * 3 * N + c * N + i];
                e2 += (h * a) * (h * a);
            }
            const double e = sqrt(e2);
            if (!(e <= err)) err = e;  /* NaN propagates */
        }
        if (err != err) { status = -3; break; }
        if (err <= tol) {
            memcpy(m, mn, sizeof(double) * 3 * N);
            t += h;
            ++acc;
        } else {
            ++rej;
        }
        double f = err > 0.0 ? 0.9 * pow(tol / err, 1.0 / (q + 1)) : 5.0;
        if (f > 5.0) f = 5.0;
        if (f < 0.2) f = 0.2;
        dt = h * f;
    }
    *dt_io = dt;
    if (accepted) *accepted = acc;
    if (rejected) *rejected = rej;
    free(k); free(mi); free(mn); free(H);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Energy of eq. (1) summed over cells (volume V = dx dy dz):                */
/*   E_ex = A V sum_{neighbour pairs} |m_j - m_i|^2 / d^2                    */
/*   E_d  = -(mu0 V / 2) sum Ms_i m_i . H_d,i                                */
/*   E_an = Ku V sum (1 - (m_i . u)^2)                                       */
/*   E_Z  = -mu0 V sum Ms_i m_i . h_ext,i                                    */
/* out = {E_ex, E_d, E_an, E_Z, E_total}; terms not in the mask are 0.       */
/* ------------------------------------------------------------------------ */
void orc_energy(const orc_problem *p, const double *m, double out[5])
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t N = (size_t)nx * ny * nz;
    const double V = p->dx * p->dy * p->dz;
    double eex = 0.0, ed = 0.0, ean = 0.0, ez = 0.0;
    if (p->terms & ORC_T_EXCH) {
        const double cx = 1.0 / (p->dx * p->dx), cy = 1.0 / (p->dy * p->dy), cz = 1.0 / (p->dz * p->dz);
        for (int c = 0; c < 3; ++c)
            for (int iz = 0; iz < nz; ++iz)
                for (int iy = 0; iy < ny; ++iy)
                    for (int ix = 0; ix < nx; ++ix) {
                        const size_t j = ((size_t)iz * ny + iy) * nx + ix, i = c * N + j;
                        const size_t sz = (size_t)nx * ny;
                        double d;
                        if (!magnetic(p, j)) continue;  /* pairs of two magnetic cells only */
                        if (ix < nx - 1 && magnetic(p, j + 1)) { d = m[i + 1] - m[i]; eex += cx * d * d; }
                        if (iy < ny - 1 && magnetic(p, j + nx)) { d = m[i + nx] - m[i]; eex += cy * d * d; }
                        if (iz < nz - 1 && magnetic(p, j + sz)) { d = m[i + sz] - m[i]; eex += cz * d * d; }
                    }
        eex *= p->A * V;
    }
    if (p->terms & ORC_T_DEMAG) {
        double *Hd = (double *)malloc(sizeof(double) * 3 * N);
        orc_demag(p, m, Hd);
        for (size_t i = 0; i < N; ++i)
            ed += p->Ms[i] * (m[i] * Hd[i] + m[N + i] * Hd[N + i] + m[2 * N + i] * Hd[2 * N + i]);
        ed *= -0.5 * ORC_MU0 * V;
        free(Hd);
    }
    if (p->terms & ORC_T_ANIS) {
        for (size_t i = 0; i < N; ++i) {
            if (!magnetic(p, i)) continue;
            const double mu = m[i] * p->u[0] + m[N + i] * p->u[1] + m[2 * N + i] * p->u[2];
            ean += 1.0 - mu * mu;
        }
        ean *= p->Ku * V;
    }
    if (p->terms & ORC_T_ZEEMAN) {
        for (size_t i = 0; i < N; ++i)
            ez += p->Ms[i] * (m[i] * p->hext[i] + m[N + i] * p->hext[N + i] + m[2 * N + i] * p->hext[2 * N + i]);
        ez *= -ORC_MU0 * V;
    }
    out[0] = eex; out[1] = ed; out[2] = ean; out[3] = ez;
    out[4] = eex + ed + ean + ez;
}

/* ------------------------------------------------------------------------ */
/* Exact discrete adjoint of the Euler rollout for                          */
/*   L = 1/2 sum_i |m_T,i - t_i|^2                                          */
/* with respect to m_0, the external-field map h_ext and the Ms map.        */
/* Per step (m = m_n, H = H(m_n), v = m + dt f, m' = v/|v|):                */
/*   w   = (lam' - (m'.lam') m') / |v|        (lam' if no renormalisation)  */
/*   g_H = dt [c1 (w x m) + c2 m x (m x w)]   (transpose of df/dH)          */
/*   lam = w + dt [c1 H x w + c2 ((m x H) x w + H x (w x m))]               */
/*         + (2A/mu0) L(g_H/Ms) - Ms (N*g_H) + (2Ku/(mu0 Ms)) (u.g_H) u     */
/*   dL/dh_ext += g_H                                                       */
/*   dL/dMs    += -m.(N*g_H) - (2A/(mu0 Ms^2)) (L m).g_H                    */
/*                - (2Ku/(mu0 Ms^2)) (m.u)(u.g_H)                           */
/* where c1 = -gamma0/(1+alpha^2), c2 = alpha c1, L is the symmetric        */
/* Neumann Laplacian and N* the (self-adjoint) demag convolution.           */
/* Returns the loss.                                                        */
/* ------------------------------------------------------------------------ */
double orc_adjoint(const orc_problem *p, const double *m0, int64_t nsteps, double dt,
                   const double *target, double *g_m0, double *g_hext, double *g_ms)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t N = (size_t)nx * ny * nz;
    const size_t S = 3 * N;
    double *traj = (double *)malloc(sizeof(double) * S * (size_t)(nsteps + 1));
    double *m = (double *)malloc(sizeof(double) * S);
    memcpy(m, m0, sizeof(double) * S);
    orc_run(p, m, nsteps, dt, traj);
    double loss = 0.0;
    double *lam = (double *)malloc(sizeof(double) * S);
    const double *mT = traj + (size_t)nsteps * S;
    for (size_t i = 0; i < S; ++i) {
        const double d = mT[i] - target[i];
        lam[i] = d;
        loss += 0.5 * d * d;
    }
    memset(g_hext, 0, sizeof(double) * S);
    memset(g_ms, 0, sizeof(double) * N);
    const double c1 = -p->gamma0 / (1.0 + p->alpha * p->alpha);
    const double c2 = p->alpha * c1;
    double *H = (double *)malloc(sizeof(double) * S);
    double *f = (double *)malloc(sizeof(double) * S);
    double *gH = (double *)malloc(sizeof(double) * S);
    double *tmp = (double *)malloc(sizeof(double) * S);
    double *conv = (double *)malloc(sizeof(double) * S);
    double *Lm = (double *)malloc(sizeof(double) * S);
    double *nl = (double *)malloc(sizeof(double) * S);
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const double *mn = traj + (size_t)s * S;
        const double *mp = traj + (size_t)(s + 1) * S;
        orc_heff(p, mn, p->terms, H);
        orc_llg_rhs(p, mn, H, f);
        /* w and g_H, and the local part of the new lambda */
        for (size_t i = 0; i < N; ++i) {
            const double a[3] = {mn[i], mn[N + i], mn[2 * N + i]};
            const double h[3] = {H[i], H[N + i], H[2 * N + i]};
            const double l[3] = {lam[i], lam[N + i], lam[2 * N + i]};
            double w[3];
            if (p->renorm) {
                double v[3], vn = 0.0;
                for (int c = 0; c < 3; ++c) { v[c] = a[c] + dt * f[c * N + i]; vn += v[c] * v[c]; }
                vn = sqrt(vn);
                const double mq[3] = {mp[i], mp[N + i], mp[2 * N + i]};
                const double dot = mq[0] * l[0] + mq[1] * l[1] + mq[2] * l[2];
                for (int c = 0; c < 3; ++c) w[c] = (l[c] - dot * mq[c]) / vn;
            } else {
                for (int c = 0; c < 3; ++c) w[c] = l[c];
            }
            double wxm[3], mxw[3], mxmxw[3], hxw[3], mxh[3], mxhxw[3], hxwxm[3];
            cross(w, a, wxm);
            cross(a, w, mxw);
            cross(a, mxw, mxmxw);
            cross(h, w, hxw);
            cross(a, h, mxh);
            cross(mxh, w, mxhxw);
            cross(h, wxm, hxwxm);
            for (int c = 0; c < 3; ++c) {
                gH[c * N + i] = dt * (c1 * wxm[c] + c2 * mxmxw[c]);
                nl[c * N + i] = w[c] + dt * (c1 * hxw[c] + c2 * (mxhxw[c] + hxwxm[c]));
            }
        }
        for (size_t i = 0; i < S; ++i) g_hext[i] += (p->terms & ORC_T_ZEEMAN) ? gH[i] : 0.0;
        if (p->terms & ORC_T_EXCH) {
            for (int c = 0; c < 3; ++c)
                for (size_t i = 0; i < N; ++i) tmp[c * N + i] = gH[c * N + i] / p->Ms[i];
            orc_laplacian(nx, ny, nz, p->dx, p->dy, p->dz, tmp, conv);
            for (size_t i = 0; i < S; ++i) nl[i] += 2.0 * p->A / ORC_MU0 * conv[i];
            orc_laplacian(nx, ny, nz, p->dx, p->dy, p->dz, mn, Lm);
            for (size_t i = 0; i < N; ++i) {
                const double dot = Lm[i] * gH[i] + Lm[N + i] * gH[N + i] + Lm[2 * N + i] * gH[2 * N + i];
                g_ms[i] -= 2.0 * p->A / (ORC_MU0 * p->Ms[i] * p->Ms[i]) * dot;
            }
        }
        if (p->terms & ORC_T_DEMAG) {
            orc_conv(nx, ny, nz, p->tab, gH, conv);
            for (size_t i = 0; i < N; ++i) {
                double dot = 0.0;
                for (int c = 0; c < 3; ++c) {
                    nl[c * N + i] -= p->Ms[i] * conv[c * N + i];
                    dot += mn[c * N + i] * conv[c * N + i];
                }
                g_ms[i] -= dot;
            }
        }
        if (p->terms & ORC_T_ANIS) {
            for (size_t i = 0; i < N; ++i) {
                const double ug = p->u[0] * gH[i] + p->u[1] * gH[N + i] + p->u[2] * gH[2 * N + i];
                const double mu = p->u[0] * mn[i] + p->u[1] * mn[N + i] + p->u[2] * mn[2 * N + i];
                const double k = 2.0 * p->Ku / (ORC_MU0 * p->Ms[i]);
                for (int c = 0; c < 3; ++c) nl[c * N + i] += k * ug * p->u[c];
                g_ms[i] -= k / p->Ms[i] * mu * ug;
            }
        }
        memcpy(lam, nl, sizeof(double) * S);
    }
    memcpy(g_m0, lam, sizeof(double) * S);
    free(traj); free(m); free(lam); free(H); free(f); free(gH); free(tmp);
    free(conv); free(Lm); free(nl);
    return loss;
}
