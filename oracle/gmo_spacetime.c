/*
 * gmo_spacetime.c -- oracle: metrics, Christoffel symbols and orthonormal
 * fluid-frame tetrads.  TEST INFRASTRUCTURE (see gmo.h).
 *
 * Minkowski-Cartesian: x = (t, x, y, z) in units of ell, g = diag(-1,1,1,1).
 *
 * Kerr-Schild in modified coordinates (the GRMHD grid of the paper's GRMHD
 * test section): x = (t, x1, x2, x3) with r = exp(x1),
 * theta = pi x2 + (1-h)/2 sin(2 pi x2), phi = x3, M = 1 (ell = r_g).
 * The KS line element is
 *   ds^2 = -(1-z)dt^2 + 2z dt dr + (1+z)dr^2 + S dth^2
 *          + sin^2th [S + a^2 (1+z) sin^2th] dph^2
 *          - 2 a z sin^2th dt dph - 2 a (1+z) sin^2th dr dph,
 *   S = r^2 + a^2 cos^2th, z = 2r/S,
 * and the modified-coordinate metric is g_mn = g^KS_mn (dX^m/dx^m)(dX^n/dx^n)
 * with the diagonal Jacobian (1, r, dth/dx2, 1).
 * Flat spherical (the sphere tests of the paper, coordinates t, ln r, theta,
 * phi): the Minkowski line element in spherical coordinates,
 *   ds^2 = -dt^2 + dr^2 + r^2 dth^2 + r^2 sin^2th dph^2,
 * with the same diagonal Jacobian (1, r, dth/dx2, 1).
 * Christoffel symbols come from the definition
 *   Gamma^m_ab = 1/2 g^mn (d_a g_nb + d_b g_na - d_n g_ab)
 * with the metric derivatives taken by complex-step differentiation
 * (d f/dx = Im f(x + i h)/h, exact to rounding for analytic f) and g^mn by
 * Gauss-Jordan inversion.  Pinned by g g^-1 = I, sqrt(-g) = S sin(th) r dth/dx2,
 * the Schwarzschild limit and geodesic invariants (test_oracle_spacetime.py).
 */
#include "gmo_internal.h"

#include <complex.h>
#include <math.h>
#include <string.h>

double gmo_r_of_x1(const gmo_grid *g, double x1) { (void)g; return exp(x1); }

double gmo_th_of_x2(const gmo_grid *g, double x2)
{
    return M_PI * x2 + 0.5 * (1.0 - g->h_slope) * sin(2.0 * M_PI * x2);
}

static void ks_mks_gcov_c(double a, double hs, double complex x1, double complex x2,
                          double complex gm[4][4])
{
    double complex r = cexp(x1);
    double complex th = M_PI * x2 + 0.5 * (1.0 - hs) * csin(2.0 * M_PI * x2);
    double complex dth = M_PI * (1.0 + (1.0 - hs) * ccos(2.0 * M_PI * x2));
    double complex c = ccos(th), s = csin(th);
    double complex s2 = s * s;
    double complex S = r * r + a * a * c * c;
    double complex z = 2.0 * r / S;
    double complex gk[4][4];
    memset(gk, 0, sizeof(gk));
    gk[0][0] = -(1.0 - z);
    gk[0][1] = gk[1][0] = z;
    gk[0][3] = gk[3][0] = -a * z * s2;
    gk[1][1] = 1.0 + z;
    gk[1][3] = gk[3][1] = -a * (1.0 + z) * s2;
    gk[2][2] = S;
    gk[3][3] = s2 * (S + a * a * (1.0 + z) * s2);
    double complex J[4] = {1.0, r, dth, 1.0};
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n)
            gm[m][n] = gk[m][n] * J[m] * J[n];
}

static void sph_gcov_c(double hs, double complex x1, double complex x2, double complex gm[4][4])
{
    double complex r = cexp(x1);
    double complex th = M_PI * x2 + 0.5 * (1.0 - hs) * csin(2.0 * M_PI * x2);
    double complex dth = M_PI * (1.0 + (1.0 - hs) * ccos(2.0 * M_PI * x2));
    double complex s = csin(th);
    memset(gm, 0, 16 * sizeof(double complex));
    gm[0][0] = -1.0;
    gm[1][1] = r * r;                    /* dr^2 with dr = r dx1 */
    gm[2][2] = r * r * dth * dth;
    gm[3][3] = r * r * s * s;
}

/* Metric of the curved-coordinate grids at complex (x1, x2). */
static void gcov_c(const gmo_grid *grid, double complex x1, double complex x2, double complex gm[4][4])
{
    if (grid->metric == GMO_METRIC_FLAT_SPH) sph_gcov_c(grid->h_slope, x1, x2, gm);
    else ks_mks_gcov_c(grid->a_spin, grid->h_slope, x1, x2, gm);
}

void gmo_gcov(const gmo_grid *grid, const double x[4], double gcov[4][4])
{
    memset(gcov, 0, 16 * sizeof(double));
    if (grid->metric == GMO_METRIC_MINKOWSKI_CART) {
        gcov[0][0] = -1.0; gcov[1][1] = gcov[2][2] = gcov[3][3] = 1.0;
        return;
    }
    double complex gm[4][4];
    gcov_c(grid, x[1], x[2], gm);
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) gcov[m][n] = creal(gm[m][n]);
}

/* Gauss-Jordan inverse with partial pivoting. */
static void invert4(const double A[4][4], double Ai[4][4])
{
    double M[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) M[i][j] = (j < 4) ? A[i][j] : (j - 4 == i ? 1.0 : 0.0);
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int i = col + 1; i < 4; ++i)
            if (fabs(M[i][col]) > fabs(M[piv][col])) piv = i;
        if (piv != col)
            for (int j = 0; j < 8; ++j) { double t = M[col][j]; M[col][j] = M[piv][j]; M[piv][j] = t; }
        double d = M[col][col];
        for (int j = 0; j < 8; ++j) M[col][j] /= d;
        for (int i = 0; i < 4; ++i) {
            if (i == col) continue;
            double f = M[i][col];
            for (int j = 0; j < 8; ++j) M[i][j] -= f * M[col][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) Ai[i][j] = M[i][j + 4];
}

void gmo_gcon(const gmo_grid *grid, const double x[4], double gcon[4][4])
{
    double g[4][4];
    gmo_gcov(grid, x, g);
    invert4(g, gcon);
}

double gmo_sqrt_neg_g(const gmo_grid *grid, const double x[4])
{
    if (grid->metric == GMO_METRIC_MINKOWSKI_CART) return 1.0;
    double g[4][4];
    gmo_gcov(grid, x, g);
    /* determinant by elimination on a copy */
    double M[4][4];
    memcpy(M, g, sizeof(M));
    double det = 1.0;
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int i = col + 1; i < 4; ++i)
            if (fabs(M[i][col]) > fabs(M[piv][col])) piv = i;
        if (piv != col) {
            for (int j = 0; j < 4; ++j) { double t = M[col][j]; M[col][j] = M[piv][j]; M[piv][j] = t; }
            det = -det;
        }
        det *= M[col][col];
        for (int i = col + 1; i < 4; ++i) {
            double f = M[i][col] / M[col][col];
            for (int j = col; j < 4; ++j) M[i][j] -= f * M[col][j];
        }
    }
    return sqrt(-det);
}

void gmo_christoffel(const gmo_grid *grid, const double x[4], double Gam[4][4][4])
{
    memset(Gam, 0, 64 * sizeof(double));
    if (grid->metric == GMO_METRIC_MINKOWSKI_CART) return;
    double dg[4][4][4];            /* dg[c][a][b] = d_c g_ab */
    memset(dg, 0, sizeof(dg));
    const double hstep = 1e-30;
    for (int c = 1; c <= 2; ++c) {
        double complex x1 = x[1], x2 = x[2];
        if (c == 1) x1 += I * hstep; else x2 += I * hstep;
        double complex gm[4][4];
        gcov_c(grid, x1, x2, gm);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) dg[c][a][b] = cimag(gm[a][b]) / hstep;
    }
    double gcon[4][4];
    gmo_gcon(grid, x, gcon);
    for (int m = 0; m < 4; ++m)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double s = 0.0;
                for (int n = 0; n < 4; ++n)
                    s += gcon[m][n] * (dg[a][n][b] + dg[b][n][a] - dg[n][a][b]);
                Gam[m][a][b] = 0.5 * s;
            }
}
