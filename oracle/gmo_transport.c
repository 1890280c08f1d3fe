/*
 * gmo_transport.c -- oracle: the superphoton Monte Carlo method itself,
 * one photon at a time.  TEST INFRASTRUCTURE (see gmo.h).
 *
 *  make:  weight table (eq:weight_calc), per-zone expected counts and
 *         stochastic rounding (Sampling procedure section);
 *  birth: position, frequency and direction by rejection (Sampling
 *         procedure section), fluid-frame tetrad, wavevector;
 *  step:  velocity Verlet with iterated corrector (geodesic section,
 *         eq:predicted_wavevector, eq:calculated_wavevector), absorption
 *         weighting with the trapezoid optical depth (eq:weight_absorption,
 *         eq:abs_optdepth), biased scattering with weight split and a
 *         child superphoton (Scattering section);
 *  tally: (frequency, inclination) bins at escape.
 *
 * Descendants of each root are processed depth-first from an explicit
 * stack.  Random streams are keyed by photon identity, so the processing
 * order does not change any photon's history.
 */
#include "gmo_internal.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MEC2 (GMO_ME * GMO_CL * GMO_CL)

static __thread char g_err[256];
void gmo_set_error(const char *msg) { snprintf(g_err, sizeof(g_err), "%s", msg); }
const char *gmo_last_error(void) { return g_err; }

struct gmo_ctx {
    gmo_grid grid;
    int nz;
    double *n_e, *theta, *B, *ucon, *bcon;   /* copies of the inputs          */
    double *A, *nu_c, *vol;                   /* per-zone emission constants   */
    int *emits;                               /* zone takes part in emission   */
    /* last make */
    int made;
    gmo_emit_params ep;
    double lnnu_min, lnnu_span;               /* ln nu_min, ln(nu_max/nu_min)  */
    double *w_node, *ln_w;                    /* [n_wnodes]                    */
    uint32_t *count;
    double *nbar, *fmax;
    uint64_t *offset;                         /* [nz+1] exclusive prefix       */
    /* hot cross-section table, built on first use */
    double *sh;
    /* electrons: thermal, or the power law with its angular factor and its
     * hot cross-section table (ln sigma/sigma_T on the thermal table's eps
     * nodes), built on first use */
    gmo_dist dist;
    double pl_ang;
    double *shpl;
    /* accumulators */
    int n_nu, n_theta;
    double *spec;
    double ledger[GMO_L_N];
    int64_t stats[GMO_S_N];
    /* per-zone tables of the learned / adaptive forms */
    double *btab; int bt_n; double bt_lo, bt_hi;      /* bias, in ln eps       */
    double *mtab; int mt_n; double mt_lo, mt_hi;      /* emission, in ln nu    */
    /* event log and score weights */
    gmo_event_rec *ev_out; uint64_t ev_cap, ev_n, root_stride;
    double *sw; int sw_n;
};

gmo_ctx *gmo_create(void)
{
    gmo_ctx *c = (gmo_ctx *)calloc(1, sizeof(gmo_ctx));
    return c;
}

static void free_zones(gmo_ctx *c)
{
    free(c->n_e); free(c->theta); free(c->B); free(c->ucon); free(c->bcon);
    free(c->A); free(c->nu_c); free(c->vol); free(c->emits);
    free(c->w_node); free(c->ln_w); free(c->count); free(c->nbar); free(c->fmax); free(c->offset);
    c->n_e = c->theta = c->B = c->ucon = c->bcon = c->A = c->nu_c = c->vol = NULL;
    c->emits = NULL; c->w_node = c->ln_w = c->nbar = c->fmax = NULL; c->count = NULL; c->offset = NULL;
    c->made = 0;
}

void gmo_destroy(gmo_ctx *c)
{
    if (!c) return;
    free_zones(c);
    free(c->sh); free(c->shpl); free(c->spec); free(c->btab); free(c->mtab); free(c->sw);
    free(c);
}

/* ---------------------------------------------------------------------
 * Geometry helpers
 * ------------------------------------------------------------------- */
/* Kerr: outer horizon (M = 1); flat spherical coordinates: none (0). */
static double horizon_r(const gmo_grid *g)
{
    return g->metric == GMO_METRIC_KS_MKS ? 1.0 + sqrt(1.0 - g->a_spin * g->a_spin) : 0.0;
}

/* Grids in (ln r, x2, phi) coordinates: Kerr-Schild and flat spherical. */
static int spherical_grid(const gmo_grid *g) { return g->metric != GMO_METRIC_MINKOWSKI_CART; }

static double dot4(const double g[4][4], const double a[4], const double b[4])
{
    double s = 0.0;
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) s += g[m][n] * a[m] * b[n];
    return s;
}

/* Zone containing code point x, or -1 outside the grid (vacuum).
 * Cartesian: half-open boxes.  KS: x1 outside the grid is vacuum, x2 is
 * clamped into [0, n2-1], x3 is periodic. */
static int zone_of(const gmo_grid *g, const double x[4])
{
    int idx[3];
    for (int j = 0; j < 3; ++j) {
        double f = floor((x[j + 1] - g->x_start[j]) / g->dx[j]);
        if (g->metric == GMO_METRIC_MINKOWSKI_CART || j == 0) {
            if (f < 0.0 || f >= g->n[j]) return -1;
            idx[j] = (int)f;
        } else if (j == 1) {
            if (f < 0.0) f = 0.0;
            if (f > g->n[j] - 1) f = g->n[j] - 1;
            idx[j] = (int)f;
        } else {
            double m = fmod(f, (double)g->n[j]);
            if (m < 0.0) m += g->n[j];
            idx[j] = (int)m;
        }
    }
    return (idx[0] * g->n[1] + idx[1]) * g->n[2] + idx[2];
}

/* Normalised fluid velocity and unit field direction at a point (the zone
 * values are renormalised with the local metric, reading). */
static void fluid_frame(const gmo_ctx *c, int z, const double g[4][4], double u[4], double bh[4],
                        int *has_b)
{
    for (int m = 0; m < 4; ++m) { u[m] = c->ucon[m * c->nz + z]; bh[m] = c->bcon[m * c->nz + z]; }
    double uu = -dot4(g, u, u);
    double nu_ = sqrt(uu);
    for (int m = 0; m < 4; ++m) u[m] /= nu_;
    double bu = dot4(g, bh, u);
    for (int m = 0; m < 4; ++m) bh[m] += bu * u[m];
    double bb = dot4(g, bh, bh);
    *has_b = (bb > 0.0 && c->B[z] > 0.0);
    if (*has_b) {
        double nb = sqrt(bb);
        for (int m = 0; m < 4; ++m) bh[m] /= nb;
    } else {
        for (int m = 0; m < 4; ++m) bh[m] = 0.0;
    }
}

/* Gram-Schmidt of v against the orthonormal vectors e[0..ne-1] (e[0]
 * timelike).  Returns 0 when the residual norm^2 is below 1e-10 of the
 * original norm^2 (degenerate). */
static int gs_add(const double g[4][4], double e[4][4], int ne, const double vin[4])
{
    double v[4] = {vin[0], vin[1], vin[2], vin[3]};
    double n0 = fabs(dot4(g, v, v));
    for (int i = 0; i < ne; ++i) {
        double p = dot4(g, v, e[i]);
        double s = (i == 0) ? p : -p;      /* e0.e0 = -1, ei.ei = +1 */
        for (int m = 0; m < 4; ++m) v[m] += s * e[i][m];
    }
    double nn = dot4(g, v, v);
    if (!(nn > 1e-10 * n0) || !(nn > 0.0)) return 0;
    nn = sqrt(nn);
    for (int m = 0; m < 4; ++m) e[ne][m] = v[m] / nn;
    return 1;
}

static void basis_vec(int j, double v[4]) { v[0] = v[1] = v[2] = v[3] = 0.0; v[j] = 1.0; }

/* Emission tetrad: e0 = u, e3 = field direction, e1 and e2 from the
 * coordinate directions 1, 2, 3 in that order (reading). */
static void emission_tetrad(const double g[4][4], const double u[4], const double bh[4],
                            double e[4][4])
{
    double t[4][4];
    memcpy(t[0], u, sizeof(double) * 4);
    memcpy(t[1], bh, sizeof(double) * 4);
    int n = 2;
    for (int j = 1; j <= 3 && n < 4; ++j) {
        double v[4];
        basis_vec(j, v);
        n += gs_add(g, t, n, v);
    }
    /* order the frame as (u, e1, e2, b) */
    memcpy(e[0], t[0], sizeof(double) * 4);
    memcpy(e[1], t[2], sizeof(double) * 4);
    memcpy(e[2], t[3], sizeof(double) * 4);
    memcpy(e[3], t[1], sizeof(double) * 4);
}

/* Scattering tetrad by Gram-Schmidt (Scattering section): e0 = u, e1 the
 * photon's direction in the fluid frame -- k with its projection on u
 * removed, divided by its own norm (equal to the fluid-frame energy only
 * while k is exactly null; along an integrated path it is null to the
 * integrator's accuracy) -- e2 from the field direction (else coordinate 1,
 * 2, 3), e3 from the first coordinate direction that is not degenerate
 * (reading). */
static void scatter_tetrad(const double g[4][4], const double u[4], const double bh[4], int has_b,
                           const double k[4], double e[4][4], double *eps)
{
    memcpy(e[0], u, sizeof(double) * 4);
    double ep = -dot4(g, k, u);
    double v[4];
    for (int m = 0; m < 4; ++m) v[m] = k[m] - ep * u[m];
    double nv = sqrt(dot4(g, v, v));
    for (int m = 0; m < 4; ++m) e[1][m] = v[m] / nv;
    int n = 2;
    if (has_b) n += gs_add(g, e, n, bh);
    for (int j = 1; j <= 3 && n < 4; ++j) {
        double v[4];
        basis_vec(j, v);
        n += gs_add(g, e, n, v);
    }
    *eps = ep;
}

static double e_inf(const double g[4][4], const double k[4])
{
    double kt = 0.0;
    for (int n = 0; n < 4; ++n) kt += g[0][n] * k[n];
    return -kt;
}

/* ---------------------------------------------------------------------
 * Zone preparation and weight table (Creation of superphotons section,
 * eq:weight_calc; Sampling procedure section).
 * ------------------------------------------------------------------- */
int gmo_load_zones(gmo_ctx *c, const gmo_grid *grid, const gmo_zones *z)
{
    if (!c || !grid || !z) { gmo_set_error("null argument"); return GMO_EINVAL; }
    for (int j = 0; j < 3; ++j)
        if (grid->n[j] < 1 || !(grid->dx[j] > 0.0)) { gmo_set_error("bad grid"); return GMO_EINVAL; }
    if (grid->metric != GMO_METRIC_MINKOWSKI_CART && grid->metric != GMO_METRIC_KS_MKS &&
        !(grid->metric == GMO_METRIC_FLAT_SPH && grid->a_spin == 0.0)) {
        gmo_set_error("unknown metric"); return GMO_EINVAL;
    }
    const gmo_dist *dd = &z->dist;
    if (dd->kind != GMO_DIST_THERMAL &&
        !(dd->kind == GMO_DIST_POWERLAW && dd->p > 1.0 && dd->g1 >= 1.0 && dd->g2 > dd->g1 && isfinite(dd->g2))) {
        gmo_set_error("bad electron distribution"); return GMO_EINVAL;
    }
    free_zones(c);
    c->grid = *grid;
    if (c->shpl && (dd->kind != c->dist.kind || dd->p != c->dist.p || dd->g1 != c->dist.g1 || dd->g2 != c->dist.g2)) {
        free(c->shpl);
        c->shpl = NULL;
    }
    c->dist = *dd;
    c->pl_ang = dd->kind == GMO_DIST_POWERLAW ? gmo_pl_ang(dd->p) : 0.0;
    int nz = grid->n[0] * grid->n[1] * grid->n[2];
    c->nz = nz;
    c->n_e = malloc(sizeof(double) * nz); c->theta = malloc(sizeof(double) * nz);
    c->B = malloc(sizeof(double) * nz);
    c->ucon = malloc(sizeof(double) * 4 * nz); c->bcon = malloc(sizeof(double) * 4 * nz);
    c->A = malloc(sizeof(double) * nz); c->nu_c = malloc(sizeof(double) * nz);
    c->vol = malloc(sizeof(double) * nz); c->emits = malloc(sizeof(int) * nz);
    memcpy(c->n_e, z->n_e, sizeof(double) * nz);
    memcpy(c->theta, z->theta_e, sizeof(double) * nz);
    memcpy(c->B, z->B, sizeof(double) * nz);
    memcpy(c->ucon, z->ucon, sizeof(double) * 4 * nz);
    memcpy(c->bcon, z->bcon, sizeof(double) * 4 * nz);
    const double L3 = grid->L_unit_cm * grid->L_unit_cm * grid->L_unit_cm;
    const double rh = horizon_r(grid);
    for (int i = 0; i < nz; ++i) {
        if (c->n_e[i] > 0.0 && !(c->theta[i] > 0.0)) { gmo_set_error("n_e > 0 needs Theta_e > 0"); return GMO_EINVAL; }
        if (c->dist.kind == GMO_DIST_POWERLAW) {
            c->A[i] = gmo_pl_A(&c->dist, c->n_e[i], c->B[i]);
            c->nu_c[i] = gmo_pl_nu_c(c->B[i]);
        } else {
            c->A[i] = gmo_A_coef(c->n_e[i], c->theta[i], c->B[i]);
            c->nu_c[i] = gmo_nu_c(c->theta[i], c->B[i]);
        }
        int i3 = i % grid->n[2], i2 = (i / grid->n[2]) % grid->n[1], i1 = i / (grid->n[2] * grid->n[1]);
        double xc[4] = {0.0, grid->x_start[0] + (i1 + 0.5) * grid->dx[0],
                        grid->x_start[1] + (i2 + 0.5) * grid->dx[1],
                        grid->x_start[2] + (i3 + 0.5) * grid->dx[2]};
        c->vol[i] = gmo_sqrt_neg_g(grid, xc) * grid->dx[0] * grid->dx[1] * grid->dx[2] * L3;
        c->emits[i] = (c->A[i] > 0.0);
        /* Kerr: no emission from zones centred inside the horizon (reading) */
        if (spherical_grid(grid) && exp(xc[1]) < rh) c->emits[i] = 0;
    }
    return GMO_OK;
}

/* Shape g(X) and its angle integral G(X_c) of the loaded electrons. */
static double shape_g(const gmo_ctx *c, double X)
{
    return c->dist.kind == GMO_DIST_POWERLAW ? gmo_pl_g(X, c->dist.p) : gmo_g_of_X(X);
}

static double shape_G(const gmo_ctx *c, double Xc)
{
    return c->dist.kind == GMO_DIST_POWERLAW ? gmo_pl_g(Xc, c->dist.p) * c->pl_ang : gmo_G_of_Xc(Xc);
}

/* j at (nu, angle) in zone z; cos_th = cosine to the field. */
static double zone_j(const gmo_ctx *c, int z, double nu, double cos_th)
{
    if (c->A[z] == 0.0) return 0.0;
    double s2 = 1.0 - cos_th * cos_th;
    if (!(s2 > 0.0)) return 0.0;
    double s = sqrt(s2);
    return c->A[z] * s * shape_g(c, nu / (c->nu_c[z] * s));
}

static double zone_J(const gmo_ctx *c, int z, double nu)
{
    if (c->A[z] == 0.0) return 0.0;
    return 4.0 * M_PI * c->A[z] * shape_G(c, nu / c->nu_c[z]);
}

/* ln w at ln nu: linear between nodes (reading), clamped at the ends. */
static double ln_weight(const gmo_ctx *c, double lnnu)
{
    int n = c->ep.n_wnodes;
    double d = c->lnnu_span / (n - 1);
    double a = (lnnu - c->lnnu_min) / d;
    int i = (int)floor(a);
    if (i < 0) i = 0;
    if (i > n - 2) i = n - 2;
    double f = a - i;
    return (1.0 - f) * c->ln_w[i] + f * c->ln_w[i + 1];
}

/* Value of a per-zone table at log variable v: linear between the nodes,
 * the end node's value outside [lo, hi]. */
static double table_at(const double *tab, int n, double lo, double hi, int z, double v)
{
    const double *t = tab + (size_t)z * n;
    double pos = (v - lo) / (hi - lo) * (n - 1);
    if (pos <= 0.0) return t[0];
    if (pos >= n - 1) return t[n - 1];
    int i = (int)floor(pos);
    double f = pos - i;
    return t[i] + f * (t[i + 1] - t[i]);
}

/* ln w_i(nu) of zone z: the weight table lowered by the zone's emission
 * modulation, when one is set. */
static double ln_weight_zone(const gmo_ctx *c, int z, double lnnu)
{
    double lw = ln_weight(c, lnnu);
    if (c->mtab) lw -= table_at(c->mtab, c->mt_n, c->mt_lo, c->mt_hi, z, lnnu);
    return lw;
}

static int set_table(double **dst, int *dn, double *dlo, double *dhi, const gmo_ctx *c,
                     const double *tab, int n, double lo, double hi)
{
    if (!tab) { free(*dst); *dst = NULL; *dn = 0; return GMO_OK; }
    if (!c->n_e) { gmo_set_error("load zones first"); return GMO_ESTATE; }
    if (n < 2 || !(hi > lo)) { gmo_set_error("bad table shape"); return GMO_EINVAL; }
    size_t m = (size_t)c->nz * n;
    for (size_t i = 0; i < m; ++i)
        if (!isfinite(tab[i])) { gmo_set_error("table entry not finite"); return GMO_EINVAL; }
    free(*dst);
    *dst = malloc(sizeof(double) * m);
    memcpy(*dst, tab, sizeof(double) * m);
    *dn = n; *dlo = lo; *dhi = hi;
    return GMO_OK;
}

int gmo_set_bias_table(gmo_ctx *c, const double *tab, int n_nodes, double lo, double hi)
{
    return set_table(&c->btab, &c->bt_n, &c->bt_lo, &c->bt_hi, c, tab, n_nodes, lo, hi);
}

int gmo_set_emission_table(gmo_ctx *c, const double *tab, int n_nodes, double lo, double hi)
{
    return set_table(&c->mtab, &c->mt_n, &c->mt_lo, &c->mt_hi, c, tab, n_nodes, lo, hi);
}

double gmo_table_value(const gmo_ctx *c, int which, int zone, double v)
{
    if (which == 0) return c->btab ? table_at(c->btab, c->bt_n, c->bt_lo, c->bt_hi, zone, v) : NAN;
    return c->mtab ? table_at(c->mtab, c->mt_n, c->mt_lo, c->mt_hi, zone, v) : NAN;
}

int gmo_set_event_log(gmo_ctx *c, gmo_event_rec *buf, uint64_t cap, uint64_t root_stride)
{
    if (buf && (cap == 0 || root_stride == 0)) { gmo_set_error("bad event log"); return GMO_EINVAL; }
    c->ev_out = buf;
    c->ev_cap = buf ? cap : 0;
    c->ev_n = 0;
    c->root_stride = root_stride;
    return GMO_OK;
}

int gmo_event_count(const gmo_ctx *c, uint64_t *n)
{
    *n = c->ev_n;
    return GMO_OK;
}

int gmo_set_score_weights(gmo_ctx *c, const double *sw, int n)
{
    free(c->sw);
    c->sw = NULL;
    c->sw_n = 0;
    if (!sw) return GMO_OK;
    if (n < 1) { gmo_set_error("bad score weights"); return GMO_EINVAL; }
    c->sw = malloc(sizeof(double) * n);
    memcpy(c->sw, sw, sizeof(double) * n);
    c->sw_n = n;
    return GMO_OK;
}

int gmo_make_superphotons(gmo_ctx *c, const gmo_emit_params *p, uint64_t *n_made)
{
    if (!c || !c->n_e) { gmo_set_error("load zones first"); return GMO_ESTATE; }
    if (!(p->nu_max > p->nu_min) || !(p->nu_min > 0.0) || p->n_wnodes < 3 || !(p->n_wnodes & 1) ||
        !(p->n_target > 0.0) || p->w_floor_rel < 0.0) {
        gmo_set_error("bad emission parameters"); return GMO_EINVAL;
    }
    int nz = c->nz, nw = p->n_wnodes;
    c->ep = *p;
    c->lnnu_min = log(p->nu_min);
    c->lnnu_span = log(p->nu_max / p->nu_min);
    free(c->w_node); free(c->ln_w); free(c->count); free(c->nbar); free(c->fmax); free(c->offset);
    c->w_node = malloc(sizeof(double) * nw); c->ln_w = malloc(sizeof(double) * nw);
    c->count = malloc(sizeof(uint32_t) * nz); c->nbar = malloc(sizeof(double) * nz);
    c->fmax = malloc(sizeof(double) * nz); c->offset = malloc(sizeof(uint64_t) * (nz + 1));
    double *nu = malloc(sizeof(double) * nw);
    for (int k = 0; k < nw; ++k) nu[k] = exp(c->lnnu_min + c->lnnu_span * k / (nw - 1));

    /* J_i(nu_k) for every zone; G depends on nu_c only, so consecutive zones
     * with the same nu_c reuse it. */
    double *Jz = malloc(sizeof(double) * (size_t)nz * nw);
    #pragma omp parallel
    {
        double *Gk = malloc(sizeof(double) * nw);
        double last_nuc = -1.0;
        #pragma omp for schedule(dynamic, 64)
        for (int i = 0; i < nz; ++i) {
            if (!c->emits[i]) {
                for (int k = 0; k < nw; ++k) Jz[(size_t)i * nw + k] = 0.0;
                continue;
            }
            if (c->nu_c[i] != last_nuc) {
                for (int k = 0; k < nw; ++k) Gk[k] = shape_G(c, nu[k] / c->nu_c[i]);
                last_nuc = c->nu_c[i];
            }
            for (int k = 0; k < nw; ++k) Jz[(size_t)i * nw + k] = 4.0 * M_PI * c->A[i] * Gk[k];
        }
        free(Gk);
    }
    /* weight table: w(nu) = Delta t Delta(ln nu) / (h N_s) sum_i V_i J_i(nu),
     * Delta t = 1 s and Delta(ln nu) = ln(nu_max/nu_min) (reading), plus a
     * floor relative to the maximum. */
    double wmax = 0.0;
    for (int k = 0; k < nw; ++k) {
        double phi = 0.0;
        for (int i = 0; i < nz; ++i) phi += c->vol[i] * Jz[(size_t)i * nw + k];
        c->w_node[k] = phi * c->lnnu_span / (GMO_HPL * p->n_target);
        if (c->w_node[k] > wmax) wmax = c->w_node[k];
    }
    if (!(wmax > 0.0)) {
        free(Jz); free(nu);
        gmo_set_error("no zone emits in the band"); return GMO_EINVAL;
    }
    for (int k = 0; k < nw; ++k) {
        c->w_node[k] += p->w_floor_rel * wmax;
        c->ln_w[k] = log(c->w_node[k]);
    }
    /* per zone: dN/dln nu = V J / (h w_i); Simpson over the nodes; bound
     * F_max.  w_i = w e^{-m_i} under an emission table. */
    const double d = c->lnnu_span / (nw - 1);
    uint64_t total = 0;
    for (int i = 0; i < nz; ++i) {
        double s = 0.0, fm = 0.0;
        for (int k = 0; k < nw; ++k) {
            double wik = c->w_node[k];
            if (c->mtab)
                wik *= exp(-table_at(c->mtab, c->mt_n, c->mt_lo, c->mt_hi, i,
                                     c->lnnu_min + c->lnnu_span * k / (nw - 1)));
            double F = Jz[(size_t)i * nw + k] / wik;
            double wk = (k == 0 || k == nw - 1) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
            s += wk * F;
            if (F > fm) fm = F;
        }
        c->nbar[i] = c->vol[i] / GMO_HPL * s * d / 3.0;
        /* the bound is the node maximum with a 2% margin for the curvature
         * of ln J between nodes (reading) */
        c->fmax[i] = GMO_FMAX_MARGIN * fm;
        double fl = floor(c->nbar[i]);
        uint32_t zs[3] = {(uint32_t)i, 0u, ((uint32_t)p->instance << 8) | 2u};
        double u = gmo_uniform_at(p->seed, zs, 0);
        uint32_t n = (uint32_t)fl + ((u < c->nbar[i] - fl) ? 1u : 0u);
        c->count[i] = n;
        c->offset[i] = total;
        total += n;
    }
    c->offset[nz] = total;
    free(Jz); free(nu);
    c->made = 1;
    if (n_made) *n_made = total;
    return GMO_OK;
}

int gmo_read_emission(const gmo_ctx *c, uint32_t *counts, double *nbar, double *fmax, double *ln_w)
{
    if (!c || !c->made) { gmo_set_error("nothing made"); return GMO_ESTATE; }
    if (counts) memcpy(counts, c->count, sizeof(uint32_t) * c->nz);
    if (nbar) memcpy(nbar, c->nbar, sizeof(double) * c->nz);
    if (fmax) memcpy(fmax, c->fmax, sizeof(double) * c->nz);
    if (ln_w) memcpy(ln_w, c->ln_w, sizeof(double) * c->ep.n_wnodes);
    return GMO_OK;
}

/* ---------------------------------------------------------------------
 * Transport
 * ------------------------------------------------------------------- */
typedef struct {
    double x[4], k[4], a[4];
    double w, w_birth, x1;         /* x1: remaining biased optical depth    */
    double nua, nus, b;            /* at the current point (window mode: the
                                      importance factor instead of b)         */
    int n_sc;
    uint32_t steps;
    gmo_rng rng;
    /* worker-local indices of the event records of the photon's ancestry
     * (its creating event first): its escape adds to every one of them */
    int n_anc;
    int64_t anc[GMO_MAX_GEN + 1];
} photon;

typedef struct {
    double *spec;
    double ledger[GMO_L_N];
    int64_t stats[GMO_S_N];
    gmo_trace_rec *trace;
    uint64_t trace_n, trace_cap;
    photon *stack;
    size_t stack_n, stack_cap;
    gmo_event_rec *ev;
    size_t ev_n, ev_cap;
} worker;

/* Append an event record to the worker's list; returns its index. */
static int64_t add_event(worker *wk, const uint32_t s[3], const uint32_t par[3], int zone, int gen,
                         double eps, double w, const double x[4])
{
    if (wk->ev_n == wk->ev_cap) {
        wk->ev_cap = wk->ev_cap ? 2 * wk->ev_cap : 256;
        wk->ev = realloc(wk->ev, sizeof(gmo_event_rec) * wk->ev_cap);
    }
    gmo_event_rec *r = &wk->ev[wk->ev_n];
    memset(r, 0, sizeof(*r));
    r->s0 = s[0]; r->s1 = s[1]; r->s2 = s[2];
    if (par) { r->p0 = par[0]; r->p1 = par[1]; r->p2 = par[2]; }
    r->zone = zone; r->gen = gen; r->eps = eps; r->w = w;
    for (int m = 0; m < 3; ++m) r->x[m] = x[m + 1];
    return (int64_t)wk->ev_n++;
}

/* ln sigma/sigma_T of the power law, linear in ln eps between the nodes,
 * clamped to the end nodes (as the thermal table). */
static double pl_sigma_lookup(const double *t, double eps)
{
    const double le0 = log(GMO_SH_E_MIN), le1 = log(GMO_SH_E_MAX);
    double b = (log(eps) - le0) / ((le1 - le0) / (GMO_SH_NE - 1));
    if (b < 0.0) b = 0.0;
    if (b > GMO_SH_NE - 1) b = GMO_SH_NE - 1;
    int j = (int)floor(b);
    if (j > GMO_SH_NE - 2) j = GMO_SH_NE - 2;
    double f = b - j;
    return exp((1.0 - f) * t[j] + f * t[j + 1]);
}

typedef struct {
    double nua, nus, b;
    int vacuum;
} coef;

/* Invariant absorption and scattering coefficients (nu alpha) at a point,
 * Absorption and Scattering sections: alpha = j/B_nu (Kirchhoff),
 * alpha_sc = n_e sigma_h.  Also the bias at the point. */
static void coefficients(const gmo_ctx *c, const gmo_track_params *tp, const double x[4],
                         const double k[4], int n_sc, coef *out)
{
    out->nua = out->nus = 0.0; out->b = 1.0; out->vacuum = 1;
    int z = zone_of(&c->grid, x);
    if (z < 0 || !(c->n_e[z] > 0.0)) return;
    out->vacuum = 0;
    double g[4][4], u[4], bh[4];
    int has_b;
    gmo_gcov(&c->grid, x, g);
    fluid_frame(c, z, g, u, bh, &has_b);
    double ef = -dot4(g, k, u);
    double nuf = ef * MEC2 / GMO_HPL;
    if (has_b && c->A[z] > 0.0) {
        double cth = dot4(g, k, bh) / ef;
        if (cth > 1.0) cth = 1.0;
        if (cth < -1.0) cth = -1.0;
        if (c->dist.kind == GMO_DIST_POWERLAW) {
            out->nua = gmo_pl_nualpha(&c->dist, c->n_e[z], c->B[z], nuf, cth);
        } else {
            double j = zone_j(c, z, nuf, cth);
            if (j > 0.0) {
                double x_ = ef / c->theta[z];
                double alpha = j * expm1(x_) / (2.0 * GMO_HPL * nuf * nuf * nuf / (GMO_CL * GMO_CL));
                out->nua = nuf * alpha;
            }
        }
    }
    if (tp->scattering)
        out->nus = nuf * c->n_e[z] * GMO_SIGT *
                   (c->dist.kind == GMO_DIST_POWERLAW ? pl_sigma_lookup(c->shpl, ef)
                                                      : gmo_sigma_hot_lookup(c->sh, c->theta[z], ef));
    double b = 1.0;
    switch (tp->bias_mode) {
    case GMO_BIAS_CONST: b = tp->bias_value; break;
    case GMO_BIAS_THETA2: b = tp->bias_value * c->theta[z] * c->theta[z]; break;
    case GMO_BIAS_GEN2:
        b = (double)(n_sc + 1) * (n_sc + 1) / (c->n_e[z] * GMO_SIGT * tp->bias_value * c->grid.L_unit_cm);
        break;
    case GMO_BIAS_TABLE:
    case GMO_BIAS_WINDOW:
        b = exp(table_at(c->btab, c->bt_n, c->bt_lo, c->bt_hi, z, log(ef)));
        break;
    }
    /* the window mode's factor is multiplied by the weight at each step */
    if (tp->bias_mode == GMO_BIAS_WINDOW) { out->b = b; return; }
    if (b < 1.0) b = 1.0;
    if (b > tp->bias_max) b = tp->bias_max;
    out->b = b;
}

/* Bias of a step from the value carried by the photon or evaluated at the
 * step's end: the value itself, or in the window mode w times the
 * importance factor, clamped to [1, bias_max]. */
static double step_bias(const gmo_track_params *tp, double w, double bf)
{
    if (tp->bias_mode != GMO_BIAS_WINDOW) return bf;
    double b = w * bf;
    if (b < 1.0) b = 1.0;
    if (b > tp->bias_max) b = tp->bias_max;
    return b;
}

static void accel_at(const gmo_grid *grid, const double x[4], const double k[4], double a[4])
{
    double G[4][4][4];
    gmo_christoffel(grid, x, G);
    for (int m = 0; m < 4; ++m) {
        double s = 0.0;
        for (int p = 0; p < 4; ++p)
            for (int q = 0; q < 4; ++q) s += G[m][p][q] * k[p] * k[q];
        a[m] = -s;
    }
}

static void record_end(const gmo_ctx *c, worker *wk, const photon *ph, int kind, int inu, int ith)
{
    (void)c;
    if (wk->trace && wk->trace_n < wk->trace_cap) {
        gmo_trace_rec *r = &wk->trace[wk->trace_n++];
        r->s0 = ph->rng.s[0]; r->s1 = ph->rng.s[1]; r->s2 = ph->rng.s[2];
        r->n_sc = ph->n_sc; r->kind = kind; r->i_nu = inu; r->i_theta = ith;
        r->n_steps = ph->steps; r->w_birth = ph->w_birth; r->w_end = ph->w;
        for (int m = 0; m < 4; ++m) { r->x[m] = ph->x[m]; r->k[m] = ph->k[m]; }
    }
}

static void push_child(worker *wk, const photon *ch)
{
    if (wk->stack_n == wk->stack_cap) {
        wk->stack_cap = wk->stack_cap ? 2 * wk->stack_cap : 64;
        wk->stack = realloc(wk->stack, sizeof(photon) * wk->stack_cap);
    }
    wk->stack[wk->stack_n++] = *ch;
}

/* Frame components -> coordinate components. */
static void from_frame(const double e[4][4], const double kf[4], double k[4])
{
    for (int m = 0; m < 4; ++m)
        k[m] = kf[0] * e[0][m] + kf[1] * e[1][m] + kf[2] * e[2][m] + kf[3] * e[3][m];
}

/* Scattering event at (x*, k*): a child with weight w_child (Scattering
 * section).  The child's stream is derived from the parent's stream and the
 * parent's counter at the event; the scattering draws (electron, angles)
 * come from the child's stream, which then continues with the child's own
 * optical-depth draw.  The parent's stream is not advanced here. */
static void scatter_event(const gmo_ctx *c, const gmo_track_params *tp, worker *wk, photon *par,
                          const double xs[4], const double ks[4], double w_child,
                          const double xa[4], const double xb[4])
{
    /* plasma of the zone holding the scatter point; when the interpolated
     * point lies in vacuum, that of the step's start, else its end (reading) */
    int z = zone_of(&c->grid, xs);
    if (z < 0 || !(c->n_e[z] > 0.0)) z = zone_of(&c->grid, xa);
    if (z < 0 || !(c->n_e[z] > 0.0)) z = zone_of(&c->grid, xb);
    photon ch;
    memset(&ch, 0, sizeof(ch));
    ch.rng.seed = par->rng.seed;
    gmo_child_stream(par->rng.seed, par->rng.s, par->rng.block, ch.rng.s);
    ch.rng.block = 0;
    double g[4][4];
    gmo_gcov(&c->grid, xs, g);
    double kchild[4];
    double eps_in = 0.0;
    if (z >= 0 && c->n_e[z] > 0.0) {
        double u[4], bh[4], e[4][4], eps;
        int has_b;
        fluid_frame(c, z, g, u, bh, &has_b);
        scatter_tetrad(g, u, bh, has_b, ks, e, &eps);
        eps_in = eps;
        double kf[4];
        gmo_scatter_in_frame_dist(&ch.rng, &c->dist, c->theta[z], eps, NULL, NULL, kf,
                                  &wk->stats[GMO_S_E_TRIALS], &wk->stats[GMO_S_ANG_TRIALS]);
        from_frame(e, kf, kchild);
    } else {
        for (int m = 0; m < 4; ++m) kchild[m] = ks[m];   /* unreachable: tau_s > 0 */
    }
    for (int m = 0; m < 4; ++m) { ch.x[m] = xs[m]; ch.k[m] = kchild[m]; }
    ch.w = ch.w_birth = w_child;
    ch.n_sc = par->n_sc + 1;
    /* event record: the child inherits the parent's ancestry plus this
     * event; a child without a record starts an empty ancestry */
    ch.n_anc = 0;
    if (c->ev_out && z >= 0 && c->n_e[z] > 0.0) {
        for (int j = 0; j < par->n_anc; ++j) ch.anc[ch.n_anc++] = par->anc[j];
        ch.anc[ch.n_anc++] = add_event(wk, ch.rng.s, par->rng.s, z, ch.n_sc, eps_in, w_child, xs);
    }
    wk->ledger[GMO_L_E_COMPTON] += w_child * (e_inf(g, kchild) - e_inf(g, ks)) * MEC2;
    wk->stats[GMO_S_SCATTER] += 1;
    (void)tp;
    push_child(wk, &ch);
}

/* Step size (reading; the paper names only "the step size"):
 * Cartesian: h * min_j dx^j/|k^j| (h = 0.25 keeps a step within a quarter
 * zone); KS: h / max_j (|k^j|/s^j) with s = (dx1, dx2, min(dx3, pi dx2)) --
 * the azimuth is resolved at least as finely as the polar angle, also on
 * axisymmetric grids with a single 2 pi zone -- at most half the coordinate
 * distance to the horizon when moving inward, and at most a tenth of the x2
 * distance to the nearer pole (k^phi grows like 1/sin^2 theta there; a
 * longer step leaves the corrector without a fixed point). */
static double step_size(const gmo_grid *G, double h, const double x[4], const double k[4])
{
    double dl;
    if (!spherical_grid(G)) {
        dl = INFINITY;
        for (int j = 1; j <= 3; ++j)
            if (k[j] != 0.0) {
                double t = G->dx[j - 1] / fabs(k[j]);
                if (t < dl) dl = t;
            }
        return dl * h;
    }
    double sc[3] = {G->dx[0], G->dx[1], fmin(G->dx[2], M_PI * G->dx[1])};
    double m = 0.0;
    for (int j = 1; j <= 3; ++j) {
        double t = fabs(k[j]) / sc[j - 1];
        if (t > m) m = t;
    }
    dl = h / m;
    if (k[1] < 0.0) {
        double r = exp(x[1]);
        double lim = 0.5 * (r - horizon_r(G)) / (r * fabs(k[1]));
        if (lim < dl) dl = lim;
    }
    double dp = fmin(x[2], 1.0 - x[2]);
    if (dp < 1e-9) dp = 1e-9;
    double lim_p = 0.1 * dp / fabs(k[2]);      /* +inf when k^2 = 0 */
    if (lim_p < dl) dl = lim_p;
    return dl;
}

/* Velocity Verlet with iterated corrector (geodesic section,
 * eq:predicted_wavevector and eq:calculated_wavevector): predictor
 * x' = x + k dl + a dl^2/2 (the printed line lacks dl^2; reading), k_p = k + a dl;
 * Gamma at x' once; repeat a' = -Gamma k_p k_p, k' = k + (a + a') dl/2,
 * error = sum|k' - k_p| / sum|k'|, k_p = k', until error < tol or max_it.
 * Returns the number of corrector passes. */
static int verlet(const gmo_grid *G, double tol, int max_it, const double x[4], const double k[4],
                  const double a[4], double dl, double xn[4], double kn[4], double an[4])
{
    double kp[4];
    for (int m = 0; m < 4; ++m) {
        xn[m] = x[m] + k[m] * dl + 0.5 * a[m] * dl * dl;
        kp[m] = k[m] + a[m] * dl;
    }
    double Gm[4][4][4];
    gmo_christoffel(G, xn, Gm);
    int it;
    for (it = 1;; ++it) {
        for (int m = 0; m < 4; ++m) {
            double s = 0.0;
            for (int p = 0; p < 4; ++p)
                for (int q = 0; q < 4; ++q) s += Gm[m][p][q] * kp[p] * kp[q];
            an[m] = -s;
        }
        double num = 0.0, den = 0.0;
        for (int m = 0; m < 4; ++m) {
            kn[m] = k[m] + 0.5 * (a[m] + an[m]) * dl;
            num += fabs(kn[m] - kp[m]);
            den += fabs(kn[m]);
        }
        for (int m = 0; m < 4; ++m) kp[m] = kn[m];
        if (num / (den + 1e-300) < tol || it >= max_it) break;
    }
    return it;
}

/* Reflection through the pole of the modified coordinates (reading). */
static void pole_reflect(double xn[4], double kn[4], double an[4])
{
    if (xn[2] < 0.0 || xn[2] > 1.0) {
        xn[2] = (xn[2] < 0.0) ? -xn[2] : 2.0 - xn[2];
        xn[3] += M_PI;
        kn[2] = -kn[2];
        an[2] = -an[2];
    }
}

/* Integrate a bare null geodesic (no plasma) with the transport's step rule
 * and integrator for n steps or until r leaves [r_min, r_max]; writes the
 * states (x, k) after every step into out[n][8].  Returns the steps taken.
 * Used by the geodesic-invariant pins. */
int gmo_integrate_geodesic(const gmo_grid *G, const double x0[4], const double k0[4], double h,
                           double tol, int max_it, int n, double r_min, double r_max, double *out)
{
    double x[4], k[4], a[4];
    memcpy(x, x0, sizeof(x));
    memcpy(k, k0, sizeof(k));
    accel_at(G, x, k, a);
    int s;
    for (s = 0; s < n; ++s) {
        double dl = step_size(G, h, x, k);
        double xn[4], kn[4], an[4];
        verlet(G, tol, max_it, x, k, a, dl, xn, kn, an);
        if (spherical_grid(G)) pole_reflect(xn, kn, an);
        memcpy(x, xn, sizeof(x)); memcpy(k, kn, sizeof(k)); memcpy(a, an, sizeof(a));
        for (int m = 0; m < 4; ++m) { out[8 * s + m] = x[m]; out[8 * s + 4 + m] = k[m]; }
        if (spherical_grid(G)) {
            double r = exp(x[1]);
            if (r < r_min || r > r_max) { ++s; break; }
        }
    }
    return s;
}

/* Run one photon (root already born or child) to termination. */
static void run_photon(const gmo_ctx *c, const gmo_track_params *tp, worker *wk, photon *ph)
{
    const gmo_grid *G = &c->grid;
    const int ks_metric = spherical_grid(G);
    const double rh = horizon_r(G);
    const double Cc = GMO_HPL * G->L_unit_cm / MEC2;   /* C = h ell / m_e c^2 */
    coef c0;
    double g[4][4];
    if (ph->n_sc > 0) {
        /* child: its own stream starts with its optical-depth draw */
        ph->x1 = -log(1.0 - gmo_rng_next(&ph->rng));
    }
    accel_at(&c->grid, ph->x, ph->k, ph->a);
    coefficients(c, tp, ph->x, ph->k, ph->n_sc, &c0);
    ph->nua = c0.nua; ph->nus = c0.nus; ph->b = c0.b;
    int gen = ph->n_sc < GMO_MAX_GEN ? ph->n_sc : GMO_MAX_GEN - 1;
    wk->stats[GMO_S_GEN0 + gen] += 1;

    for (;;) {
        if ((int64_t)ph->steps >= tp->max_steps) {
            gmo_gcov(G, ph->x, g);
            double e = e_inf(g, ph->k);
            wk->ledger[GMO_L_W_STUCK] += ph->w; wk->ledger[GMO_L_E_STUCK] += ph->w * e * MEC2;
            wk->stats[GMO_S_STUCK] += 1;
            record_end(c, wk, ph, GMO_END_STUCK, -1, -1);
            return;
        }
        // far-field rule: an outgoing photon beyond r_far (outside the plasma
        // and the photon orbits, so it never comes back) steps step_far
        // times further
        double h = tp->step_h;
        if (spherical_grid(G) && tp->step_far > 1.0 && ph->k[1] > 0.0 && exp(ph->x[1]) > tp->r_far)
            h *= tp->step_far;
        double dl = step_size(G, h, ph->x, ph->k);
        double xn[4], kn[4], an[4];
        wk->stats[GMO_S_VERLET_IT] += verlet(G, tp->verlet_tol, tp->verlet_max_it, ph->x, ph->k, ph->a, dl, xn, kn, an);
        if (ks_metric) pole_reflect(xn, kn, an);
        coef c1;
        coefficients(c, tp, xn, kn, ph->n_sc, &c1);
        ph->steps += 1;
        wk->stats[GMO_S_STEPS] += 1;

        double tau_a = 0.5 * (ph->nua + c1.nua) * Cc * dl;
        double tau_s = tp->scattering ? 0.5 * (ph->nus + c1.nus) * Cc * dl : 0.0;
        double bf = c1.vacuum ? ph->b : c1.b;
        double b = step_bias(tp, ph->w, bf);
        gmo_gcov(G, ph->x, g);
        double e_old = e_inf(g, ph->k);

        if (tp->scattering && ph->n_sc < tp->n_sc_max && b * tau_s > ph->x1) {
            /* the scattering point: the same integrator advanced over the
             * fraction f of the step from its start (reading) */
            double f = ph->x1 / (b * tau_s);
            double xs[4], ks[4], as[4];
            wk->stats[GMO_S_VERLET_IT] += verlet(G, tp->verlet_tol, tp->verlet_max_it, ph->x, ph->k,
                                                 ph->a, f * dl, xs, ks, as);
            if (ks_metric) pole_reflect(xs, ks, as);
            double wb = ph->w;
            ph->w *= exp(-f * tau_a);
            wk->ledger[GMO_L_W_ABS] += wb - ph->w;
            wk->ledger[GMO_L_E_ABS] += (wb - ph->w) * e_old * MEC2;
            gmo_gcov(G, xs, g);
            double e_s = e_inf(g, ks);
            wk->ledger[GMO_L_E_DRIFT] += ph->w * (e_s - e_old) * MEC2;
            scatter_event(c, tp, wk, ph, xs, ks, ph->w / b, ph->x, xn);
            ph->w *= (1.0 - 1.0 / b);
            ph->x1 = -log(1.0 - gmo_rng_next(&ph->rng));
            for (int m = 0; m < 4; ++m) { ph->x[m] = xs[m]; ph->k[m] = ks[m]; }
            accel_at(&c->grid, ph->x, ph->k, ph->a);
            coefficients(c, tp, ph->x, ph->k, ph->n_sc, &c0);
            ph->nua = c0.nua; ph->nus = c0.nus;
            if (!c0.vacuum) ph->b = c0.b;
            if (b == 1.0) {   /* all weight went to the child */
                record_end(c, wk, ph, GMO_END_SPLIT, -1, -1);
                return;
            }
        } else {
            if (tp->scattering) {
                if (ph->n_sc < tp->n_sc_max) {
                    ph->x1 -= b * tau_s;
                } else {   /* generation cap: extinction without a child (reading) */
                    double wb = ph->w;
                    ph->w *= exp(-tau_s);
                    wk->ledger[GMO_L_W_CAPLOSS] += wb - ph->w;
                    wk->ledger[GMO_L_E_CAPLOSS] += (wb - ph->w) * e_old * MEC2;
                }
            }
            double wb = ph->w;
            ph->w *= exp(-tau_a);
            wk->ledger[GMO_L_W_ABS] += wb - ph->w;
            wk->ledger[GMO_L_E_ABS] += (wb - ph->w) * e_old * MEC2;
            for (int m = 0; m < 4; ++m) { ph->x[m] = xn[m]; ph->k[m] = kn[m]; ph->a[m] = an[m]; }
            ph->nua = c1.nua; ph->nus = c1.nus; ph->b = bf;
            gmo_gcov(G, ph->x, g);
            double e_new = e_inf(g, ph->k);
            wk->ledger[GMO_L_E_DRIFT] += ph->w * (e_new - e_old) * MEC2;

            /* ---- termination ---- */
            int escaped = 0, captured = 0;
            if (!ks_metric) {
                for (int j = 0; j < 3; ++j) {
                    double lo = G->x_start[j], hi = G->x_start[j] + G->n[j] * G->dx[j];
                    if (ph->x[j + 1] < lo || ph->x[j + 1] >= hi) escaped = 1;
                }
            } else {
                double r = exp(ph->x[1]);
                if (r >= G->r_record) escaped = 1;
                else if (r < rh * (1.0 + tp->horizon_eps)) captured = 1;
            }
            if (escaped) {
                double nuinf = e_new * MEC2 / GMO_HPL;
                double dln = log(tp->nu_hi / tp->nu_lo) / tp->n_nu;
                double fi = floor((log(nuinf) - log(tp->nu_lo)) / dln);
                double E = ph->w * e_new * MEC2;
                if (!(fi >= 0.0 && fi < tp->n_nu)) {
                    wk->ledger[GMO_L_W_OOB] += ph->w; wk->ledger[GMO_L_E_OOB] += E;
                    wk->stats[GMO_S_OOB] += 1;
                    record_end(c, wk, ph, GMO_END_OOB, -1, -1);
                    return;
                }
                double th;
                if (!ks_metric) {
                    double kk = sqrt(ph->k[1] * ph->k[1] + ph->k[2] * ph->k[2] + ph->k[3] * ph->k[3]);
                    th = acos(ph->k[3] / kk);
                } else {
                    th = gmo_th_of_x2(G, ph->x[2]);
                }
                int ith = (int)floor(th * tp->n_theta / M_PI);
                if (ith < 0) ith = 0;
                if (ith > tp->n_theta - 1) ith = tp->n_theta - 1;
                int inu = (int)fi;
                double *bin = &wk->spec[((size_t)ith * tp->n_nu + inu) * 3];
                bin[0] += E; bin[1] += E * E; bin[2] += 1.0;
                /* the escape scores for every event of the photon's ancestry */
                double sc = E * (c->sw ? c->sw[(size_t)ith * tp->n_nu + inu] : 1.0);
                for (int j = 0; j < ph->n_anc; ++j) wk->ev[ph->anc[j]].score += sc;
                wk->ledger[GMO_L_W_ESC] += ph->w; wk->ledger[GMO_L_E_ESC] += E;
                wk->stats[GMO_S_ESCAPED] += 1;
                record_end(c, wk, ph, GMO_END_ESCAPE, inu, ith);
                return;
            }
            if (captured) {
                wk->ledger[GMO_L_W_CAPT] += ph->w; wk->ledger[GMO_L_E_CAPT] += ph->w * e_new * MEC2;
                wk->stats[GMO_S_CAPTURED] += 1;
                record_end(c, wk, ph, GMO_END_CAPTURE, -1, -1);
                return;
            }
        }
        /* ---- Russian roulette (reading) ---- */
        if (ph->w < tp->roulette_frac * ph->w_birth) {
            gmo_gcov(G, ph->x, g);
            double e = e_inf(g, ph->k);
            if (gmo_rng_next(&ph->rng) < tp->roulette_p) {
                double gain = ph->w * (1.0 / tp->roulette_p - 1.0);
                wk->ledger[GMO_L_W_ROUL] += gain; wk->ledger[GMO_L_E_ROUL] += gain * e * MEC2;
                ph->w /= tp->roulette_p;
                wk->stats[GMO_S_ROUL_SURVIVE] += 1;
            } else {
                wk->ledger[GMO_L_W_ROUL] -= ph->w; wk->ledger[GMO_L_E_ROUL] -= ph->w * e * MEC2;
                wk->stats[GMO_S_ROUL_KILL] += 1;
                double wk_w = ph->w;
                ph->w = 0.0;
                record_end(c, wk, ph, GMO_END_ROULETTE, -1, -1);
                (void)wk_w;
                return;
            }
        }
    }
}

/* Birth of root p in zone i (Sampling procedure section). */
static void birth(const gmo_ctx *c, worker *wk, uint64_t p, int z, photon *ph)
{
    const gmo_grid *G = &c->grid;
    memset(ph, 0, sizeof(*ph));
    ph->rng.seed = c->ep.seed;
    ph->rng.s[0] = (uint32_t)p; ph->rng.s[1] = (uint32_t)(p >> 32);
    ph->rng.s[2] = ((uint32_t)c->ep.instance << 8) | 1u;
    ph->rng.block = 0;
    int i3 = z % G->n[2], i2 = (z / G->n[2]) % G->n[1], i1 = z / (G->n[2] * G->n[1]);
    int id[3] = {i1, i2, i3};
    ph->x[0] = 0.0;
    for (int j = 0; j < 3; ++j) ph->x[j + 1] = G->x_start[j] + (id[j] + gmo_rng_next(&ph->rng)) * G->dx[j];
    /* frequency by rejection against max_k dN/dln nu at the nodes */
    double lnnu, nu;
    for (int64_t it = 0;; ++it) {
        lnnu = c->lnnu_min + gmo_rng_next(&ph->rng) * c->lnnu_span;
        nu = exp(lnnu);
        double u2 = gmo_rng_next(&ph->rng);
        double F = zone_J(c, z, nu) / exp(ln_weight_zone(c, z, lnnu));
        wk->stats[GMO_S_NU_TRIALS] += 1;
        if (F > c->fmax[z]) wk->stats[GMO_S_OVERSHOOT] += 1;
        if (u2 < F / c->fmax[z] || it >= GMO_MAX_TRIALS) break;
    }
    /* direction by rejection against j(pi/2) */
    double cth;
    double jmax = zone_j(c, z, nu, 0.0);
    for (int64_t it = 0;; ++it) {
        cth = 2.0 * gmo_rng_next(&ph->rng) - 1.0;
        double u4 = gmo_rng_next(&ph->rng);
        wk->stats[GMO_S_DIR_TRIALS] += 1;
        if (u4 < zone_j(c, z, nu, cth) / jmax || it >= GMO_MAX_TRIALS) break;
    }
    double phi = 2.0 * M_PI * gmo_rng_next(&ph->rng);
    double g[4][4], u[4], bh[4], e[4][4];
    int has_b;
    gmo_gcov(G, ph->x, g);
    fluid_frame(c, z, g, u, bh, &has_b);
    emission_tetrad(g, u, bh, e);
    double eps = GMO_HPL * nu / MEC2;
    double sth = sqrt(1.0 - cth * cth);
    double kf[4] = {eps, eps * sth * cos(phi), eps * sth * sin(phi), eps * cth};
    from_frame(e, kf, ph->k);
    ph->w = ph->w_birth = exp(ln_weight_zone(c, z, lnnu));
    ph->x1 = -log(1.0 - gmo_rng_next(&ph->rng));
    ph->n_sc = 0;
    ph->n_anc = 0;
    if (c->ev_out && p % c->root_stride == 0)
        ph->anc[ph->n_anc++] = add_event(wk, ph->rng.s, NULL, z, 0, eps, ph->w, ph->x);
    wk->ledger[GMO_L_W_EMIT] += ph->w;
    wk->ledger[GMO_L_E_EMIT] += ph->w * e_inf(g, ph->k) * MEC2;
    wk->stats[GMO_S_ROOTS] += 1;
}

static int zone_of_root(const gmo_ctx *c, uint64_t p)
{
    int lo = 0, hi = c->nz;             /* offset[lo] <= p < offset[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (c->offset[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

int gmo_track_scatter(gmo_ctx *c, const gmo_track_params *tp, uint64_t root_begin,
                      uint64_t root_end, int n_threads, gmo_trace_rec *trace, uint64_t trace_cap,
                      uint64_t *trace_n)
{
    if (!c || !c->made) { gmo_set_error("make superphotons first"); return GMO_ESTATE; }
    if (tp->n_nu < 1 || tp->n_theta < 1 || !(tp->nu_hi > tp->nu_lo) || !(tp->nu_lo > 0.0) ||
        !(tp->bias_max >= 1.0) || !(tp->step_h > 0.0) || tp->verlet_max_it < 1 ||
        tp->n_sc_max < 0 || !(tp->roulette_p > 0.0 && tp->roulette_p <= 1.0) ||
        !(tp->step_far == 0.0 || tp->step_far >= 1.0)) {
        gmo_set_error("bad track parameters"); return GMO_EINVAL;
    }
    if ((tp->bias_mode == GMO_BIAS_TABLE || tp->bias_mode == GMO_BIAS_WINDOW) && !c->btab) {
        gmo_set_error("bias table not set"); return GMO_ESTATE;
    }
    if (c->sw && c->sw_n != tp->n_nu * tp->n_theta) {
        gmo_set_error("score weights do not match the tally"); return GMO_EINVAL;
    }
    if (root_end > c->offset[c->nz]) root_end = c->offset[c->nz];
    if (c->spec && (c->n_nu != tp->n_nu || c->n_theta != tp->n_theta)) {
        gmo_set_error("tally shape changed without reset"); return GMO_EINVAL;
    }
    if (!c->spec) {
        c->n_nu = tp->n_nu; c->n_theta = tp->n_theta;
        c->spec = calloc((size_t)tp->n_nu * tp->n_theta * 3, sizeof(double));
    }
    if (tp->scattering && !c->sh) {
        /* the table depends on nothing but its fixed nodes: built once per
         * process and copied into each context */
        static double *sh_cache = NULL;
        c->sh = malloc(sizeof(double) * GMO_SH_NT * GMO_SH_NE);
        #pragma omp critical(gmo_sh_cache)
        {
            if (!sh_cache) {
                double *t = malloc(sizeof(double) * GMO_SH_NT * GMO_SH_NE);
                gmo_sigma_hot_table(t);
                sh_cache = t;
            }
        }
        memcpy(c->sh, sh_cache, sizeof(double) * GMO_SH_NT * GMO_SH_NE);
    }
    if (tp->scattering && c->dist.kind == GMO_DIST_POWERLAW && !c->shpl) {
        c->shpl = malloc(sizeof(double) * GMO_SH_NE);
        const double le0 = log(GMO_SH_E_MIN), le1 = log(GMO_SH_E_MAX);
        #pragma omp parallel for schedule(dynamic, 4)
        for (int j = 0; j < GMO_SH_NE; ++j)
            c->shpl[j] = log(gmo_sigma_pl_direct(&c->dist, exp(le0 + (le1 - le0) * j / (GMO_SH_NE - 1))));
    }
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    int nt = 1; (void)n_threads;
#endif
    worker *W = calloc(nt, sizeof(worker));
    size_t nbins = (size_t)tp->n_nu * tp->n_theta * 3;
    for (int t = 0; t < nt; ++t) {
        W[t].spec = calloc(nbins, sizeof(double));
        if (trace) { W[t].trace = malloc(sizeof(gmo_trace_rec) * (trace_cap ? trace_cap : 1)); W[t].trace_cap = trace_cap; }
    }
    int64_t nroots = (int64_t)(root_end > root_begin ? root_end - root_begin : 0);
    #pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        worker *wk = &W[omp_get_thread_num()];
#else
        worker *wk = &W[0];
#endif
        #pragma omp for schedule(static, 1024)
        for (int64_t q = 0; q < nroots; ++q) {
            uint64_t p = root_begin + (uint64_t)q;
            photon ph;
            birth(c, wk, p, zone_of_root(c, p), &ph);
            /* roots have block counter > 0 after birth; children start at 0 */
            run_photon(c, tp, wk, &ph);
            while (wk->stack_n > 0) {
                photon ch = wk->stack[--wk->stack_n];
                wk->stats[GMO_S_CHILDREN] += 1;
                run_photon(c, tp, wk, &ch);
            }
        }
    }
    uint64_t tn = 0;
    for (int t = 0; t < nt; ++t) {
        for (size_t i = 0; i < nbins; ++i) c->spec[i] += W[t].spec[i];
        for (int i = 0; i < GMO_L_N; ++i) c->ledger[i] += W[t].ledger[i];
        for (int i = 0; i < GMO_S_N; ++i) c->stats[i] += W[t].stats[i];
        if (trace)
            for (uint64_t r = 0; r < W[t].trace_n && tn < trace_cap; ++r) trace[tn++] = W[t].trace[r];
        for (size_t r = 0; r < W[t].ev_n; ++r, ++c->ev_n)
            if (c->ev_n < c->ev_cap) c->ev_out[c->ev_n] = W[t].ev[r];
        free(W[t].spec); free(W[t].trace); free(W[t].stack); free(W[t].ev);
    }
    free(W);
    if (trace_n) *trace_n = tn;
    return GMO_OK;
}

int gmo_read_spectrum(gmo_ctx *c, double *spec, double *ledger, int64_t *stats, int reset)
{
    if (!c) { gmo_set_error("null context"); return GMO_EINVAL; }
    size_t nb = (size_t)c->n_nu * c->n_theta * 3;
    if (spec && c->spec) memcpy(spec, c->spec, sizeof(double) * nb);
    if (ledger) memcpy(ledger, c->ledger, sizeof(c->ledger));
    if (stats) memcpy(stats, c->stats, sizeof(c->stats));
    if (reset) {
        if (c->spec) memset(c->spec, 0, sizeof(double) * nb);
        memset(c->ledger, 0, sizeof(c->ledger));
        memset(c->stats, 0, sizeof(c->stats));
    }
    return GMO_OK;
}
