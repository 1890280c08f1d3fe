/*
 * gmo_physics.c -- oracle: random numbers, quadrature, emissivity, Planck
 * function, Klein-Nishina and hot cross sections, electron and photon
 * samplers.  TEST INFRASTRUCTURE (see gmo.h).  Plain double precision.
 */
#include "gmo_internal.h"

#include <math.h>
#include <string.h>
#include <stdlib.h>

/* ======================================================================
 * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).  A counter of
 * four 32-bit words and a key of two words go through ten rounds; each
 * round multiplies words 0 and 2 by fixed constants (64-bit products),
 * xors the high halves with the other words and the key, and the key
 * is bumped by the two Weyl increments between rounds.
 * Pinned against an independent Python implementation and the published
 * known-answer vectors in tests/test_oracle_rng.py.
 * ==================================================================== */
void gmo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * c[0];
        uint64_t p1 = (uint64_t)M1 * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* One uniform in [0,1) per counter block: the first two output words give
 * 53 random bits, u = (w0 * 2^21 + (w1 >> 11)) * 2^-53.  The counter is
 * (block, s0, s1, s2); the key is the 64-bit seed split into two words. */
double gmo_uniform_at(uint64_t seed, const uint32_t stream[3], uint32_t block)
{
    uint32_t ctr[4] = {block, stream[0], stream[1], stream[2]};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    gmo_philox4x32_10(ctr, key, o);
    uint64_t bits = ((uint64_t)o[0] << 21) | (uint64_t)(o[1] >> 11);
    return (double)bits * 0x1.0p-53;
}

double gmo_rng_next(gmo_rng *r)
{
    double u = gmo_uniform_at(r->seed, r->s, r->block);
    r->block += 1;
    return u;
}

/* Stream of a child created when the parent's counter stood at `block`:
 * the first three words of Philox under a second key (seed_lo xor the
 * golden-ratio word, seed_hi) applied to (block, parent stream), with the
 * top bit of the third word set so it can never equal a root stream
 * (third word = instance<<8 | 1) or a zone stream (instance<<8 | 2). */
void gmo_child_stream(uint64_t seed, const uint32_t parent[3], uint32_t block, uint32_t child[3])
{
    uint32_t ctr[4] = {block, parent[0], parent[1], parent[2]};
    uint32_t key[2] = {(uint32_t)seed ^ 0x9E3779B9u, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    gmo_philox4x32_10(ctr, key, o);
    child[0] = o[0]; child[1] = o[1]; child[2] = o[2] | 0x80000000u;
}

/* ======================================================================
 * Adaptive Gauss-Kronrod (7-point Gauss embedded in 15-point Kronrod)
 * quadrature with recursive bisection.  Nodes and weights are the
 * standard published values (Kronrod extension of Gauss-Legendre).
 * ==================================================================== */
static const double XGK[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double WGK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

/* One 15-point Kronrod panel.  Error estimate as in QUADPACK's qk15:
 * the Gauss-Kronrod difference, scaled down when it is small relative to
 * the spread of the integrand (K15 is far more accurate than G7), and never
 * below 50 machine epsilons of the integral of |f| (rounding floor). */
static double gk15(double (*f)(double, void *), void *ctx, double a, double b, double *err)
{
    double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double fv1[7], fv2[7];
    double fc = f(c, ctx);
    double resk = fc * WGK[7], resg = fc * WG[3], resabs = fabs(fc) * WGK[7];
    for (int j = 0; j < 7; ++j) {
        double dx = h * XGK[j];
        double f1 = f(c - dx, ctx), f2 = f(c + dx, ctx);
        fv1[j] = f1; fv2[j] = f2;
        resk += WGK[j] * (f1 + f2);
        resabs += WGK[j] * (fabs(f1) + fabs(f2));
        if (j & 1) resg += WG[j / 2] * (f1 + f2);
    }
    double mean = 0.5 * resk;
    double resasc = WGK[7] * fabs(fc - mean);
    for (int j = 0; j < 7; ++j) resasc += WGK[j] * (fabs(fv1[j] - mean) + fabs(fv2[j] - mean));
    double e = fabs((resk - resg) * h);
    resasc *= fabs(h);
    resabs *= fabs(h);
    if (resasc != 0.0 && e != 0.0) {
        double t = 200.0 * e / resasc;
        e = resasc * fmin(1.0, t * sqrt(t));
    }
    /* at the rounding floor the panel cannot be improved: report 0 */
    if (e <= 50.0 * 2.220446049250313e-16 * resabs) e = 0.0;
    *err = e;
    return resk * h;
}

typedef struct { double (*f)(double, void *); void *ctx; long panels; } quad_state;

/* Recursive bisection; each half gets half of the absolute tolerance.  A
 * panel whose estimate is already at the rounding floor, or the panel
 * budget, stops the recursion. */
static double adapt(quad_state *q, double a, double b, double whole, double err,
                    double abs_tol, int depth)
{
    if (err <= abs_tol || depth >= 40 || q->panels > 200000) return whole;
    double m = 0.5 * (a + b), el, er;
    double left = gk15(q->f, q->ctx, a, m, &el);
    double right = gk15(q->f, q->ctx, m, b, &er);
    q->panels += 2;
    return adapt(q, a, m, left, el, 0.5 * abs_tol, depth + 1) +
           adapt(q, m, b, right, er, 0.5 * abs_tol, depth + 1);
}

/* Integral of f over [a,b] to a relative tolerance.  A first pass over 16
 * equal panels sets the scale of the absolute tolerance. */
double gmo_quad(double (*f)(double, void *), void *ctx, double a, double b, double rel_tol)
{
    if (b <= a) return 0.0;
    const int P = 16;
    double pv[16], pe[16], scale = 0.0;
    for (int i = 0; i < P; ++i) {
        double lo = a + (b - a) * i / P, hi = a + (b - a) * (i + 1) / P;
        pv[i] = gk15(f, ctx, lo, hi, &pe[i]);
        scale += fabs(pv[i]);
    }
    double abs_tol = rel_tol * scale / P;
    if (abs_tol == 0.0) abs_tol = 1e-300;
    quad_state q = {f, ctx, 0};
    double sum = 0.0;
    for (int i = 0; i < P; ++i) {
        double lo = a + (b - a) * i / P, hi = a + (b - a) * (i + 1) / P;
        sum += adapt(&q, lo, hi, pv[i], pe[i], abs_tol, 0);
    }
    return sum;
}

/* ======================================================================
 * Modified Bessel function K_2 from its integral representation
 * K_2(x) = int_0^inf exp(-x cosh t) cosh(2t) dt.  The factor exp(-x) is
 * taken out so the integrand is O(1) at t = 0.
 * Pinned against scipy.special.kv (test_oracle_physics.py).
 * ==================================================================== */
static double k2_integrand(double t, void *ctx)
{
    double x = *(double *)ctx;
    return exp(-x * (cosh(t) - 1.0)) * cosh(2.0 * t);
}

double gmo_k2(double x)
{
    /* beyond T the integrand is below exp(-740) relative to its value at 0 */
    double T = acosh(1.0 + 745.0 / x);
    double I = gmo_quad(k2_integrand, &x, 0.0, T, 1e-14);
    return exp(-x) * I;
}

/* Emissivity section: K_2(1/Theta) replaced by 2 Theta^2 in the large
 * temperature limit.  Reading: exact K_2 for Theta <= 100, 2 Theta^2 above. */
double gmo_k2_of_theta(double theta_e)
{
    if (theta_e > 100.0) return 2.0 * theta_e * theta_e;
    return gmo_k2(1.0 / theta_e);
}

/* ======================================================================
 * Thermal synchrotron emissivity, Emissivity section (eq:emissivity),
 * fit of Leung et al. (2011):
 *   j = sqrt(2) pi e^2 n_e nu_s / (3 c K_2(1/Theta)) (X^1/2 + 2^(11/12) X^(1/6))^2 exp(-X^(1/3)),
 *   X = nu / nu_s,  nu_s = (2/9) (e B / (2 pi m_e c)) Theta^2 sin(theta).
 * Written as j = A sin(theta) g(X) with nu_s = nu_c sin(theta).
 * ==================================================================== */
double gmo_g_of_X(double X)
{
    if (!(X > 0.0) || isinf(X)) return 0.0;
    double s = pow(X, 0.5) + pow(2.0, 11.0 / 12.0) * pow(X, 1.0 / 6.0);
    return s * s * exp(-pow(X, 1.0 / 3.0));
}

double gmo_nu_c(double theta_e, double B)
{
    return (2.0 / 9.0) * (GMO_EE * B / (2.0 * M_PI * GMO_ME * GMO_CL)) * theta_e * theta_e;
}

double gmo_A_coef(double n_e, double theta_e, double B)
{
    if (!(n_e > 0.0) || !(B > 0.0) || !(theta_e > 0.0)) return 0.0;
    double nuc = gmo_nu_c(theta_e, B);
    return sqrt(2.0) * M_PI * GMO_EE * GMO_EE * n_e * nuc /
           (3.0 * GMO_CL * gmo_k2_of_theta(theta_e));
}

double gmo_jnu(double n_e, double theta_e, double B, double nu, double cos_th)
{
    double A = gmo_A_coef(n_e, theta_e, B);
    if (A == 0.0) return 0.0;
    double s2 = 1.0 - cos_th * cos_th;
    if (!(s2 > 0.0)) return 0.0;
    double s = sqrt(s2);
    double X = nu / (gmo_nu_c(theta_e, B) * s);
    return A * s * gmo_g_of_X(X);
}

/* Angle integral: int j dOmega = 2 pi A int_{-1}^{1} s g(X_c/s) dmu
 * = 4 pi A G(X_c), G(X_c) = int_0^1 s g(X_c/s) dmu, s = sqrt(1-mu^2).
 * With mu = sin(phi): G = int_0^{pi/2} cos^2(phi) g(X_c / cos(phi)) dphi.
 * The integrand peaks at phi = 0, where it equals g(X_c); it is integrated
 * as g(X_c) times the ratio g(X_c/c)/g(X_c) written out,
 *   [(X/c)^{1/2} + 2^{11/12}(X/c)^{1/6}]^2 / [X^{1/2} + 2^{11/12} X^{1/6}]^2
 *     * exp(-X^{1/3} (c^{-1/3} - 1)),
 * which stays of order one where g itself is subnormal (X_c near 4e8). */
static double G_ratio_integrand(double phi, void *ctx)
{
    double Xc = *(double *)ctx;
    double c = cos(phi);
    if (!(c > 0.0)) return 0.0;
    const double k = pow(2.0, 11.0 / 12.0);
    double X = Xc / c;
    double num = pow(X, 0.5) + k * pow(X, 1.0 / 6.0);
    double den = pow(Xc, 0.5) + k * pow(Xc, 1.0 / 6.0);
    double e = exp(-pow(Xc, 1.0 / 3.0) * (pow(c, -1.0 / 3.0) - 1.0));
    return c * c * (num / den) * (num / den) * e;
}

double gmo_G_of_Xc(double Xc)
{
    if (!(Xc > 0.0) || isinf(Xc)) return 0.0;
    double g0 = gmo_g_of_X(Xc);
    if (g0 == 0.0) return 0.0;
    return g0 * gmo_quad(G_ratio_integrand, &Xc, 0.0, 0.5 * M_PI, 1e-13);
}

double gmo_Jnu(double n_e, double theta_e, double B, double nu)
{
    double A = gmo_A_coef(n_e, theta_e, B);
    if (A == 0.0) return 0.0;
    return 4.0 * M_PI * A * gmo_G_of_Xc(nu / gmo_nu_c(theta_e, B));
}

/* Planck function B_nu(T) with h nu / k T = (h nu / m_e c^2) / Theta. */
double gmo_planck(double nu, double theta_e)
{
    double x = GMO_HPL * nu / (GMO_ME * GMO_CL * GMO_CL * theta_e);
    return 2.0 * GMO_HPL * nu * nu * nu / (GMO_CL * GMO_CL) / expm1(x);
}

/* ======================================================================
 * Klein-Nishina total cross section in units of sigma_T, Scattering
 * section:  sigma/sigma_T = 3/(4 e^2) [2 + e^2(1+e)/(1+2e)^2
 *                                       + (e^2-2e-2)/(2e) ln(1+2e)].
 * For small e the paper adopts the leading terms 1 - 2e.  Reading: below
 * e = 0.02 the Taylor series of the same function is carried to tenth
 * order (coefficients 1, -2, 26/5, -133/10, 1144/35, -544/7, 3784/21,
 * -6148/15, 151552/165, -111872/55, 637952/143), which meets the closed
 * form to ~1e-12 at the switch; the closed form uses log1p.  Pinned against
 * a 50-digit mpmath evaluation and against sympy's series.
 * ==================================================================== */
double gmo_sigma_kn(double e)
{
    if (e < 0.02) {
        static const double c[11] = {1.0, -2.0, 26.0 / 5.0, -133.0 / 10.0, 1144.0 / 35.0,
                                     -544.0 / 7.0, 3784.0 / 21.0, -6148.0 / 15.0,
                                     151552.0 / 165.0, -111872.0 / 55.0, 637952.0 / 143.0};
        double s = c[10];
        for (int i = 9; i >= 0; --i) s = s * e + c[i];
        return s;
    }
    double e2 = e * e, d = 1.0 + 2.0 * e;
    return 0.75 / e2 * (2.0 + e2 * (1.0 + e) / (d * d) + (e2 - 2.0 * e - 2.0) / (2.0 * e) * log1p(2.0 * e));
}

/* ======================================================================
 * Hot (Maxwell-Juttner averaged) cross section, Scattering section:
 *   sigma_h = (1/n) int d^3p (dn/d^3p) (1 - mu beta) sigma_KN(eps_e),
 * with eps_e = gamma eps (1 - beta mu), the photon energy in the electron
 * rest frame, isotropic electrons, and the thermal distribution
 *   dn/dgamma proportional to gamma^2 beta exp(-gamma/Theta).
 * The normalisation is taken from the same quadrature as the numerator.
 * Outer variable v with gamma = 1 + v^2 (removes the sqrt at gamma=1).
 * ==================================================================== */
typedef struct { double theta, eps, gamma, beta; } hot_ctx;

static double hot_inner(double mu, void *vc)
{
    hot_ctx *h = (hot_ctx *)vc;
    double w = 1.0 - h->beta * mu;
    return 0.5 * w * gmo_sigma_kn(h->gamma * h->eps * w);
}

static double mj_weight_v(double v, double theta)
{
    double x = v * v;              /* gamma - 1 */
    double gam = 1.0 + x;
    /* gamma^2 beta dgamma = gamma sqrt(x(x+2)) * 2 v dv, times exp(-x/Theta) */
    return gam * sqrt(x * (x + 2.0)) * 2.0 * v * exp(-x / theta);
}

static double hot_outer(double v, void *vc)
{
    hot_ctx *h = (hot_ctx *)vc;
    double x = v * v;
    double wt = mj_weight_v(v, h->theta);
    if (wt == 0.0) return 0.0;
    hot_ctx in = *h;
    in.gamma = 1.0 + x;
    in.beta = sqrt(x * (x + 2.0)) / (1.0 + x);
    return wt * gmo_quad(hot_inner, &in, -1.0, 1.0, 1e-12);
}

static double hot_norm(double v, void *vc)
{
    hot_ctx *h = (hot_ctx *)vc;
    return mj_weight_v(v, h->theta);
}

double gmo_sigma_hot_direct(double theta_e, double eps)
{
    hot_ctx h = {theta_e, eps, 0.0, 0.0};
    /* exp(-x/Theta) < e^-740 beyond x = 740 Theta */
    double vmax = sqrt(740.0 * theta_e);
    double num = gmo_quad(hot_outer, &h, 0.0, vmax, 1e-12);
    double den = gmo_quad(hot_norm, &h, 0.0, vmax, 1e-13);
    return num / den;
}

/* Table nodes: 64 in ln Theta over [1e-2, 1e3], 256 in ln eps over
 * [1e-12, 1e6] (reading: the paper tabulates sigma_h a priori without
 * stating ranges).  Entries are ln(sigma_h / sigma_T). */
void gmo_sigma_hot_table(double *ln_table)
{
    const double lt0 = log(GMO_SH_TH_MIN), lt1 = log(GMO_SH_TH_MAX);
    const double le0 = log(GMO_SH_E_MIN), le1 = log(GMO_SH_E_MAX);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int idx = 0; idx < GMO_SH_NT * GMO_SH_NE; ++idx) {
        int i = idx / GMO_SH_NE, j = idx % GMO_SH_NE;
        double th = exp(lt0 + (lt1 - lt0) * i / (GMO_SH_NT - 1));
        double ep = exp(le0 + (le1 - le0) * j / (GMO_SH_NE - 1));
        ln_table[idx] = log(gmo_sigma_hot_direct(th, ep));
    }
}

/* Bilinear interpolation of ln sigma_h in (ln Theta, ln eps), clamped to
 * the table edges (reading). */
double gmo_sigma_hot_lookup(const double *t, double theta_e, double eps)
{
    const double lt0 = log(GMO_SH_TH_MIN), lt1 = log(GMO_SH_TH_MAX);
    const double le0 = log(GMO_SH_E_MIN), le1 = log(GMO_SH_E_MAX);
    double dt = (lt1 - lt0) / (GMO_SH_NT - 1), de = (le1 - le0) / (GMO_SH_NE - 1);
    double a = (log(theta_e) - lt0) / dt;
    double b = (log(eps) - le0) / de;
    if (a < 0.0) a = 0.0;
    if (a > GMO_SH_NT - 1) a = GMO_SH_NT - 1;
    if (b < 0.0) b = 0.0;
    if (b > GMO_SH_NE - 1) b = GMO_SH_NE - 1;
    int i = (int)floor(a), j = (int)floor(b);
    if (i > GMO_SH_NT - 2) i = GMO_SH_NT - 2;
    if (j > GMO_SH_NE - 2) j = GMO_SH_NE - 2;
    double fa = a - i, fb = b - j;
    double v = (1 - fa) * (1 - fb) * t[i * GMO_SH_NE + j] + (1 - fa) * fb * t[i * GMO_SH_NE + j + 1] +
               fa * (1 - fb) * t[(i + 1) * GMO_SH_NE + j] + fa * fb * t[(i + 1) * GMO_SH_NE + j + 1];
    return exp(v);
}

/* ======================================================================
 * Power-law electrons (non-thermal distributions, named as future work in
 * the paper's Conclusions): isotropic n(gamma) = n_e C gamma^-p on
 * [g1, g2], C = (p - 1) / (g1^{1-p} - g2^{1-p}).  Synchrotron emission and
 * absorption take the textbook asymptotic forms of a power law (Rybicki &
 * Lightman, eqs. 6.36 and 6.53; valid for nu_c(g1) << nu << nu_c(g2)),
 * per steradian, s = sin(angle to the field):
 *   j_nu = sqrt3 e^3 n_e C B s / (4 pi m c^2 (p + 1))
 *          Gamma((3p + 19)/12) Gamma((3p - 1)/12) (2 pi m c nu / (3 e B s))^{-(p-1)/2},
 *   alpha_nu = sqrt3 e^3 / (8 pi m) (3 e / (2 pi m^3 c^5))^{p/2} C_E (B s)^{(p+2)/2}
 *          Gamma((3p + 2)/12) Gamma((3p + 22)/12) nu^{-(p+4)/2},
 * C_E = n_e C (m c^2)^{p-1} the coefficient of the energy distribution.
 * In the form j = A s g(X) that the emission sampler uses: X = nu / (nu_c s)
 * with nu_c = 3 e B / (2 pi m c), g(X) = X^{-(p-1)/2}.
 * ==================================================================== */
static double pl_C(const gmo_dist *d)
{
    return (d->p - 1.0) / (pow(d->g1, 1.0 - d->p) - pow(d->g2, 1.0 - d->p));
}

double gmo_pl_nu_c(double B) { return 3.0 * GMO_EE * B / (2.0 * M_PI * GMO_ME * GMO_CL); }

double gmo_pl_A(const gmo_dist *d, double n_e, double B)
{
    if (!(n_e > 0.0) || !(B > 0.0)) return 0.0;
    const double p = d->p;
    return sqrt(3.0) * GMO_EE * GMO_EE * GMO_EE * n_e * pl_C(d) * B * tgamma((3.0 * p + 19.0) / 12.0) *
           tgamma((3.0 * p - 1.0) / 12.0) / (4.0 * M_PI * GMO_ME * GMO_CL * GMO_CL * (p + 1.0));
}

double gmo_pl_g(double X, double p)
{
    if (!(X > 0.0) || isinf(X)) return 0.0;
    return pow(X, -0.5 * (p - 1.0));
}

double gmo_pl_jnu(const gmo_dist *d, double n_e, double B, double nu, double cos_th)
{
    double s2 = 1.0 - cos_th * cos_th;
    if (!(s2 > 0.0)) return 0.0;
    double s = sqrt(s2);
    return gmo_pl_A(d, n_e, B) * s * gmo_pl_g(nu / (gmo_pl_nu_c(B) * s), d->p);
}

static double pl_ang_integrand(double mu, void *ctx)
{
    double p = *(const double *)ctx;
    return pow(1.0 - mu * mu, 0.25 * (p + 1.0));
}

/* G's angular factor: int_0^1 s g(X_c / s) dmu = X_c^{-(p-1)/2} times this. */
double gmo_pl_ang(double p)
{
    return gmo_quad(pl_ang_integrand, &p, 0.0, 1.0, 1e-13);
}

double gmo_pl_Jnu(const gmo_dist *d, double n_e, double B, double nu)
{
    return 4.0 * M_PI * gmo_pl_A(d, n_e, B) * gmo_pl_g(nu / gmo_pl_nu_c(B), d->p) * gmo_pl_ang(d->p);
}

double gmo_pl_nualpha(const gmo_dist *d, double n_e, double B, double nu, double cos_th)
{
    double s2 = 1.0 - cos_th * cos_th;
    if (!(s2 > 0.0) || !(n_e > 0.0) || !(B > 0.0)) return 0.0;
    const double p = d->p, m = GMO_ME, c = GMO_CL, e = GMO_EE;
    /* the textbook form takes the coefficient of the energy distribution,
     * n_e C (m c^2)^{p-1} */
    double alpha = sqrt(3.0) * e * e * e / (8.0 * M_PI * m) *
                   pow(3.0 * e / (2.0 * M_PI * m * m * m * pow(c, 5.0)), 0.5 * p) * n_e * pl_C(d) *
                   pow(m * c * c, p - 1.0) *
                   pow(B * sqrt(s2), 0.5 * (p + 2.0)) * tgamma((3.0 * p + 2.0) / 12.0) *
                   tgamma((3.0 * p + 22.0) / 12.0) * pow(nu, -0.5 * (p + 4.0));
    return nu * alpha;
}

/* Hot cross section of the power law, Scattering section with the power
 * law in place of the thermal distribution:
 *   sigma / sigma_T = C int_{g1}^{g2} gamma^-p dgamma int_{-1}^{1} dmu/2 (1 - beta mu) sigma_KN(gamma eps (1 - beta mu)),
 * outer variable ln gamma. */
typedef struct { double eps, p, gamma, beta; } pl_ctx;

static double pl_inner(double mu, void *vc)
{
    pl_ctx *h = (pl_ctx *)vc;
    double w = 1.0 - h->beta * mu;
    return 0.5 * w * gmo_sigma_kn(h->gamma * h->eps * w);
}

static double pl_outer(double u, void *vc)
{
    pl_ctx in = *(pl_ctx *)vc;
    in.gamma = exp(u);
    in.beta = sqrt((in.gamma - 1.0) * (in.gamma + 1.0)) / in.gamma;
    return pow(in.gamma, 1.0 - in.p) * gmo_quad(pl_inner, &in, -1.0, 1.0, 1e-12);
}

double gmo_sigma_pl_direct(const gmo_dist *d, double eps)
{
    pl_ctx h = {eps, d->p, 0.0, 0.0};
    return pl_C(d) * gmo_quad(pl_outer, &h, log(d->g1), log(d->g2), 1e-12);
}

/* ======================================================================
 * Electron sampling for a scattering event, Scattering section: the
 * electron momentum is drawn from the thermal distribution by rejection,
 * then a second rejection on the Klein-Nishina cross section.  The paper
 * points to igrmonty for the sampler; the reading here is an exact
 * sampler of the same joint density
 *   p(gamma, mu) ~ f_MJ(gamma) (1 - beta mu) sigma_KN(gamma eps (1 - beta mu)),
 * which is the integrand of sigma_h:
 *  (a) x = gamma - 1 from the mixture of Gamma(s, Theta) laws with
 *      s = 3/2, 2, 5/2, 3 and weights sqrt2 G(3/2) T^3/2, G(2) T^2,
 *      sqrt2 G(5/2) T^5/2, G(3) T^3, which bounds gamma sqrt(gamma^2-1),
 *      accepted with probability sqrt(2+x)/(sqrt2 + sqrt x);
 *  (b) mu by inverting the CDF of (1 - beta mu)/2 on [-1,1];
 *  (c) accept (gamma, mu) with probability sigma_KN(eps_e)/sigma_T.
 * Draw order: component, exponentials, the two normal uniforms (for a
 * half-integer shape), the x acceptance, mu, the KN acceptance.
 * ==================================================================== */
static double exp_draw(gmo_rng *r) { return -log(1.0 - gmo_rng_next(r)); }

void gmo_sample_electron_rng(gmo_rng *r, double theta, double eps, double *gamma,
                             double *beta_out, double *mu, int64_t *trials)
{
    const double sq2 = sqrt(2.0), spi = sqrt(M_PI);
    double w1 = sq2 * (0.5 * spi) * pow(theta, 1.5);
    double w2 = 1.0 * theta * theta;
    double w3 = sq2 * (0.75 * spi) * pow(theta, 2.5);
    double w4 = 2.0 * theta * theta * theta;
    double wsum = w1 + w2 + w3 + w4;
    for (int64_t it = 0;; ++it) {
        double x;
        for (;;) {
            double uc = gmo_rng_next(r) * wsum;
            double s;
            if (uc < w1) {
                s = exp_draw(r);
                double ua = gmo_rng_next(r), ub = gmo_rng_next(r);
                double c = cos(2.0 * M_PI * ub);
                s += -log(1.0 - ua) * c * c;        /* Z^2/2 */
            } else if (uc < w1 + w2) {
                s = exp_draw(r) + exp_draw(r);
            } else if (uc < w1 + w2 + w3) {
                s = exp_draw(r) + exp_draw(r);
                double ua = gmo_rng_next(r), ub = gmo_rng_next(r);
                double c = cos(2.0 * M_PI * ub);
                s += -log(1.0 - ua) * c * c;
            } else {
                s = exp_draw(r) + exp_draw(r) + exp_draw(r);
            }
            x = theta * s;
            double acc = sqrt(2.0 + x) / (sq2 + sqrt(x));
            if (gmo_rng_next(r) < acc) break;
        }
        double g = 1.0 + x;
        double beta = sqrt(x * (x + 2.0)) / g;
        double c = 1.0 + 0.5 * beta - 2.0 * gmo_rng_next(r);
        double m = -2.0 * c / (1.0 + sqrt(1.0 + 2.0 * beta * c));
        double ee = g * eps * (1.0 - beta * m);
        double ukn = gmo_rng_next(r);
        if (ukn < gmo_sigma_kn(ee) || it >= GMO_MAX_TRIALS) {
            *gamma = g; *beta_out = beta; *mu = m;
            if (trials) *trials += it + 1;
            return;
        }
    }
}

/* Power-law electron for a scattering event: the same joint density with
 * the power law in place of the thermal one,
 *   p(gamma, mu) ~ gamma^-p (1 - beta mu) sigma_KN(gamma eps (1 - beta mu)),
 *  (a) gamma by inverting the power law's distribution function,
 *      gamma = [g1^{1-p} - u (g1^{1-p} - g2^{1-p})]^{1/(1-p)};
 *  (b) mu as for the thermal electrons; (c) accept with sigma_KN / sigma_T.
 * Draw order: gamma, mu, the KN acceptance. */
static void sample_electron_pl(gmo_rng *r, const gmo_dist *d, double eps, double *gamma,
                               double *beta_out, double *mu, int64_t *trials)
{
    const double a = pow(d->g1, 1.0 - d->p), b = pow(d->g2, 1.0 - d->p);
    for (int64_t it = 0;; ++it) {
        double g = pow(a - gmo_rng_next(r) * (a - b), 1.0 / (1.0 - d->p));
        double beta = sqrt((g - 1.0) * (g + 1.0)) / g;
        double c = 1.0 + 0.5 * beta - 2.0 * gmo_rng_next(r);
        double m = -2.0 * c / (1.0 + sqrt(1.0 + 2.0 * beta * c));
        double ee = g * eps * (1.0 - beta * m);
        if (gmo_rng_next(r) < gmo_sigma_kn(ee) || it >= GMO_MAX_TRIALS) {
            *gamma = g; *beta_out = beta; *mu = m;
            if (trials) *trials += it + 1;
            return;
        }
    }
}

void gmo_sample_electron(uint64_t seed, const uint32_t stream[3], uint32_t *block,
                         double theta_e, double eps, double *gamma, double *mu, int64_t *trials)
{
    gmo_rng r = {seed, {stream[0], stream[1], stream[2]}, *block};
    double beta;
    gmo_sample_electron_rng(&r, theta_e, eps, gamma, &beta, mu, trials);
    *block = r.block;
}

/* ---- small 3-vector helpers ---- */
static double dot3(const double a[3], const double b[3]) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1]*b[2] - a[2]*b[1];
    c[1] = a[2]*b[0] - a[0]*b[2];
    c[2] = a[0]*b[1] - a[1]*b[0];
}

/* Scatter a photon of fluid-frame energy eps moving along e1 of an
 * orthonormal fluid frame (e0 = fluid velocity).  Returns the scattered
 * photon's frame components kout = (eps', kx, ky, kz).  Steps:
 *  1. electron (gamma, mu) as above; azimuth phi_e uniform;
 *     electron direction v = mu e1 + sqrt(1-mu^2)(cos phi_e e2 + sin phi_e e3);
 *  2. boost the photon into the electron rest frame;
 *  3. scattering angle by rejection on the Klein-Nishina differential
 *     cross section (Thomson when eps_e < 1e-4, reading), azimuth uniform
 *     about the incoming rest-frame direction;
 *  4. boost back to the fluid frame. */
void gmo_scatter_in_frame(gmo_rng *r, double theta, double eps, double *gamma_out,
                          double *mu_out, double kout[4], int64_t *e_trials, int64_t *ang_trials)
{
    gmo_scatter_in_frame_dist(r, NULL, theta, eps, gamma_out, mu_out, kout, e_trials, ang_trials);
}

void gmo_scatter_in_frame_dist(gmo_rng *r, const gmo_dist *d, double theta, double eps,
                               double *gamma_out, double *mu_out, double kout[4], int64_t *e_trials,
                               int64_t *ang_trials)
{
    double g, beta, mu;
    if (d && d->kind == GMO_DIST_POWERLAW) sample_electron_pl(r, d, eps, &g, &beta, &mu, e_trials);
    else gmo_sample_electron_rng(r, theta, eps, &g, &beta, &mu, e_trials);
    double phe = 2.0 * M_PI * gmo_rng_next(r);
    double sm = sqrt(fmax(0.0, 1.0 - mu * mu));
    double v[3] = {mu, sm * cos(phe), sm * sin(phe)};

    /* photon in the fluid frame: energy eps along x */
    double kf[3] = {eps, 0.0, 0.0};
    double kpar = dot3(kf, v);
    double ee = g * (eps - beta * kpar);                 /* rest-frame energy */
    double kpar_e = g * (kpar - beta * eps);
    double ke[3];
    for (int i = 0; i < 3; ++i) ke[i] = kf[i] - kpar * v[i] + kpar_e * v[i];
    double ne[3] = {ke[0] / ee, ke[1] / ee, ke[2] / ee};

    double cth, es;
    for (int64_t it = 0;; ++it) {
        cth = 2.0 * gmo_rng_next(r) - 1.0;
        es = (ee < 1e-4) ? ee : ee / (1.0 + ee * (1.0 - cth));
        double rr = es / ee;
        double acc = 0.5 * rr * rr * (rr + 1.0 / rr - (1.0 - cth * cth));
        double ua = gmo_rng_next(r);
        if (ua < acc || it >= GMO_MAX_TRIALS) {
            if (ang_trials) *ang_trials += it + 1;
            break;
        }
    }
    double psi = 2.0 * M_PI * gmo_rng_next(r);
    double sth = sqrt(fmax(0.0, 1.0 - cth * cth));

    /* basis about ne: p along v x ne, else e2 made orthogonal to ne, else e3 */
    double p[3], q[3];
    cross3(v, ne, p);
    double pn = dot3(p, p);
    if (pn < 1e-20) {
        double e2[3] = {0.0, 1.0, 0.0}, e3[3] = {0.0, 0.0, 1.0};
        double d = dot3(e2, ne);
        for (int i = 0; i < 3; ++i) p[i] = e2[i] - d * ne[i];
        pn = dot3(p, p);
        if (pn < 1e-20) {
            d = dot3(e3, ne);
            for (int i = 0; i < 3; ++i) p[i] = e3[i] - d * ne[i];
            pn = dot3(p, p);
        }
    }
    pn = sqrt(pn);
    for (int i = 0; i < 3; ++i) p[i] /= pn;
    cross3(ne, p, q);
    double ns[3];
    for (int i = 0; i < 3; ++i)
        ns[i] = cth * ne[i] + sth * (cos(psi) * p[i] + sin(psi) * q[i]);

    /* rest frame -> fluid frame: boost by -beta v */
    double ks[3] = {es * ns[0], es * ns[1], es * ns[2]};
    double kspar = dot3(ks, v);
    double ef = g * (es + beta * kspar);
    double kfpar = g * (kspar + beta * es);
    kout[0] = ef;
    for (int i = 0; i < 3; ++i) kout[1 + i] = ks[i] + (kfpar - kspar) * v[i];
    if (gamma_out) *gamma_out = g;
    if (mu_out) *mu_out = mu;
}

void gmo_sample_scatter_frame_dist(uint64_t seed, const uint32_t stream[3], uint32_t *block,
                                   const gmo_dist *d, double theta_e, double eps, double *gamma_out,
                                   double *mu_out, double kout[4], int64_t *e_trials, int64_t *ang_trials)
{
    gmo_rng r = {seed, {stream[0], stream[1], stream[2]}, *block};
    gmo_scatter_in_frame_dist(&r, d, theta_e, eps, gamma_out, mu_out, kout, e_trials, ang_trials);
    *block = r.block;
}

void gmo_sample_scatter_frame(uint64_t seed, const uint32_t stream[3], uint32_t *block,
                              double theta_e, double eps, double *gamma_out, double *mu_out,
                              double kout[4], int64_t *e_trials, int64_t *ang_trials)
{
    gmo_rng r = {seed, {stream[0], stream[1], stream[2]}, *block};
    gmo_scatter_in_frame(&r, theta_e, eps, gamma_out, mu_out, kout, e_trials, ang_trials);
    *block = r.block;
}
