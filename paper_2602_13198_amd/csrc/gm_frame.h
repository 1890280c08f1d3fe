// gm_frame.h -- metric traits, fluid-frame tetrads and the Compton
// scattering event (device side).
#pragma once

#include "gm_physics.h"

namespace gm {

// ---------------------------------------------------------------------------
// Flat spacetime in Cartesian coordinates, x in units of ell.
// ---------------------------------------------------------------------------
struct Minkowski {
    static constexpr bool kCurved = false;
    GM_D static void gcov(const double *, double g[4][4])
    {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) g[m][n] = (m == n) ? (m == 0 ? -1.0 : 1.0) : 0.0;
    }
};

GM_D double dot4(const double g[4][4], const double *a, const double *b)
{
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double t = 0.0;
#pragma unroll
        for (int n = 0; n < 4; ++n) t += g[m][n] * b[n];
        s += a[m] * t;
    }
    return s;
}

// Inner products with the metric at a point, without forming a 4x4 matrix
// whose zeros would still be multiplied: flat (Cartesian Minkowski), and a
// general matrix for the paths that hold one.
struct GFlat {
    GM_D double dot(const double *a, const double *b) const
    {
        return -a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
    }
};

struct GMat {
    const double (*g)[4];
    GM_D double dot(const double *a, const double *b) const { return dot4(g, a, b); }
};

GM_D double e_inf(const double g[4][4], const double *k)
{
    return -(g[0][0] * k[0] + g[0][1] * k[1] + g[0][2] * k[2] + g[0][3] * k[3]);
}

// Packed zone record (16 doubles, 128 bytes): u (4), field direction (4),
// emission coefficient A, nu_c, Theta_e, n_e, ln Theta_e, 1/Theta_e, field
// flag (1 when B > 0 and the direction exists), 1/nu_c.  In flat spacetime u
// and the field direction are stored already normalised; in curved
// spacetime they are stored as given and normalised at each point.
enum { Z_U0 = 0, Z_B0 = 4, Z_A = 8, Z_NUC = 9, Z_TH = 10, Z_NE = 11, Z_LNTH = 12, Z_INVTH = 13,
       Z_HASB = 14, Z_INVNUC = 15, Z_STRIDE = 16 };

// Unit fluid velocity and field direction at a point: the zone's u (given
// in u) is normalised with the local metric, the field direction (in bh)
// projected normal to u and normalised (absent when the zone has no field
// or it is degenerate here).
template <class G>
GM_D bool fluid_frame_vec(bool zone_has_b, const G &gm, double u[4], double bh[4])
{
    const double iun = rsqrt(-gm.dot(u, u));
#pragma unroll
    for (int m = 0; m < 4; ++m) u[m] *= iun;
    double bu = gm.dot(bh, u);
#pragma unroll
    for (int m = 0; m < 4; ++m) bh[m] += bu * u[m];
    double bb = gm.dot(bh, bh);
    bool has_b = (bb > 0.0) && zone_has_b;
    double inv = has_b ? 1.0 / sqrt(bb) : 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) bh[m] = has_b ? bh[m] * inv : 0.0;
    return has_b;
}

// The two frame products the opacities need, without forming the unit
// vectors: with u_n = u / sqrt(-u.u) and b' = b + (b.u_n) u_n (b projected
// normal to u_n), eps = -k.u_n and kb = k.b' / |b'|, where
// |b'|^2 = b.b + (b.u_n)^2 and k.b' = k.b - (b.u_n) eps.  kb is 0 and the
// result false when the zone has no field or b' vanishes here.
template <class G, class T>
GM_D bool frame_products(bool zone_has_b, const G &gm, const T *uz, const T *bz, const double *k,
                         double &eps, double &kb)
{
    double u[4], b[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) { u[m] = (double)uz[m]; b[m] = (double)bz[m]; }
    const double iun = rsqrt(-gm.dot(u, u));
    eps = -gm.dot(k, u) * iun;
    const double bu = gm.dot(b, u) * iun;
    const double n2 = gm.dot(b, b) + bu * bu;
    const bool has_b = zone_has_b && n2 > 0.0;
    kb = has_b ? (gm.dot(k, b) - bu * eps) * rsqrt(n2) : 0.0;
    return has_b;
}

// Same from a packed FP64 zone record.
template <class G>
GM_D bool fluid_frame_m(const double *zr, const G &gm, double u[4], double bh[4])
{
#pragma unroll
    for (int m = 0; m < 4; ++m) { u[m] = zr[Z_U0 + m]; bh[m] = zr[Z_B0 + m]; }
    return fluid_frame_vec(zr[Z_HASB] != 0.0, gm, u, bh);
}

GM_D bool fluid_frame(const double *zr, const double g[4][4], double u[4], double bh[4])
{
    return fluid_frame_m(zr, GMat{g}, u, bh);
}

// Flat spacetime: the normalised vectors were stored by the zone preparation.
GM_D bool fluid_frame_flat(const double *zr, double u[4], double bh[4])
{
#pragma unroll
    for (int m = 0; m < 4; ++m) { u[m] = zr[Z_U0 + m]; bh[m] = zr[Z_B0 + m]; }
    return zr[Z_HASB] != 0.0;
}

// Add v, made orthonormal to e[0..ne-1] (e[0] timelike), as e[ne]; false
// when its residual norm^2 is below 1e-10 of the original (degenerate).
GM_D bool gram_schmidt(const double g[4][4], double e[4][4], int ne, const double *vin)
{
    double v[4] = {vin[0], vin[1], vin[2], vin[3]};
    double n0 = fabs(dot4(g, v, v));
    for (int i = 0; i < ne; ++i) {
        double p = dot4(g, v, e[i]);
        double s = (i == 0) ? p : -p;
#pragma unroll
        for (int m = 0; m < 4; ++m) v[m] += s * e[i][m];
    }
    double nn = dot4(g, v, v);
    if (!(nn > 1e-10 * n0) || !(nn > 0.0)) return false;
    double inv = 1.0 / sqrt(nn);
#pragma unroll
    for (int m = 0; m < 4; ++m) e[ne][m] = v[m] * inv;
    return true;
}

// Emission tetrad: e0 = u, e3 = field direction, e1 and e2 from the first
// non-degenerate coordinate directions 1, 2, 3.
GM_D void emission_tetrad(const double g[4][4], const double u[4], const double bh[4],
                          double e[4][4])
{
    double t[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) { t[0][m] = u[m]; t[1][m] = bh[m]; }
    int n = 2;
    for (int j = 1; j <= 3 && n < 4; ++j) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        v[j] = 1.0;
        n += gram_schmidt(g, t, n, v) ? 1 : 0;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        e[0][m] = t[0][m]; e[1][m] = t[2][m]; e[2][m] = t[3][m]; e[3][m] = t[1][m];
    }
}

// Scattering tetrad (Gram-Schmidt): e0 = u; e1 the photon's fluid-frame
// direction, i.e. k minus its projection on u, normalised by its own norm
// (which equals the fluid-frame energy only for an exactly null k; an
// integrated k is null only to the integrator's accuracy, and a unit e1
// keeps the frame orthonormal regardless); e2 from the field direction
// (else coordinate 1, 2, 3), e3 from the next non-degenerate coordinate
// direction.  Returns the fluid-frame energy -k.u.
GM_D double scatter_tetrad(const double g[4][4], const double u[4], const double bh[4], bool has_b,
                           const double k[4], double e[4][4])
{
    double ep = -dot4(g, k, u);
    double v[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = k[m] - ep * u[m];
    double inv = 1.0 / sqrt(dot4(g, v, v));
#pragma unroll
    for (int m = 0; m < 4; ++m) { e[0][m] = u[m]; e[1][m] = v[m] * inv; }
    int n = 2;
    if (has_b) n += gram_schmidt(g, e, n, bh) ? 1 : 0;
    for (int j = 1; j <= 3 && n < 4; ++j) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        v[j] = 1.0;
        n += gram_schmidt(g, e, n, v) ? 1 : 0;
    }
    return ep;
}

// ---------------------------------------------------------------------------
// Scattering event in the fluid frame (Scattering section).  The photon has
// energy eps along e1.  The electron (gamma, mu) is drawn from the joint law
// f_thermal(gamma) (1 - beta mu) sigma_KN(gamma eps (1 - beta mu)), which is
// the integrand of the hot cross section:
//   gamma - 1 from the mixture of Gamma(s, Theta), s = 3/2, 2, 5/2, 3, with
//   weights sqrt2 G(3/2) T^1.5, G(2) T^2, sqrt2 G(5/2) T^2.5, G(3) T^3,
//   accepted with probability sqrt(2+x)/(sqrt2 + sqrt x); mu by inverting the
//   CDF of (1 - beta mu)/2; the pair accepted with probability sigma_KN/sigma_T.
// Then the photon is boosted to the electron rest frame, scattered by
// rejection on the Klein-Nishina differential cross section (Thomson below
// eps_e = 1e-4), and boosted back.  Returns the frame components of the
// scattered photon.  Draws come from the child's stream in a fixed order.
// ---------------------------------------------------------------------------
struct ScatterCount { uint32_t e_trials, ang_trials; };

GM_D double exp_variate(Rng &r, uint32_t k0, uint32_t k1) { return -log(1.0 - rng_uniform(r, k0, k1)); }

// Power-law electrons: gamma by inverting the distribution function of the
// power law, gamma = [g1^{1-p} - u (g1^{1-p} - g2^{1-p})]^{1/(1-p)}; mu and
// the Klein-Nishina acceptance as for the thermal electrons.  Draws: gamma,
// mu, the acceptance.
GM_D void electron_power_law(Rng &r, uint32_t k0, uint32_t k1, const Elec &E, double eps, double &gam,
                             double &beta, double &mu, ScatterCount &cnt)
{
    for (int64_t it = 0;; ++it) {
        gam = exp(E.inv1mp * log(E.ga - rng_uniform(r, k0, k1) * (E.ga - E.gb)));
        beta = sqrt((gam - 1.0) * (gam + 1.0)) / gam;
        double c = 1.0 + 0.5 * beta - 2.0 * rng_uniform(r, k0, k1);
        mu = -2.0 * c / (1.0 + sqrt(1.0 + 2.0 * beta * c));
        double ee = gam * eps * (1.0 - beta * mu);
        if (rng_uniform(r, k0, k1) < sigma_kn(ee) || it >= kMaxTrials) {
            cnt.e_trials += (uint32_t)(it + 1);
            return;
        }
    }
}

GM_D void scatter_in_frame(Rng &r, uint32_t k0, uint32_t k1, const Elec &El, double theta, double eps,
                           double kout[4], ScatterCount &cnt)
{
    const double sq2 = 1.4142135623730951, spi = 1.7724538509055159;
    double w1 = sq2 * (0.5 * spi) * pow(theta, 1.5);
    double w2 = theta * theta;
    double w3 = sq2 * (0.75 * spi) * pow(theta, 2.5);
    double w4 = 2.0 * theta * theta * theta;
    double wsum = w1 + w2 + w3 + w4;
    double gam, beta, mu;
    if (El.kind != 0) electron_power_law(r, k0, k1, El, eps, gam, beta, mu, cnt);
    else for (int64_t it = 0;; ++it) {
        double x;
        for (;;) {
            double uc = rng_uniform(r, k0, k1) * wsum;
            double s;
            if (uc < w1) {
                s = exp_variate(r, k0, k1);
                double ua = rng_uniform(r, k0, k1), ub = rng_uniform(r, k0, k1);
                double c = cos(2.0 * kPi * ub);
                s += -log(1.0 - ua) * c * c;
            } else if (uc < w1 + w2) {
                s = exp_variate(r, k0, k1);
                s += exp_variate(r, k0, k1);
            } else if (uc < w1 + w2 + w3) {
                s = exp_variate(r, k0, k1);
                s += exp_variate(r, k0, k1);
                double ua = rng_uniform(r, k0, k1), ub = rng_uniform(r, k0, k1);
                double c = cos(2.0 * kPi * ub);
                s += -log(1.0 - ua) * c * c;
            } else {
                s = exp_variate(r, k0, k1);
                s += exp_variate(r, k0, k1);
                s += exp_variate(r, k0, k1);
            }
            x = theta * s;
            double acc = sqrt(2.0 + x) / (sq2 + sqrt(x));
            if (rng_uniform(r, k0, k1) < acc) break;
        }
        gam = 1.0 + x;
        beta = sqrt(x * (x + 2.0)) / gam;
        double c = 1.0 + 0.5 * beta - 2.0 * rng_uniform(r, k0, k1);
        mu = -2.0 * c / (1.0 + sqrt(1.0 + 2.0 * beta * c));
        double ee = gam * eps * (1.0 - beta * mu);
        double ukn = rng_uniform(r, k0, k1);
        if (ukn < sigma_kn(ee) || it >= kMaxTrials) {
            cnt.e_trials += (uint32_t)(it + 1);
            break;
        }
    }
    double phe = 2.0 * kPi * rng_uniform(r, k0, k1);
    double sm = sqrt(fmax(0.0, 1.0 - mu * mu));
    double v[3] = {mu, sm * cos(phe), sm * sin(phe)};
    // photon (eps, eps, 0, 0) -> electron rest frame
    double kpar = eps * v[0];
    double ee = gam * (eps - beta * kpar);
    double kpar_e = gam * (kpar - beta * eps);
    double ke[3] = {eps - kpar * v[0] + kpar_e * v[0], -kpar * v[1] + kpar_e * v[1],
                    -kpar * v[2] + kpar_e * v[2]};
    double ne[3] = {ke[0] / ee, ke[1] / ee, ke[2] / ee};
    double cth, es;
    for (int64_t it = 0;; ++it) {
        cth = 2.0 * rng_uniform(r, k0, k1) - 1.0;
        es = (ee < 1e-4) ? ee : ee / (1.0 + ee * (1.0 - cth));
        double rr = es / ee;
        double acc = 0.5 * rr * rr * (rr + 1.0 / rr - (1.0 - cth * cth));
        double ua = rng_uniform(r, k0, k1);
        if (ua < acc || it >= kMaxTrials) {
            cnt.ang_trials += (uint32_t)(it + 1);
            break;
        }
    }
    double psi = 2.0 * kPi * rng_uniform(r, k0, k1);
    double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
    // basis about ne: along v x ne, else frame axis 2 (then 3) made normal to ne
    double p[3] = {v[1] * ne[2] - v[2] * ne[1], v[2] * ne[0] - v[0] * ne[2], v[0] * ne[1] - v[1] * ne[0]};
    double pn = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    if (pn < 1e-20) {
        double d = ne[1];
        p[0] = -d * ne[0]; p[1] = 1.0 - d * ne[1]; p[2] = -d * ne[2];
        pn = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        if (pn < 1e-20) {
            d = ne[2];
            p[0] = -d * ne[0]; p[1] = -d * ne[1]; p[2] = 1.0 - d * ne[2];
            pn = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        }
    }
    pn = sqrt(pn);
    p[0] /= pn; p[1] /= pn; p[2] /= pn;
    double q[3] = {ne[1] * p[2] - ne[2] * p[1], ne[2] * p[0] - ne[0] * p[2], ne[0] * p[1] - ne[1] * p[0]};
    double cp = cos(psi), sp = sin(psi);
    double ks[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) ks[i] = es * (cth * ne[i] + sth * (cp * p[i] + sp * q[i]));
    // electron rest frame -> fluid frame
    double kspar = ks[0] * v[0] + ks[1] * v[1] + ks[2] * v[2];
    double ef = gam * (es + beta * kspar);
    double kfpar = gam * (kspar + beta * es);
    kout[0] = ef;
#pragma unroll
    for (int i = 0; i < 3; ++i) kout[1 + i] = ks[i] + (kfpar - kspar) * v[i];
}

}  // namespace gm
