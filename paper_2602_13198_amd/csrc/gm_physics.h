// gm_physics.h -- emissivity, opacities and cross sections (device side).
#pragma once

#include "gm_common.h"

namespace gm {

// ---------------------------------------------------------------------------
// Thermal synchrotron emissivity (Emissivity section, eq:emissivity, fit of
// Leung et al. 2011): j = A sin(theta) g(nu / (nu_c sin(theta))),
//   A = sqrt(2) pi e^2 n_e nu_c / (3 c K2(1/Theta)),
//   nu_c = (2/9) (e B / (2 pi m_e c)) Theta^2,
//   g(X) = (X^1/2 + 2^(11/12) X^(1/6))^2 exp(-X^(1/3)).
// X^(1/6) and X^(1/2) are built from one cube root.
// ---------------------------------------------------------------------------
GM_HD double g_shape(double X)
{
    if (!(X > 0.0) || X > 1.7e308) return 0.0;
    const double a = 1.8877486253633869;     // 2^(11/12)
    double y = cbrt(X);                      // X^1/3
    double s6 = sqrt(y);                     // X^1/6
    double t = y * s6 + a * s6;              // X^1/2 + a X^1/6
    return t * t * exp(-y);
}

// e^x - 1 for the Kirchhoff factor (x = h nu / k T >= 0): the series to
// x^5 below 1e-3 (truncation below x^6 / 720 < 2e-21 relative), else
// exp(x) - 1 (relative error below 2e-13 there).  Shares exp's code with
// the other exponentials of the opacity evaluation instead of bringing a
// second set of polynomial constants into the tracker's registers.
GM_HD double expm1_kirchhoff(double x)
{
    if (x < 1e-3) return x * (1.0 + x * (0.5 + x * (1.0 / 6.0 + x * (1.0 / 24.0 + x * (1.0 / 120.0)))));
    return exp(x) - 1.0;
}

GM_HD double nu_crit(double theta_e, double B)
{
    return (2.0 / 9.0) * (kE * B / (2.0 * kPi * kMe * kC)) * theta_e * theta_e;
}

// Angle integral G(Xc) = int_0^1 s g(Xc/s) dmu, s = sqrt(1 - mu^2), so that
// int j dOmega = 4 pi A G(nu/nu_c).  Evaluated from a piecewise Chebyshev
// expansion of ln G in t = ln Xc built on the host (pieces of width h over
// [t_lo, t_hi]); below t_lo the leading small-Xc form C0 Xc^(1/3), above
// t_hi zero (G < 1e-190 there).
struct GCheb {
    const double *coef;   // [n_pieces][deg]
    double t_lo, t_hi, inv_h, ln_c0;
    int n_pieces, deg;
};

GM_HD double lnG_of_t(const GCheb &T, double t)
{
    if (t < T.t_lo) return T.ln_c0 + t * (1.0 / 3.0);
    double a = (t - T.t_lo) * T.inv_h;
    int p = (int)a;
    if (p >= T.n_pieces) p = T.n_pieces - 1;
    double s = 2.0 * (a - (double)p) - 1.0;
    const double *c = T.coef + (size_t)p * T.deg;
    // Clenshaw: sum' c_k T_k(s) with c_0 halved
    double b1 = 0.0, b2 = 0.0;
    for (int k = T.deg - 1; k >= 1; --k) {
        double b0 = fma(2.0 * s, b1, c[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(s, b1, 0.5 * c[0] - b2);
}

GM_HD double G_of_Xc(const GCheb &T, double Xc)
{
    if (!(Xc > 0.0)) return 0.0;
    double t = log(Xc);
    if (t > T.t_hi) return 0.0;
    return exp(lnG_of_t(T, t));
}

// ---------------------------------------------------------------------------
// Klein-Nishina total cross section / sigma_T (Scattering section).  Below
// e = 0.02 the tenth-order Taylor series of the closed form (the paper's
// small-e form 1 - 2e carried further); above, the closed form with log1p.
// ---------------------------------------------------------------------------
GM_HD double sigma_kn(double e)
{
    if (e < 0.02) {
        double s = 637952.0 / 143.0;
        s = fma(s, e, -111872.0 / 55.0);
        s = fma(s, e, 151552.0 / 165.0);
        s = fma(s, e, -6148.0 / 15.0);
        s = fma(s, e, 3784.0 / 21.0);
        s = fma(s, e, -544.0 / 7.0);
        s = fma(s, e, 1144.0 / 35.0);
        s = fma(s, e, -133.0 / 10.0);
        s = fma(s, e, 26.0 / 5.0);
        s = fma(s, e, -2.0);
        return fma(s, e, 1.0);
    }
    double e2 = e * e, d = 1.0 + 2.0 * e;
    return 0.75 / e2 * (2.0 + e2 * (1.0 + e) / (d * d) + (e2 - 2.0 * e - 2.0) / (2.0 * e) * log1p(2.0 * e));
}

// Bilinear interpolation of ln(sigma_h/sigma_T) on the table, clamped at
// the edges.
struct ShTable {
    const double *t;      // [kShNT][kShNE]
    double lt0, inv_dt, le0, inv_de;
};

// In two halves, so that a caller can request the four table entries early
// and interpolate once other work has covered their latency.
struct ShFetch {
    double t00, t01, t10, t11, fa, fb;
};

GM_HD ShFetch sigma_hot_fetch(const ShTable &S, double ln_theta, double ln_eps)
{
    double a = (ln_theta - S.lt0) * S.inv_dt;
    double b = (ln_eps - S.le0) * S.inv_de;
    a = fmin(fmax(a, 0.0), (double)(kShNT - 1));
    b = fmin(fmax(b, 0.0), (double)(kShNE - 1));
    int i = min((int)a, kShNT - 2), j = min((int)b, kShNE - 2);
    const double *r0 = S.t + i * kShNE + j, *r1 = r0 + kShNE;
    return ShFetch{r0[0], r0[1], r1[0], r1[1], a - i, b - j};
}

GM_HD double sigma_hot_finish(const ShFetch &f)
{
    double v = (1.0 - f.fa) * ((1.0 - f.fb) * f.t00 + f.fb * f.t01) + f.fa * ((1.0 - f.fb) * f.t10 + f.fb * f.t11);
    return exp(v);
}


// ---------------------------------------------------------------------------
// Electrons of a plasma.  Thermal: the emissivity above, Kirchhoff
// absorption and the thermal hot cross section.  Power law (the paper's
// Conclusions name non-thermal distributions as future work): isotropic
// n(gamma) = n_e C gamma^-p on [g1, g2], C = (p - 1)/(g1^{1-p} - g2^{1-p}),
// with the asymptotic synchrotron forms of a power law, written in the
// variable X = nu / (nu_c s) of the thermal form with nu_c = 3 e B /
// (2 pi m c) and s the sine of the angle to the field:
//   j = A s X^{-(p-1)/2},  A = sqrt3 e^3 n_e C B Gamma((3p+19)/12) Gamma((3p-1)/12) / (4 pi m c^2 (p+1)),
//   nu alpha = A_a X^{-(p+2)/2},  A_a = sqrt3 e^2 n_e C Gamma((3p+2)/12) Gamma((3p+22)/12) / (12 m c),
// the second from the absorption integral of a smooth distribution,
// alpha = (p+2)/(8 pi m nu^2) int n(gamma)/gamma P(nu, gamma) dgamma, with
// the single-electron spectrum's moments; the angle integral of j is
// 4 pi A X_c^{-(p-1)/2} (sqrt(pi)/2) Gamma((p+5)/4)/Gamma((p+7)/4).
// ---------------------------------------------------------------------------
struct Elec {
    int kind;                  // 0 thermal, 1 power law
    double p;
    double ga, gb, inv1mp;     // g1^{1-p}, g2^{1-p}, 1/(1-p): the inverse distribution function
    double eg, ea;             // exponents -(p-1)/2 (emission), -(p+2)/2 (absorption)
    double ang;                // angular factor of the emission's angle integral
    const double *sig;         // [kShNE] ln(sigma/sigma_T) on the thermal table's eps nodes
    double le0, inv_de;
};

// emission shape g(X) and its angle integral G(X_c) of the electrons
GM_HD double shape_g(const Elec &E, double X)
{
    if (E.kind == 0) return g_shape(X);
    return (X > 0.0 && X < 1.7e308) ? exp(E.eg * log(X)) : 0.0;
}

GM_HD double shape_G(const Elec &E, const GCheb &G, double Xc)
{
    if (E.kind == 0) return G_of_Xc(G, Xc);
    return (Xc > 0.0 && Xc < 1.7e308) ? exp(E.eg * log(Xc)) * E.ang : 0.0;
}

// hot cross section of the power law: linear in ln eps between the nodes,
// clamped at the ends
GM_HD double sigma_pl(const Elec &E, double eps)
{
    double b = fmin(fmax((log(eps) - E.le0) * E.inv_de, 0.0), (double)(kShNE - 1));
    int j = min((int)b, kShNE - 2);
    double f = b - j;
    return exp((1.0 - f) * E.sig[j] + f * E.sig[j + 1]);
}

// ---------------------------------------------------------------------------
// K2(x) = int_0^inf exp(-x cosh t) cosh(2t) dt by the trapezoid rule in t,
// which converges geometrically for this analytic integrand (error of
// order exp(-pi^2/h)); exp(-x) is factored out.
// ---------------------------------------------------------------------------
GM_HD double bessel_k2(double x)
{
    const double h = 0.0625;
    double sum = 0.5;               // t = 0 term: exp(0) cosh(0) / 2
    for (int k = 1; k < 4096; ++k) {
        double t = k * h;
        double e = exp(t), ei = 1.0 / e;
        double ch = 0.5 * (e + ei);
        double arg = x * (ch - 1.0);
        if (arg > 745.0) break;
        double c2 = 0.5 * (e * e + ei * ei);
        sum += exp(-arg) * c2;
    }
    return exp(-x) * h * sum;
}

// Emissivity section: K2(1/Theta) -> 2 Theta^2 at large Theta (switch at 100).
GM_HD double k2_of_theta(double theta_e)
{
    if (theta_e > 100.0) return 2.0 * theta_e * theta_e;
    return bessel_k2(1.0 / theta_e);
}

GM_HD double emis_coef(double n_e, double theta_e, double B)
{
    if (!(n_e > 0.0) || !(B > 0.0) || !(theta_e > 0.0)) return 0.0;
    return 1.4142135623730951 * kPi * kE * kE * n_e * nu_crit(theta_e, B) /
           (3.0 * kC * k2_of_theta(theta_e));
}

}  // namespace gm
