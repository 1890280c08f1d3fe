// gm_host_tables.h -- host-side construction of the device lookup tables.
#pragma once

#include <cmath>
#include <vector>

namespace gm {
namespace host {

// Emissivity shape g(X) (same fit as the device code, host arithmetic).
inline double g_shape_h(double X)
{
    if (!(X > 0.0) || std::isinf(X)) return 0.0;
    const double a = 1.8877486253633869;     // 2^(11/12)
    double y = std::cbrt(X), s6 = std::sqrt(y);
    double t = y * s6 + a * s6;
    return t * t * std::exp(-y);
}

// G(Xc) = int_0^{pi/2} cos^2(phi) g(Xc / cos(phi)) dphi  (mu = sin phi) by
// tanh-sinh quadrature: phi = pi/4 (1 + tanh(pi/2 sinh t)), levels of
// halved step until two successive levels agree to 1e-15.  The distance to
// the upper end is carried separately so cos(phi) = sin(distance) keeps its
// relative accuracy near pi/2.
inline double G_quad(double Xc)
{
    const double half = M_PI / 4.0;
    auto f_at = [&](double t) -> double {
        double s = 0.5 * M_PI * std::sinh(t);
        double ch = std::cosh(s);
        double w = 0.5 * M_PI * std::cosh(t) / (ch * ch);
        double c;
        if (t > 0.0) {                              // near pi/2: distance = half (1 - tanh s)
            double d = half * 2.0 / (std::exp(2.0 * s) + 1.0);
            c = std::sin(d);
        } else {
            double phi = half * (1.0 + std::tanh(s));
            c = std::cos(phi);
        }
        if (!(c > 0.0)) return 0.0;
        return w * c * c * g_shape_h(Xc / c);
    };
    double h = 1.0;
    double sum = f_at(0.0);
    for (int k = 1;; ++k) {
        double a = f_at(k * h), b = f_at(-k * h);
        sum += a + b;
        if ((a == 0.0 && b == 0.0 && k * h > 1.0) || k * h > 6.0) break;
    }
    double prev = half * h * sum;
    for (int level = 1; level < 14; ++level) {
        h *= 0.5;
        double add = 0.0;
        for (int k = 1;; k += 2) {
            double a = f_at(k * h), b = f_at(-k * h);
            add += a + b;
            if ((a == 0.0 && b == 0.0 && k * h > 1.0) || k * h > 6.0) break;
        }
        sum += add;
        double cur = half * h * sum;
        if (level >= 4 && std::fabs(cur - prev) <= 1e-15 * std::fabs(cur)) return cur;
        prev = cur;
    }
    return prev;
}

// Piecewise Chebyshev expansion of ln G(e^t) on [t_lo, t_hi].
struct GChebHost {
    std::vector<double> coef;
    double t_lo, t_hi, h, ln_c0;
    int n_pieces, deg;
};

inline GChebHost build_G_cheb(double t_lo = -104.0, double t_hi = 18.5, double h = 0.5, int deg = 16)
{
    GChebHost T;
    T.t_lo = t_lo;
    T.t_hi = t_hi;
    T.h = h;
    T.deg = deg;
    T.n_pieces = (int)std::ceil((t_hi - t_lo) / h);
    // G -> C0 Xc^(1/3) as Xc -> 0, C0 = 2^(11/6) (sqrt(pi)/2) Gamma(4/3)/Gamma(11/6)
    T.ln_c0 = (11.0 / 6.0) * std::log(2.0) + 0.5 * std::log(M_PI) - std::log(2.0) +
              std::lgamma(4.0 / 3.0) - std::lgamma(11.0 / 6.0);
    T.coef.assign((size_t)T.n_pieces * deg, 0.0);
    std::vector<double> fv(deg);
    for (int p = 0; p < T.n_pieces; ++p) {
        double mid = t_lo + (p + 0.5) * h;
        for (int j = 0; j < deg; ++j) {
            double s = std::cos(M_PI * (j + 0.5) / deg);
            fv[j] = std::log(G_quad(std::exp(mid + 0.5 * h * s)));
        }
        for (int k = 0; k < deg; ++k) {
            double c = 0.0;
            for (int j = 0; j < deg; ++j) c += fv[j] * std::cos(M_PI * k * (j + 0.5) / deg);
            T.coef[(size_t)p * deg + k] = 2.0 * c / deg;
        }
    }
    return T;
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
inline void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace host
}  // namespace gm
