// gm_kerr.h -- Kerr spacetime in modified Kerr-Schild coordinates (device).
//
// Coordinates (t, x1, x2, x3): r = exp(x1), theta = pi x2 + (1-h)/2 sin(2 pi x2),
// phi = x3, mass M (1 for the black hole, lengths in r_g; 0 with a = 0 for
// flat spacetime in spherical coordinates, the sphere grids of the paper's
// tests).  The Kerr-Schild line element
//   ds^2 = -(1-z)dt^2 + 2z dt dr + (1+z)dr^2 + S dth^2 + sin^2th [S + a^2(1+z)sin^2th] dph^2
//          - 2az sin^2th dt dph - 2a(1+z) sin^2th dr dph,   S = r^2 + a^2 cos^2th, z = 2Mr/S,
// carried to the modified coordinates by the Jacobian (1, r, dtheta/dx2, 1).
// Seven components are non-zero: g00 g01 g03 g11 g13 g22 g33.  Their x1 and
// x2 derivatives come from forward-mode dual numbers; the inverse is the
// closed form of the Kerr-Schild inverse metric,
//   g^tt = -(1+z), g^tr = z, g^rr = D/S, g^rph = a/S, g^thth = 1/S, g^phph = 1/(S sin^2),
// D = r^2 - 2Mr + a^2, divided by the Jacobian factors.
#pragma once

#include "gm_common.h"

namespace gm {

// Metric tag of the Kerr path (the flat one is Minkowski).
struct KerrMKS {
    static constexpr bool kCurved = true;
};

struct D3 {
    double v, d1, d2;      // value, d/dx1, d/dx2
};
GM_HD D3 operator+(D3 x, D3 y) { return {x.v + y.v, x.d1 + y.d1, x.d2 + y.d2}; }
GM_HD D3 operator-(D3 x, D3 y) { return {x.v - y.v, x.d1 - y.d1, x.d2 - y.d2}; }
GM_HD D3 operator*(D3 x, D3 y) { return {x.v * y.v, x.d1 * y.v + x.v * y.d1, x.d2 * y.v + x.v * y.d2}; }
GM_HD D3 operator*(double s, D3 x) { return {s * x.v, s * x.d1, s * x.d2}; }
GM_HD D3 operator+(double s, D3 x) { return {s + x.v, x.d1, x.d2}; }

// The seven metric components (and optionally their derivatives) at a point.
struct KMetric {
    double r;
    double g00, g01, g03, g11, g13, g22, g33;             // covariant
    double u00, u01, u11, u13, u22, u33;                  // contravariant (g^03 = g^02 = ... = 0)
    double d1[7], d2[7];                                  // d/dx1, d/dx2 of g00 g01 g03 g11 g13 g22 g33
};

// sin(pi x) and cos(pi x): on the device the library's sincospi, whose
// reduction of a multiple of pi is exact and short (the tracker evaluates
// two per point); the host's check of the zones uses sin and cos.
GM_HD void sincos_pi(double x, double *s, double *c)
{
#ifdef __HIP_DEVICE_COMPILE__
    sincospi(x, s, c);
#else
    *s = ::sin(kPi * x);
    *c = ::cos(kPi * x);
#endif
}

template <bool DERIV>
GM_HD void kerr_metric(double a, double M, double hs, double x1, double x2, KMetric &K)
{
    double r = exp(x1);
    // theta = pi (x2 + (1-h)/(2 pi) sin(2 pi x2)): both sines from sincospi
    double st, ct;
    sincos_pi(2.0 * x2, &st, &ct);
    double dth = kPi * (1.0 + (1.0 - hs) * ct);
    double s, c;
    sincos_pi(x2 + (0.5 / kPi) * (1.0 - hs) * st, &s, &c);
    K.r = r;
    if (!DERIV) {
        double s2 = s * s, S = r * r + a * a * c * c, z = 2.0 * M * r / S;
        K.g00 = z - 1.0;
        K.g01 = z * r;
        K.g03 = -a * z * s2;
        K.g11 = (1.0 + z) * r * r;
        K.g13 = -a * (1.0 + z) * s2 * r;
        K.g22 = S * dth * dth;
        K.g33 = s2 * (S + a * a * (1.0 + z) * s2);
        double D = r * r - 2.0 * M * r + a * a;
        K.u00 = -(1.0 + z);
        K.u01 = z / r;
        K.u11 = D / (S * r * r);
        K.u13 = a / (S * r);
        K.u22 = 1.0 / (S * dth * dth);
        K.u33 = 1.0 / (S * s2);
        return;
    }
    D3 R{r, r, 0.0};
    D3 Dth{dth, 0.0, -2.0 * kPi * kPi * (1.0 - hs) * st};
    D3 Sn{s, 0.0, c * dth}, Cs{c, 0.0, -s * dth};
    D3 S2 = Sn * Sn, C2 = Cs * Cs;
    D3 S = R * R + (a * a) * C2;
    // one reciprocal, of Sigma r^2 dth^2, serves 1/Sigma and the inverse
    // metric's quotients below
    const double q = 1.0 / (S.v * r * r * dth * dth);
    const double iS = q * (r * r * dth * dth);
    D3 Z;
    Z.v = 2.0 * M * r * iS;
    Z.d1 = (2.0 * M * R.d1 - Z.v * S.d1) * iS;
    Z.d2 = (-Z.v * S.d2) * iS;
    D3 one{1.0, 0.0, 0.0};
    D3 Zp = 1.0 + Z;
    D3 g[7];
    g[0] = Z - one;
    g[1] = Z * R;
    g[2] = (-a) * (Z * S2);
    g[3] = Zp * (R * R);
    g[4] = (-a) * (Zp * S2 * R);
    g[5] = S * (Dth * Dth);
    g[6] = S2 * (S + (a * a) * (Zp * S2));
    K.g00 = g[0].v; K.g01 = g[1].v; K.g03 = g[2].v; K.g11 = g[3].v; K.g13 = g[4].v; K.g22 = g[5].v; K.g33 = g[6].v;
#pragma unroll
    for (int i = 0; i < 7; ++i) { K.d1[i] = g[i].d1; K.d2[i] = g[i].d2; }
    // inverse: the reciprocal q serves four quotients; the sin^2 quotient
    // keeps its own division (infinite on the axis, as before)
    double D = r * r - 2.0 * M * r + a * a;
    double Sv = S.v, z = Z.v;
    const double iSr2 = q * (dth * dth);                   // 1 / (Sigma r^2)
    K.u00 = -(1.0 + z);
    K.u01 = z * (iSr2 * Sv * r);                           // z / r
    K.u11 = D * iSr2;
    K.u13 = a * (iSr2 * r);                                // a / (Sigma r)
    K.u22 = q * (r * r);                                   // 1 / (Sigma dth^2)
    K.u33 = 1.0 / (Sv * S2.v);
}

// g(a, b) from the seven non-zero components.
struct GKerr {
    const KMetric &K;
    GM_HD double dot(const double *a, const double *b) const
    {
        return K.g00 * (a[0] * b[0]) + K.g01 * (a[0] * b[1] + a[1] * b[0]) + K.g03 * (a[0] * b[3] + a[3] * b[0])
             + K.g11 * (a[1] * b[1]) + K.g13 * (a[1] * b[3] + a[3] * b[1]) + K.g22 * (a[2] * b[2])
             + K.g33 * (a[3] * b[3]);
    }
};

GM_HD void kerr_full(const KMetric &K, double g[4][4])
{
    g[0][0] = K.g00; g[0][1] = K.g01; g[0][2] = 0.0; g[0][3] = K.g03;
    g[1][0] = K.g01; g[1][1] = K.g11; g[1][2] = 0.0; g[1][3] = K.g13;
    g[2][0] = 0.0;   g[2][1] = 0.0;   g[2][2] = K.g22; g[2][3] = 0.0;
    g[3][0] = K.g03; g[3][1] = K.g13; g[3][2] = 0.0; g[3][3] = K.g33;
}

GM_HD double kerr_einf(const KMetric &K, const double *k)
{
    return -(K.g00 * k[0] + K.g01 * k[1] + K.g03 * k[3]);
}

// Geodesic acceleration a^m = -Gamma^m_ab k^a k^b in the contracted form
//   a^m = -g^mn [ (d_a g_nb) k^a k^b - 1/2 (d_n g_ab) k^a k^b ],
// only x1 and x2 derivatives being non-zero.
GM_HD void kerr_accel(const KMetric &K, const double *k, double *acc)
{
    // (d_c g_nb) k^b for c = 1, 2 and n = 0..3
    double A1[4], A2[4];
    A1[0] = K.d1[0] * k[0] + K.d1[1] * k[1] + K.d1[2] * k[3];
    A1[1] = K.d1[1] * k[0] + K.d1[3] * k[1] + K.d1[4] * k[3];
    A1[2] = K.d1[5] * k[2];
    A1[3] = K.d1[2] * k[0] + K.d1[4] * k[1] + K.d1[6] * k[3];
    A2[0] = K.d2[0] * k[0] + K.d2[1] * k[1] + K.d2[2] * k[3];
    A2[1] = K.d2[1] * k[0] + K.d2[3] * k[1] + K.d2[4] * k[3];
    A2[2] = K.d2[5] * k[2];
    A2[3] = K.d2[2] * k[0] + K.d2[4] * k[1] + K.d2[6] * k[3];
    double Q1 = k[0] * A1[0] + k[1] * A1[1] + k[2] * A1[2] + k[3] * A1[3];
    double Q2 = k[0] * A2[0] + k[1] * A2[1] + k[2] * A2[2] + k[3] * A2[3];
    double F0 = k[1] * A1[0] + k[2] * A2[0];
    double F1 = k[1] * A1[1] + k[2] * A2[1] - 0.5 * Q1;
    double F2 = k[1] * A1[2] + k[2] * A2[2] - 0.5 * Q2;
    double F3 = k[1] * A1[3] + k[2] * A2[3];
    acc[0] = -(K.u00 * F0 + K.u01 * F1);
    acc[1] = -(K.u01 * F0 + K.u11 * F1 + K.u13 * F3);
    acc[2] = -(K.u22 * F2);
    acc[3] = -(K.u13 * F1 + K.u33 * F3);
}

GM_HD double theta_of_x2(double hs, double x2)
{
    return kPi * x2 + 0.5 * (1.0 - hs) * sin(2.0 * kPi * x2);
}

// sqrt(-g) of the modified coordinates: Sigma |sin theta| r dtheta/dx2.
GM_HD double kerr_sqrt_neg_g(double a, double hs, double x1, double x2)
{
    double r = exp(x1);
    double th = theta_of_x2(hs, x2);
    double c = cos(th);
    double dth = kPi * (1.0 + (1.0 - hs) * cos(2.0 * kPi * x2));
    return (r * r + a * a * c * c) * fabs(sin(th)) * r * dth;
}

// Outer horizon M + sqrt(M^2 - a^2); 0 in flat spacetime.
GM_HD double kerr_horizon(double a, double M) { return M > 0.0 ? M + sqrt(M * M - a * a) : 0.0; }

}  // namespace gm
