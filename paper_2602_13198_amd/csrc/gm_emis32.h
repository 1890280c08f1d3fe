// gm_emis32.h -- the FP32 form of the opacity evaluation (device side).
//
// Emissivity, Kirchhoff absorption and the hot cross section are evaluated
// in single precision from a 64-byte zone record, in logarithms so that no
// intermediate leaves the FP32 range (1/K2(1/Theta) alone reaches ~1e43 at
// Theta = 0.01), with the hardware exp2/log: the opacities (nu alpha) come
// out as one exp of a sum of logs.  The frame products (-k.u, the pitch
// angle) stay in double, as do the geodesic state, step control, optical
// depth sums, weights and tallies.
#pragma once

#include "gm_physics.h"

namespace gm {

// FP32 zone record: u (4), field direction (4) -- normalised in flat
// spacetime, raw in Kerr -- ln A, ln(1/nu_c), Theta_e, 1/Theta_e,
// ln Theta_e, ln(n_e sigma_T), field flag, n_e.
enum { F_U0 = 0, F_B0 = 4, F_LNA = 8, F_LNINVNUC = 9, F_TH = 10, F_INVTH = 11, F_LNTH = 12,
       F_LNNESIG = 13, F_HASB = 14, F_NE = 15, F_STRIDE = 16 };

struct ShTable32 {
    const float *t;       // [kShNT][kShNE] ln(sigma_h / sigma_T)
    float lt0, inv_dt, le0, inv_de;
};

// ln g(X) for the emissivity shape g = (X^1/2 + 2^(11/12) X^1/6)^2 e^{-X^1/3},
// from ln X:  ln g = ln X / 3 + 2 ln(X^1/3 + 2^(11/12)) - X^1/3.
GM_D float ln_g_shape32(float lnX)
{
    const float a = 1.8877486f;                         // 2^(11/12)
    float x3 = __builtin_amdgcn_exp2f(lnX * (1.4426950f / 3.0f));
    return lnX * (1.0f / 3.0f) + 2.0f * __logf(x3 + a) - x3;
}

// ln(e^x - 1), accurate for small x; x itself above 15.
GM_D float ln_expm1_32(float x)
{
    return x > 15.0f ? x : __logf(expm1f(x));
}

// Bilinear interpolation of ln(sigma_h/sigma_T), clamped at the table edges.
GM_D float ln_sigma_hot32(const ShTable32 &S, float ln_theta, float ln_eps)
{
    float a = (ln_theta - S.lt0) * S.inv_dt;
    float b = (ln_eps - S.le0) * S.inv_de;
    a = fminf(fmaxf(a, 0.0f), (float)(kShNT - 1));
    b = fminf(fmaxf(b, 0.0f), (float)(kShNE - 1));
    int i = min((int)a, kShNT - 2), j = min((int)b, kShNE - 2);
    float fa = a - (float)i, fb = b - (float)j;
    const float *r0 = S.t + i * kShNE + j, *r1 = r0 + kShNE;
    return (1.0f - fa) * ((1.0f - fb) * r0[0] + fb * r0[1]) + fa * ((1.0f - fb) * r1[0] + fb * r1[1]);
}

}  // namespace gm
