// gm_track.h -- the superphoton transport kernel (device side).
//
// One lane carries one superphoton for its whole life.  A persistent grid
// processes one scattering generation per launch: waves claim photons from
// the generation's source (roots, or the children written by the previous
// generation) with one atomic per wave for all their idle lanes, and push
// the children they create into the next generation's buffer with one
// atomic per wave.  Tallies, ledgers and counters go to LDS and are merged
// into HBM when the block finishes.
#pragma once

#include "gm_frame.h"

namespace gm {

// Child superphotons in structure-of-arrays form.
struct ChildSoA {
    double *x[4], *k[4], *w;
    uint32_t *s0, *s1, *s2;
    int32_t *n_sc;
};

struct TraceRec {
    uint32_t s0, s1, s2;
    int32_t n_sc, kind, i_nu, i_theta;
    uint32_t n_steps;
    double w_birth, w_end;
    double x[4], k[4];
};

struct TrackArgs {
    // instance geometry and plasma
    const double *zrec;
    int n[3];
    double xs[3], dx[3];
    double C;                      // h ell / (m_e c^2): converts d(lambda) to cm s
    int inst;
    uint32_t key0, key1;
    // roots of the instance
    const uint32_t *zone_of_root;
    const unsigned long long *n_roots;
    double lnnu_min, lnnu_span, inv_dlnw;
    int n_wnodes;
    const double *ln_w, *fmax;
    GCheb G;
    // generation being processed
    int gen;
    ChildSoA src;
    const unsigned long long *src_count;
    unsigned long long *src_cursor;
    ChildSoA dst;
    unsigned long long *dst_count;
    unsigned long long dst_cap, backpressure;
    int *overflow;
    // tallies of the instance
    double *spec, *ledger;
    unsigned long long *stats;
    int n_nu, n_theta;
    double ln_nu_lo, inv_dln_nu;
    // transport parameters
    int scattering, bias_mode, n_sc_max, verlet_max_it;
    double bias_value, bias_max, step_h, verlet_tol, roulette_frac, roulette_p;
    long long max_steps;
    double L_unit_cm;
    ShTable sh;
    // optional trace
    TraceRec *trace;
    unsigned long long *trace_n;
    unsigned long long trace_cap;
};

struct Photon {
    double x[4], k[4];
    double w, w_birth, x1;         // x1: remaining biased optical depth
    double nua, nus, b;            // invariant opacities and bias at the current point
    double acc_wabs, acc_wcap;     // weight lost to absorption / the generation cap
    Rng rng;
    int n_sc;
    uint32_t steps;
};

struct Coef {
    double nua, nus, b;
    bool vacuum;
};

struct BlockAcc {
    double *spec, *ledger;
    unsigned long long *stats;
};

GM_D void lds_add(double *p, double v) { atomicAdd(p, v); }
GM_D void lds_inc(unsigned long long *p, unsigned long long v) { atomicAdd(p, v); }

// Zone holding a Cartesian point, or -1 outside the grid (vacuum).
GM_D int zone_cart(const TrackArgs &A, const double *x)
{
    int id[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double f = floor((x[j + 1] - A.xs[j]) / A.dx[j]);
        if (!(f >= 0.0) || f >= (double)A.n[j]) return -1;
        id[j] = (int)f;
    }
    return (id[0] * A.n[1] + id[1]) * A.n[2] + id[2];
}

// Invariant absorption and scattering coefficients (nu alpha) at a point
// (Absorption and Scattering sections): alpha = j / B_nu (Kirchhoff),
// alpha_sc = n_e sigma_h; and the bias at that point.
template <class M>
GM_D Coef coefficients(const TrackArgs &A, const double *x, const double *k, int n_sc)
{
    Coef c{0.0, 0.0, 1.0, true};
    int z = zone_cart(A, x);
    if (z < 0) return c;
    const double *zr = A.zrec + (size_t)z * Z_STRIDE;
    double ne = zr[Z_NE];
    if (!(ne > 0.0)) return c;
    c.vacuum = false;
    double g[4][4], u[4], bh[4];
    M::gcov(x, g);
    bool has_b = fluid_frame(zr, g, u, bh);
    double ef = -dot4(g, k, u);
    double nuf = ef * (kMeC2 / kH);
    double Az = zr[Z_A];
    double th = zr[Z_TH];
    if (has_b && Az > 0.0) {
        double cth = dot4(g, k, bh) / ef;
        cth = fmin(fmax(cth, -1.0), 1.0);
        double s2 = 1.0 - cth * cth;
        if (s2 > 0.0) {
            double s = sqrt(s2);
            double j = Az * s * g_shape(nuf / (zr[Z_NUC] * s));
            if (j > 0.0) {
                double alpha = j * expm1(ef / th) / (2.0 * kH * nuf * nuf * nuf / (kC * kC));
                c.nua = nuf * alpha;
            }
        }
    }
    if (A.scattering) c.nus = nuf * ne * kSigT * sigma_hot(A.sh, zr[Z_LNTH], ef);
    double b;
    if (A.bias_mode == 0) b = A.bias_value;
    else if (A.bias_mode == 1) b = A.bias_value * th * th;
    else b = (double)((n_sc + 1) * (n_sc + 1)) / (ne * kSigT * A.bias_value * A.L_unit_cm);
    c.b = fmin(fmax(b, 1.0), A.bias_max);
    return c;
}

GM_D void write_trace(const TrackArgs &A, const Photon &ph, int kind, int inu, int ith)
{
    if (!A.trace) return;
    unsigned long long i = atomicAdd(A.trace_n, 1ull);
    if (i >= A.trace_cap) return;
    TraceRec &r = A.trace[i];
    r.s0 = ph.rng.s0; r.s1 = ph.rng.s1; r.s2 = ph.rng.s2;
    r.n_sc = ph.n_sc; r.kind = kind; r.i_nu = inu; r.i_theta = ith;
    r.n_steps = ph.steps; r.w_birth = ph.w_birth; r.w_end = ph.w;
#pragma unroll
    for (int m = 0; m < 4; ++m) { r.x[m] = ph.x[m]; r.k[m] = ph.k[m]; }
}

// Book a finished photon: accumulated losses, end kind, trace.
template <class M>
GM_D void finish(const TrackArgs &A, BlockAcc &B, const Photon &ph, int kind, int inu, int ith)
{
    double g[4][4];
    M::gcov(ph.x, g);
    double e = e_inf(g, ph.k) * kMeC2;
    if (ph.acc_wabs != 0.0) { lds_add(&B.ledger[L_W_ABS], ph.acc_wabs); lds_add(&B.ledger[L_E_ABS], ph.acc_wabs * e); }
    if (ph.acc_wcap != 0.0) { lds_add(&B.ledger[L_W_CAPLOSS], ph.acc_wcap); lds_add(&B.ledger[L_E_CAPLOSS], ph.acc_wcap * e); }
    double we = ph.w * e;
    switch (kind) {
    case END_ESCAPE: lds_add(&B.ledger[L_W_ESC], ph.w); lds_add(&B.ledger[L_E_ESC], we); lds_inc(&B.stats[S_ESCAPED], 1); break;
    case END_OOB: lds_add(&B.ledger[L_W_OOB], ph.w); lds_add(&B.ledger[L_E_OOB], we); lds_inc(&B.stats[S_OOB], 1); break;
    case END_CAPTURE: lds_add(&B.ledger[L_W_CAPT], ph.w); lds_add(&B.ledger[L_E_CAPT], we); lds_inc(&B.stats[S_CAPTURED], 1); break;
    case END_STUCK: lds_add(&B.ledger[L_W_STUCK], ph.w); lds_add(&B.ledger[L_E_STUCK], we); lds_inc(&B.stats[S_STUCK], 1); break;
    default: break;
    }
    lds_inc(&B.stats[S_STEPS], ph.steps);
    lds_inc(&B.stats[S_VERLET_IT], ph.steps);   // flat: one corrector pass per step
    write_trace(A, ph, kind, inu, ith);
}

// Birth of root photon p (Sampling procedure section): position uniform in
// the zone, frequency by rejection against the zone's bound on dN/d ln nu,
// direction by rejection against j(pi/2), fluid-frame tetrad, weight w(nu).
template <class M>
GM_D void birth(const TrackArgs &A, BlockAcc &B, unsigned long long p, Photon &ph)
{
    uint32_t z = A.zone_of_root[p];
    const double *zr = A.zrec + (size_t)z * Z_STRIDE;
    ph.rng = Rng{(uint32_t)p, (uint32_t)(p >> 32), ((uint32_t)A.inst << 8) | 1u, 0u};
    int i3 = (int)(z % (uint32_t)A.n[2]);
    int i2 = (int)((z / (uint32_t)A.n[2]) % (uint32_t)A.n[1]);
    int i1 = (int)(z / ((uint32_t)A.n[2] * (uint32_t)A.n[1]));
    ph.x[0] = 0.0;
    ph.x[1] = A.xs[0] + (i1 + rng_uniform(ph.rng, A.key0, A.key1)) * A.dx[0];
    ph.x[2] = A.xs[1] + (i2 + rng_uniform(ph.rng, A.key0, A.key1)) * A.dx[1];
    ph.x[3] = A.xs[2] + (i3 + rng_uniform(ph.rng, A.key0, A.key1)) * A.dx[2];
    const double Az = zr[Z_A], nuc = zr[Z_NUC];
    const double fm = A.fmax[z];
    const double dlnw = A.lnnu_span / (A.n_wnodes - 1);
    double lnnu, nu, lnw;
    uint32_t trials = 0, over = 0;
    for (int64_t it = 0;; ++it) {
        lnnu = A.lnnu_min + rng_uniform(ph.rng, A.key0, A.key1) * A.lnnu_span;
        nu = exp(lnnu);
        double u2 = rng_uniform(ph.rng, A.key0, A.key1);
        double a = (lnnu - A.lnnu_min) / dlnw;
        int i = (int)floor(a);
        i = max(0, min(i, A.n_wnodes - 2));
        double f = a - i;
        lnw = (1.0 - f) * A.ln_w[i] + f * A.ln_w[i + 1];
        double F = 4.0 * kPi * Az * G_of_Xc(A.G, nu / nuc) / exp(lnw);
        ++trials;
        over += (F > fm) ? 1u : 0u;
        if (u2 < F / fm || it >= kMaxTrials) break;
    }
    double jmax = Az * g_shape(nu / nuc);
    double cth;
    uint32_t dtr = 0;
    for (int64_t it = 0;; ++it) {
        cth = 2.0 * rng_uniform(ph.rng, A.key0, A.key1) - 1.0;
        double u4 = rng_uniform(ph.rng, A.key0, A.key1);
        ++dtr;
        double s2 = 1.0 - cth * cth;
        double j = 0.0;
        if (s2 > 0.0) {
            double s = sqrt(s2);
            j = Az * s * g_shape(nu / (nuc * s));
        }
        if (u4 < j / jmax || it >= kMaxTrials) break;
    }
    double phi = 2.0 * kPi * rng_uniform(ph.rng, A.key0, A.key1);
    double g[4][4], u[4], bh[4], e[4][4];
    M::gcov(ph.x, g);
    fluid_frame(zr, g, u, bh);
    emission_tetrad(g, u, bh, e);
    double eps = kH * nu / kMeC2;
    double sth = sqrt(1.0 - cth * cth);
    double kf[4] = {eps, eps * sth * cos(phi), eps * sth * sin(phi), eps * cth};
#pragma unroll
    for (int m = 0; m < 4; ++m) ph.k[m] = kf[0] * e[0][m] + kf[1] * e[1][m] + kf[2] * e[2][m] + kf[3] * e[3][m];
    ph.w = ph.w_birth = exp(lnw);
    ph.x1 = -log(1.0 - rng_uniform(ph.rng, A.key0, A.key1));
    ph.n_sc = 0;
    ph.steps = 0;
    ph.acc_wabs = ph.acc_wcap = 0.0;
    lds_add(&B.ledger[L_W_EMIT], ph.w);
    lds_add(&B.ledger[L_E_EMIT], ph.w * e_inf(g, ph.k) * kMeC2);
    lds_inc(&B.stats[S_ROOTS], 1);
    lds_inc(&B.stats[S_NU_TRIALS], trials);
    if (over) lds_inc(&B.stats[S_OVERSHOOT], over);
    lds_inc(&B.stats[S_DIR_TRIALS], dtr);
    lds_inc(&B.stats[S_GEN0], 1);
    Coef c = coefficients<M>(A, ph.x, ph.k, 0);
    ph.nua = c.nua; ph.nus = c.nus; ph.b = c.b;
}

template <class M>
GM_D void load_child(const TrackArgs &A, BlockAcc &B, unsigned long long i, Photon &ph)
{
#pragma unroll
    for (int m = 0; m < 4; ++m) { ph.x[m] = A.src.x[m][i]; ph.k[m] = A.src.k[m][i]; }
    ph.w = ph.w_birth = A.src.w[i];
    ph.rng = Rng{A.src.s0[i], A.src.s1[i], A.src.s2[i], 0u};
    ph.n_sc = A.src.n_sc[i];
    ph.steps = 0;
    ph.acc_wabs = ph.acc_wcap = 0.0;
    ph.x1 = -log(1.0 - rng_uniform(ph.rng, A.key0, A.key1));
    lds_inc(&B.stats[S_CHILDREN], 1);
    lds_inc(&B.stats[S_GEN0 + min(ph.n_sc, 15)], 1);
    Coef c = coefficients<M>(A, ph.x, ph.k, ph.n_sc);
    ph.nua = c.nua; ph.nus = c.nus; ph.b = c.b;
}

// State carried from a step into the wave's scattering pass.
struct Pending {
    double xn[4], kn[4];
    double f, b, tau_a;
};

// Tally an escaping photon into its (theta, nu) bin.
template <class M>
GM_D void tally_escape(const TrackArgs &A, BlockAcc &B, const Photon &ph)
{
    double g[4][4];
    M::gcov(ph.x, g);
    double einf = e_inf(g, ph.k);
    double nuinf = einf * (kMeC2 / kH);
    double fi = floor((log(nuinf) - A.ln_nu_lo) * A.inv_dln_nu);
    if (!(fi >= 0.0 && fi < (double)A.n_nu)) {
        finish<M>(A, B, ph, END_OOB, -1, -1);
        return;
    }
    double kk = sqrt(ph.k[1] * ph.k[1] + ph.k[2] * ph.k[2] + ph.k[3] * ph.k[3]);
    double th = acos(ph.k[3] / kk);
    int ith = (int)floor(th * A.n_theta / kPi);
    ith = max(0, min(ith, A.n_theta - 1));
    int inu = (int)fi;
    double E = ph.w * einf * kMeC2;
    double *bin = B.spec + ((size_t)ith * A.n_nu + inu) * 3;
    lds_add(&bin[0], E);
    lds_add(&bin[1], E * E);
    lds_add(&bin[2], 1.0);
    finish<M>(A, B, ph, END_ESCAPE, inu, ith);
}

// One transport step (geodesic section: velocity Verlet; Absorption
// section: trapezoid optical depth; Scattering section: biased scattering
// test).  Returns 1 when the photon scatters in this step (handled by the
// wave's scattering pass), else 0; `alive` drops when the photon ends.
template <class M>
GM_D int step(const TrackArgs &A, BlockAcc &B, Photon &ph, Pending &pd, bool &alive, bool &stepped)
{
    stepped = false;
    if ((long long)ph.steps >= A.max_steps) {
        finish<M>(A, B, ph, END_STUCK, -1, -1);
        alive = false;
        return 0;
    }
    double dl = 1.0 / 0.0;
#pragma unroll
    for (int j = 1; j <= 3; ++j)
        if (ph.k[j] != 0.0) dl = fmin(dl, A.dx[j - 1] / fabs(ph.k[j]));
    dl *= A.step_h;
    double xn[4], kn[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) { xn[m] = ph.x[m] + ph.k[m] * dl; kn[m] = ph.k[m]; }
    Coef c1 = coefficients<M>(A, xn, kn, ph.n_sc);
    ph.steps += 1;
    stepped = true;
    double tau_a = 0.5 * (ph.nua + c1.nua) * A.C * dl;
    double tau_s = A.scattering ? 0.5 * (ph.nus + c1.nus) * A.C * dl : 0.0;
    double b = c1.vacuum ? ph.b : c1.b;
    if (A.scattering && ph.n_sc < A.n_sc_max && b * tau_s > ph.x1) {
#pragma unroll
        for (int m = 0; m < 4; ++m) { pd.xn[m] = xn[m]; pd.kn[m] = kn[m]; }
        pd.f = ph.x1 / (b * tau_s);
        pd.b = b;
        pd.tau_a = tau_a;
        return 1;
    }
    if (A.scattering) {
        if (ph.n_sc < A.n_sc_max) {
            ph.x1 -= b * tau_s;
        } else {   // generation cap: extinction without a child
            double wb = ph.w;
            ph.w *= exp(-tau_s);
            ph.acc_wcap += wb - ph.w;
        }
    }
    double wb = ph.w;
    ph.w *= exp(-tau_a);
    ph.acc_wabs += wb - ph.w;
#pragma unroll
    for (int m = 0; m < 4; ++m) { ph.x[m] = xn[m]; ph.k[m] = kn[m]; }
    ph.nua = c1.nua; ph.nus = c1.nus; ph.b = b;
    bool escaped = false;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double lo = A.xs[j], hi = A.xs[j] + A.n[j] * A.dx[j];
        escaped |= (ph.x[j + 1] < lo) || (ph.x[j + 1] >= hi);
    }
    if (escaped) {
        tally_escape<M>(A, B, ph);
        alive = false;
    }
    return 0;
}

// Russian roulette for low-weight photons (reading: below roulette_frac of
// the birth weight, survive with probability roulette_p).
template <class M>
GM_D void roulette(const TrackArgs &A, BlockAcc &B, Photon &ph, bool &alive)
{
    if (!(ph.w < A.roulette_frac * ph.w_birth)) return;
    double g[4][4];
    M::gcov(ph.x, g);
    double e = e_inf(g, ph.k) * kMeC2;
    if (rng_uniform(ph.rng, A.key0, A.key1) < A.roulette_p) {
        double gain = ph.w * (1.0 / A.roulette_p - 1.0);
        lds_add(&B.ledger[L_W_ROUL], gain);
        lds_add(&B.ledger[L_E_ROUL], gain * e);
        ph.w /= A.roulette_p;
        lds_inc(&B.stats[S_ROUL_SURVIVE], 1);
    } else {
        lds_add(&B.ledger[L_W_ROUL], -ph.w);
        lds_add(&B.ledger[L_E_ROUL], -ph.w * e);
        lds_inc(&B.stats[S_ROUL_KILL], 1);
        ph.w = 0.0;
        finish<M>(A, B, ph, END_ROULETTE, -1, -1);
        alive = false;
    }
}

// Scattering pass for the lanes whose step found a scattering point: the
// child is built from the parent's stream (Scattering section), pushed
// with one atomic per wave, and the parent continues from the scattering
// point with weight w (1 - 1/b).
template <class M>
GM_D void scatter_pass(const TrackArgs &A, BlockAcc &B, Photon &ph, const Pending &pd, bool want,
                       bool &alive)
{
    double xs[4], kc[4];
    double wchild = 0.0;
    uint32_t blk_at = 0;
    Rng crng{0, 0, 0, 0};
    if (want) {
        double ks[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            xs[m] = ph.x[m] + pd.f * (pd.xn[m] - ph.x[m]);
            ks[m] = ph.k[m] + pd.f * (pd.kn[m] - ph.k[m]);
        }
        double wb = ph.w;
        ph.w *= exp(-pd.f * pd.tau_a);
        ph.acc_wabs += wb - ph.w;
        wchild = ph.w / pd.b;
        // plasma of the scattering point, else of the step's start, else its end
        int z = zone_cart(A, xs);
        if (z >= 0 && !(A.zrec[(size_t)z * Z_STRIDE + Z_NE] > 0.0)) z = -1;
        if (z < 0) {
            z = zone_cart(A, ph.x);
            if (z >= 0 && !(A.zrec[(size_t)z * Z_STRIDE + Z_NE] > 0.0)) z = -1;
        }
        if (z < 0) {
            z = zone_cart(A, pd.xn);
            if (z >= 0 && !(A.zrec[(size_t)z * Z_STRIDE + Z_NE] > 0.0)) z = -1;
        }
        blk_at = ph.rng.block;
        double g[4][4];
        M::gcov(xs, g);
        if (z >= 0) {
            const double *zr = A.zrec + (size_t)z * Z_STRIDE;
            double u[4], bh[4], e[4][4];
            bool has_b = fluid_frame(zr, g, u, bh);
            double eps = scatter_tetrad(g, u, bh, has_b, ks, e);
            double kf[4];
            ScatterCount cnt{0, 0};
            scatter_in_frame(ph.rng, A.key0, A.key1, zr[Z_TH], eps, kf, cnt);
#pragma unroll
            for (int m = 0; m < 4; ++m) kc[m] = kf[0] * e[0][m] + kf[1] * e[1][m] + kf[2] * e[2][m] + kf[3] * e[3][m];
            lds_inc(&B.stats[S_E_TRIALS], cnt.e_trials);
            lds_inc(&B.stats[S_ANG_TRIALS], cnt.ang_trials);
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) kc[m] = ks[m];
        }
        lds_add(&B.ledger[L_E_COMPTON], wchild * (e_inf(g, kc) - e_inf(g, ks)) * kMeC2);
        lds_inc(&B.stats[S_SCATTER], 1);
        crng = child_rng(ph.rng, blk_at, A.key0, A.key1);
        // the parent continues from the scattering point
        ph.w *= (1.0 - 1.0 / pd.b);
        ph.x1 = -log(1.0 - rng_uniform(ph.rng, A.key0, A.key1));
#pragma unroll
        for (int m = 0; m < 4; ++m) { ph.x[m] = xs[m]; ph.k[m] = ks[m]; }
        Coef c0 = coefficients<M>(A, ph.x, ph.k, ph.n_sc);
        ph.nua = c0.nua; ph.nus = c0.nus;
        if (!c0.vacuum) ph.b = c0.b;
        if (pd.b == 1.0) {
            finish<M>(A, B, ph, END_SPLIT, -1, -1);
            alive = false;
        }
    }
    // one slot reservation per wave
    uint64_t mask = __ballot(want);
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(A.dst_count, (unsigned long long)__popcll(mask));
    base = bcast_u64(base, 0);
    if (want) {
        unsigned long long i = base + rank_in_mask(mask);
        if (i < A.dst_cap) {
#pragma unroll
            for (int m = 0; m < 4; ++m) { A.dst.x[m][i] = xs[m]; A.dst.k[m][i] = kc[m]; }
            A.dst.w[i] = wchild;
            A.dst.s0[i] = crng.s0; A.dst.s1[i] = crng.s1; A.dst.s2[i] = crng.s2;
            A.dst.n_sc[i] = ph.n_sc + 1;
        } else {
            atomicOr(A.overflow, 1);
        }
    }
}

constexpr int kRefillMin = 16;   // claim new photons once this many lanes idle

template <class M>
__global__ __launch_bounds__(256) void track_kernel(TrackArgs A)
{
    extern __shared__ double lds[];
    BlockAcc B;
    B.ledger = lds;
    B.stats = reinterpret_cast<unsigned long long *>(lds + L_N);
    B.spec = lds + L_N + S_N;
    const int nspec = A.n_theta * A.n_nu * 3;
    for (int i = threadIdx.x; i < L_N + S_N + nspec; i += blockDim.x) lds[i] = 0.0;
    __syncthreads();

    // a generation never reads past its queue's capacity (an overflowed
    // count is reported to the host through A.overflow)
    const unsigned long long n_src =
        (A.gen == 0) ? *A.n_roots : min(*A.src_count, A.dst_cap);
    Photon ph;
    Pending pd;
    bool alive = false, exhausted = false;
    for (;;) {
        uint64_t idle = __ballot(!alive);
        int nidle = __popcll(idle);
        if (!exhausted && (nidle >= kRefillMin || nidle == 64)) {
            unsigned long long base = 0;
            if (lane_id() == 0) {
                bool hold = (A.gen == 0) &&
                            (__hip_atomic_load(A.dst_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= A.backpressure);
                base = hold ? ~0ull : atomicAdd(A.src_cursor, (unsigned long long)nidle);
            }
            base = bcast_u64(base, 0);
            if (base == ~0ull || base + (unsigned long long)nidle >= n_src) exhausted = true;
            if (base != ~0ull && !alive) {
                unsigned long long idx = base + rank_in_mask(idle);
                if (idx < n_src) {
                    alive = true;
                    if (A.gen == 0) birth<M>(A, B, idx, ph);
                    else load_child<M>(A, B, idx, ph);
                }
            }
        }
        if (!__any(alive)) break;
        bool stepped = false;
        int want = 0;
        if (alive) want = step<M>(A, B, ph, pd, alive, stepped);
        if (__any(want)) scatter_pass<M>(A, B, ph, pd, want != 0, alive);
        if (alive && stepped) roulette<M>(A, B, ph, alive);
    }

    __syncthreads();
    for (int i = threadIdx.x; i < nspec; i += blockDim.x) {
        double v = B.spec[i];
        if (v != 0.0) atomicAdd(&A.spec[i], v);
    }
    for (int i = threadIdx.x; i < L_N; i += blockDim.x) {
        double v = B.ledger[i];
        if (v != 0.0) atomicAdd(&A.ledger[i], v);
    }
    for (int i = threadIdx.x; i < S_N; i += blockDim.x) {
        unsigned long long v = B.stats[i];
        if (v) atomicAdd(&A.stats[i], v);
    }
}

}  // namespace gm
