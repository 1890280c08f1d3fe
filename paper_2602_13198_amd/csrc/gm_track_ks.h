// gm_track_ks.h -- superphoton transport in Kerr spacetime, modified
// Kerr-Schild coordinates (device side).
//
// Same queue structure as the flat path: the tracker keeps one lane per
// photon for its whole life and writes scattering events to the next
// generation's queue; scatter_kernel_ks turns events into children.  Each
// tracker iteration evaluates the metric (with its x1/x2 derivatives) at
// exactly one point:
//   step     the Verlet predictor point of a new step; the corrector reuses
//            the derivatives there for every pass,
//   substep  the scattering point: a Verlet step over the fraction f of the
//            step that found the scattering, from that step's start; the
//            scattering, the parent's restart there and its roulette follow
//            in the same iteration,
//   load     the point of a photon just taken from the queue,
// so the cases share one code path and a wave does not diverge on them.
// Energies at infinity -k_t change along the path: each photon keeps its
// current e_inf, and its absorption, cap-loss and drift ledgers are summed
// per photon with the e_inf at the start of each step.
#pragma once

#include "gm_track.h"

namespace gm {

struct PhotonK {
    double x[3], k[4], a[4];       // position (x1, x2, x3), wavevector, geodesic acceleration
    double w, wb, x1;              // weight, birth weight, remaining biased depth
    double nua, nus, b;            // opacities and bias at the current point; while a
                                   // substep is pending, nua holds its length and nus
                                   // the bias of the scattering it leads to
    double r, e;                   // r and e_inf = -k_t at the current point
    double acc_wabs, acc_eabs;     // weight (and weight x e_inf) absorbed
    double acc_wcap, acc_ecap;     // ... extinguished at the generation cap
    double acc_edrift;             // sum of w * (change of e_inf) along steps
    Rng rng;
    int n_sc, inst;
    uint32_t ev;                   // event-log record that created the photon
    int zone_end;                  // zone of the end of the step that found a scattering
    uint32_t steps, vit;
    int ncoef;                     // opacity evaluations (one per iteration)
};

enum { MODE_STEP = 0, MODE_SUBSTEP = 1, MODE_LOAD = 2 };

GM_D void load_photon_ks(const PhotonQ &Q, unsigned long long i, PhotonK &ph)
{
#pragma unroll
    for (int m = 0; m < 3; ++m) ph.x[m] = Q.x[m][i];
#pragma unroll
    for (int m = 0; m < 4; ++m) ph.k[m] = Q.k[m][i];
    ph.w = Q.w[i]; ph.wb = Q.wb[i]; ph.x1 = Q.x1[i];
    ph.rng = Rng{Q.s0[i], Q.s1[i], Q.s2[i], Q.blk[i]};
    ph.n_sc = Q.n_sc[i];
    ph.inst = Q.inst[i];
    ph.ev = Q.ev[i];
    ph.steps = 0;
    ph.vit = 0;
    ph.ncoef = 0;
    ph.acc_wabs = ph.acc_eabs = ph.acc_wcap = ph.acc_ecap = ph.acc_edrift = 0.0;
}

GM_D void write_trace_ks(const TArgs &A, const PhotonK &ph, int kind, int inu, int ith)
{
    if (!A.trace) return;
    unsigned long long i = atomicAdd(A.trace_n, 1ull);
    if (i >= A.trace_cap) return;
    TraceRec &r = A.trace[i];
    r.s0 = ph.rng.s0; r.s1 = ph.rng.s1; r.s2 = ph.rng.s2;
    r.n_sc = ph.n_sc; r.kind = kind; r.i_nu = inu; r.i_theta = ith;
    r.n_steps = ph.steps; r.w_birth = ph.wb; r.w_end = ph.w;
    r.x[0] = 0.0;               // the coordinate time is not carried
#pragma unroll
    for (int m = 0; m < 3; ++m) r.x[m + 1] = ph.x[m];
#pragma unroll
    for (int m = 0; m < 4; ++m) r.k[m] = ph.k[m];
}

// Book a finished photon: tally at the record radius (frequency at infinity
// from -k_t, inclination from the polar coordinate), ledgers, trace.
GM_D void finish_ks(const TArgs &A, BlockAcc &B, const PhotonK &ph, int kind)
{
    double e = ph.e * kMeC2;
    int inu = -1, ith = -1;
    if (kind == END_ESCAPE) {
        double nuinf = ph.e * (kMeC2 / kH);
        double fi = floor((log(nuinf) - A.ln_nu_lo) * A.inv_dln_nu);
        if (!(fi >= 0.0 && fi < (double)A.n_nu)) {
            kind = END_OOB;
        } else {
            double th = theta_of_x2(A.h_slope, ph.x[1]);
            ith = max(0, min((int)floor(th * A.n_theta / kPi), A.n_theta - 1));
            inu = (int)fi;
            double E = ph.w * e;
            double *bin = (B.spec ? B.spec : A.spec) + ((size_t)ith * A.n_nu + inu) * 3;
            lds_add(&bin[0], E);
            lds_add(&bin[1], E * E);
            lds_add(&bin[2], 1.0);
            score_escape(A, ph.ev, ith, inu, E);
        }
    }
    if (ph.acc_wabs != 0.0) { lds_add(&B.ledger[L_W_ABS], ph.acc_wabs); lds_add(&B.ledger[L_E_ABS], ph.acc_eabs * kMeC2); }
    if (ph.acc_wcap != 0.0) { lds_add(&B.ledger[L_W_CAPLOSS], ph.acc_wcap); lds_add(&B.ledger[L_E_CAPLOSS], ph.acc_ecap * kMeC2); }
    if (ph.acc_edrift != 0.0) lds_add(&B.ledger[L_E_DRIFT], ph.acc_edrift * kMeC2);
    double we = ph.w * e;
    switch (kind) {
    case END_ESCAPE: lds_add(&B.ledger[L_W_ESC], ph.w); lds_add(&B.ledger[L_E_ESC], we); lds_inc(&B.stats[S_ESCAPED], 1); break;
    case END_OOB: lds_add(&B.ledger[L_W_OOB], ph.w); lds_add(&B.ledger[L_E_OOB], we); lds_inc(&B.stats[S_OOB], 1); break;
    case END_CAPTURE: lds_add(&B.ledger[L_W_CAPT], ph.w); lds_add(&B.ledger[L_E_CAPT], we); lds_inc(&B.stats[S_CAPTURED], 1); break;
    case END_STUCK: lds_add(&B.ledger[L_W_STUCK], ph.w); lds_add(&B.ledger[L_E_STUCK], we); lds_inc(&B.stats[S_STUCK], 1); break;
    default: break;
    }
    lds_inc(&B.stats[S_STEPS], ph.steps);
    lds_inc(&B.stats[S_VERLET_IT], ph.vit);
    lds_inc(&B.stats[S_COEF], (unsigned long long)ph.ncoef);
    write_trace_ks(A, ph, kind, inu, ith);
}

// Step size: step_h over the largest rate of zone crossing (times step_far
// for an outgoing photon beyond r_far), the azimuth
// scaled like the polar angle at most; moving inward, at most half the
// coordinate distance to the horizon; at most a tenth of the x2 distance to
// the nearer pole (k^phi grows like 1/sin^2 theta there, and a longer step
// leaves the corrector without a fixed point).
GM_D double step_ks(const TArgs &A, const PhotonK &ph)
{
    // the least of the quotients num/den (positive denominators) is chosen by
    // cross-multiplied comparisons, so the step costs one division
    double num = (ph.k[1] > 0.0 && ph.r > A.r_far) ? A.step_h * A.step_far : A.step_h;
    double den = fmax(fmax(fabs(ph.k[1]) * A.inv_sc[0], fabs(ph.k[2]) * A.inv_sc[1]),
                      fabs(ph.k[3]) * A.inv_sc[2]);
    if (ph.k[1] < 0.0) {
        const double n1 = 0.5 * (ph.r - A.r_h), d1 = ph.r * fabs(ph.k[1]);
        if (n1 * den < num * d1) { num = n1; den = d1; }
    }
    const double dp = fmax(fmin(ph.x[1], 1.0 - ph.x[1]), 1e-9);
    const double n2 = 0.1 * dp, d2 = fabs(ph.k[2]);   // no bound when k^2 = 0
    if (n2 * den < num * d2) { num = n2; den = d2; }
    return num / den;
}

// Plasma zone of a scattering point: the point's own zone when it holds
// plasma, else that of the step's start, else of its end; -1 if none does.
GM_D int plasma_zone(const TArgs &A, int z)
{
    return (z >= 0 && A.zrec[(size_t)z * Z_STRIDE + Z_NE] > 0.0) ? z : -1;
}

// Kerr tracker (geodesic section: velocity Verlet with an iterated
// corrector; Absorption and Scattering sections).  Scheduling as in the
// flat tracker: lanes idle until enough of the wave is idle, then claim
// queue entries together and run the finished photons' bookkeeping.  CB:
// every instance of the launch has the constant bias.
template <int WAVES, bool F32, bool BATCHED, bool CB>
__global__ __launch_bounds__(256, WAVES) void track_kernel_ks(TArgs L)
{
    extern __shared__ double lds[];
    const int stride = L.lds_stride;
    lds_zero(lds, L.n_inst, stride);
    EvStage ev = ev_stage(lds, L.n_inst, stride);
    const unsigned long long n_src = min(*L.src_count, L.cap);
    PhotonK ph;
    ph.inst = 0;
    bool alive = false, exhausted = false;
    int mode = MODE_STEP;
    int ended = 0;
    for (;;) {
        uint64_t idle = __ballot(!alive);
        int nidle = __popcll(idle);
        if (nidle >= L.refill_min || nidle == 64) {
            // bookkeeping of the lanes that ended (one instance at a time)
            if constexpr (BATCHED) {
                for (uint64_t todo = __ballot(ended != 0); todo;) {
                    const int iu = uniform_inst(todo, ph.inst);
                    const bool mine = ended != 0 && ph.inst == iu;
                    todo &= ~__ballot(mine);
                    if (mine) {
                        BlockAcc B = lds_acc(lds, stride, iu);
                        finish_ks(L.insts[iu], B, ph, ended);
                        ended = 0;
                    }
                }
            } else if (ended) {
                BlockAcc B = lds_acc(lds, stride, 0);
                finish_ks(L, B, ph, ended);
                ended = 0;
            }
            if (!exhausted) {
                unsigned long long base = 0;
                if (lane_id() == 0) base = atomicAdd(L.src_cursor, (unsigned long long)nidle);
                base = bcast_u64(base, 0);
                if (base + (unsigned long long)nidle >= n_src) exhausted = true;
                if (!alive) {
                    unsigned long long idx = base + rank_in_mask(idle);
                    if (idx < n_src) {
                        load_photon_ks(L.src, idx, ph);
                        alive = true;
                        mode = MODE_LOAD;
                    }
                }
            }
        }
        if (!__any(alive)) break;
        bool scat = false;
        double wchild = 0.0;
        int zs = -1;
        Rng ev_rng{0u, 0u, 0u, 0u};
        if (alive && mode == MODE_STEP && (long long)ph.steps >= L.max_steps) {
            ended = END_STUCK;
            alive = false;
        }
        // one step (or restart, or load evaluation) of this lane's photon
        // with the arguments of its instance
        auto advance = [&](const TArgs &A, BlockAcc &B) {
            // ---- the point of this iteration ----
            double P[3], kn[4], an[4], a_fresh[4] = {0.0, 0.0, 0.0, 0.0};
            double dl = 0.0;
            bool found_sc = false;
            if (mode == MODE_STEP) dl = step_ks(A, ph);
            else if (mode == MODE_SUBSTEP) dl = ph.nua;
            if (mode != MODE_LOAD) {
#pragma unroll
                for (int m = 0; m < 3; ++m) P[m] = ph.x[m] + ph.k[m + 1] * dl + 0.5 * ph.a[m + 1] * dl * dl;
            } else {
#pragma unroll
                for (int m = 0; m < 3; ++m) P[m] = ph.x[m];
            }
            // the zone of the point (-1 beyond the outermost plasma zone: no
            // zone lookup and no record load, most steps on the way out), and
            // a touch of its record now (the record is one cache line), so
            // that the line arrives while the metric and the corrector are
            // computed; the pole reflection below moves the point to another
            // zone, whose record then comes later
            const bool beyond = floor((P[0] - A.xs[0]) * A.inv_dx[0]) > A.i1_plasma_max;
            int zn = beyond ? -1 : zone_ks(A, P[0], P[1], P[2]);
            double ne_touch = 0.0;
            if (zn >= 0) {
                if constexpr (F32) ne_touch = (double)A.zrec32[(size_t)zn * F_STRIDE + F_NE];
                else ne_touch = A.zrec[(size_t)zn * Z_STRIDE + Z_NE];
            }
            KMetric K;
            kerr_metric<true>(A.a_spin, A.mass, A.h_slope, P[0], P[1], K);
            if (mode != MODE_LOAD) {
                // corrector: a' at the predicted wavevector, k' = k + (a + a') dl / 2
                double kp[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) kp[m] = ph.k[m] + ph.a[m] * dl;
                int it = 0;
                for (;;) {
                    ++it;
                    kerr_accel(K, kp, an);
                    double num = 0.0, den = 0.0;
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        kn[m] = ph.k[m] + 0.5 * (ph.a[m] + an[m]) * dl;
                        num += fabs(kn[m] - kp[m]);
                        den += fabs(kn[m]);
                        kp[m] = kn[m];
                    }
                    // relative change num / den below the tolerance (den > 0)
                    if (num < A.verlet_tol * (den + 1e-300) || it >= A.verlet_max_it) break;
                }
                ph.vit += (uint32_t)it;
                // the scattering point restarts with the acceleration of the
                // final wavevector there
                if (mode == MODE_SUBSTEP) kerr_accel(K, kn, a_fresh);
                // through the pole of the modified coordinates: reflect (the
                // metric is even about the pole, so reflected position,
                // wavevector and acceleration form a geodesic state again)
                if (P[1] < 0.0 || P[1] > 1.0) {
                    P[1] = (P[1] < 0.0) ? -P[1] : 2.0 - P[1];
                    P[2] += kPi;
                    kn[2] = -kn[2];
                    an[2] = -an[2];
                    a_fresh[2] = -a_fresh[2];
                    if (!beyond) zn = zone_ks(A, P[0], P[1], P[2]);
                }
            } else {
#pragma unroll
                for (int m = 0; m < 4; ++m) kn[m] = ph.k[m];
                kerr_accel(K, kn, a_fresh);
            }
            const double e_here = kerr_einf(K, kn);
            if (mode == MODE_SUBSTEP) {
                // ---- scattering at (P, kn): child event, parent's split ----
                const double b_sc = ph.nus;
                ph.acc_edrift += ph.w * (e_here - ph.e);
                wchild = ph.w / b_sc;
                zs = plasma_zone(A, zn);      // beyond: no plasma either way
                if (zs < 0) zs = plasma_zone(A, zone_ks(A, ph.x[0], ph.x[1], ph.x[2]));
                if (zs < 0) zs = plasma_zone(A, ph.zone_end);
                ev_rng = ph.rng;              // the parent's stream at the event
                ph.w *= (1.0 - 1.0 / b_sc);
                ph.x1 = -log(1.0 - rng_uniform(ph.rng, A.key0, A.key1));
                ph.e = e_here;
                scat = true;
                if (b_sc == 1.0) {    // all weight went to the child
                    ended = END_SPLIT;
                    alive = false;
                }
#pragma unroll
                for (int m = 0; m < 3; ++m) ph.x[m] = P[m];
#pragma unroll
                for (int m = 0; m < 4; ++m) ph.k[m] = kn[m];
            }
            settle(ne_touch);
            Coef c1 = coefficients_at<false, F32, CB>(A, A.el, zn, GKerr{K}, kn, ph.n_sc);
            ph.ncoef += 1;
            if (mode != MODE_STEP) {
                // restart at the scattering point, or first evaluation of a
                // loaded photon: fresh acceleration and opacities here
#pragma unroll
                for (int m = 0; m < 4; ++m) ph.a[m] = a_fresh[m];
                ph.nua = c1.nua; ph.nus = c1.nus;
                ph.r = K.r;
                if (mode == MODE_LOAD) {
                    ph.b = c1.b;
                    ph.e = e_here;
                } else if (!c1.vacuum) {
                    ph.b = c1.b;
                }
            } else {
                ph.steps += 1;
                // ---- optical depths by the trapezoid rule ----
                double tau_a = 0.5 * (ph.nua + c1.nua) * A.C * dl;
                double tau_s = A.scattering ? 0.5 * (ph.nus + c1.nus) * A.C * dl : 0.0;
                const double bf = c1.vacuum ? ph.b : c1.b;
                const double b = step_bias<CB>(A, ph.w, bf);
                const double e_old = ph.e;
                if (A.scattering && ph.n_sc < A.n_sc_max && b * tau_s > ph.x1) {
                    // ---- scattering inside the step, at the fraction f: absorb
                    // up to there now, reach the point on the next iteration ----
                    double f = ph.x1 / (b * tau_s);
                    double wbf = ph.w;
                    ph.w *= exp(-f * tau_a);
                    ph.acc_wabs += wbf - ph.w;
                    ph.acc_eabs += (wbf - ph.w) * e_old;
                    ph.nua = f * dl;
                    ph.nus = b;
                    ph.zone_end = zn;
                    found_sc = true;
                } else {
                    if (A.scattering) {
                        if (ph.n_sc < A.n_sc_max) {
                            ph.x1 -= b * tau_s;
                        } else {   // generation cap: extinction without a child
                            double wbc = ph.w;
                            ph.w *= exp(-tau_s);
                            ph.acc_wcap += wbc - ph.w;
                            ph.acc_ecap += (wbc - ph.w) * e_old;
                        }
                    }
                    double wba = ph.w;
                    if (tau_a != 0.0) ph.w *= exp(-tau_a);      // vacuum steps skip the exp
                    ph.acc_wabs += wba - ph.w;
                    ph.acc_eabs += (wba - ph.w) * e_old;
#pragma unroll
                    for (int m = 0; m < 3; ++m) ph.x[m] = P[m];
#pragma unroll
                    for (int m = 0; m < 4; ++m) { ph.k[m] = kn[m]; ph.a[m] = an[m]; }
                    ph.nua = c1.nua; ph.nus = c1.nus; ph.b = bf;
                    ph.r = K.r;
                    ph.e = e_here;
                    ph.acc_edrift += ph.w * (e_here - e_old);
                    if (K.r >= A.r_record) {
                        ended = END_ESCAPE;
                        alive = false;
                    } else if (K.r < A.r_capture) {
                        ended = END_CAPTURE;
                        alive = false;
                    }
                }
            }
            // ---- next iteration's kind; Russian roulette below roulette_frac
            // of the birth weight after a completed step or a scattering ----
            const bool roulette_now = alive && (mode == MODE_SUBSTEP || (mode == MODE_STEP && !found_sc));
            mode = found_sc ? MODE_SUBSTEP : MODE_STEP;
            if (roulette_now && ph.w < A.roulette_frac * ph.wb) {
                double e = ph.e * kMeC2;
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
                    ended = END_ROULETTE;
                    alive = false;
                }
            }
        };
        if constexpr (BATCHED) {
            // one instance at a time, with wave-uniform instance arguments
            for (uint64_t todo = __ballot(alive); todo;) {
                const int iu = uniform_inst(todo, ph.inst);
                const bool mine = ((todo >> lane_id()) & 1ull) && ph.inst == iu;
                todo &= ~__ballot(mine);
                if (mine) {
                    BlockAcc B = lds_acc(lds, stride, iu);
                    advance(L.insts[iu], B);
                }
            }
        } else if (alive) {
            BlockAcc B = lds_acc(lds, stride, 0);
            advance(L, B);
        }
        // ---- scattering events (the parent now sits at the scattering
        // point with the wavevector it scattered) ----
        uint64_t smask = __ballot(scat);
        if (smask) ev_push(L, ev, smask, scat, ph.inst, ph.x, ph.k, wchild, ev_rng, ph.n_sc + 1, ph.ev, zs);
    }
    ev_flush(L, ev);
    if constexpr (BATCHED) {
        for (uint64_t todo = __ballot(ended != 0); todo;) {
            const int iu = uniform_inst(todo, ph.inst);
            const bool mine = ended != 0 && ph.inst == iu;
            todo &= ~__ballot(mine);
            if (mine) {
                BlockAcc B = lds_acc(lds, stride, iu);
                finish_ks(L.insts[iu], B, ph, ended);
                ended = 0;
            }
        }
    } else if (ended) {
        BlockAcc B = lds_acc(lds, stride, 0);
        finish_ks(L, B, ph, ended);
        ended = 0;
    }
    lds_flush_all(L, lds, stride);
}

// Scattering events -> child photons in Kerr spacetime, one thread per
// event: fluid frame at the scattering point, electron and angle draws from
// the child's stream, then the child's optical-depth draw.  The child's
// opacities and acceleration are evaluated when the tracker loads it.
template <bool BATCHED>
__global__ __launch_bounds__(256, 2) void scatter_kernel_ks(TArgs L)
{
    extern __shared__ double lds[];
    const int stride = L_N + S_N;
    lds_zero(lds, L.n_inst, stride);
    const unsigned long long n = min(*L.dst_count, L.cap);
    const PhotonQ &Q = L.dst;
    // event i -> child: in place, or (batched) complete record at slot o of L.out
    auto event = [&](unsigned long long i, unsigned long long o) {
        const int ii = Q.inst[i];
        const TArgs &A = L.insts[ii];
        BlockAcc B = lds_acc(lds, stride, ii);
        double ks[4] = {Q.k[0][i], Q.k[1][i], Q.k[2][i], Q.k[3][i]};
        int z = Q.zone[i];
        int n_sc = Q.n_sc[i];
        double wchild = Q.w[i];
        const Rng r_par{Q.s0[i], Q.s1[i], Q.s2[i], 0u};
        const uint32_t pev = Q.ev[i];
        Rng r = child_rng(r_par, Q.blk[i], A.key0, A.key1);
        const Rng r_child = r;
        uint32_t cev = kNoEvent;
        KMetric K;
        kerr_metric<false>(A.a_spin, A.mass, A.h_slope, Q.x[0][i], Q.x[1][i], K);
        double g[4][4];
        kerr_full(K, g);
        double kc[4];
        if (z >= 0) {
            const double *zr = A.zrec + (size_t)z * Z_STRIDE;
            double u[4], bh[4], e[4][4];
            bool has_b = fluid_frame(zr, g, u, bh);
            double eps = scatter_tetrad(g, u, bh, has_b, ks, e);
            if (A.evlog) {
                double xe[3] = {Q.x[0][i], Q.x[1][i], Q.x[2][i]};
                cev = log_event(A, r_child, &r_par, z, n_sc, eps, wchild, xe, pev);
            }
            double kf[4];
            ScatterCount cnt{0, 0};
            scatter_in_frame(r, A.key0, A.key1, A.el, zr[Z_TH], eps, kf, cnt);
#pragma unroll
            for (int m = 0; m < 4; ++m) kc[m] = kf[0] * e[0][m] + kf[1] * e[1][m] + kf[2] * e[2][m] + kf[3] * e[3][m];
            lds_inc(&B.stats[S_E_TRIALS], cnt.e_trials);
            lds_inc(&B.stats[S_ANG_TRIALS], cnt.ang_trials);
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) kc[m] = ks[m];
        }
        lds_add(&B.ledger[L_E_COMPTON], wchild * (kerr_einf(K, kc) - kerr_einf(K, ks)) * kMeC2);
        lds_inc(&B.stats[S_SCATTER], 1);
        lds_inc(&B.stats[S_CHILDREN], 1);
        lds_inc(&B.stats[S_GEN0 + min(n_sc, 15)], 1);
        double x1 = -log(1.0 - rng_uniform(r, A.key0, A.key1));
        const PhotonQ &O = BATCHED ? L.out : Q;
        if (BATCHED) {
#pragma unroll
            for (int m = 0; m < 3; ++m) O.x[m][o] = Q.x[m][i];
            O.w[o] = wchild;
            O.n_sc[o] = n_sc;
            O.inst[o] = ii;
        }
        O.s0[o] = r_child.s0; O.s1[o] = r_child.s1; O.s2[o] = r_child.s2;
#pragma unroll
        for (int m = 0; m < 4; ++m) O.k[m][o] = kc[m];
        O.wb[o] = wchild;
        O.x1[o] = x1;
        O.blk[o] = r.block;
        O.ev[o] = cev;
    };
    if constexpr (BATCHED) {
        for_events_grouped(L, n, event);
    } else {
        for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (unsigned long long)gridDim.x * blockDim.x)
            event(i, i);
    }
    lds_flush_all(L, lds, stride);
}

}  // namespace gm
