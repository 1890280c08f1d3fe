// gm_track.h -- superphoton transport kernels (device side).
//
// Three kernels per scattering generation, connected by photon queues in
// structure-of-arrays form:
//   birth_kernel    one thread per root: position, frequency and direction
//                   sampling, tetrad, weight, opacities -> generation-0 queue;
//   track_kernel    persistent grid, one lane per photon for its whole life:
//                   geodesic steps, absorption, scattering decision, tally at
//                   escape; a scattering event updates the parent and writes
//                   the event (point, incoming wavevector, child weight and
//                   stream) into the next generation's queue;
//   scatter_kernel  one thread per event: electron and scattering-angle
//                   sampling, the child's wavevector and opacities, in place.
// Waves of the tracker claim queue entries for all their idle lanes with one
// atomic, and reserve event slots with one atomic per wave.  Tallies,
// ledgers and counters accumulate in LDS and are merged into HBM per block.
#pragma once

#include <climits>

#include "gm_emis32.h"
#include "gm_frame.h"
#include "gm_kerr.h"

namespace gm {

// Photon queue (one generation), structure of arrays.
struct PhotonQ {
    double *x[3], *k[4];
    double *w, *wb, *x1, *nua, *nus, *b;
    uint32_t *s0, *s1, *s2, *blk;
    uint32_t *ev;                  // event-log record that created the photon (kNoEvent: none);
                                   // in an event queue: the scattering photon's record
    int32_t *n_sc, *zone, *inst;
};

// One event of the event log (records of the learned and adaptive forms):
// the emission of a root or a scattering, keyed by the stream of the photon
// it created.  score sums w E s_bin over that photon and all its
// descendants that escape into a tally bin (E the energy at infinity in
// erg, s_bin the bin's score weight); parent is the record of the photon
// that scattered, so scores propagate up the ancestry.  88 bytes.
struct EventRec {
    uint32_t s0, s1, s2;           // stream of the photon the event created
    uint32_t p0, p1, p2;           // stream of the photon that scattered (0: emission)
    int32_t zone, gen;             // plasma zone; generation of the created photon
    uint32_t parent, pad;          // record of the scattering photon (kNoEvent: none)
    double eps;                    // fluid-frame energy of the incoming (scattering) or
                                   // emitted photon, m_e c^2
    double w;                      // weight of the created photon
    double score;
    double x[3];                   // event position, code coordinates
};

struct TraceRec {
    uint32_t s0, s1, s2;
    int32_t n_sc, kind, i_nu, i_theta;
    uint32_t n_steps;
    double w_birth, w_end;
    double x[4], k[4];
};

struct TArgs {
    // instance geometry and plasma
    const double *zrec;
    const float *zrec32;           // FP32 records (precision form)
    int n[3];
    double xs[3], dx[3], inv_dx[3], xe[3];
    double inv_n3;                 // 1 / n[2]
    double C;                      // h ell / (m_e c^2): converts d(lambda) to cm s
    int inst;
    uint32_t key0, key1;
    // roots of the instance (birth kernel)
    const uint32_t *zone_of_root;
    unsigned long long root_begin, root_count;
    double lnnu_min, lnnu_span;
    int n_wnodes;
    const double *ln_w, *fmax;
    GCheb G;
    // queues of the generation being processed
    int gen;
    PhotonQ src, dst;
    unsigned long long *src_count, *src_cursor, *dst_count;
    unsigned long long cap;
    int *overflow;
    // batched launch: per-instance argument blocks (instance fields; the
    // queue fields of a launch are those of the launch's own arguments),
    // combined root offsets [n_inst + 1], LDS doubles per instance
    const struct TArgs *insts;
    int n_inst;
    const unsigned long long *root_off;
    int lds_stride;
    // batched scattering: per-instance event counts and slot cursors of the
    // generation, and the queue the children are written to, grouped by
    // instance (the generation's consumed source queue)
    unsigned long long *inst_count, *inst_cursor;
    PhotonQ out;
    // tallies of the instance
    double *spec, *ledger;
    unsigned long long *stats;
    int n_nu, n_theta;
    double ln_nu_lo, inv_dln_nu;
    // transport parameters
    int scattering, bias_mode, n_sc_max;
    double bias_value, bias_max, step_h, roulette_frac, roulette_p;
    double step_far, r_far;        // far-field step factor beyond r_far (1, +inf: off)
    long long max_steps;
    double L_unit_cm;
    ShTable sh;
    ShTable32 sh32;
    float ln_c2_2h;                // ln(c^2 / (2 h)), set on the host from the CGS constants
    // Kerr (modified Kerr-Schild): spin, polar slope, horizon, capture and
    // record radii, corrector, reciprocal step scales (dx1, dx2, min(dx3, pi dx2))
    double a_spin, mass, h_slope, r_h, r_capture, r_record;   // mass 1 (Kerr) or 0 (flat spherical)
    Elec el;                       // electrons (the same in every instance of a shared launch)
    double i1_plasma_max;          // no zone with a larger first-axis index holds plasma
    double verlet_tol;
    int verlet_max_it;
    double inv_sc[3];
    // scheduling: claim new photons once this many lanes of a wave idle
    int refill_min;
    // optional trace and scattering-event log
    TraceRec *trace;
    unsigned long long *trace_n;
    unsigned long long trace_cap;
    EventRec *evlog;
    unsigned long long *evlog_n;
    unsigned long long evlog_cap;
    unsigned long long root_stride;   // roots with id % root_stride == 0 log their emission
    const double *sw;                 // score weights [n_theta][n_nu] (NULL: 1)
    // bias table: ln of the bias (mode 3) or of the importance factor
    // (mode 4) per zone on ln(eps) nodes over [lnb_lo, lnb_hi]
    const double *lnb;
    int lnb_n;
    double lnb_lo, lnb_hi;
    // emission table: ln w_i(nu) = ln w(nu) - m_i(ln nu), nodes over [mt_lo, mt_hi]
    const double *mtab;
    int mt_n;
    double mt_lo, mt_hi;
};

struct Coef {
    double nua, nus, b;
    bool vacuum;
};

// The instance fields a flat step reads.  A batched launch gathers them once
// per change of a wave's instance instead of re-reading them field by field
// from the per-instance argument blocks on every step.
struct StepArgs {
    const double *zrec;
    const float *zrec32;
    int n[3];
    double xs[3], xe[3], inv_dx[3];
    double C, step_h, roulette_frac, roulette_p;
    int scattering, n_sc_max, bias_mode;
    uint32_t key0, key1;
    double bias_value, bias_max, L_unit_cm;
    ShTable sh;
    ShTable32 sh32;
    float ln_c2_2h;
    const double *lnb;
    int lnb_n;
    double lnb_lo, lnb_hi;
};

GM_D StepArgs step_args(const TArgs &T)
{
    StepArgs S;
    S.zrec = T.zrec; S.zrec32 = T.zrec32;
#pragma unroll
    for (int j = 0; j < 3; ++j) { S.n[j] = T.n[j]; S.xs[j] = T.xs[j]; S.xe[j] = T.xe[j]; S.inv_dx[j] = T.inv_dx[j]; }
    S.C = T.C; S.step_h = T.step_h; S.roulette_frac = T.roulette_frac; S.roulette_p = T.roulette_p;
    S.scattering = T.scattering; S.n_sc_max = T.n_sc_max; S.bias_mode = T.bias_mode;
    S.key0 = T.key0; S.key1 = T.key1;
    S.bias_value = T.bias_value; S.bias_max = T.bias_max; S.L_unit_cm = T.L_unit_cm;
    S.sh = T.sh; S.sh32 = T.sh32; S.ln_c2_2h = T.ln_c2_2h;
    S.lnb = T.lnb; S.lnb_n = T.lnb_n; S.lnb_lo = T.lnb_lo; S.lnb_hi = T.lnb_hi;
    return S;
}

// Per-block accumulators in LDS.
struct BlockAcc {
    double *spec, *ledger;
    unsigned long long *stats;
};

GM_D void lds_add(double *p, double v) { atomicAdd(p, v); }
GM_D void lds_inc(unsigned long long *p, unsigned long long v) { atomicAdd(p, v); }

// LDS holds one accumulator block (ledger, counters, tally) per instance of
// the launch, `stride` doubles apart.
GM_D void lds_zero(double *lds, int n_inst, int stride)
{
    for (int i = threadIdx.x; i < n_inst * stride; i += blockDim.x) lds[i] = 0.0;
    __syncthreads();
}

// The tally is in LDS when the stride leaves room for it, else the
// instance's tally in HBM is added to directly (spec = NULL here).
GM_D BlockAcc lds_acc(double *lds, int stride, int inst)
{
    BlockAcc B;
    double *base = lds + (size_t)inst * stride;
    B.ledger = base;
    B.stats = reinterpret_cast<unsigned long long *>(base + L_N);
    B.spec = stride > L_N + S_N ? base + L_N + S_N : nullptr;
    return B;
}

GM_D void lds_flush_all(const TArgs &L, double *lds, int stride)
{
    __syncthreads();
    const int nspec = stride - L_N - S_N;
    for (int ii = 0; ii < L.n_inst; ++ii) {
        const TArgs &A = L.insts[ii];
        BlockAcc B = lds_acc(lds, stride, ii);
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
}

// Scattering events of a wave staged in LDS and written to the event queue
// in batches: one queue reservation (a device-wide atomic, served beyond the
// XCD's L2) per batch instead of one per step of the wave, and coalesced
// stores of consecutive slots instead of scattered single-lane ones.  Each
// wave of the block owns kEvCap slots after the block's tallies; `n` is
// wave-uniform.
constexpr int kEvCap = 64;
constexpr int kEvDoubles = kEvCap * 8 + kEvCap * 7 / 2;   // 8 doubles + 7 ints per event
constexpr size_t kEvBytesPerBlock = (size_t)(256 / 64) * kEvDoubles * 8;

struct EvStage {
    double *d;    // [8][kEvCap]: x1, x2, x3, k0..k3, w
    int *i;       // [7][kEvCap]: instance | generation << 8, parent stream s0 s1 s2 and
                  // block, parent's event record, zone
    int n;
};

GM_D EvStage ev_stage(double *lds, int n_inst, int stride)
{
    EvStage S;
    S.d = lds + (size_t)n_inst * stride + (size_t)(threadIdx.x >> 6) * kEvDoubles;
    S.i = reinterpret_cast<int *>(S.d + 8 * kEvCap);
    S.n = 0;
    return S;
}

// Write the wave's staged events to consecutive queue slots (whole wave).
GM_D void ev_flush(const TArgs &L, EvStage &S)
{
    if (S.n == 0) return;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(L.dst_count, (unsigned long long)S.n);
    base = bcast_u64(base, 0);
    const int l = lane_id();
    if (l < S.n) {
        const unsigned long long q = base + (unsigned long long)l;
        if (q < L.cap) {
            const PhotonQ &Q = L.dst;
#pragma unroll
            for (int m = 0; m < 3; ++m) Q.x[m][q] = S.d[m * kEvCap + l];
#pragma unroll
            for (int m = 0; m < 4; ++m) Q.k[m][q] = S.d[(3 + m) * kEvCap + l];
            Q.w[q] = S.d[7 * kEvCap + l];
            Q.inst[q] = S.i[l] & 0xff;
            Q.n_sc[q] = S.i[l] >> 8;
            Q.s0[q] = (uint32_t)S.i[kEvCap + l];
            Q.s1[q] = (uint32_t)S.i[2 * kEvCap + l];
            Q.s2[q] = (uint32_t)S.i[3 * kEvCap + l];
            Q.blk[q] = (uint32_t)S.i[4 * kEvCap + l];
            Q.ev[q] = (uint32_t)S.i[5 * kEvCap + l];
            Q.zone[q] = S.i[6 * kEvCap + l];
        } else {
            atomicOr(L.overflow, 1);
        }
    }
    S.n = 0;
}

// Stage the events of the lanes in `smask` (whole wave; `scat` is this
// lane's bit): scattering point x, incoming wavevector k, child weight, the
// parent's stream and counter block at the event (the scattering kernel
// derives the child's stream from them), child generation, the parent's
// event record and the plasma zone.
GM_D void ev_push(const TArgs &L, EvStage &S, uint64_t smask, bool scat, int inst, const double *x,
                  const double *k, double w, const Rng &r, int n_sc, uint32_t pev, int zone)
{
    const int nn = __popcll(smask);
    if (S.n + nn > kEvCap) ev_flush(L, S);
    if (scat) {
        const int j = S.n + (int)rank_in_mask(smask);
#pragma unroll
        for (int m = 0; m < 3; ++m) S.d[m * kEvCap + j] = x[m];
#pragma unroll
        for (int m = 0; m < 4; ++m) S.d[(3 + m) * kEvCap + j] = k[m];
        S.d[7 * kEvCap + j] = w;
        S.i[j] = inst | (n_sc << 8);
        S.i[kEvCap + j] = (int)r.s0;
        S.i[2 * kEvCap + j] = (int)r.s1;
        S.i[3 * kEvCap + j] = (int)r.s2;
        S.i[4 * kEvCap + j] = (int)r.block;
        S.i[5 * kEvCap + j] = (int)pev;
        S.i[6 * kEvCap + j] = zone;
    }
    S.n += nn;
}

// Append an event to the log (emission: parent stream NULL); returns its
// index, or kNoEvent when the log is full (the event is still counted).
GM_D uint32_t log_event(const TArgs &A, const Rng &made, const Rng *par, int z, int gen, double eps, double w,
                        const double *x, uint32_t parent)
{
    unsigned long long i = atomicAdd(A.evlog_n, 1ull);
    if (i >= A.evlog_cap) return kNoEvent;
    EventRec &e = A.evlog[i];
    e.s0 = made.s0; e.s1 = made.s1; e.s2 = made.s2;
    e.p0 = par ? par->s0 : 0u; e.p1 = par ? par->s1 : 0u; e.p2 = par ? par->s2 : 0u;
    e.zone = z;
    e.gen = gen;
    e.parent = parent;
    e.pad = 0u;
    e.eps = eps;
    e.w = w;
    e.score = 0.0;
    e.x[0] = x[0]; e.x[1] = x[1]; e.x[2] = x[2];
    return (uint32_t)i;
}

// An escape into tally bin (ith, inu) with energy E adds to the score of the
// photon's own record; scores reach the ancestors' records afterwards
// (score_propagate_kernel).
GM_D void score_escape(const TArgs &A, uint32_t ev, int ith, int inu, double E)
{
    if (!A.evlog || ev == kNoEvent) return;
    double s = A.sw ? E * A.sw[(size_t)ith * A.n_nu + inu] : E;
    atomicAdd(&A.evlog[ev].score, s);
}

// Instance of a root in the launch's combined root range (binary search of
// the combined offsets).
GM_D int inst_of_root(const TArgs &L, unsigned long long g)
{
    int lo = 0, hi = L.n_inst;               // root_off[lo] <= g < root_off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (L.root_off[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// The instance of the first lane of `mask`, as a wave-uniform value.
GM_D int uniform_inst(uint64_t mask, int inst)
{
    int first = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)mask) - 1);
    return __builtin_amdgcn_readlane(inst, first);
}

// Zone holding a Cartesian point, or -1 outside the grid (vacuum).
template <class Args>
GM_D int zone_cart(const Args &A, double x1, double x2, double x3)
{
    double f1 = floor((x1 - A.xs[0]) * A.inv_dx[0]);
    double f2 = floor((x2 - A.xs[1]) * A.inv_dx[1]);
    double f3 = floor((x3 - A.xs[2]) * A.inv_dx[2]);
    bool in = (f1 >= 0.0) && (f1 < (double)A.n[0]) && (f2 >= 0.0) && (f2 < (double)A.n[1]) &&
              (f3 >= 0.0) && (f3 < (double)A.n[2]);
    return in ? ((int)f1 * A.n[1] + (int)f2) * A.n[2] + (int)f3 : -1;
}

// Zone holding a modified Kerr-Schild point: x1 outside the grid is vacuum
// (-1), x2 is clamped to the first/last polar zone, x3 is periodic.
GM_D int zone_ks(const TArgs &A, double x1, double x2, double x3)
{
    double f1 = floor((x1 - A.xs[0]) * A.inv_dx[0]);
    if (!(f1 >= 0.0 && f1 < (double)A.n[0])) return -1;
    double f2 = floor((x2 - A.xs[1]) * A.inv_dx[1]);
    f2 = fmin(fmax(f2, 0.0), (double)(A.n[1] - 1));
    double f3 = floor((x3 - A.xs[2]) * A.inv_dx[2]);
    // f3 mod n3 for the integer-valued f3: the quotient from a multiply by
    // 1/n3 is off by at most one, which the two corrections undo
    const double n3 = (double)A.n[2];
    f3 -= n3 * floor(f3 * A.inv_n3);
    f3 = (f3 >= n3) ? f3 - n3 : f3;
    f3 = (f3 < 0.0) ? f3 + n3 : f3;
    return ((int)f1 * A.n[1] + (int)f2) * A.n[2] + (int)f3;
}

// Bias of a point (Scattering section): constant, Theta_e^2-scaled,
// growing with the generation and falling with the density, or from the
// zone's table (exp of its entry interpolated in ln eps), clamped to
// [1, bias_max].  In the weight-window mode (4) the table gives an
// importance factor, returned unclamped: the bias of a step is the
// photon's weight times it (step_bias).  Any b >= 1 keeps the estimator
// unbiased: the child carries w/b, the parent keeps w(1 - 1/b).  CB: the
// caller knows at compile time that the bias is the constant one (mode 0),
// which spares the tracker the registers of the other modes.
template <bool CB = false, class Args>
GM_D double bias_at(const Args &A, int z, double theta, double ne, int n_sc, double eps)
{
    if constexpr (CB) return fmin(fmax(A.bias_value, 1.0), A.bias_max);
    double b;
    if (A.bias_mode == 0) b = A.bias_value;
    else if (A.bias_mode == 1) b = A.bias_value * theta * theta;
    else if (A.bias_mode == 2) b = (double)((n_sc + 1) * (n_sc + 1)) / (ne * kSigT * A.bias_value * A.L_unit_cm);
    else {
        b = exp(zone_table(A.lnb, A.lnb_n, A.lnb_lo, A.lnb_hi, z, log(eps)));
        if (A.bias_mode == 4) return b;
    }
    return fmin(fmax(b, 1.0), A.bias_max);
}

// Bias of a step from the value carried by the photon or evaluated at the
// step's end: the value itself, or in the weight-window mode the weight at
// the step's start times the importance factor, clamped to [1, bias_max].
template <bool CB = false, class Args>
GM_D double step_bias(const Args &A, double w, double bf)
{
    if (CB || A.bias_mode != 4) return bf;
    return fmin(fmax(w * bf, 1.0), A.bias_max);
}

// Invariant absorption and scattering coefficients (nu alpha) at a point
// (Absorption and Scattering sections): alpha = j / B_nu (Kirchhoff),
// alpha_sc = n_e sigma_h; and the bias at that point.  gm gives inner
// products with the metric at the point; FLAT zones carry their unit u and
// field direction already.
template <bool FLAT, bool CB = false, class Args, class G>
GM_D Coef coefficients_at64(const Args &A, const Elec &el, int z, const G &gm, const double *k, int n_sc)
{
    Coef c{0.0, 0.0, 1.0, true};
    if (z < 0) return c;
    // the whole 128-byte record in one round of 16-byte loads, before the
    // vacuum test, so that the record costs one memory latency, not two
    double zr[Z_STRIDE];
    {
        const double2 *src = reinterpret_cast<const double2 *>(A.zrec + (size_t)z * Z_STRIDE);
#pragma unroll
        for (int m = 0; m < Z_STRIDE / 2; ++m) {
            double2 v = src[m];
            zr[2 * m] = v.x;
            zr[2 * m + 1] = v.y;
        }
#pragma unroll
        for (int m = 0; m < Z_STRIDE; ++m) settle(zr[m]);
    }
    double ne = zr[Z_NE];
    if (!(ne > 0.0)) return c;
    c.vacuum = false;
    double ef, kb;                 // -k.u and k.(field direction) at the point
    bool has_b;
    if constexpr (FLAT) {
        double u[4], bh[4];
        has_b = fluid_frame_flat(zr, u, bh);
        ef = -gm.dot(k, u);
        kb = gm.dot(k, bh);
    } else {
        has_b = frame_products(zr[Z_HASB] != 0.0, gm, zr + Z_U0, zr + Z_B0, k, ef, kb);
    }
    // the thermal hot cross section's table entries are requested before the
    // absorption is computed, which then covers their latency
    const bool sh_thermal = A.scattering && el.kind == 0;
    ShFetch shf{};
    if (sh_thermal) shf = sigma_hot_fetch(A.sh, zr[Z_LNTH], log(ef));
    double inv_ef = 1.0 / ef;
    double nuf = ef * (kMeC2 / kH);
    double Az = zr[Z_A];
    if (has_b && Az > 0.0) {
        double cth = kb * inv_ef;
        cth = fmin(fmax(cth, -1.0), 1.0);
        double s2 = 1.0 - cth * cth;
        if (s2 > 0.0) {
            double rs = rsqrt(s2);                      // 1 / sin(theta)
            double s = s2 * rs;
            const double X = nuf * zr[Z_INVNUC] * rs;
            if (el.kind != 0) {
                // power law: nu alpha = A_a X^{-(p+2)/2}, A_a in the 1/Theta slot
                c.nua = zr[Z_INVTH] * exp(el.ea * log(X));
            } else {
                double j = Az * s * g_shape(X);
                if (j > 0.0) {
                    // nu alpha = j (e^{h nu / kT} - 1) c^2 / (2 h nu^2), Kirchhoff
                    double inv_nu = inv_ef * (kH / kMeC2);
                    c.nua = j * expm1_kirchhoff(ef * zr[Z_INVTH]) * (kC * kC / (2.0 * kH)) * inv_nu * inv_nu;
                }
            }
        }
    }
    if (sh_thermal) {
        settle(shf.t00); settle(shf.t01); settle(shf.t10); settle(shf.t11);
        c.nus = nuf * ne * kSigT * sigma_hot_finish(shf);
    } else if (A.scattering) {
        c.nus = nuf * ne * kSigT * sigma_pl(el, ef);
    }
    c.b = bias_at<CB>(A, z, zr[Z_TH], ne, n_sc, ef);
    return c;
}

// The same in the FP32 form: frame products in double, then emissivity,
// absorption and the hot cross section as FP32 logarithms and one exp each.
template <bool FLAT, bool CB = false, class Args, class G>
GM_D Coef coefficients_at32(const Args &A, const Elec &el, int z, const G &gm, const double *k, int n_sc)
{
    (void)el;                      // thermal electrons only (power laws run in FP64)
    Coef c{0.0, 0.0, 1.0, true};
    if (z < 0) return c;
    // the 64-byte record in one round of 16-byte loads, as in FP64
    float zf[F_STRIDE];
    {
        const float4 *src = reinterpret_cast<const float4 *>(A.zrec32 + (size_t)z * F_STRIDE);
#pragma unroll
        for (int m = 0; m < F_STRIDE / 4; ++m) {
            float4 v = src[m];
            zf[4 * m] = v.x; zf[4 * m + 1] = v.y; zf[4 * m + 2] = v.z; zf[4 * m + 3] = v.w;
        }
#pragma unroll
        for (int m = 0; m < F_STRIDE; ++m) settle(zf[m]);
    }
    float nef = zf[F_NE];
    if (!(nef > 0.0f)) return c;
    c.vacuum = false;
    double ef, kb;                 // -k.u and k.(field direction) at the point
    bool has_b = zf[F_HASB] != 0.0f;
    if constexpr (FLAT) {
        double u[4], bh[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) { u[m] = (double)zf[F_U0 + m]; bh[m] = (double)zf[F_B0 + m]; }
        ef = -gm.dot(k, u);
        kb = gm.dot(k, bh);
    } else {
        has_b = frame_products(has_b, gm, zf + F_U0, zf + F_B0, k, ef, kb);
    }
    float lnnu = __logf((float)(ef * (kMeC2 / kH)));
    float lnA = zf[F_LNA];
    if (has_b && lnA > -1e30f) {
        double cth = fmin(fmax(kb / ef, -1.0), 1.0);
        float s2 = (float)(1.0 - cth * cth);
        if (s2 > 0.0f) {
            float lns = 0.5f * __logf(s2);
            float lnj = lnA + lns + ln_g_shape32(lnnu + zf[F_LNINVNUC] - lns);
            float x = (float)ef * zf[F_INVTH];
            // nu alpha = j (e^{h nu/kT} - 1) c^2 / (2 h nu^2)
            c.nua = (double)__expf(lnj + ln_expm1_32(x) + A.ln_c2_2h - 2.0f * lnnu);
        }
    }
    if (A.scattering)
        c.nus = (double)__expf(lnnu + zf[F_LNNESIG] + ln_sigma_hot32(A.sh32, zf[F_LNTH], __logf((float)ef)));
    c.b = bias_at<CB>(A, z, (double)zf[F_TH], (double)nef, n_sc, ef);
    return c;
}

template <bool FLAT, bool F32 = false, bool CB = false, class Args, class G>
GM_D Coef coefficients_at(const Args &A, const Elec &el, int z, const G &gm, const double *k, int n_sc)
{
    if constexpr (F32) return coefficients_at32<FLAT, CB>(A, el, z, gm, k, n_sc);
    else return coefficients_at64<FLAT, CB>(A, el, z, gm, k, n_sc);
}

// Flat spacetime (Cartesian Minkowski metric).
template <class M, bool F32 = false, class Args>
GM_D Coef coefficients(const Args &A, const Elec &el, int z, const double *x, const double *k, int n_sc)
{
    static_assert(!M::kCurved, "the flat form");
    (void)x;
    return coefficients_at<true, F32>(A, el, z, GFlat{}, k, n_sc);
}

// ---------------------------------------------------------------------------
// Birth of root photons (Sampling procedure section): position uniform in
// the zone, frequency by rejection against the zone's bound on dN/d ln nu,
// direction by rejection against j(pi/2), fluid-frame tetrad, weight w(nu),
// remaining optical depth, opacities at the birth point.
//
// In two kernels.  birth_sample_kernel runs the two rejection loops with
// each lane taking its own roots' trials one after another (lane i of a
// grid of T lanes takes roots i, i + T, i + 2T, ... of the chunk), so a
// wave waits for its slowest lane's total over many roots, not for the
// slowest lane at every root (the trials per root have a long geometric
// tail).  It leaves nu, ln w, cos theta and the stream's block counter
// after the last trial in the root's generation-0 queue slots (x1, w, k^0,
// blk), which birth_kernel reads and then overwrites.  The position's three
// draws, the stream's first three blocks, are made by birth_kernel, so
// every root draws exactly the numbers of a single pass.
__global__ __launch_bounds__(256) void birth_sample_kernel(TArgs L)
{
    extern __shared__ double lds[];
    const int stride = L_N + S_N;
    lds_zero(lds, L.n_inst, stride);
    const PhotonQ &Q = L.dst;
    const unsigned long long T = (unsigned long long)gridDim.x * blockDim.x;
    unsigned long long q = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    // the lane's current root: phase 0 set-up, 1 frequency trials, 2 direction trials
    int phase = 0, ii = 0;
    const TArgs *Ap = L.insts;
    uint32_t z = 0, trials = 0, over = 0, dtr = 0;
    int64_t it = 0;
    Rng rng{0u, 0u, 0u, 0u};
    double Az = 0.0, nuc = 0.0, fm = 0.0, nu = 0.0, lnw = 0.0, jmax = 0.0;
    while (q < L.root_count) {
        if (phase == 0) {
            const unsigned long long gq = L.root_begin + q;
            ii = inst_of_root(L, gq);
            Ap = L.insts + ii;
            const unsigned long long p = gq - L.root_off[ii];
            z = Ap->zone_of_root[p];
            const double *zr = Ap->zrec + (size_t)z * Z_STRIDE;
            Az = zr[Z_A];
            nuc = zr[Z_NUC];
            fm = Ap->fmax[z];
            rng = Rng{(uint32_t)p, (uint32_t)(p >> 32), ((uint32_t)Ap->inst << 8) | 1u, 3u};
            trials = over = dtr = 0;
            it = 0;
            phase = 1;
        }
        const TArgs &A = *Ap;
        if (phase == 1) {
            const double lnnu = A.lnnu_min + rng_uniform(rng, A.key0, A.key1) * A.lnnu_span;
            nu = exp(lnnu);
            const double u2 = rng_uniform(rng, A.key0, A.key1);
            const double dlnw = A.lnnu_span / (A.n_wnodes - 1);
            const double a = (lnnu - A.lnnu_min) / dlnw;
            int i = (int)floor(a);
            i = max(0, min(i, A.n_wnodes - 2));
            const double f = a - i;
            lnw = (1.0 - f) * A.ln_w[i] + f * A.ln_w[i + 1];
            if (A.mtab) lnw -= zone_table(A.mtab, A.mt_n, A.mt_lo, A.mt_hi, (int)z, lnnu);
            const double F = 4.0 * kPi * Az * shape_G(A.el, A.G, nu / nuc) / exp(lnw);
            ++trials;
            over += (F > fm) ? 1u : 0u;
            if (u2 < F / fm || it >= kMaxTrials) {
                jmax = Az * shape_g(A.el, nu / nuc);
                it = 0;
                phase = 2;
            } else {
                ++it;
            }
        } else {
            const double cth = 2.0 * rng_uniform(rng, A.key0, A.key1) - 1.0;
            const double u4 = rng_uniform(rng, A.key0, A.key1);
            ++dtr;
            const double s2 = 1.0 - cth * cth;
            double j = 0.0;
            if (s2 > 0.0) {
                const double s = sqrt(s2);
                j = Az * s * shape_g(A.el, nu / (nuc * s));
            }
            if (u4 < j / jmax || it >= kMaxTrials) {
                Q.x1[q] = nu;
                Q.w[q] = lnw;
                Q.k[0][q] = cth;
                Q.blk[q] = rng.block;
                BlockAcc B = lds_acc(lds, stride, ii);
                lds_inc(&B.stats[S_NU_TRIALS], trials);
                if (over) lds_inc(&B.stats[S_OVERSHOOT], over);
                lds_inc(&B.stats[S_DIR_TRIALS], dtr);
                q += T;
                phase = 0;
            } else {
                ++it;
            }
        }
    }
    lds_flush_all(L, lds, stride);
}

// ---------------------------------------------------------------------------
template <class M, bool F32>
__global__ __launch_bounds__(256) void birth_kernel(TArgs L)
{
    extern __shared__ double lds[];
    const int stride = L_N + S_N;
    lds_zero(lds, L.n_inst, stride);
    unsigned long long q = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < L.root_count) {
        const unsigned long long gq = L.root_begin + q;
        const int ii = inst_of_root(L, gq);
        const TArgs &A = L.insts[ii];
        BlockAcc B = lds_acc(lds, stride, ii);
        unsigned long long p = gq - L.root_off[ii];
        uint32_t z = A.zone_of_root[p];
        const double *zr = A.zrec + (size_t)z * Z_STRIDE;
        Rng rng{(uint32_t)p, (uint32_t)(p >> 32), ((uint32_t)A.inst << 8) | 1u, 0u};
        int i3 = (int)(z % (uint32_t)A.n[2]);
        int i2 = (int)((z / (uint32_t)A.n[2]) % (uint32_t)A.n[1]);
        int i1 = (int)(z / ((uint32_t)A.n[2] * (uint32_t)A.n[1]));
        double x[4];
        x[0] = 0.0;
        x[1] = A.xs[0] + (i1 + rng_uniform(rng, A.key0, A.key1)) * A.dx[0];
        x[2] = A.xs[1] + (i2 + rng_uniform(rng, A.key0, A.key1)) * A.dx[1];
        x[3] = A.xs[2] + (i3 + rng_uniform(rng, A.key0, A.key1)) * A.dx[2];
        // frequency, its weight and the direction from birth_sample_kernel;
        // the stream continues after its last trial
        const PhotonQ &Q = L.dst;
        const double nu = Q.x1[q], lnw = Q.w[q], cth = Q.k[0][q];
        rng.block = Q.blk[q];
        double phi = 2.0 * kPi * rng_uniform(rng, A.key0, A.key1);
        double g[4][4], u[4], bh[4], e[4][4];
        if constexpr (M::kCurved) {
            KMetric K;
            kerr_metric<false>(A.a_spin, A.mass, A.h_slope, x[1], x[2], K);
            kerr_full(K, g);
            fluid_frame(zr, g, u, bh);
        } else {
            M::gcov(x, g);
            fluid_frame_flat(zr, u, bh);
        }
        emission_tetrad(g, u, bh, e);
        double eps = kH * nu / kMeC2;
        double sth = sqrt(1.0 - cth * cth);
        double kf[4] = {eps, eps * sth * cos(phi), eps * sth * sin(phi), eps * cth};
        double k[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) k[m] = kf[0] * e[0][m] + kf[1] * e[1][m] + kf[2] * e[2][m] + kf[3] * e[3][m];
        double w = exp(lnw);
        double x1 = -log(1.0 - rng_uniform(rng, A.key0, A.key1));
        // flat: opacities at the birth point now; Kerr: the tracker's first
        // evaluation of a loaded photon computes them with the acceleration
        Coef c{0.0, 0.0, 1.0, true};
        if constexpr (!M::kCurved) c = coefficients<M, F32>(A, A.el, zone_cart(A, x[1], x[2], x[3]), x, k, 0);
        // write generation-0 queue entry q
        Q.inst[q] = ii;
#pragma unroll
        for (int m = 0; m < 3; ++m) Q.x[m][q] = x[m + 1];
#pragma unroll
        for (int m = 0; m < 4; ++m) Q.k[m][q] = k[m];
        Q.w[q] = w; Q.wb[q] = w; Q.x1[q] = x1;
        Q.nua[q] = c.nua; Q.nus[q] = c.nus; Q.b[q] = c.b;
        Q.s0[q] = rng.s0; Q.s1[q] = rng.s1; Q.s2[q] = rng.s2; Q.blk[q] = rng.block;
        Q.n_sc[q] = 0;
        Q.ev[q] = (A.evlog && A.root_stride != 0 && p % A.root_stride == 0)
                      ? log_event(A, rng, nullptr, (int)z, 0, eps, w, x + 1, kNoEvent) : kNoEvent;
        lds_add(&B.ledger[L_W_EMIT], w);
        lds_add(&B.ledger[L_E_EMIT], w * e_inf(g, k) * kMeC2);
        lds_inc(&B.stats[S_ROOTS], 1);
        lds_inc(&B.stats[S_GEN0], 1);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *L.src_count = L.root_count;
    lds_flush_all(L, lds, stride);
}

// ---------------------------------------------------------------------------
// The tracker.
// ---------------------------------------------------------------------------
struct Photon {
    double x[3], k[4];
    double w, wb, x1;              // weight, birth weight, remaining biased depth
    double nua, nus, b;            // opacities and bias at the current point
    double acc_wabs, acc_wcap;     // weight lost to absorption / the generation cap
    Rng rng;
    int n_sc, inst;
    uint32_t ev;                   // event-log record that created the photon
    uint32_t steps, nsub;          // steps; partial steps to scattering points
    // opacities and bias of the last zone evaluated: in flat spacetime they
    // depend only on the zone, k (fixed for a photon) and n_sc, so a step
    // ending in the same zone reuses them (bitwise the same values)
    int cz, ncoef;
    bool cvac;
    double cnua, cnus, cb;
};

GM_D void load_photon(const PhotonQ &Q, unsigned long long i, Photon &ph)
{
#pragma unroll
    for (int m = 0; m < 3; ++m) ph.x[m] = Q.x[m][i];
#pragma unroll
    for (int m = 0; m < 4; ++m) ph.k[m] = Q.k[m][i];
    ph.w = Q.w[i]; ph.wb = Q.wb[i]; ph.x1 = Q.x1[i];
    ph.nua = Q.nua[i]; ph.nus = Q.nus[i]; ph.b = Q.b[i];
    ph.rng = Rng{Q.s0[i], Q.s1[i], Q.s2[i], Q.blk[i]};
    ph.n_sc = Q.n_sc[i];
    ph.inst = Q.inst[i];
    ph.ev = Q.ev[i];
    ph.steps = 0;
    ph.nsub = 0;
    ph.cz = INT_MIN;
    ph.ncoef = 0;
    ph.acc_wabs = ph.acc_wcap = 0.0;
}

GM_D void write_trace(const TArgs &A, const Photon &ph, int kind, int inu, int ith)
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

// Book a finished photon: tally (escape), accumulated losses, end kind,
// trace.  Flat spacetime: the energy at infinity is k^t.
GM_D void finish(const TArgs &A, BlockAcc &B, const Photon &ph, int kind)
{
    double e = ph.k[0] * kMeC2;
    int inu = -1, ith = -1;
    if (kind == END_ESCAPE) {
        double nuinf = ph.k[0] * (kMeC2 / kH);
        double fi = floor((log(nuinf) - A.ln_nu_lo) * A.inv_dln_nu);
        if (!(fi >= 0.0 && fi < (double)A.n_nu)) {
            kind = END_OOB;
        } else {
            double kk = sqrt(ph.k[1] * ph.k[1] + ph.k[2] * ph.k[2] + ph.k[3] * ph.k[3]);
            double th = acos(ph.k[3] / kk);
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
    if (ph.acc_wabs != 0.0) { lds_add(&B.ledger[L_W_ABS], ph.acc_wabs); lds_add(&B.ledger[L_E_ABS], ph.acc_wabs * e); }
    if (ph.acc_wcap != 0.0) { lds_add(&B.ledger[L_W_CAPLOSS], ph.acc_wcap); lds_add(&B.ledger[L_E_CAPLOSS], ph.acc_wcap * e); }
    double we = ph.w * e;
    switch (kind) {
    case END_ESCAPE: lds_add(&B.ledger[L_W_ESC], ph.w); lds_add(&B.ledger[L_E_ESC], we); lds_inc(&B.stats[S_ESCAPED], 1); break;
    case END_OOB: lds_add(&B.ledger[L_W_OOB], ph.w); lds_add(&B.ledger[L_E_OOB], we); lds_inc(&B.stats[S_OOB], 1); break;
    case END_STUCK: lds_add(&B.ledger[L_W_STUCK], ph.w); lds_add(&B.ledger[L_E_STUCK], we); lds_inc(&B.stats[S_STUCK], 1); break;
    default: break;
    }
    lds_inc(&B.stats[S_STEPS], ph.steps);
    lds_inc(&B.stats[S_VERLET_IT], ph.steps + ph.nsub);   // flat: one corrector pass per (partial) step
    lds_inc(&B.stats[S_COEF], (unsigned long long)ph.ncoef);
    write_trace(A, ph, kind, inu, ith);
}

// Flat-spacetime tracker (geodesic section with Gamma = 0; Absorption and
// Scattering sections).  Each lane evaluates the opacities at one point per
// iteration: the end of a trial step, or -- on the iteration after a
// scattering -- the scattering point the parent restarts from.  A photon
// that ends keeps its state in the idle lane; its bookkeeping (tally,
// ledger, trace) runs in the wave's next refill pass together with the
// other lanes that ended, instead of diverging from the stepping lanes.
template <int WAVES, bool F32, bool BATCHED>
__global__ __launch_bounds__(256, WAVES) void track_kernel_flat(TArgs L)
{
    extern __shared__ double lds[];
    const int stride = L.lds_stride;
    lds_zero(lds, L.n_inst, stride);
    EvStage ev = ev_stage(lds, L.n_inst, stride);
    const unsigned long long n_src = min(*L.src_count, L.cap);
    Photon ph;
    ph.inst = 0;
    StepArgs cur{};                         // batched: the step fields of this lane's instance
    int cur_inst = -1;
    bool alive = false, exhausted = false, restart = false;
    int ended = 0;                          // end kind awaiting bookkeeping
    // one instance: the arguments every step reads, held in registers
    TArgs Lh = L;
    if constexpr (!BATCHED) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            keep_vgpr(Lh.inv_dx[j]); keep_vgpr(Lh.xs[j]); keep_vgpr(Lh.xe[j]); keep_vgpr(Lh.n[j]);
        }
        keep_vgpr(Lh.step_h); keep_vgpr(Lh.C); keep_vgpr(Lh.roulette_frac);
        keep_vgpr(Lh.bias_value); keep_vgpr(Lh.bias_max);
        keep_vgpr(Lh.scattering); keep_vgpr(Lh.n_sc_max); keep_vgpr(Lh.bias_mode);
        keep_vgpr(Lh.key0); keep_vgpr(Lh.key1);
        if constexpr (!F32) {
            keep_vgpr(Lh.sh.lt0); keep_vgpr(Lh.sh.inv_dt);
            keep_vgpr(Lh.sh.le0); keep_vgpr(Lh.sh.inv_de);
        }
    }
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
                        finish(L.insts[iu], B, ph, ended);
                        ended = 0;
                    }
                }
            } else if (ended) {
                BlockAcc B = lds_acc(lds, stride, 0);
                finish(L, B, ph, ended);
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
                        load_photon(L.src, idx, ph);
                        alive = true;
                        restart = false;
                        if constexpr (BATCHED) {
                            if (ph.inst != cur_inst) {
                                cur = step_args(L.insts[ph.inst]);
                                cur_inst = ph.inst;
                            }
                        }
                    }
                }
            }
        }
        if (!__any(alive)) break;
        bool scat = false;
        double wchild = 0.0;
        int zs = -1;
        Rng ev_rng{0u, 0u, 0u, 0u};
        if (alive && !restart && (long long)ph.steps >= L.max_steps) {
            ended = END_STUCK;
            alive = false;
        }
        // one step (or restart, or load evaluation) of this lane's photon
        // with the arguments of its instance
        auto advance = [&](const auto &A, BlockAcc &B) {
            // ---- the point where the opacities are needed ----
            double dl = 0.0;
            double xn[3];
            if (restart) {
#pragma unroll
                for (int m = 0; m < 3; ++m) xn[m] = ph.x[m];
            } else {
                // step: step_h times the smallest zone-crossing parameter
                double rate = fmax(fmax(fabs(ph.k[1]) * A.inv_dx[0], fabs(ph.k[2]) * A.inv_dx[1]),
                                   fabs(ph.k[3]) * A.inv_dx[2]);
                dl = A.step_h / rate;
#pragma unroll
                for (int m = 0; m < 3; ++m) xn[m] = ph.x[m] + ph.k[m + 1] * dl;
            }
            int zn = zone_cart(A, xn[0], xn[1], xn[2]);
            Coef c1;
            if (zn == ph.cz) {
                c1 = Coef{ph.cnua, ph.cnus, ph.cb, ph.cvac};
            } else {
                double xv[4] = {0.0, xn[0], xn[1], xn[2]};
                c1 = coefficients<Minkowski, F32>(A, L.el, zn, xv, ph.k, ph.n_sc);   // one distribution per launch
                ph.cz = zn;
                ph.cnua = c1.nua; ph.cnus = c1.nus; ph.cb = c1.b; ph.cvac = c1.vacuum;
                ph.ncoef += 1;
            }
            if (restart) {
                ph.nua = c1.nua; ph.nus = c1.nus;
                if (!c1.vacuum) ph.b = c1.b;
                restart = false;
            } else {
                ph.steps += 1;
                // ---- optical depths by the trapezoid rule ----
                double tau_a = 0.5 * (ph.nua + c1.nua) * A.C * dl;
                double tau_s = A.scattering ? 0.5 * (ph.nus + c1.nus) * A.C * dl : 0.0;
                const double bf = c1.vacuum ? ph.b : c1.b;
                const double b = step_bias(A, ph.w, bf);
                if (A.scattering && ph.n_sc < A.n_sc_max && b * tau_s > ph.x1) {
                    // ---- scattering point: the step's start advanced over
                    // the fraction f of the step (a straight line here) ----
                    double f = ph.x1 / (b * tau_s);
                    double fdl = f * dl;
                    double xs[3];
#pragma unroll
                    for (int m = 0; m < 3; ++m) xs[m] = ph.x[m] + ph.k[m + 1] * fdl;
                    ph.nsub += 1;
                    double wbf = ph.w;
                    ph.w *= exp(-f * tau_a);
                    ph.acc_wabs += wbf - ph.w;
                    wchild = ph.w / b;
                    // plasma of the scattering point, else of the step's start, else its end
                    zs = zone_cart(A, xs[0], xs[1], xs[2]);
                    if (zs >= 0 && !(A.zrec[(size_t)zs * Z_STRIDE + Z_NE] > 0.0)) zs = -1;
                    if (zs < 0) {
                        zs = zone_cart(A, ph.x[0], ph.x[1], ph.x[2]);
                        if (zs >= 0 && !(A.zrec[(size_t)zs * Z_STRIDE + Z_NE] > 0.0)) zs = -1;
                    }
                    if (zs < 0) {
                        zs = zn;
                        if (zs >= 0 && !(A.zrec[(size_t)zs * Z_STRIDE + Z_NE] > 0.0)) zs = -1;
                    }
                    ev_rng = ph.rng;              // the parent's stream at the event
                    // the parent continues from the scattering point; its
                    // opacities there are evaluated on the next iteration
                    ph.w *= (1.0 - 1.0 / b);
                    ph.x1 = -log(1.0 - rng_uniform(ph.rng, A.key0, A.key1));
#pragma unroll
                    for (int m = 0; m < 3; ++m) ph.x[m] = xs[m];
                    restart = true;
                    scat = true;
                    if (b == 1.0) {    // all weight went to the child
                        ended = END_SPLIT;
                        alive = false;
                    }
                } else {
                    if (A.scattering) {
                        if (ph.n_sc < A.n_sc_max) {
                            ph.x1 -= b * tau_s;
                        } else {   // generation cap: extinction without a child
                            double wbc = ph.w;
                            ph.w *= exp(-tau_s);
                            ph.acc_wcap += wbc - ph.w;
                        }
                    }
                    double wba = ph.w;
                    ph.w *= exp(-tau_a);
                    ph.acc_wabs += wba - ph.w;
#pragma unroll
                    for (int m = 0; m < 3; ++m) ph.x[m] = xn[m];
                    ph.nua = c1.nua; ph.nus = c1.nus; ph.b = bf;
                    bool esc = false;
#pragma unroll
                    for (int j = 0; j < 3; ++j) esc |= (ph.x[j] < A.xs[j]) || (ph.x[j] >= A.xe[j]);
                    if (esc) {
                        ended = END_ESCAPE;
                        alive = false;
                    }
                }
                // ---- Russian roulette below roulette_frac of the birth weight ----
                if (alive && ph.w < A.roulette_frac * ph.wb) {
                    double e = ph.k[0] * kMeC2;
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
            }
        };
        if constexpr (BATCHED) {
            // every lane with its own instance's fields: one pass for the
            // wave whatever instances its photons belong to
            if (alive) {
                BlockAcc B = lds_acc(lds, stride, ph.inst);
                advance(cur, B);
            }
        } else if (alive) {
            BlockAcc B = lds_acc(lds, stride, 0);
            advance(Lh, B);
        }
        // ---- scattering events, staged per wave in LDS: the scattering
        // point and the incoming wavevector (the parent's own, unchanged in
        // flat spacetime) ----
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
                finish(L.insts[iu], B, ph, ended);
                ended = 0;
            }
        }
    } else if (ended) {
        BlockAcc B = lds_acc(lds, stride, 0);
        finish(L, B, ph, ended);
        ended = 0;
    }
    lds_flush_all(L, lds, stride);
}

// Events of the generation per instance (batched launches).
__global__ __launch_bounds__(256) void count_events_kernel(TArgs L)
{
    __shared__ unsigned int hist[64];
    if (threadIdx.x < 64) hist[threadIdx.x] = 0u;
    __syncthreads();
    const unsigned long long n = min(*L.dst_count, L.cap);
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
        atomicAdd(&hist[L.dst.inst[i]], 1u);
    __syncthreads();
    if (threadIdx.x < L.n_inst && hist[threadIdx.x])
        atomicAdd(&L.inst_count[threadIdx.x], (unsigned long long)hist[threadIdx.x]);
}

// Batched scattering: the events of a block's 256-event window are given
// slots in the output queue grouped by instance (per-block reservation per
// instance); calls ev(i, slot) for every event of the window.  Every thread
// of the block runs the same number of windows.
template <class Ev>
GM_D void for_events_grouped(const TArgs &L, unsigned long long n, Ev ev)
{
    __shared__ unsigned long long off[64], lbase[64];
    __shared__ unsigned int lcount[64];
    if (threadIdx.x == 0) {
        unsigned long long acc = 0;
        for (int k = 0; k < L.n_inst; ++k) { off[k] = acc; acc += L.inst_count[k]; }
    }
    for (unsigned long long base = (unsigned long long)blockIdx.x * blockDim.x; base < n;
         base += (unsigned long long)gridDim.x * blockDim.x) {
        if (threadIdx.x < 64) lcount[threadIdx.x] = 0u;
        __syncthreads();
        const unsigned long long i = base + threadIdx.x;
        const bool valid = i < n;
        const int ii = valid ? L.dst.inst[i] : 0;
        const unsigned int local = valid ? atomicAdd(&lcount[ii], 1u) : 0u;
        __syncthreads();
        if (threadIdx.x < L.n_inst && lcount[threadIdx.x])
            lbase[threadIdx.x] = off[threadIdx.x] + atomicAdd(&L.inst_cursor[threadIdx.x], (unsigned long long)lcount[threadIdx.x]);
        __syncthreads();
        if (valid) ev(i, lbase[ii] + local);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Scattering events -> child photons (Scattering section), one thread per
// event of the generation just tracked.  Draws come from the child's stream
// (derived from the parent's stream and counter at the event): electron
// (gamma, mu), electron azimuth, scattering angle and azimuth, then the
// child's own optical-depth draw.
// ---------------------------------------------------------------------------
template <bool F32, bool BATCHED>
__global__ __launch_bounds__(256, 2) void scatter_kernel_flat(TArgs L)
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
        double x[4] = {0.0, Q.x[0][i], Q.x[1][i], Q.x[2][i]};
        double ks[4] = {Q.k[0][i], Q.k[1][i], Q.k[2][i], Q.k[3][i]};
        int z = Q.zone[i];
        int n_sc = Q.n_sc[i];
        double wchild = Q.w[i];
        const Rng r_par{Q.s0[i], Q.s1[i], Q.s2[i], 0u};
        const uint32_t pev = Q.ev[i];
        Rng r = child_rng(r_par, Q.blk[i], A.key0, A.key1);
        const Rng r_child = r;
        uint32_t cev = kNoEvent;
        double g[4][4];
        Minkowski::gcov(x, g);
        double kc[4];
        if (z >= 0) {
            const double *zr = A.zrec + (size_t)z * Z_STRIDE;
            double u[4], bh[4], e[4][4];
            bool has_b = fluid_frame_flat(zr, u, bh);
            double eps = scatter_tetrad(g, u, bh, has_b, ks, e);
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
        if (A.evlog && z >= 0)
            cev = log_event(A, r_child, &r_par, z, n_sc, -dot4(g, ks, A.zrec + (size_t)z * Z_STRIDE + Z_U0), wchild,
                            x + 1, pev);
        lds_add(&B.ledger[L_E_COMPTON], wchild * (e_inf(g, kc) - e_inf(g, ks)) * kMeC2);
        lds_inc(&B.stats[S_SCATTER], 1);
        lds_inc(&B.stats[S_CHILDREN], 1);
        lds_inc(&B.stats[S_GEN0 + min(n_sc, 15)], 1);
        double x1 = -log(1.0 - rng_uniform(r, A.key0, A.key1));
        Coef c = coefficients<Minkowski, F32>(A, A.el, zone_cart(A, x[1], x[2], x[3]), x, kc, n_sc);
        const PhotonQ &O = BATCHED ? L.out : Q;
        if (BATCHED) {
#pragma unroll
            for (int m = 0; m < 3; ++m) O.x[m][o] = x[m + 1];
            O.w[o] = wchild;
            O.n_sc[o] = n_sc;
            O.inst[o] = ii;
        }
        O.s0[o] = r_child.s0; O.s1[o] = r_child.s1; O.s2[o] = r_child.s2;
#pragma unroll
        for (int m = 0; m < 4; ++m) O.k[m][o] = kc[m];
        O.wb[o] = wchild;
        O.x1[o] = x1;
        O.nua[o] = c.nua; O.nus[o] = c.nus; O.b[o] = c.b;
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

// Scores of one generation's records reach their parents' records
// (records [lo, hi) of one track call; launched from the highest generation
// down, so a record's score is complete when it is passed on).
__global__ __launch_bounds__(256) void score_propagate_kernel(EventRec *ev, unsigned long long lo,
                                                              unsigned long long hi, int gen)
{
    for (unsigned long long i = lo + (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        const EventRec &e = ev[i];
        if (e.gen == gen && e.parent != kNoEvent && e.score != 0.0) atomicAdd(&ev[e.parent].score, e.score);
    }
}

}  // namespace gm
