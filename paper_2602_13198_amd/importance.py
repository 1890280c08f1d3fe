"""Importance-driven forms of the transport and their time to 1 % spectral
error against the plain uniform bias.

The paper names tuning the scattering bias "on the fly" as future work
(Conclusions).  Two forms are built here, both from records the method
itself produces (the library's event log: one record per scattering and per
sampled root emission, each carrying the score of the photon it created --
the sum, over that photon and every descendant that escapes into a tally
bin, of its escaping energy times the bin's score weight):

* adaptive: no network.  The importance of a photon created at (zone,
  photon energy) is estimated from the records that fall in a coarse
  spatial cell and an energy node -- summed scores over summed weights
  (per unit weight, for the bias) or over the number of records (per
  photon, for the emission) -- shrunk towards the overall mean where
  records are few;
* learned: a network 6 -> 64 -> 64 -> 2 (the library's matrix-core kernels,
  BF16 operands, FP32 accumulation) trained on the same records with the
  log-link Poisson deviance, whose minimiser is the log of the mean
  importance (also for records whose score is zero); its first output is
  the importance of a scattered photon, its second that of an emitted one.

Both give the same two tables: the weight-window bias b = clamp(c_b w I_sc,
1, b_max), so that children carry weights near 1/(c_b I_sc), and the
defensive emission proposal w_i(nu) = w(nu) / [(1 - alpha) + alpha S_em /
S_bar] (S_em the score a root born there carries, S_bar its mean over the
plain roots), which spends roots where they contribute most and keeps at
least 1 - alpha of the plain roots elsewhere.  Any b >= 1 and any positive emission weight keep the
estimator unbiased (child w/b and parent w(1 - 1/b), Scattering section;
the expected emitted luminosity of eq:weight_calc does not depend on w).
c_b and the emission table's shift hold the children and roots to the plain
run's budget.

Score weights are the relative-error weights of the measure, 1 / L(bin) on
the bins the pilot rounds resolve; the pilot rounds are plain rounds and
their cost is counted in the form's time.  The host part here prepares
training arrays and drives the library; transport, the records' scores,
network training, the cell sums and both tables (inference over every
zone and node) run in the library's kernels."""
from __future__ import annotations

import math
import time

import numpy as np

from . import convergence as CV
from . import gm as GM

MEC2_OVER_H = 1.2355899341e20          # m_e c^2 / h in Hz
LN_EPS = (math.log(1e-12), math.log(1e6))


# ---------------------------------------------------------------------------
# zone geometry and features
# ---------------------------------------------------------------------------
def zone_geometry(wl):
    """Per zone: (i1, i2, i3), radius feature (Kerr: ln r; flat: |x| over the
    half-size) and cos theta of the zone centre."""
    g = wl.grid
    n1, n2, n3 = g["n"]
    i1, i2, i3 = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    i1, i2, i3 = i1.reshape(-1), i2.reshape(-1), i3.reshape(-1)
    xc = [g["x_start"][j] + (idx + 0.5) * g["dx"][j] for j, idx in enumerate((i1, i2, i3))]
    if g["metric"] == 0:
        half = 0.5 * max(n * d for n, d in zip(g["n"], g["dx"]))
        rr = np.sqrt(xc[0] ** 2 + xc[1] ** 2 + xc[2] ** 2)
        rad = rr / half
        cth = np.where(rr > 0, xc[2] / np.maximum(rr, 1e-300), 0.0)
    else:
        hs = g["h_slope"]
        th = np.pi * xc[1] + 0.5 * (1 - hs) * np.sin(2 * np.pi * xc[1])
        rad = xc[0]
        cth = np.cos(th)
    return (i1, i2, i3), rad, cth


_FEATURES = {}


def zone_features(wl):
    """[nz][8]: ln Theta_e, ln n_e, ln(B + 1e-10), 0 (the photon energy's
    slot), radius feature, cos theta, 0, 0 -- the zone's part of a feature
    row (kept for the workload object once computed)."""
    key = id(wl)
    hit = _FEATURES.get(key)
    if hit is not None and hit[0] is wl:
        return hit[1]
    f = _zone_features(wl)
    _FEATURES.clear()
    _FEATURES[key] = (wl, f)
    return f


def _zone_features(wl):
    _, rad, cth = zone_geometry(wl)
    tiny = 1e-300
    zf = np.zeros((len(rad), 8))
    zf[:, 0] = np.log(np.maximum(wl.theta_e, 1e-3))
    zf[:, 1] = np.log(np.maximum(wl.n_e, tiny))
    zf[:, 2] = np.log(wl.B + 1e-10)
    zf[:, 4], zf[:, 5] = rad, cth
    return zf


def rows(zf, zone, ln_e):
    """Feature rows [n][8] (6 used) for zones and log photon energies: one
    gather of the zones' rows, then the energy slot."""
    X = zf[zone]
    X[:, 3] = ln_e
    return X


# ---------------------------------------------------------------------------
# records
# ---------------------------------------------------------------------------
def pilot(ctx, wl, inst, rounds, seed0, n_s, root_stride=4, track=None):
    """Plain rounds with the event log on.  Round 0 only measures the
    spectrum, whose resolved bins (relative standard error <= 10 %, >= 100
    superphotons) get the score weight 1 / L(bin); the next `rounds` rounds
    log their records into one device buffer, where they stay (the caller
    reads them if it needs them on the host)."""
    track = dict(track or wl.track)
    emit = dict(wl.emit, n_target=float(n_s))
    ctx.reset_spectrum(inst)
    ctx.make_superphotons(dict(emit, seed=seed0), instance=inst)
    ctx.track_scatter(track)
    sp, _ = ctx.read_spectrum(inst, reset=True)
    S1, S2, N = sp[..., 0], sp[..., 1], sp[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        rse = np.where(S1 > 0, np.sqrt(S2) / S1, np.inf)
    sw = np.where((N >= 100) & (rse <= 0.1), 1.0 / np.maximum(S1, 1e-300), 0.0)
    ctx.set_score_weights(inst, sw)
    ctx.set_event_log(int(rounds * 6 * n_s) + 100000, root_stride)
    for r in range(rounds):
        ctx.make_superphotons(dict(emit, seed=seed0 + 1 + r), instance=inst)
        ctx.track_scatter(track)
    ctx.read_spectrum(inst, reset=True)
    ctx.set_score_weights(inst, None)
    return sw


def event_columns(ev):
    """The event log's fields the tables use, as contiguous columns, in the
    order of the created photons' streams: the log's own order follows the
    device's scheduling, and the network's batches and held-out rows are
    taken by position, so sorting makes its training repeatable."""
    key = (ev["s0"].astype(np.uint64) | (ev["s1"].astype(np.uint64) << np.uint64(32)))
    order = np.argsort(key)          # 64 bits of a distinct stream per record
    return {k: np.ascontiguousarray(ev[k][order]) for k in ("zone", "gen", "eps", "w", "score")}


def split_records(ev):
    """(scatter records, emission records) with positive weight, as column
    dicts (zone, eps, w, score); an emission record stands for the pilot's
    root stride of roots."""
    gen, w, score = ev["gen"], ev["w"], ev["score"]
    ok = (w > 0) & np.isfinite(w) & np.isfinite(score)
    return tuple({k: ev[k][m] for k in ("zone", "eps", "w", "score")} for m in (ok & (gen > 0), ok & (gen == 0)))


# ---------------------------------------------------------------------------
# the learned form: the network on the library's kernels
# ---------------------------------------------------------------------------
class Network:
    """Standardised features, Poisson-deviance training, inference."""

    def __init__(self, seed=1):
        self.seed = seed

    @staticmethod
    def initial_params(seed):
        rng = np.random.default_rng(seed)
        parts = []
        for fan_in, fan_out in ((6, 64), (64, 64), (64, 2)):
            lim = math.sqrt(6.0 / (fan_in + fan_out))
            parts.append(rng.uniform(-lim, lim, fan_in * fan_out))
            parts.append(np.zeros(fan_out))
        return np.concatenate(parts).astype(np.float32)

    def standardise(self, X):
        Z = np.zeros((len(X), 8), dtype=np.float32)
        Z[:, :6] = (X[:, :6] - self.mu) * (1.0 / self.sd)
        return Z

    def fit(self, ctx, X, T, C, steps=800, batch=16384, lr=2e-3):
        """X rows, T [n][2] targets (>= 0, normalised to mean 1 per output),
        C [n][2] weights (0 where a row does not train an output)."""
        import torch
        # feature means and standard deviations from the first two moments
        n6 = max(len(X), 1)
        m1 = X.sum(0)[:6] / n6
        m2 = np.einsum("ij,ij->j", X, X)[:6] / n6
        self.mu = m1
        self.sd = np.sqrt(np.maximum(m2 - m1 * m1, 0.0)) + 1e-6
        Z = self.standardise(X)
        n = len(Z)
        ctx.mlp_set_params(self.initial_params(self.seed))
        ctx.mlp_set_loss(GM.MLP_POISSON)
        Xd = torch.as_tensor(Z, device="cuda")
        Td = torch.as_tensor(T.astype(np.float32), device="cuda")
        # each output's weights sum to 1 over a batch on average
        b = min(batch, n)
        Cn = C / np.maximum(C.sum(0, keepdims=True), 1e-30) * (n / b)
        Cd = torch.as_tensor(Cn.astype(np.float32), device="cuda")
        gen = torch.Generator(device="cuda")
        gen.manual_seed(self.seed)
        hist = []
        # batches are consecutive slices of the rows in a fresh random order
        # per pass over them; each pass's steps run in one library call, the
        # learning rate falling as lr 0.1^(s / steps) over the whole fit
        per_pass = max(n // b, 1)
        s = 0
        while s < steps:
            k = min(per_pass, steps - s)
            if n > batch:
                perm = torch.randperm(n, device="cuda", generator=gen)
                Xp, Tp, Cp = Xd[perm], Td[perm], Cd[perm]
            else:
                Xp, Tp, Cp = Xd, Td, Cd
            want = s == 0 or s + k == steps
            L = ctx.mlp_train_steps(Xp, Tp, Cp, b, k, lr * 0.1 ** (s / steps), 0.1 ** (k / steps), want_loss=want)
            if s == 0:
                hist.append((0, L[0]))
            if s + k == steps:
                hist.append((steps - 1, L[1]))
            s += k
        ctx.mlp_set_loss(GM.MLP_SQUARED)
        return hist

    def predict(self, ctx, X, chunk=1 << 22):
        out = []
        for a in range(0, len(X), chunk):
            out.append(ctx.mlp_forward(self.standardise(X[a:a + chunk])).cpu().numpy().astype(np.float64))
        return np.concatenate(out) if out else np.zeros((0, 2))


# ---------------------------------------------------------------------------
# tables (built on the device by the library)
# ---------------------------------------------------------------------------
def heldout_deviance(net, ctx, X, T, C, hold):
    """Poisson deviance e^y - t y per output on the held-out rows, of the
    network and of the best constant predictor (ln of the training rows'
    mean target): [(network, constant), ...]."""
    y = net.predict(ctx, X[hold])
    out = []
    for o in range(T.shape[1]):
        w = C[hold, o] > 0
        tr = (~hold) & (C[:, o] > 0)
        if not w.any() or not tr.any():
            out.append((math.inf, math.inf))
            continue
        t, yy = T[hold, o][w], y[w, o]
        c = math.log(max(T[tr, o].mean(), 1e-300))
        out.append((float(np.mean(np.exp(yy) - t * yy)), float(np.mean(math.exp(c) - t * c))))
    return out


def emission_band(ev, nodes, pad=0.5):
    """ln nu range of the emission records (the band the plain roots are
    born in), padded by `pad` node spacings on each side; ev is the records
    (host columns) or the (eps_min, eps_max) pair the library finds on the
    device."""
    if isinstance(ev, tuple):
        lo, hi = (math.log(e * MEC2_OVER_H) for e in ev)
    else:
        m = (ev["gen"] == 0) & (ev["w"] > 0)
        ln_nu = np.log(ev["eps"][m] * MEC2_OVER_H)
        lo, hi = float(ln_nu.min()), float(ln_nu.max())
    d = (hi - lo) / max(nodes - 1, 1)
    return lo - pad * d, hi + pad * d


def build_tables(ctx, wl, inst, b_plain, b_max, n_s, mode, net_seed=1, use_bias=True, use_emission=True,
                 alpha=0.5, nodes=16, em_nodes=32, train_steps=1000, train_batch=16384):
    """Tables of the adaptive ("cells") or learned ("network") form from the
    records in the context's event log, built on the device; sets the
    instance's weight-window bias table and defensive emission table.
    Window bias: ln(c_b I_sc) with c_b = records / summed score, so that
    the mean bias over the pilot's scattering opportunities is the plain b
    (the parent's weight at a pilot scattering is b times its child's, and
    the sum over records of w_child I_sc is the summed score).  Emission:
    em_nodes nodes over the band the pilot's roots were born in; S_em is
    the score a root born at (zone, nu) carries (per photon, not per unit
    weight: a root density r times the plain one and weights divided by r
    leave the estimator unbiased, and its variance, the plain roots' mean
    of (w S)^2 / r, is least for r proportional to w S, the plain root's
    score); the table is ln((1 - alpha) + alpha S_em / S_bar) with S_bar
    the mean of S_em over the plain roots (the expected roots of the table
    ln S_em over those of the plain method), so that the plain roots' mean
    of the density ratio is 1 and every region keeps at least 1 - alpha of
    its plain roots; a last shift, fixed by the expected roots, absorbs
    what the interpolation between nodes leaves.  The network trains on
    nine rows in ten; an output whose Poisson deviance on the held-out
    rows is not below that of the constant mean builds no table (the form
    falls back to the plain bias, resp. emission; info["fallback"])."""
    info, t0 = {}, time.perf_counter()
    e = wl.emit
    emit_round = dict(e, n_target=float(n_s))
    nb0 = ctx.expected_roots(emit_round, inst)
    # the cells need the records on the device only; the network trains on
    # host rows
    ev = event_columns(ctx.read_event_log()) if mode != "cells" else None
    info["read_s"] = time.perf_counter() - t0
    lo_nu, hi_nu = emission_band(ctx.event_band(), em_nodes)
    info["emission_band_hz"] = [math.exp(lo_nu), math.exp(hi_nu)]
    m_bias = GM.Context.importance_map(GM.TABLE_BIAS, nodes, LN_EPS[0], LN_EPS[1], GM.IMP_LINEAR)
    m_em = GM.Context.importance_map(GM.TABLE_EMISSION, em_nodes, lo_nu, hi_nu, GM.IMP_LINEAR, per_photon=1)
    if mode == "cells":
        del ev
        tot_sc = ctx.cells_accumulate(inst, m_bias)
        if use_bias:
            m_bias.b = math.log(tot_sc[2] / max(tot_sc[0], 1e-300))
            ctx.cells_fill_table(inst, m_bias)
        tot_em = ctx.cells_accumulate(inst, m_em)
        b_I = 0.0                                            # the cells' table is ln S itself
        fill = lambda m: ctx.cells_fill_table(inst, m)       # noqa: E731
        info["records"] = [int(tot_sc[2]), int(tot_em[2])]
    else:
        sc, em = split_records(ev)
        n_sc, n_em = len(sc["zone"]), len(em["zone"])
        del ev
        zf = zone_features(wl)
        X = np.concatenate([rows(zf, sc["zone"], np.log(sc["eps"])), rows(zf, em["zone"], np.log(em["eps"]))])
        t_sc, t_em = sc["score"] / sc["w"], em["score"]
        m_sc, m_em_mean = max(t_sc.mean(), 1e-300), max(t_em.mean(), 1e-300)
        T = np.zeros((len(X), 2))
        Cw = np.zeros((len(X), 2))
        T[:n_sc, 0], Cw[:n_sc, 0] = t_sc / m_sc, 1.0
        T[n_sc:, 1], Cw[n_sc:, 1] = t_em / m_em_mean, 1.0
        net = Network(seed=net_seed)
        t1 = time.perf_counter()
        info["features_s"] = t1 - t0 - info["read_s"]
        # every tenth row held out: a table is built only from an output that
        # predicts those rows better than the constant mean does
        hold = (np.arange(len(X)) % 10) == 0
        Ct = Cw.copy()
        Ct[hold] = 0.0
        hist = net.fit(ctx, X, T, Ct, steps=train_steps, batch=train_batch)
        info["train_s"] = time.perf_counter() - t1
        info["loss_first_last"] = [hist[0][1], hist[-1][1]]
        info["records"] = [n_sc, n_em]
        t2 = time.perf_counter()
        dev = heldout_deviance(net, ctx, X, T, Cw, hold)
        info["heldout_deviance"] = dev
        info["heldout_s"] = time.perf_counter() - t2
        if use_bias and not dev[0][0] < dev[0][1]:
            use_bias = False
            info["fallback"] = info.get("fallback", []) + ["bias"]
        if use_emission and not dev[1][0] < dev[1][1]:
            use_emission = False
            info["fallback"] = info.get("fallback", []) + ["emission"]
        if use_bias:
            # ln I = y + ln(mean t); c_b = records / summed score
            m_bias.b = math.log(m_sc) + math.log(n_sc / max(sc["score"].sum(), 1e-300))
            ctx.mlp_fill_table(inst, m_bias, 0, net.mu, net.sd)
        b_I = math.log(m_em_mean)                            # ln S = y + ln(mean t)
        fill = lambda m: ctx.mlp_fill_table(inst, m, 1, net.mu, net.sd)   # noqa: E731
    t3 = time.perf_counter()
    if use_emission:
        # the table ln S once, then mapped in place: the plain roots' mean of
        # S is the expected roots of the table ln S over the plain ones
        m_em.b = b_I
        fill(m_em)
        i_bar = ctx.expected_roots(emit_round, inst) / nb0
        m_em.kind, m_em.alpha, m_em.a, m_em.b = GM.IMP_MIXTURE, alpha, 1.0, -math.log(max(i_bar, 1e-300))
        ctx.remap_table(inst, m_em)
        nb1 = ctx.expected_roots(emit_round, inst)
        m_em.kind, m_em.a, m_em.b, m_em.shift = GM.IMP_LINEAR, 1.0, 0.0, math.log(nb0 / max(nb1, 1e-300))
        ctx.remap_table(inst, m_em)
        info["emission_shift"] = m_em.shift
    info["bias_table"], info["emission_table"] = bool(use_bias), bool(use_emission)
    info["tables_s"] = time.perf_counter() - t0
    info["emission_table_s"] = info["tables_s"] - (t3 - t0)
    return info


# ---------------------------------------------------------------------------
# the comparison
# ---------------------------------------------------------------------------
FORMS = {
    # name: (table source, weight-window bias, emission proposal)
    "adaptive": ("cells", True, True),
    "learned": ("network", True, True),
}


def compare_forms(ctx, wl, inst, seeds=3, ref_rounds=24, round_div=32, pilot_rounds=1, b_max=100.0,
                  forms=("adaptive", "learned"), log=None, alpha=0.5, variants=None):
    """Time to 1 % spectral error of the plain uniform bias and of the
    adaptive and learned forms on one workload (median over seeds), against
    one plain reference of ref_rounds rounds of N_s."""
    import torch
    n_s = wl.emit["n_target"]
    n_round = n_s / round_div
    b_plain = wl.track["bias_value"]
    t0 = time.perf_counter()
    L_ref, cnt_ref, rse_ref, n_ref = CV.reference(ctx, wl, inst, ref_rounds, 100000)
    t_ref = time.perf_counter() - t0
    # bins resolved by the reference (>= 1e3 superphotons) whose relative
    # standard error in one measured round is at most 10 %
    rse_round = rse_ref * math.sqrt(round_div)
    mask = (cnt_ref * ref_rounds >= 1e3) & (rse_round <= 0.1)
    if log:
        log("reference: %d rounds, %.3g superphotons, %.1f s, %d masked bins" % (ref_rounds, n_ref, t_ref, mask.sum()))
    out = {"target_eps_err": 0.01, "round_superphotons_target": n_round,
           "reference": {"rounds": ref_rounds, "n_s_per_round": n_s, "superphotons": n_ref, "seconds": t_ref,
                         "masked_bins": int(mask.sum()),
                         "mask": "bins holding >= 1e3 superphotons in the reference whose relative standard "
                                 "error per measured round (N_s/%d) is <= 10%%" % round_div,
                         "seeds": "disjoint from every measured run"}}
    runs = [CV.time_to_error(ctx, wl, inst, L_ref, mask, 200000 + 1000 * k, n_round, max_rounds=512)
            for k in range(seeds)]
    secs = [r["seconds"] for r in runs]
    med_p = float(np.median(secs)) if all(s is not None for s in secs) else None
    out["plain"] = {"bias": "constant b = %g" % b_plain, "seconds_median": med_p, "seconds": secs,
                    "superphotons": [r["superphotons"] for r in runs],
                    "final_eps": [r["final_eps"] for r in runs]}
    if log:
        log("plain: %s" % secs)
    root_stride = 4
    variants = dict(FORMS, **(variants or {}))
    for name in forms:
        form, use_bias, use_em = variants[name]
        res = []
        infos = []
        for k in range(seeds):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            try:
                pilot(ctx, wl, inst, pilot_rounds, 300000 + 1000 * k, n_round, root_stride)
                info = build_tables(ctx, wl, inst, b_plain, b_max, n_round, form, net_seed=1 + k,
                                    use_bias=use_bias, use_emission=use_em, alpha=alpha)
                ctx.set_event_log(0)
                torch.cuda.synchronize()
                t_prep = time.perf_counter() - ta
                over = dict(bias_mode=GM.BIAS_WINDOW, bias_max=b_max) if info["bias_table"] else None
                r = CV.time_to_error(ctx, wl, inst, L_ref, mask, 400000 + 1000 * k, n_round, max_rounds=512,
                                     track_overrides=over)
            except GM.GmError as exc:          # reported, not hidden: the form has no time then
                ctx.set_emission_table(inst, None)
                ctx.set_event_log(0)
                ctx.read_spectrum(inst, reset=True)
                res.append(None)
                infos.append({"error": str(exc)})
                if log:
                    log("%s seed %d failed: %s" % (form, k, exc))
                continue
            ctx.set_emission_table(inst, None)
            info["prep_s"] = t_prep
            res.append((r["seconds"] + t_prep) if r["seconds"] is not None else None)
            infos.append(dict(info, superphotons=r["superphotons"], final_eps=r["final_eps"],
                              transport_s=r["seconds"]))
            if log:
                log("%s seed %d: prep %.2f s, transport %s s, final eps %.4f, %.3g superphotons"
                    % (name, k, t_prep, r["seconds"], r["final_eps"], r["superphotons"]))
        med = float(np.median(res)) if all(s is not None for s in res) else None
        parts = []
        if use_bias:
            parts.append("weight-window bias b = clamp(c_b w I_sc, 1, %g)" % b_max)
        if use_em:
            parts.append("defensive emission proposal w / [(1 - %g) + %g S_em / S_bar] (S_em the score per root, "
                         "S_bar its plain mean)" % (alpha, alpha))
        out[name] = {
            "seconds_median": med, "seconds": res, "runs": infos,
            "what": ("importance per (8x8x8-zone cell, energy node) from summed scores / summed weights"
                     if form == "cells" else
                     "network 6-64-64-2 trained on the library's matrix-core kernels (Poisson deviance)")
                    + "; " + " and ".join(parts) + "; %d plain pilot rounds counted in the time" % pilot_rounds,
            "plain_over_form": (med_p / med) if (med_p and med) else None,
        }
    ctx.read_spectrum(inst, reset=True)
    return out
