"""Importance-driven forms of the transport and their time to 1 % spectral
error against the plain uniform bias.

The paper names tuning the scattering bias "on the fly" as future work
(Conclusions).  Two forms are built here, both from records the method
itself produces (the library's event log: one record per scattering and per
sampled root emission, each carrying the score of the photon it created --
the sum, over that photon and every descendant that escapes into a tally
bin, of its escaping energy times the bin's score weight):

* adaptive: no network.  The importance of a unit-weight photon created at
  (zone, photon energy) is estimated by the ratio of summed scores to summed
  weights of the records that fall in a coarse spatial cell and an energy
  node, shrunk towards the overall mean where records are few;
* learned: a network 6 -> 64 -> 64 -> 2 (the library's matrix-core kernels,
  BF16 operands, FP32 accumulation) trained on the same records with the
  log-link Poisson deviance, whose minimiser is the log of the mean
  importance (also for records whose score is zero); its first output is
  the importance of a scattered photon, its second that of an emitted one.

Both give the same two tables: the weight-window bias b = clamp(c_b w I_sc,
1, b_max), so that children carry weights near 1/(c_b I_sc), and the
emission proposal w_i(nu) = c_w / I_em(zone, nu), which spends roots where
they contribute most.  Any b >= 1 and any positive emission weight keep the
estimator unbiased (child w/b and parent w(1 - 1/b), Scattering section;
the expected emitted luminosity of eq:weight_calc does not depend on w).
c_b and c_w hold the children and roots to the plain run's budget.

Score weights are the relative-error weights of the measure, 1 / L(bin) on
the bins the pilot rounds resolve; the pilot rounds are plain rounds and
their cost is counted in the form's time.  The host part here prepares
arrays and drives the library; transport, network training and inference
run in the library's kernels."""
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


def zone_features(wl):
    """[nz][5]: ln Theta_e, ln n_e, ln(B + 1e-10), radius feature, cos theta."""
    _, rad, cth = zone_geometry(wl)
    tiny = 1e-300
    return np.stack([np.log(np.maximum(wl.theta_e, 1e-3)), np.log(np.maximum(wl.n_e, tiny)),
                     np.log(wl.B + 1e-10), rad, cth], axis=1)


def rows(zf, zone, ln_e):
    """Feature rows [n][8] (6 used) for zones and log photon energies."""
    X = np.zeros((len(zone), 8))
    X[:, [0, 1, 2, 4, 5]] = zf[zone]
    X[:, 3] = ln_e
    return X


# ---------------------------------------------------------------------------
# records
# ---------------------------------------------------------------------------
def pilot(ctx, wl, inst, rounds, seed0, n_s, root_stride=4, track=None):
    """Plain rounds with the event log on: the records (with scores under
    unit score weights first, to learn the spectrum) are collected after
    the score weights are set from the pilot's own first round."""
    track = dict(track or wl.track)
    emit = dict(wl.emit, n_target=float(n_s))
    ev_all, spec_acc = [], None
    # round 0: the spectrum, for the relative-error score weights
    ctx.read_spectrum(inst, reset=True)
    ctx.make_superphotons(dict(emit, seed=seed0), instance=inst)
    ctx.track_scatter(track)
    sp, _ = ctx.read_spectrum(inst, reset=True)
    S1, S2, N = sp[..., 0], sp[..., 1], sp[..., 2]
    # relative-error weights on the bins this round resolves (relative
    # standard error <= 10 %, >= 100 superphotons)
    with np.errstate(divide="ignore", invalid="ignore"):
        rse = np.where(S1 > 0, np.sqrt(S2) / S1, np.inf)
    sw = np.where((N >= 100) & (rse <= 0.1), 1.0 / np.maximum(S1, 1e-300), 0.0)
    ctx.set_score_weights(inst, sw)
    for r in range(rounds):
        cap = int(6 * n_s) + 100000
        ctx.set_event_log(cap, root_stride)
        ctx.make_superphotons(dict(emit, seed=seed0 + 1 + r), instance=inst)
        ctx.track_scatter(track)
        sp, _ = ctx.read_spectrum(inst, reset=True)
        spec_acc = sp if spec_acc is None else spec_acc + sp
        ev = ctx.read_event_log()
        ev_all.append(ev)
    ctx.set_event_log(0)
    ctx.set_score_weights(inst, None)
    return np.concatenate(ev_all), sw, spec_acc


def split_records(ev, root_stride):
    """(scatter records, emission records) with positive weight; emission
    records stand for root_stride roots each."""
    ok = (ev["w"] > 0) & np.isfinite(ev["w"]) & np.isfinite(ev["score"])
    ev = ev[ok]
    return ev[ev["gen"] > 0], ev[ev["gen"] == 0]


# ---------------------------------------------------------------------------
# the adaptive form: cell x energy-node ratio estimates
# ---------------------------------------------------------------------------
class CellTable:
    """Importance per (coarse cell, ln-energy node) from summed scores over
    summed weights, shrunk towards the overall ratio with `prior` records'
    worth of weight.  Cells are blocks of (c1, c2, c3) zones."""

    def __init__(self, wl, blocks=(8, 8, 8), n_nodes=16, lo=LN_EPS[0], hi=LN_EPS[1], prior=20.0):
        g = wl.grid
        self.n = g["n"]
        self.blocks = blocks
        self.nc = [max(1, -(-self.n[j] // blocks[j])) for j in range(3)]
        (i1, i2, i3), _, _ = zone_geometry(wl)
        self.cell_of_zone = ((i1 // blocks[0]) * self.nc[1] + (i2 // blocks[1])) * self.nc[2] + (i3 // blocks[2])
        self.n_cells = self.nc[0] * self.nc[1] * self.nc[2]
        self.n_nodes, self.lo, self.hi, self.prior = n_nodes, lo, hi, prior

    def node(self, ln_e):
        p = (ln_e - self.lo) / (self.hi - self.lo) * (self.n_nodes - 1)
        return np.clip(np.rint(p), 0, self.n_nodes - 1).astype(np.int64)

    def fit(self, zone, ln_e, w, score):
        """ln importance [n_cells][n_nodes] (NaN where no record)."""
        idx = self.cell_of_zone[zone] * self.n_nodes + self.node(ln_e)
        m = self.n_cells * self.n_nodes
        sw = np.bincount(idx, weights=w, minlength=m)
        ss = np.bincount(idx, weights=score, minlength=m)
        cnt = np.bincount(idx, minlength=m)
        tot = ss.sum() / max(w.sum(), 1e-300)
        wbar = w.sum() / max(len(w), 1)
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = (ss + self.prior * wbar * tot) / (sw + self.prior * wbar)
        ratio = np.where(cnt > 0, ratio, np.nan)
        self.ln_I = np.log(np.maximum(ratio, 1e-300)).reshape(self.n_cells, self.n_nodes)
        self.ln_tot = math.log(max(tot, 1e-300))
        return self.ln_I

    def zone_table(self, n_zone_nodes, lo, hi):
        """Per zone [nz][n_zone_nodes] ln importance on nodes over [lo, hi]
        (cells without records take the overall value)."""
        x = np.linspace(lo, hi, n_zone_nodes)
        k = self.node(x)
        t = self.ln_I[:, k]
        t = np.where(np.isfinite(t), t, self.ln_tot)
        return t[self.cell_of_zone]


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
        Z = np.zeros_like(X, dtype=np.float32)
        Z[:, :6] = (X[:, :6] - self.mu) / self.sd
        return Z

    def fit(self, ctx, X, T, C, steps=800, batch=16384, lr=2e-3):
        """X rows, T [n][2] targets (>= 0, normalised to mean 1 per output),
        C [n][2] weights (0 where a row does not train an output)."""
        import torch
        self.mu = X[:, :6].mean(0)
        self.sd = X[:, :6].std(0) + 1e-6
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
        for s in range(steps):
            if n > batch:
                idx = torch.randint(0, n, (batch,), device="cuda", generator=gen)
                xb, tb, cb = Xd[idx].contiguous(), Td[idx].contiguous(), Cd[idx].contiguous()
            else:
                xb, tb, cb = Xd, Td, Cd
            want = (s % 100 == 0) or s == steps - 1
            lr_s = lr * (0.1 ** (s / steps))
            L = ctx.mlp_train_step(xb, tb, cb, lr_s, want_loss=want)
            if want:
                hist.append((s, L))
        ctx.mlp_set_loss(GM.MLP_SQUARED)
        return hist

    def predict(self, ctx, X, chunk=1 << 22):
        out = []
        for a in range(0, len(X), chunk):
            out.append(ctx.mlp_forward(self.standardise(X[a:a + chunk])).cpu().numpy().astype(np.float64))
        return np.concatenate(out) if out else np.zeros((0, 2))


# ---------------------------------------------------------------------------
# tables from importances
# ---------------------------------------------------------------------------
def window_table(ln_I_sc_zone, sc, sc_lnI, b_plain, b_max):
    """ln(c_b I) per zone and node, c_b chosen so that the mean bias over the
    pilot's scattering opportunities equals b_plain (the parent's weight at
    a pilot scattering is b_plain times its child's)."""
    w_par = sc["w"] * b_plain
    lo, hi = -60.0, 60.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        b = np.clip(w_par * np.exp(mid + sc_lnI), 1.0, b_max)
        if b.mean() > b_plain:
            hi = mid
        else:
            lo = mid
    return ln_I_sc_zone + 0.5 * (lo + hi)


def emission_modulation(ctx, wl, inst, ln_I_em_zone, ln_I_mean, n_nodes, n_s, alpha=0.5):
    """Defensive emission proposal: zone i's superphotons at nu get the
    weight w(nu) / [(1 - alpha) + alpha I_em(zone, nu) / I_mean] (times the
    constant that keeps the expected roots at the plain run's), I_mean the
    plain run's mean importance per unit weight.  Where the importance is
    high the proposal emits up to alpha I/I_mean times more roots; nowhere
    does it emit fewer than 1 - alpha of the plain number, which bounds the
    weights by w / (1 - alpha) however wrong the estimate.  The expected
    count scales exactly with the constant, so it is found from one make at
    a constant low enough that the make allocates almost nothing."""
    e = wl.emit
    lo, hi = math.log(e["nu_min"]), math.log(e["nu_max"])
    nb0 = float(ctx.read_emission(inst)["nbar"].sum())
    ratio = np.exp(np.clip(ln_I_em_zone - ln_I_mean, -50.0, 50.0))
    m = np.log((1.0 - alpha) + alpha * ratio)
    shift = m.max() + 20.0
    ctx.set_emission_table(inst, m - shift, lo, hi)
    ctx.make_superphotons(dict(e, n_target=float(n_s), seed=1), instance=inst)
    nb1 = float(ctx.read_emission(inst)["nbar"].sum())
    m = m - shift + math.log(nb0 / max(nb1, 1e-300))
    ctx.set_emission_table(inst, m, lo, hi)
    return m, lo, hi


def build_tables(ctx, wl, inst, ev, root_stride, b_plain, b_max, n_s, mode, net_seed=1, log=None,
                 use_bias=True, use_emission=True, alpha=0.5):
    """Tables of the adaptive ("cells") or learned ("network") form from the
    pilot records; sets the instance's bias (window) and emission tables."""
    sc, em = split_records(ev, root_stride)
    nodes = 16
    zf = zone_features(wl)
    nz = wl.n_zones
    ln_nodes_eps = np.linspace(LN_EPS[0], LN_EPS[1], nodes)
    e = wl.emit
    lo_nu, hi_nu = math.log(e["nu_min"]), math.log(e["nu_max"])
    ln_nodes_nu = np.linspace(lo_nu, hi_nu, nodes)
    # emission records carry the fluid-frame energy of the emitted photon;
    # the emission table is in ln nu of the fluid frame (the comoving emitter)
    em_lnnu = np.log(em["eps"] * MEC2_OVER_H)
    info = {"scatter_records": int(len(sc)), "emission_records": int(len(em))}
    t_sc = sc["score"] / sc["w"]
    t_em = em["score"] / em["w"]
    n_sc_mean, n_em_mean = max(t_sc.mean(), 1e-300), max(t_em.mean(), 1e-300)
    if mode == "cells":
        ct = CellTable(wl, n_nodes=nodes)
        ct.fit(sc["zone"], np.log(sc["eps"]), sc["w"], sc["score"])
        sc_lnI = ct.ln_I[ct.cell_of_zone[sc["zone"]], ct.node(np.log(sc["eps"]))]
        sc_lnI = np.where(np.isfinite(sc_lnI), sc_lnI, ct.ln_tot)
        lnI_sc = ct.zone_table(nodes, LN_EPS[0], LN_EPS[1])
        ce = CellTable(wl, n_nodes=nodes, lo=lo_nu, hi=hi_nu)
        ce.fit(em["zone"], em_lnnu, em["w"], em["score"])
        lnI_em = ce.zone_table(nodes, lo_nu, hi_nu)
    else:
        X = np.concatenate([rows(zf, sc["zone"], np.log(sc["eps"])), rows(zf, em["zone"], em_lnnu - math.log(MEC2_OVER_H))])
        T = np.zeros((len(X), 2))
        C = np.zeros((len(X), 2))
        T[:len(sc), 0] = t_sc / n_sc_mean
        C[:len(sc), 0] = 1.0
        T[len(sc):, 1] = t_em / n_em_mean
        C[len(sc):, 1] = 1.0
        net = Network(seed=net_seed)
        t0 = time.perf_counter()
        hist = net.fit(ctx, X, T, C)
        info["train_s"] = time.perf_counter() - t0
        info["loss_first_last"] = [hist[0][1], hist[-1][1]]
        y_sc = net.predict(ctx, rows(zf, sc["zone"], np.log(sc["eps"])))[:, 0]
        sc_lnI = y_sc + math.log(n_sc_mean)
        # tables on zones with plasma only (others never scatter or emit)
        on = np.flatnonzero(wl.n_e > 0)
        zon = np.repeat(on, nodes)
        Xs = rows(zf, zon, np.tile(ln_nodes_eps, len(on)))
        ys = net.predict(ctx, Xs)
        lnI_sc = np.full((nz, nodes), math.log(n_sc_mean))
        lnI_sc[on] = ys[:, 0].reshape(len(on), nodes) + math.log(n_sc_mean)
        emits = np.flatnonzero(wl.B > 0)
        zem = np.repeat(emits, nodes)
        Xe = rows(zf, zem, np.tile(ln_nodes_nu - math.log(MEC2_OVER_H), len(emits)))
        ye = net.predict(ctx, Xe)
        lnI_em = np.full((nz, nodes), math.log(n_em_mean))
        lnI_em[emits] = ye[:, 1].reshape(len(emits), nodes) + math.log(n_em_mean)
    if use_bias:
        wt = window_table(lnI_sc, sc, sc_lnI, b_plain, b_max)
        ctx.set_bias_table(inst, wt, LN_EPS[0], LN_EPS[1])
        info["bias_table_range"] = [float(np.min(wt)), float(np.max(wt))]
    if use_emission:
        m, _, _ = emission_modulation(ctx, wl, inst, lnI_em, math.log(n_em_mean), nodes, n_s, alpha)
        info["emission_table_range"] = [float(np.min(m)), float(np.max(m))]
    return info


# ---------------------------------------------------------------------------
# the comparison
# ---------------------------------------------------------------------------
FORMS = {
    # name: (table source, weight-window bias, emission proposal)
    "adaptive": ("cells", True, True),
    "learned": ("network", True, True),
}


def compare_forms(ctx, wl, inst, seeds=3, ref_rounds=24, round_div=32, pilot_rounds=4, b_max=100.0,
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
                ev, sw, _ = pilot(ctx, wl, inst, pilot_rounds, 300000 + 1000 * k, n_round, root_stride)
                info = build_tables(ctx, wl, inst, ev, root_stride, b_plain, b_max, n_round, form,
                                    net_seed=1 + k, log=log, use_bias=use_bias, use_emission=use_em,
                                    alpha=alpha)
                del ev
                torch.cuda.synchronize()
                t_prep = time.perf_counter() - ta
                over = dict(bias_mode=GM.BIAS_WINDOW, bias_max=b_max) if use_bias else None
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
            parts.append("defensive emission proposal w / [(1 - %g) + %g I_em / I_mean]" % (alpha, alpha))
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
