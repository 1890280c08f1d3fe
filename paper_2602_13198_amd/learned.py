"""The learned form: a per-(zone, photon energy) scattering bias from a small
network trained on records the method itself generates.

Any bias b >= 1 leaves the estimator unbiased (the child carries w/b, the
parent w(1 - 1/b), Scattering section), so the network only moves sampling
effort: more scattering where scattered photons are worth more to the
recorded spectrum, less where they are not.  The paper names such bias
tuning as future work (Conclusions).

Records: a plain run with the scattering-event log and the photon trace
enabled.  For every scattering event at zone z with incoming fluid-frame
energy eps, the child's own trace record says whether it escaped, with what
weight and in which frequency bin.  Features (6): ln Theta_e, ln n_e, ln B
of the zone, ln eps, the zone's radius (flat: |x| over the grid half-size;
Kerr: ln r) and cos theta of its centre.  Targets (2): ln of the child's
escaping energy per unit scattered energy, w_end e_esc / (w_child eps), with
a floor of 1e-3 for photons that did not escape; and the escape indicator.

With a bin weight (the mask of an error measure over the reference
luminosity of each bin), the first target becomes the child's importance
for that measure: its escaping energy per unit child weight times the
weight of the bin it lands in (weight-window splitting: b proportional to
the importance).

Table: the network's first output on every zone x 32 ln-eps nodes, through
the MFMA inference kernel; ln b = ln b_plain + (y - mean over the training
events), clamped to [0, ln b_max].  The host part here only prepares
arrays and drives the ABI; every network evaluation and training step runs
in the library's kernels."""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gm as GM

M_E_C2_OVER_H = 8.187105776823886e-07 / 6.62607015e-27     # m_e c^2 / h in Hz
LN_FLOOR = math.log(1e-3)


def zone_features(wl, eps):
    """Feature rows [nz * len(eps)][8] (zone-major) for all zones of a workload."""
    g = wl.grid
    n1, n2, n3 = g["n"]
    i1, i2, i3 = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    xc = [g["x_start"][j] + (idx.reshape(-1) + 0.5) * g["dx"][j] for j, idx in enumerate((i1, i2, i3))]
    if g["metric"] == 0:
        half = 0.5 * max(n * d for n, d in zip(g["n"], g["dx"]))
        rr = np.sqrt(xc[0] ** 2 + xc[1] ** 2 + xc[2] ** 2)
        rad = rr / half
        cth = np.where(rr > 0, xc[2] / np.maximum(rr, 1e-300), 0.0)
    else:
        hs = g["h_slope"]
        th = np.pi * xc[1] + 0.5 * (1 - hs) * np.sin(2 * np.pi * xc[1])
        rad = xc[0]                       # ln r
        cth = np.cos(th)
    tiny = 1e-300
    zf = np.stack([np.log(np.maximum(wl.theta_e, tiny)), np.log(np.maximum(wl.n_e, tiny)),
                   np.log(np.maximum(wl.B, tiny)), rad, cth], axis=1)
    nz, ne = zf.shape[0], len(eps)
    X = np.zeros((nz * ne, 8))
    X[:, 0] = np.repeat(zf[:, 0], ne)
    X[:, 1] = np.repeat(zf[:, 1], ne)
    X[:, 2] = np.repeat(zf[:, 2], ne)
    X[:, 3] = np.tile(np.log(eps), nz)
    X[:, 4] = np.repeat(zf[:, 3], ne)
    X[:, 5] = np.repeat(zf[:, 4], ne)
    return X


def event_features(wl, zone, eps):
    """Feature rows for individual events (zone index, eps)."""
    base = zone_features(wl, np.array([1.0]))          # one row per zone, ln eps = 0
    X = base[zone].copy()
    X[:, 3] = np.log(eps)
    return X


def collect_records(ctx, wl, instance, rounds, seed0, track=None, bin_weight=None):
    """Plain rounds with the event log and trace on; returns (X, T).

    Without bin_weight the first target is ln of the child's escaping energy
    per unit scattered energy.  With bin_weight [n_theta][n_nu] (e.g. the
    mask of an error measure divided by the reference luminosity of each
    bin) it is ln of the child's importance for that measure: its escaping
    energy w_end e_esc, per unit child weight, times the weight of the bin
    it lands in; floored at 1e-3 of the median non-zero value."""
    track = dict(track or wl.track)
    xs, ts = [], []
    for r in range(rounds):
        ctx.set_trace(4 * int(wl.emit["n_target"]) + 1000)
        ctx.set_event_log(2 * int(wl.emit["n_target"]) + 1000)
        ctx.make_superphotons(dict(wl.emit, seed=seed0 + r), instance=instance)
        ctx.track_scatter(track)
        ev = ctx.read_event_log()
        tr = ctx.read_trace()
        ctx.read_spectrum(instance, reset=True)
        ctx.set_trace(0)
        ctx.set_event_log(0)
        # children of fully absorbed parents carry weight 0: no information
        ev = ev[ev["w"] > 0.0]
        if len(ev) == 0:
            continue
        key_t = (tr["s0"].astype(np.uint64) << np.uint64(32)) | tr["s1"].astype(np.uint64)
        key_e = (ev["s0"].astype(np.uint64) << np.uint64(32)) | ev["s1"].astype(np.uint64)
        order = np.argsort(key_t)
        pos = np.searchsorted(key_t[order], key_e)
        pos = np.minimum(pos, len(order) - 1)
        idx = order[pos]
        ok = (key_t[idx] == key_e) & (tr["s2"][idx] == ev["s2"])
        ev, rec = ev[ok], tr[idx[ok]]
        n_nu, lo, hi = track["n_nu"], track["nu_lo"], track["nu_hi"]
        dln = math.log(hi / lo) / n_nu
        esc = rec["kind"] == 1
        nu_esc = np.exp(math.log(lo) + (rec["i_nu"] + 0.5) * dln)
        e_esc = nu_esc / M_E_C2_OVER_H
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            if bin_weight is None:
                val = np.where(esc, rec["w_end"] * e_esc / (ev["w"] * ev["eps"]), 0.0)
                floor = 1e-3
            else:
                bw = np.where(esc, bin_weight[np.clip(rec["i_theta"], 0, None), np.clip(rec["i_nu"], 0, None)], 0.0)
                val = np.where(esc, rec["w_end"] / ev["w"] * e_esc * bw, 0.0)
                nzv = val[(val > 0) & np.isfinite(val)]
                floor = 1e-3 * (np.median(nzv) if len(nzv) else 1.0)
            T = np.stack([np.log(val + floor), esc.astype(float)], axis=1)
        Xe = event_features(wl, ev["zone"], ev["eps"])
        good = np.all(np.isfinite(Xe), axis=1) & np.all(np.isfinite(T), axis=1)
        collect_records.dropped = getattr(collect_records, "dropped", 0) + int((~good).sum())
        xs.append(Xe[good])
        ts.append(T[good])
    return np.concatenate(xs), np.concatenate(ts)


class LearnedBias:
    """Standardisation of the features, the network's parameters (held by the
    library context) and the bias table built from it."""

    def __init__(self, n_eps=32, ln_eps_lo=math.log(1e-12), ln_eps_hi=math.log(1e6), seed=0):
        self.n_eps, self.lo, self.hi = n_eps, ln_eps_lo, ln_eps_hi
        self.seed = seed
        self.mu = self.sd = None
        self.t_mu, self.t_sd = np.zeros(2), np.ones(2)
        self.y_ref = 0.0

    def standardise(self, X):
        Z = np.zeros_like(X, dtype=np.float32)
        Z[:, :6] = (X[:, :6] - self.mu) / self.sd
        return Z

    @staticmethod
    def initial_params(seed):
        rng = np.random.default_rng(seed)
        parts = []
        for fan_in, fan_out in ((6, 64), (64, 64), (64, 2)):
            lim = math.sqrt(6.0 / (fan_in + fan_out))
            parts.append(rng.uniform(-lim, lim, fan_in * fan_out))
            parts.append(np.zeros(fan_out))
        return np.concatenate(parts).astype(np.float32)

    def fit(self, ctx, X, T, steps=600, batch=8192, lr=3e-3, log=None, anchor_quantile=None):
        """Adam on the library's kernels; returns the loss history (sampled)."""
        self.mu = X[:, :6].mean(0)
        self.sd = X[:, :6].std(0) + 1e-6
        self.t_mu = T.mean(0)
        self.t_sd = T.std(0) + 1e-6
        Z = self.standardise(X)
        n = len(Z)
        Cw = np.full((n, 2), 1.0 / min(batch, n), np.float32)
        ctx.mlp_set_params(self.initial_params(self.seed))
        Xd = torch.as_tensor(Z, device="cuda")
        Td = torch.as_tensor(((T - self.t_mu) / self.t_sd).astype(np.float32), device="cuda")
        Cd = torch.as_tensor(Cw, device="cuda")
        gen = torch.Generator(device="cuda")
        gen.manual_seed(self.seed)
        hist = []
        for s in range(steps):
            if n > batch:
                idx = torch.randint(0, n, (batch,), device="cuda", generator=gen)
                xb, tb, cb = Xd[idx].contiguous(), Td[idx].contiguous(), Cd[:batch]
            else:
                xb, tb, cb = Xd, Td, Cd
            want = (s % 50 == 0) or s == steps - 1
            L = ctx.mlp_train_step(xb, tb, cb, lr, want_loss=want)
            if want:
                hist.append((s, L))
                if log:
                    log("step %d loss %.4f" % (s, L))
        y = self.predict(ctx, X)
        # b = b_plain where the predicted importance equals its mean over the
        # training events, or the given quantile of it
        self.y_ref = float(np.mean(y[:, 0]) if anchor_quantile is None
                           else np.quantile(y[:, 0], anchor_quantile))
        return hist

    def predict(self, ctx, X):
        """Network outputs in the targets' units for raw feature rows."""
        y = ctx.mlp_forward(self.standardise(X)).cpu().numpy().astype(np.float64)
        return y * self.t_sd + self.t_mu

    def table(self, ctx, wl, b_plain, b_max, gain=1.0):
        """ln b [nz][n_eps] for a workload from the trained network:
        b proportional to the predicted importance (splitting where children
        are worth more), scaled so that the mean over the training events is
        b_plain."""
        eps = np.exp(np.linspace(self.lo, self.hi, self.n_eps))
        X = zone_features(wl, eps)
        y = self.predict(ctx, X)[:, 0]
        lnb = math.log(b_plain) + gain * (y - self.y_ref)
        lnb = np.clip(lnb, 0.0, math.log(b_max))
        return lnb.reshape(-1, self.n_eps)

    def apply(self, ctx, wl, instance, b_plain, b_max):
        t = self.table(ctx, wl, b_plain, b_max)
        ctx.set_bias_table(instance, t, self.lo, self.hi)
        return t
