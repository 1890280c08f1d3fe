"""Spectral error and time-to-error measurement (Tests section,
eq:conv_parameter), host side.

eps_err(L, L_ref, mask) is the paper's convergence parameter: the relative
error |L_ref - L| / L_ref integrated over log10(nu) and divided by the
log10(nu) span, here per inclination bin over the masked frequency bins
(rectangle rule on the uniform log-nu bins) and averaged over inclination
bins that hold any masked bin.

time_to_error runs the transport in rounds on one instance, reads the
accumulating tally after every round (no reset), and returns the wall time
at which eps_err first falls to the target, interpolated log-log between
rounds."""
from __future__ import annotations

import math
import time

import numpy as np


def eps_err(L: np.ndarray, L_ref: np.ndarray, mask: np.ndarray) -> float:
    """L, L_ref: [n_theta, n_nu] luminosity estimates; mask: bool, same shape."""
    vals = []
    for it in range(L.shape[0]):
        m = mask[it]
        if not m.any():
            continue
        vals.append(float(np.mean(np.abs(L_ref[it, m] - L[it, m]) / L_ref[it, m])))
    return float(np.mean(vals)) if vals else float("nan")


def reference(ctx, wl, instance: int, rounds: int, seed0: int, precision: int = 0):
    """Plain high-statistics reference: `rounds` make+track rounds at the
    workload's N_s with seeds seed0, seed0+1, ...  Returns (L_ref per round
    [n_theta, n_nu], superphoton counts per round, relative standard error
    of one round's bin estimate, total superphotons).  The bin estimate of a
    round is a sum over photons, so its variance is estimated by the summed
    (wE)^2 of the round."""
    if getattr(ctx, "n_theta", None):              # clear what earlier calls left
        ctx.read_spectrum(instance, reset=True)
    n = 0
    for r in range(rounds):
        ctx.make_superphotons(dict(wl.emit, seed=seed0 + r), instance=instance)
        st = ctx.track_scatter(dict(wl.track, precision=precision))
        n += int(st[0] + st[1])
    spec, _ = ctx.read_spectrum(instance, reset=True)
    S1, S2 = spec[..., 0], spec[..., 1]
    with np.errstate(divide="ignore", invalid="ignore"):
        rse = np.where(S1 > 0, np.sqrt(S2 * rounds) / S1, np.inf)
    return S1 / rounds, spec[..., 2] / rounds, rse, n


def error_mask(counts_per_round, rse_per_round, min_count=1e3, max_rse=0.1):
    """Bins included in eps_err: at least min_count superphotons per round
    and a per-round relative standard error of at most max_rse (bins whose
    estimate is dominated by a few heavy photons would otherwise set the
    error for the whole spectrum)."""
    return (counts_per_round >= min_count) & (rse_per_round <= max_rse)


def time_to_error(ctx, wl, instance: int, L_ref, mask, seed0: int, n_s_round: float,
                  target: float = 0.01, max_rounds: int = 256, track_overrides=None):
    """Accumulate rounds of N_s = n_s_round until eps_err <= target.  Returns
    dict(seconds, superphotons, rounds, history=[(t, n, eps)])."""
    import torch
    track = dict(wl.track, **(track_overrides or {}))
    emit = dict(wl.emit, n_target=float(n_s_round))
    ctx.read_spectrum(instance, reset=True)
    torch.cuda.synchronize()
    hist = []
    t0 = time.perf_counter()
    n = 0
    for r in range(1, max_rounds + 1):
        ctx.make_superphotons(dict(emit, seed=seed0 + r), instance=instance)
        st = ctx.track_scatter(track)
        n += int(st[0] + st[1])
        spec, _ = ctx.read_spectrum(instance)
        t = time.perf_counter() - t0
        L = spec[..., 0] / r          # every round estimates L whatever its N_s (w ~ 1/N_s)
        e = eps_err(L, L_ref, mask)
        hist.append((t, n, e))
        if e <= target:
            break
    ctx.read_spectrum(instance, reset=True)
    # log-log interpolation of the first crossing
    sec, nsp = hist[-1][0], hist[-1][1]
    if hist[-1][2] <= target and len(hist) > 1:
        (t1, n1, e1), (t2, n2, e2) = hist[-2], hist[-1]
        if e1 > target and e2 > 0:
            f = (math.log(target) - math.log(e1)) / (math.log(e2) - math.log(e1))
            sec = math.exp(math.log(t1) + f * (math.log(t2) - math.log(t1)))
            nsp = math.exp(math.log(n1) + f * (math.log(n2) - math.log(n1)))
    return dict(seconds=sec if hist[-1][2] <= target else None, superphotons=nsp,
                rounds=len(hist), final_eps=hist[-1][2], history=hist)
