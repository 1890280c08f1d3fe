"""Helpers shared by the GPU parity tests: matching per-photon trace records
of the HIP path and the oracle by random-stream id."""
import numpy as np

KEY = ["s2", "s1", "s0"]


def index(tr):
    """dict: (s0, s1, s2) -> record."""
    return {(int(r["s0"]), int(r["s1"]), int(r["s2"])): r for r in tr}


def compare_traces(gpu, ora, rtol=1e-10, atol_x=1e-10, subset=False):
    """Compare records photon by photon.

    Exact: termination kind, generation, tally bin, step count.  Within
    rtol: birth and final weight, final wavevector; positions within atol_x
    (code units, O(1)).  Returns (n_compared, list of mismatching keys).  With
    subset=True only the oracle's photons are required on the GPU side."""
    G, O = index(gpu), index(ora)
    if not subset:
        missing = set(G) ^ set(O)
    else:
        missing = set(O) - set(G)
    bad = list(missing)
    n = 0
    for key, o in O.items():
        g = G.get(key)
        if g is None:
            continue
        n += 1
        ok = (g["kind"] == o["kind"] and g["n_sc"] == o["n_sc"] and g["i_nu"] == o["i_nu"]
              and g["i_theta"] == o["i_theta"] and g["n_steps"] == o["n_steps"])
        for f in ("w_birth", "w_end"):
            ok &= abs(g[f] - o[f]) <= rtol * max(abs(o[f]), 1e-300)
        kscale = np.max(np.abs(o["k"]))
        ok &= bool(np.all(np.abs(g["k"] - o["k"]) <= rtol * kscale))
        ok &= bool(np.all(np.abs(g["x"][1:] - o["x"][1:]) <= atol_x * max(1.0, np.max(np.abs(o["x"][1:])))))
        if not ok:
            bad.append(key)
    return n, bad


def describe(gpu, ora, keys, limit=5):
    G, O = index(gpu), index(ora)
    out = []
    for k in keys[:limit]:
        out.append("%s\n  gpu %s\n  ora %s" % (k, G.get(k), O.get(k)))
    return "\n".join(out)


def ledger_residuals(L):
    """Photon-number and energy identities of the ledger (numpy array)."""
    (w_emit, e_emit, w_esc, e_esc, w_oob, e_oob, w_abs, e_abs, w_capt, e_capt, w_cap, e_cap,
     w_roul, e_roul, w_stuck, e_stuck, e_compton, e_drift) = L
    wr = (w_emit + w_roul) / (w_esc + w_oob + w_abs + w_capt + w_cap + w_stuck) - 1
    er = (e_emit + e_roul + e_compton + e_drift) / (e_esc + e_oob + e_abs + e_capt + e_cap + e_stuck) - 1
    return wr, er
