"""Host logic of the importance forms (no GPU): the held-out deviance that
decides whether a trained network output builds a table, and the emission
band taken from the event records."""
import math

import numpy as np

from paper_2602_13198_amd import importance as IM


class _FakeNet:
    """Predicts fixed log-means, standing in for the network."""

    def __init__(self, y):
        self.y = y

    def predict(self, ctx, X):
        return self.y[X[:, 0].astype(int)]


def test_heldout_deviance_prefers_the_better_predictor():
    """A predictor of the true log-mean beats the constant mean on held-out
    Poisson counts; a wrong one loses to it (and then builds no table)."""
    rng = np.random.default_rng(0)
    n = 20000
    lam = np.exp(rng.normal(0.0, 1.0, n))                 # per-row mean
    T = np.stack([rng.poisson(lam), rng.poisson(lam)], axis=1).astype(float)
    T /= T.mean(axis=0)
    lam_n = lam / lam.mean()
    C = np.ones_like(T)
    X = np.zeros((n, 8))
    X[:, 0] = np.arange(n)
    hold = (np.arange(n) % 10) == 0
    good = _FakeNet(np.stack([np.log(lam_n), np.log(lam_n)], axis=1))
    (dn0, dc0), (dn1, dc1) = IM.heldout_deviance(good, None, X, T, C, hold)
    assert dn0 < dc0 and dn1 < dc1
    bad = _FakeNet(np.stack([-np.log(lam_n), np.full(n, 3.0)], axis=1))
    (bn0, bc0), (bn1, bc1) = IM.heldout_deviance(bad, None, X, T, C, hold)
    assert bn0 > bc0 and bn1 > bc1
    # rows that train no output are left out of that output's deviance
    C2 = C.copy()
    C2[:, 1] = 0.0
    assert IM.heldout_deviance(good, None, X, T, C2, hold)[1] == (math.inf, math.inf)


def test_emission_band_covers_the_records():
    """The band spans the emission records' ln nu, padded by half a node
    spacing on each side; scattering records and weightless ones are
    ignored."""
    dt = np.dtype([("gen", "<i4"), ("w", "<f8"), ("eps", "<f8")])
    ev = np.zeros(5, dt)
    nu = np.array([1e9, 3e9, 2e10, 5e12, 7e8])
    ev["eps"] = nu / IM.MEC2_OVER_H
    ev["w"] = [1.0, 1.0, 1.0, 1.0, 0.0]
    ev["gen"] = [0, 0, 0, 1, 0]
    lo, hi = IM.emission_band(ev, nodes=11)
    d = (math.log(2e10) - math.log(1e9)) / 10
    assert math.isclose(lo, math.log(1e9) - 0.5 * d, rel_tol=1e-12)
    assert math.isclose(hi, math.log(2e10) + 0.5 * d, rel_tol=1e-12)


def test_event_columns_do_not_depend_on_the_log_order():
    """The device writes the event log in scheduling order; the columns the
    network trains on come out the same for any order of the same records
    (sorted by the created photons' streams), and the split keeps every
    record with a positive finite weight and score, scatterings apart from
    emissions."""
    from paper_2602_13198_amd import gm as GM
    rng = np.random.default_rng(4)
    n = 5000
    ev = np.zeros(n, GM.EVENT_DTYPE)
    ev["s0"] = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    ev["s1"] = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    ev["zone"] = rng.integers(0, 1000, n)
    ev["gen"] = rng.integers(0, 3, n)
    ev["eps"] = rng.uniform(1e-9, 1e-3, n)
    ev["w"] = np.where(rng.random(n) < 0.05, 0.0, rng.random(n))
    ev["score"] = rng.random(n)
    a = IM.event_columns(ev)
    b = IM.event_columns(ev[rng.permutation(n)])
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    sc, em = IM.split_records(a)
    ok = ev["w"] > 0
    assert len(sc["zone"]) == (ok & (ev["gen"] > 0)).sum()
    assert len(em["zone"]) == (ok & (ev["gen"] == 0)).sum()
    assert np.all(sc["w"] > 0) and np.all(em["w"] > 0)
