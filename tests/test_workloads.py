"""Checks of the synthetic 3-D inputs (the corona torus and the survey): the
structure each generator promises, measured with the oracle's metric where
geometry enters.  They pin inputs, not the method."""
import math

import numpy as np

from paper_2602_13198_amd import workloads as W


def _centres(g):
    n1, n2, n3 = g["n"]
    x1 = g["x_start"][0] + (np.arange(n1) + 0.5) * g["dx"][0]
    x2 = g["x_start"][1] + (np.arange(n2) + 0.5) * g["dx"][1]
    x3 = g["x_start"][2] + (np.arange(n3) + 0.5) * g["dx"][2]
    return x1, x2, x3


def test_corona_radial_thomson_depth():
    """n_0 sigma_T r_g ln(r_c / r_h) = 0.1: the radial Thomson depth of the
    corona along a polar column (no torus there) from the horizon to
    r_c = 40 r_g, by the zone sum, is 0.1 to the grid's resolution."""
    wl = W.corona_torus(n1=96, n2=48, n3=8, n_target=1e5)
    g = wl.grid
    n1, n2, n3 = g["n"]
    x1, _, _ = _centres(g)
    r = np.exp(x1)
    ne = wl.n_e.reshape(n1, n2, n3)
    for j in (1, n2 - 2):
        col = ne[:, j, 3]
        tau = np.sum(col * r * g["dx"][0]) * W.SIGMA_T * g["L_unit_cm"]
        # one zone width of ln r at either end of the column, relative to ln(r_c / r_h)
        assert abs(tau - 0.1) < 0.1 * 2 * g["dx"][0] / math.log(40.0 / wl.meta["r_h"]), tau
    cor = wl.meta["corona"]
    assert cor.sum() > 0.2 * wl.n_zones
    assert np.all(wl.B[cor] == 0.0) and np.all(wl.theta_e[cor] == 1.0)
    # the torus keeps its field and emission
    assert (wl.B > 0).sum() > 1000


def test_corona_velocity_is_timelike(oracle_lib):
    """The normal observer's velocity is timelike in every corona zone,
    inside the ergosphere too (checked with the oracle's Kerr-Schild metric
    at the zone centres)."""
    wl = W.corona_torus(n1=48, n2=24, n3=4, n_target=1e5)
    g = wl.grid
    n1, n2, n3 = g["n"]
    x1, x2, x3 = _centres(g)
    cor = wl.meta["corona"].reshape(n1, n2, n3)
    u = wl.ucon.reshape(4, n1, n2, n3)
    rng = np.random.default_rng(0)
    idx = np.argwhere(cor)
    inner = idx[np.exp(x1[idx[:, 0]]) < 2.0]          # ergosphere region near the equator
    assert len(inner) > 0
    pick = np.concatenate([inner[:40], idx[rng.choice(len(idx), 200, replace=False)]])
    for i1, i2, i3 in pick:
        x = np.array([0.0, x1[i1], x2[i2], x3[i3]])
        gm_ = oracle_lib.gcov(g, x)
        uu = u[:, i1, i2, i3]
        assert uu @ gm_ @ uu < 0.0, (i1, i2, i3)


def test_torus_3d_perturbations():
    """Seeded log-normal factors exp(0.05 Z - 0.05^2 / 2), iid per zone: in
    3-D the density of a zone varies around the axisymmetric torus with
    mean 1 and standard deviation ~0.05 over the azimuth."""
    wl = W.torus(n1=48, n2=24, n3=64, n_target=1e5)
    n1, n2, n3 = wl.grid["n"]
    ne = wl.n_e.reshape(n1, n2, n3)
    on = ne[:, :, 0] > 0
    ratio = ne[on] / ne[on].mean(axis=1, keepdims=True)
    assert abs(ratio.std() - 0.05) < 0.005
    assert np.allclose(ratio.mean(axis=1), 1.0)


def test_survey_instances():
    """64 instances: every spin x R_high pair with four density scales
    within [M_c / 10, 10 M_c], N_s within [1e5, 1e7], distinct instance ids;
    n_e scales with M_unit and B with its square root; the bias coefficient
    with M_unit and R_high as stated."""
    S = W.survey(n1=24, n2=12, n3=8)
    assert len(S) == 64
    assert [w.emit["instance"] for w in S] == list(range(64))
    pairs = {(w.meta["a"], w.meta["R_high"]) for w in S}
    assert len(pairs) == 16
    for w in S:
        assert 1e26 <= w.meta["M_unit"] <= 1e28
        assert 1e5 <= w.emit["n_target"] <= 1e7
    a, b = S[0], S[1]
    on = a.n_e > 0
    np.testing.assert_allclose(b.n_e[on] / a.n_e[on], b.meta["M_unit"] / a.meta["M_unit"], rtol=1e-12)
    onb = a.B > 0
    np.testing.assert_allclose(b.B[onb] / a.B[onb], math.sqrt(b.meta["M_unit"] / a.meta["M_unit"]), rtol=1e-12)
    # R_high only lowers the temperature (before the floor)
    hot = [w for w in S if w.meta["a"] == 0.9375]
    t1 = [w for w in hot if w.meta["R_high"] == 1.0][0].theta_e
    t160 = [w for w in hot if w.meta["R_high"] == 160.0][0].theta_e
    assert np.all(t160 <= t1 + 1e-15) and t160.max() < t1.max()
    # the bias coefficient keeps b tau_T of the hottest, densest zone: with
    # b = c Theta_e^2 and tau_T ~ n_e ~ M_unit, c M_unit Theta_max^2 is the
    # same for every instance of a spin
    for a_ in {w.meta["a"] for w in S}:
        v = [w.track["bias_value"] * w.meta["M_unit"] * w.theta_e.max() ** 2 for w in S if w.meta["a"] == a_]
        np.testing.assert_allclose(v, v[0], rtol=1e-9)


def test_outer_plasma_radius_bounds_the_plasma():
    """The far-field rule's least r_far: every zone with plasma lies inside
    it, and a zone of the next first-axis row outward would not."""
    wl = W.torus(n1=64, n2=32, step_h=0.125, n_target=1000)
    r_out = wl.outer_plasma_radius()
    n1 = wl.grid["n"][0]
    rows = np.flatnonzero(wl.n_e.reshape(n1, -1).max(axis=1) > 0.0)
    x0, dx = wl.grid["x_start"][0], wl.grid["dx"][0]
    assert np.exp(x0 + rows[-1] * dx) < r_out <= np.exp(x0 + (rows[-1] + 1) * dx) * (1 + 1e-12)
    far = wl.with_far_steps(4.0)
    assert far.track["step_far"] == 4.0 and far.track["r_far"] == max(r_out, 4.0)
    assert wl.track.get("step_far", 0.0) == 0.0
