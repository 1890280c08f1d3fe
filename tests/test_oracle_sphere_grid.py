"""Pins of the oracle on the flat spherical grid of the paper's sphere tests
(coordinates t, ln r, theta, phi; Tests section, optically thin sphere):
the metric is Minkowski carried through the coordinate map, null geodesics
are straight lines, the thin sphere's spectrum matches the angle-resolved
emissivity integrated over the grid's volume, the 2500-bin tally is the
fine split of the coarse one, and the scattering sphere's ledgers close."""
import math

import numpy as np
import pytest
import scipy.integrate as si

from paper_2602_13198_amd import workloads as W

from test_oracle_transport import jnu_paper, ledger_residuals


def cart_jacobian(x1, x2, x3, h):
    """d(X, Y, Z)/d(x1, x2, x3) for r = e^x1, theta = pi x2 + (1-h)/2 sin 2 pi x2, phi = x3."""
    r = math.exp(x1)
    th = math.pi * x2 + 0.5 * (1 - h) * math.sin(2 * math.pi * x2)
    dth = math.pi * (1 + (1 - h) * math.cos(2 * math.pi * x2))
    st, ct, sp_, cp = math.sin(th), math.cos(th), math.sin(x3), math.cos(x3)
    d_r = np.array([st * cp, st * sp_, ct]) * r                 # d/dx1 = r d/dr
    d_t = np.array([ct * cp, ct * sp_, -st]) * r * dth          # d/dx2
    d_p = np.array([-st * sp_, st * cp, 0.0]) * r               # d/dx3
    return np.stack([d_r, d_t, d_p], axis=1)                    # [cartesian][coordinate]


@pytest.mark.parametrize("h", [1.0, 0.3])
def test_flat_spherical_metric_is_minkowski(oracle_lib, h):
    """g_mn = J^T diag(-1, 1, 1, 1) J with the Jacobian of the coordinate
    map written out by hand; sqrt(-g) = r^3 sin(theta) dtheta/dx2."""
    grid = dict(metric=W.METRIC_FLAT_SPH, n=[8, 8, 1], x_start=[-2.0, 0.0, 0.0], dx=[0.5, 0.125, 2 * math.pi],
                a_spin=0.0, h_slope=h, L_unit_cm=1.0, r_record=100.0)
    rng = np.random.default_rng(3)
    for _ in range(20):
        x = np.array([0.0, rng.uniform(-3, 5), rng.uniform(0.02, 0.98), rng.uniform(0, 2 * math.pi)])
        J = np.zeros((4, 4))
        J[0, 0] = 1.0
        J[1:, 1:] = cart_jacobian(x[1], x[2], x[3], h)
        ref = J.T @ np.diag([-1.0, 1.0, 1.0, 1.0]) @ J
        g = oracle_lib.gcov(grid, x)
        np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        th = math.pi * x[2] + 0.5 * (1 - h) * math.sin(2 * math.pi * x[2])
        dth = math.pi * (1 + (1 - h) * math.cos(2 * math.pi * x[2]))
        assert oracle_lib.sqrt_neg_g(grid, x) == pytest.approx(math.exp(3 * x[1]) * math.sin(th) * dth, rel=1e-12)


@pytest.mark.parametrize("impact", [0.7, 0.05])
def test_geodesics_are_straight_lines(oracle_lib, impact):
    """A null geodesic integrated in (ln r, x2, phi) stays on the straight
    line through its start along its start direction, also when it passes
    close to the centre (impact parameter 0.05 of its start radius): its
    largest distance from the line falls as the square of the step (the
    integrator is second order; an error in the metric or its Christoffel
    symbols would leave a distance that does not vanish), and e = -k_t
    stays 1."""
    grid = dict(metric=W.METRIC_FLAT_SPH, n=[64, 32, 1], x_start=[math.log(1e-3), 0.0, 0.0],
                dx=[math.log(1e7) / 64, 1 / 32, 2 * math.pi], a_spin=0.0, h_slope=1.0, L_unit_cm=1.0,
                r_record=1e4)
    # start at r = 10 on the x axis, aimed back past the centre, tilted out of the z = 0 plane
    P0 = np.array([10.0, 0.0, 0.0])
    d = np.array([-1.0, impact / 10.0 * 0.6, impact / 10.0 * 0.8])
    d /= np.linalg.norm(d)
    r0 = np.linalg.norm(P0)
    x0 = np.array([0.0, math.log(r0), math.acos(P0[2] / r0) / math.pi, math.atan2(P0[1], P0[0])])
    J = cart_jacobian(x0[1], x0[2], x0[3], 1.0)
    kc = np.linalg.solve(J, d)                   # coordinate components of the unit direction
    k0 = np.array([1.0, *kc])
    worst = []
    for h in (0.1, 0.05):
        out = oracle_lib.integrate_geodesic(grid, x0, k0, h=h, tol=1e-13, max_it=30, n=200000, r_min=1e-4,
                                            r_max=1e3)
        r = np.exp(out[:, 1])
        th = math.pi * out[:, 2]
        X = np.stack([r * np.sin(th) * np.cos(out[:, 3]), r * np.sin(th) * np.sin(out[:, 3]), r * np.cos(th)], 1)
        rel = X - P0
        dist = np.linalg.norm(rel - (rel @ d)[:, None] * d[None, :], axis=1)
        worst.append(dist.max() / r[-1])
        # it went past the centre and out again
        assert r.min() < 1.5 * impact * r0 and r[-1] > 500.0
        # e = -k_t of the flat metric is k^t, constant
        np.testing.assert_allclose(out[:, 4], 1.0, rtol=1e-12)
    assert 3.6 < worst[0] / worst[1] < 4.4, worst
    assert worst[1] < 1e-3


def _voxel_volume(wl):
    """Emitting volume as the transport counts it: sum over zones of the
    fill fraction times sqrt(-g) at the centre times the coordinate cell."""
    g = wl.grid
    n1, n2, _ = g["n"]
    x1 = g["x_start"][0] + (np.arange(n1) + 0.5) * g["dx"][0]
    x2 = (np.arange(n2) + 0.5) * g["dx"][1]
    sg = np.exp(3 * x1)[:, None] * np.sin(math.pi * x2)[None, :] * math.pi
    return float((wl.meta["frac"][:, None] * sg).sum() * g["dx"][0] * g["dx"][1] * g["dx"][2])


def _expectation(wl, track, V):
    m = wl.meta
    nb, nt = track["n_nu"], track["n_theta"]
    edges = np.exp(np.linspace(math.log(track["nu_lo"]), math.log(track["nu_hi"]), nb + 1))
    th_edges = np.linspace(0, math.pi, nt + 1)
    E = np.zeros((nt, nb))
    for i in range(nb):
        lo, hi = max(edges[i], wl.emit["nu_min"]), min(edges[i + 1], wl.emit["nu_max"])
        if hi <= lo:
            continue
        for t in range(nt):
            c1, c0 = math.cos(th_edges[t]), math.cos(th_edges[t + 1])
            f = lambda c, lnnu: jnu_paper(m["n_e0"], m["theta_e"], m["B"], math.exp(lnnu), c) * math.exp(lnnu)
            E[t, i] = 2 * math.pi * V * si.dblquad(f, math.log(lo), math.log(hi), c0, c1, epsabs=0, epsrel=1e-8)[0]
    return E


def test_log_r_thin_sphere_matches_analytic(oracle_lib):
    """eq:Lnu_analytic_thin_test on the log-r grid (the paper's sphere at
    n_e = 1e13: tau ~ 1e-4, absorption below the noise): every (theta, nu)
    bin with 30 or more superphotons agrees with the angle-resolved
    emissivity times the grid's emitting volume, chi^2/dof <= 1.2, and the
    grid's volume is the sphere's to its radial resolution."""
    wl = W.paper_thin_sphere(n1=512, n2=32, n_target=40000, seed=11, n_nu=80, dln_nu=0.3)
    res, _ = oracle_lib.run(wl)
    V = _voxel_volume(wl)
    assert V == pytest.approx(4 * math.pi / 3, rel=0.02)
    E = _expectation(wl, wl.track, V)
    S1, S2, N = res.spectrum[..., 0], res.spectrum[..., 1], res.spectrum[..., 2]
    use = N >= 30
    chi2 = ((S1[use] - E[use]) ** 2 / S2[use]).sum()
    dof = use.sum()
    assert dof >= 120
    assert chi2 / dof < 1.2, chi2 / dof
    assert S1.sum() == pytest.approx(E.sum(), rel=5 * math.sqrt(S2.sum()) / S1.sum())
    st = res.stats_dict()
    assert st["ESCAPED"] == st["ROOTS"] and st["STUCK"] == 0


def test_fine_tally_splits_the_coarse_one(oracle_lib):
    """The same photons tallied in 2500 bins of 0.01 in ln nu and in 250 of
    0.1: every coarse bin is the sum of its ten fine bins (photons whose
    ln nu falls within rounding of a shared edge may move by one bin)."""
    kw = dict(n1=256, n2=16, n_target=6000, seed=12)
    fine, _ = oracle_lib.run(W.paper_thin_sphere(**kw))
    coarse, _ = oracle_lib.run(W.paper_thin_sphere(n_nu=250, dln_nu=0.1, **kw))
    F, C = fine.spectrum, coarse.spectrum
    assert F.shape[1] == 2500 and C.shape[1] == 250
    Fs = F.reshape(F.shape[0], 250, 10, 3).sum(axis=2)
    moved = np.abs(Fs[..., 2] - C[..., 2]).sum()
    assert moved <= 2
    if moved == 0:
        np.testing.assert_allclose(Fs[..., 0], C[..., 0], rtol=1e-12, atol=0)
    assert F[..., 2].sum() == C[..., 2].sum() > 3000


def test_paper_scattering_sphere_ledgers(oracle_lib):
    """The scattering sphere (n_e = 1e18, Theta_e = 3, generation bias
    (n_sc + 1)^2 / tau_T): photon number and energy ledgers close to 1e-12,
    every generation up to the cap is populated, and the inverse-Compton
    photons reach above the synchrotron band."""
    wl = W.paper_scattering_sphere(n1=256, n2=16, n_target=3000, seed=13, n_nu=250, dln_nu=0.1)
    res, _ = oracle_lib.run(wl)
    wr, er = ledger_residuals(res)
    assert abs(wr) < 1e-12 and abs(er) < 1e-12
    st = res.stats_dict()
    assert all(st["GEN"][g] > 0 for g in range(5)), st["GEN"][:6]
    assert st["STUCK"] == 0
