"""Pins for the oracle's special functions and physics coefficients.

Each check compares against something other than the oracle's own formula:
scipy/mpmath special functions, closed-form limits, inequalities proven from
the fit, or values the paper prints."""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ME, CL, HPL, KB, EE = 9.1093837015e-28, 2.99792458e10, 6.62607015e-27, 1.380649e-16, 4.80320471e-10


def test_k2_against_scipy(oracle_lib):
    for x in np.logspace(-2, 2, 60):
        assert oracle_lib.k2(x) == pytest.approx(sp.kv(2, x), rel=2e-14)


def test_k2_large_theta_limit(oracle_lib):
    # Emissivity section: K2(1/Theta) ~ 2 Theta^2 at large Theta; the switch at 100
    assert oracle_lib.k2_of_theta(150.0) == 2 * 150.0**2
    assert oracle_lib.k2_of_theta(100.0) == pytest.approx(2 * 100.0**2, rel=3e-5)
    assert oracle_lib.k2_of_theta(4.0) == pytest.approx(sp.kv(2, 0.25), rel=2e-14)


def test_emissivity_matches_paper_form(oracle_lib):
    """j written with nu_s = nu_c sin(theta) as in eq:emissivity (mpmath, 30 digits)."""
    mp.mp.dps = 30
    rng = np.random.default_rng(3)
    for _ in range(50):
        th = 10 ** rng.uniform(-0.3, 2)
        B = 10 ** rng.uniform(-2, 2)
        ne = 10 ** rng.uniform(0, 10)
        nu = 10 ** rng.uniform(7, 13)
        c = rng.uniform(-0.99, 0.99)
        s = mp.sqrt(1 - mp.mpf(c) ** 2)
        nus = mp.mpf(2) / 9 * (EE * B / (2 * mp.pi * ME * CL)) * th**2 * s
        X = nu / nus
        K2 = 2 * th**2 if th > 100 else mp.besselk(2, 1 / mp.mpf(th))
        j = mp.sqrt(2) * mp.pi * EE**2 * ne * nus / (3 * CL * K2) * \
            (mp.sqrt(X) + mp.mpf(2) ** (mp.mpf(11) / 12) * X ** (mp.mpf(1) / 6)) ** 2 * mp.exp(-mp.cbrt(X))
        assert oracle_lib.jnu(ne, th, B, nu, c) == pytest.approx(float(j), rel=1e-12)


def test_direction_ratio_bounded(oracle_lib):
    """j(theta) <= j(pi/2): d ln g / d ln X <= 1 for the fit, so the
    direction rejection test of the Sampling procedure section is a valid
    probability."""
    for nu in np.logspace(7, 14, 30):
        jmax = oracle_lib.jnu(1e6, 4.0, 1.0, nu, 0.0)
        for c in np.linspace(-0.999, 0.999, 41):
            assert oracle_lib.jnu(1e6, 4.0, 1.0, nu, c) <= jmax * (1 + 1e-15)


def test_angle_integral_small_X_closed_form(oracle_lib):
    """G(Xc) -> 2^(11/6) Xc^(1/3) int_0^1 (1-mu^2)^(1/3) dmu as Xc -> 0, with
    int_0^1 (1-mu^2)^(1/3) dmu = (sqrt(pi)/2) Gamma(4/3)/Gamma(11/6)."""
    C0 = 2 ** (11 / 6) * math.sqrt(math.pi) / 2 * math.gamma(4 / 3) / math.gamma(11 / 6)
    for X in (1e-36, 1e-30):
        assert oracle_lib.G_of_Xc(X) == pytest.approx(C0 * X ** (1 / 3), rel=2e-10)


def test_angle_integral_large_X_laplace(oracle_lib):
    """Laplace's method about mu = 0: G ~ g(X) sqrt(pi / (2 |D|)),
    D = d ln g / d ln X; relative error O(1/|D|)."""
    a = 2 ** (11 / 12)
    for X in (1e6, 1e7):
        D = 2 * (0.5 * X**0.5 + a * X ** (1 / 6) / 6) / (X**0.5 + a * X ** (1 / 6)) - X ** (1 / 3) / 3
        lap = oracle_lib.g_of_X(X) * math.sqrt(math.pi / (2 * abs(D)))
        assert oracle_lib.G_of_Xc(X) == pytest.approx(lap, rel=6.0 / abs(D))


def test_angle_integral_against_mu_quadrature(oracle_lib):
    """The oracle integrates in phi (mu = sin phi); here in mu directly."""
    for X in (1e-6, 1e-2, 1.0, 30.0, 1e3, 1e5):
        f = lambda mu: math.sqrt(1 - mu * mu) * oracle_lib.g_of_X(X / math.sqrt(1 - mu * mu))
        ref = si.quad(f, 0, 1, epsabs=0, epsrel=1e-13, limit=500, points=[1 - 1e-6, 1 - 1e-3])[0]
        assert oracle_lib.G_of_Xc(X) == pytest.approx(ref, rel=1e-12)


def test_planck_limits(oracle_lib):
    th = 3.0
    T = th * ME * CL**2 / KB
    nu = 1e6
    assert oracle_lib.planck(nu, th) == pytest.approx(2 * nu**2 * KB * T / CL**2, rel=1e-9)
    nu = 50 * KB * T / HPL
    wien = 2 * HPL * nu**3 / CL**2 * math.exp(-HPL * nu / (KB * T))
    assert oracle_lib.planck(nu, th) == pytest.approx(wien, rel=1e-20 + 2 * math.exp(-50))


def test_paper_worked_optical_depth(oracle_lib):
    """Thin-sphere section: tau = alpha L ~ 1e-4 (order of magnitude)."""
    g = json.load(open(os.path.join(GOLD, "thin_sphere_worked_example.json")))
    j = oracle_lib.jnu(g["n_e"], g["theta_e"], g["B"], g["nu"], g["cos_theta"])
    alpha = j / oracle_lib.planck(g["nu"], g["theta_e"])
    tau = alpha * g["L_cm"]
    f = g["tolerance_factor"]
    assert g["tau_printed"] / f < tau < g["tau_printed"] * f


def _kn_textbook(e):
    """Rybicki & Lightman (7.5): sigma/sigma_T = 3/4 [ (1+x)/x^3 (2x(1+x)/(1+2x) - ln(1+2x))
    + ln(1+2x)/(2x) - (1+3x)/(1+2x)^2 ], 50 digits."""
    x = mp.mpf(e)
    L = mp.log(1 + 2 * x)
    return mp.mpf(3) / 4 * ((1 + x) / x**3 * (2 * x * (1 + x) / (1 + 2 * x) - L)
                            + L / (2 * x) - (1 + 3 * x) / (1 + 2 * x) ** 2)


def test_klein_nishina_against_textbook_form(oracle_lib):
    mp.mp.dps = 50
    for e in np.logspace(-8, 4, 400):
        assert oracle_lib.sigma_kn(e) == pytest.approx(float(_kn_textbook(e)), rel=2e-12)
    assert oracle_lib.sigma_kn(1e-9) == pytest.approx(1 - 2e-9, rel=1e-15)


def test_klein_nishina_series_coefficients(oracle_lib):
    import sympy as s
    e = s.symbols("e", positive=True)
    f = s.Rational(3, 4) / e**2 * (2 + e**2 * (1 + e) / (1 + 2 * e) ** 2
                                    + (e**2 - 2 * e - 2) / (2 * e) * s.log(1 + 2 * e))
    coeffs = s.Poly(s.series(f, e, 0, 11).removeO(), e).all_coeffs()[::-1]
    x = 0.013
    want = sum(float(c) * x**i for i, c in enumerate(coeffs))
    assert oracle_lib.sigma_kn(x) == pytest.approx(want, rel=1e-15)


def _kratio(n, th):
    return sp.kv(n, 1 / th)


@pytest.mark.parametrize("theta", [0.05, 1.0, 4.0, 50.0])
def test_hot_cross_section_thomson_slope(oracle_lib, theta):
    """sigma_h = 1 - 2 eps <gamma (1 - beta mu)^2> + O(eps^2) and for the
    thermal distribution <gamma (1 + beta^2/3)> = K1/K2 + 4 Theta, so
    d sigma_h / d eps at 0 is -2 (K1(1/Theta)/K2(1/Theta) + 4 Theta)."""
    eps = 1e-9
    slope = -2 * (_kratio(1, theta) / _kratio(2, theta) + 4 * theta)
    got = (oracle_lib.sigma_hot_direct(theta, eps) - 1.0) / eps
    assert got == pytest.approx(slope, rel=2e-3)


def test_hot_cross_section_cold_limit(oracle_lib):
    """Theta -> 0 reduces sigma_h to sigma_KN (first-order in Theta)."""
    for e in (1e-3, 0.1, 1.0, 10.0):
        assert oracle_lib.sigma_hot_direct(1e-4, e) == pytest.approx(oracle_lib.sigma_kn(e), rel=5e-3)


def test_hot_table_nodes_and_lookup(oracle_lib, sigma_hot_table):
    t = sigma_hot_table
    assert t.shape == (64, 256)
    assert np.all(np.isfinite(t)) and np.all(t <= 1e-12)
    # a node is returned exactly by the lookup
    lt = np.linspace(math.log(1e-2), math.log(1e3), 64)
    le = np.linspace(math.log(1e-12), math.log(1e6), 256)
    th, ep = math.exp(lt[20]), math.exp(le[100])
    assert oracle_lib.sigma_hot_lookup(t, th, ep) == pytest.approx(math.exp(t[20, 100]), rel=1e-12)
    # clamped outside
    assert oracle_lib.sigma_hot_lookup(t, 1e-6, 1e-20) == pytest.approx(math.exp(t[0, 0]), rel=1e-12)
    # interpolation error between nodes stays small where sigma_h varies most
    for th in (0.3, 4.0, 30.0):
        for ep in (3e-3, 0.3, 3.0, 300.0):
            assert oracle_lib.sigma_hot_lookup(t, th, ep) == pytest.approx(
                oracle_lib.sigma_hot_direct(th, ep), rel=2e-3)
