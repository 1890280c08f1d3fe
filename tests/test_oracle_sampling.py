"""Statistical pins for the oracle's scattering samplers (Scattering
section): thermal electron moments, the Klein-Nishina angular law, Compton
kinematics, the Thomson-limit energy gain, and the acceptance rate that ties
the sampler to the hot cross section."""
import math

import numpy as np
import pytest
import scipy.special as sp


def _k(n, th):
    return sp.kv(n, 1.0 / th)


def _electrons(oracle_lib, theta, eps, n, seed=5):
    g = np.empty(n)
    m = np.empty(n)
    trials = 0
    for i in range(n):
        gi, mi, _, t = oracle_lib.sample_electron(seed, [i, 0, 0x77], 0, theta, eps)
        g[i], m[i] = gi, mi
        trials += t
    return g, m, trials


@pytest.mark.parametrize("theta", [0.3, 4.0])
def test_thermal_electron_moments(oracle_lib, theta):
    """At eps -> 0 the Klein-Nishina acceptance is 1 and gamma follows the
    thermal law: <gamma> = K1/K2 + 3 Theta, <gamma^2 - 1> = 3 Theta K3/K2;
    mu follows (1 - beta mu)/2, so <mu | gamma> = -beta/3."""
    n = 40000
    g, m, _ = _electrons(oracle_lib, theta, 1e-14, n)
    mean_g = _k(1, theta) / _k(2, theta) + 3 * theta
    mean_p2 = 3 * theta * _k(3, theta) / _k(2, theta)
    assert abs(g.mean() - mean_g) < 5 * g.std() / math.sqrt(n)
    p2 = g * g - 1
    assert abs(p2.mean() - mean_p2) < 5 * p2.std() / math.sqrt(n)
    beta = np.sqrt(p2) / g
    d = m + beta / 3
    assert abs(d.mean()) < 5 * d.std() / math.sqrt(n)


def test_thermal_electron_cdf(oracle_lib):
    """Kolmogorov-Smirnov against the thermal CDF of gamma."""
    theta = 1.0
    n = 20000
    g, _, _ = _electrons(oracle_lib, theta, 1e-14, n, seed=9)
    from scipy import integrate, stats
    pdf = lambda x: (1 + x) * math.sqrt(x * (x + 2)) * math.exp(-x / theta)
    norm = theta * _k(2, theta) * math.exp(1 / theta)
    xs = np.sort(g - 1)
    grid = np.linspace(0, xs[-1], 4000)
    cdf_grid = np.concatenate([[0], np.cumsum([integrate.quad(pdf, a, b)[0]
                                               for a, b in zip(grid[:-1], grid[1:])])]) / norm
    cdf = np.interp(xs, grid, cdf_grid)
    D = np.max(np.abs(cdf - np.arange(1, n + 1) / n))
    assert D < 1.95 / math.sqrt(n)    # ~ 0.1 % tail of the KS law


def test_acceptance_rate_equals_hot_cross_section(oracle_lib):
    """The (gamma, mu) proposal has density f(gamma)(1 - beta mu)/2, so the
    Klein-Nishina acceptance probability is sigma_h/sigma_T and the mean
    number of outer trials is sigma_T/sigma_h."""
    for theta, eps in ((4.0, 1.0), (0.5, 3.0)):
        n = 15000
        _, _, trials = _electrons(oracle_lib, theta, eps, n, seed=11)
        sh = oracle_lib.sigma_hot_direct(theta, eps)
        p = 1.0 / (trials / n)
        # n successes out of `trials` Bernoulli(sigma_h) draws
        assert abs(p - sh) < 5 * sh * math.sqrt((1 - sh) / n)


def test_klein_nishina_angles_and_compton_kinematics(oracle_lib):
    """Electrons at rest (Theta = 1e-12): the scattered energy obeys
    e' = e / (1 + e (1 - cos T)) and cos T follows the Klein-Nishina
    differential cross section."""
    eps = 1.0
    n = 30000
    cs = np.empty(n)
    for i in range(n):
        _, _, k, _, _, _ = oracle_lib.sample_scatter_frame(3, [i, 1, 0x55], 0, 1e-12, eps)
        c = k[1] / k[0]
        cs[i] = c
        assert k[0] == pytest.approx(eps / (1 + eps * (1 - c)), rel=1e-5)
        assert k[0] ** 2 == pytest.approx(k[1] ** 2 + k[2] ** 2 + k[3] ** 2, rel=1e-12)
    edges = np.linspace(-1, 1, 41)
    h, _ = np.histogram(cs, edges)

    def dsig(c):
        r = 1 / (1 + eps * (1 - c))
        return r * r * (r + 1 / r - (1 - c * c))
    from scipy.integrate import quad
    w = np.array([quad(dsig, a, b)[0] for a, b in zip(edges[:-1], edges[1:])])
    e = n * w / w.sum()
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 / 39 < 1.6


@pytest.mark.parametrize("theta", [0.5, 4.0])
def test_thomson_limit_energy_gain(oracle_lib, theta):
    """Thomson limit, thermal electrons: <e'/e> = 1 + 4 Theta K3/K2 (the
    mean of (4/3) gamma^2 beta^2 over the scattering-rate weighted law)."""
    eps = 1e-10
    n = 60000
    r = np.empty(n)
    for i in range(n):
        _, _, k, _, _, _ = oracle_lib.sample_scatter_frame(21, [i, 2, 0x66], 0, theta, eps)
        r[i] = k[0] / eps
    want = 1 + 4 * theta * _k(3, theta) / _k(2, theta)
    assert abs(r.mean() - want) < 5 * r.std() / math.sqrt(n)
