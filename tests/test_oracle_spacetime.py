"""Pins for the oracle's Kerr-Schild metric in modified coordinates, its
Christoffel symbols and the geodesic integrator (geodesic section)."""
import math

import numpy as np
import pytest


def grid(a=0.9375, h=0.3):
    return dict(metric=1, n=[64, 32, 1], x_start=[math.log(1.2), 0.0, 0.0],
                dx=[0.11, 1 / 32, 2 * math.pi], a_spin=a, h_slope=h, L_unit_cm=1.0, r_record=1000.0)


def theta_of(x2, h):
    return math.pi * x2 + 0.5 * (1 - h) * math.sin(2 * math.pi * x2)


def dtheta(x2, h):
    return math.pi * (1 + (1 - h) * math.cos(2 * math.pi * x2))


def ks_inverse_textbook(r, th, a):
    """Contravariant Kerr-Schild metric (t, r, theta, phi), M = 1."""
    S = r * r + a * a * math.cos(th) ** 2
    D = r * r - 2 * r + a * a
    g = np.zeros((4, 4))
    g[0, 0] = -(1 + 2 * r / S)
    g[0, 1] = g[1, 0] = 2 * r / S
    g[1, 1] = D / S
    g[1, 3] = g[3, 1] = a / S
    g[2, 2] = 1 / S
    g[3, 3] = 1 / (S * math.sin(th) ** 2)
    return g


def random_points(n, seed=0):
    rng = np.random.default_rng(seed)
    pts = []
    for _ in range(n):
        pts.append(np.array([0.0, math.log(rng.uniform(1.5, 500)), rng.uniform(0.02, 0.98),
                             rng.uniform(0, 2 * math.pi)]))
    return pts


def test_metric_inverse_against_textbook(oracle_lib):
    G = grid()
    for x in random_points(40):
        r, th = math.exp(x[1]), theta_of(x[2], G["h_slope"])
        J = np.array([1.0, r, dtheta(x[2], G["h_slope"]), 1.0])
        gcon_mks = ks_inverse_textbook(r, th, G["a_spin"]) / np.outer(J, J)
        gcov = oracle_lib.gcov(G, x)
        np.testing.assert_allclose(gcov @ gcon_mks, np.eye(4), atol=1e-12)
        np.testing.assert_allclose(oracle_lib.gcon(G, x), gcon_mks, rtol=1e-11, atol=1e-14)


def test_schwarzschild_limit(oracle_lib):
    G = grid(a=0.0, h=1.0)       # h = 1: theta = pi x2
    for x in random_points(10, seed=1):
        r, th = math.exp(x[1]), math.pi * x[2]
        ks = np.zeros((4, 4))
        ks[0, 0] = -(1 - 2 / r)
        ks[0, 1] = ks[1, 0] = 2 / r
        ks[1, 1] = 1 + 2 / r
        ks[2, 2] = r * r
        ks[3, 3] = r * r * math.sin(th) ** 2
        J = np.array([1.0, r, math.pi, 1.0])
        np.testing.assert_allclose(oracle_lib.gcov(G, x), ks * np.outer(J, J), rtol=1e-14, atol=1e-14)


def test_sqrt_neg_g_closed_form(oracle_lib):
    G = grid()
    for x in random_points(20, seed=2):
        r, th = math.exp(x[1]), theta_of(x[2], G["h_slope"])
        S = r * r + G["a_spin"] ** 2 * math.cos(th) ** 2
        want = S * abs(math.sin(th)) * r * dtheta(x[2], G["h_slope"])
        assert oracle_lib.sqrt_neg_g(G, x) == pytest.approx(want, rel=1e-12)


def test_christoffel_against_finite_differences(oracle_lib):
    G = grid()
    h = 1e-5
    for x in random_points(12, seed=3):
        gcon = oracle_lib.gcon(G, x)
        dg = np.zeros((4, 4, 4))
        for c in (1, 2):
            e = np.zeros(4)
            e[c] = h
            dg[c] = (oracle_lib.gcov(G, x + e) - oracle_lib.gcov(G, x - e)) / (2 * h)
        fd = 0.5 * (np.einsum("mn,anb->mab", gcon, dg) + np.einsum("mn,bna->mab", gcon, dg)
                    - np.einsum("mn,nab->mab", gcon, dg))
        Gam = oracle_lib.christoffel(G, x)
        scale = np.max(np.abs(Gam))
        np.testing.assert_allclose(Gam, fd, atol=1e-7 * scale)
        np.testing.assert_allclose(Gam, np.transpose(Gam, (0, 2, 1)), atol=1e-15 * scale)


def null_k(oracle_lib, G, x, k_spatial):
    g = oracle_lib.gcov(G, x)
    ks = np.asarray(k_spatial, float)
    A = g[0, 0]
    B = 2 * g[0, 1:] @ ks
    Cq = ks @ g[1:, 1:] @ ks
    k0 = (-B - math.sqrt(B * B - 4 * A * Cq)) / (2 * A)
    return np.concatenate([[k0], ks])


def invariants(oracle_lib, G, x, k):
    g = oracle_lib.gcov(G, x)
    kl = g @ k
    h = G["h_slope"]
    th = theta_of(x[2], h)
    kth = kl[2] / dtheta(x[2], h)          # covariant theta component
    a = G["a_spin"]
    E, L = -kl[0], kl[3]
    Q = kth ** 2 + math.cos(th) ** 2 * (L * L / math.sin(th) ** 2 - a * a * E * E)
    return k @ g @ k, E, L, Q


def test_geodesic_invariants(oracle_lib):
    """Null norm, energy -k_t, angular momentum k_phi and Carter's constant
    are conserved along photon paths, with errors falling as the square of
    the step (velocity Verlet is second order): 2.5x smaller steps cut the
    drift ~6x."""
    G = grid()
    rng = np.random.default_rng(4)
    ratios = []
    for _ in range(12):
        x = np.array([0.0, math.log(rng.uniform(5, 40)), rng.uniform(0.2, 0.8), 0.3])
        ks = rng.normal(size=3) * np.array([0.3, 0.05, 0.05])
        k = null_k(oracle_lib, G, x, ks)
        n0, E0, L0, Q0 = invariants(oracle_lib, G, x, k)
        drift = {}
        for h in (0.05, 0.02):
            path = oracle_lib.integrate_geodesic(G, x, k, h=h, n=100000, r_min=1.6, r_max=900)
            d = np.zeros(4)
            for row in path[:: max(1, len(path) // 200)]:
                n, E, L, Q = invariants(oracle_lib, G, row[:4], row[4:])
                d = np.maximum(d, [abs(n) / E0 ** 2, abs(E / E0 - 1), abs(L - L0) / (abs(L0) + E0),
                                   abs(Q - Q0) / (abs(Q0) + E0 * E0)])
            drift[h] = d
            escaped = math.exp(path[-1, 1]) > 899
        if escaped:
            assert np.all(drift[0.02] < [1e-3, 1e-5, 1e-3, 1e-3]), drift[0.02]
        ratios.append(drift[0.05][2:] / drift[0.02][2:])
    med = np.median(np.array(ratios), axis=0)
    assert np.all((med > 4.0) & (med < 9.0)), med


def deflection(oracle_lib, b, h, dx1=0.01):
    G = dict(grid(a=0.0, h=1.0), dx=[dx1, 1 / 32, 2 * math.pi])
    r0 = 100 * b
    # start in the equatorial plane at (x, y) = (-sqrt(r0^2 - b^2), b), moving +x
    X, Y = -math.sqrt(r0 * r0 - b * b), b
    r, ph = math.hypot(X, Y), math.atan2(Y, X)
    x = np.array([0.0, math.log(r), 0.5, ph])
    k = null_k(oracle_lib, G, x, [math.cos(ph) / r, 0.0, -math.sin(ph) / r])
    path = oracle_lib.integrate_geodesic(G, x, k, h=h, n=2000000, r_min=2.5, r_max=r0 * 1.01)
    xe, ke = path[-1, :4], path[-1, 4:]
    re, phe = math.exp(xe[1]), xe[3]
    vr, vph = ke[1] * re, ke[3] * re          # dr/dl and r dphi/dl
    vx = vr * math.cos(phe) - vph * math.sin(phe)
    vy = vr * math.sin(phe) + vph * math.cos(phe)
    return -math.atan2(vy, vx)


def test_weak_field_deflection(oracle_lib):
    """Schwarzschild light bending at impact parameter b = 200:
    4/b + 15 pi/(4 b^2) to second order, approached as the step shrinks."""
    b = 200.0
    want = 4 / b + 15 * math.pi / (4 * b * b)
    coarse, fine = deflection(oracle_lib, b, 0.5), deflection(oracle_lib, b, 0.1)
    assert fine == pytest.approx(want, rel=0.01)
    assert abs(fine - want) < 0.2 * abs(coarse - want)
