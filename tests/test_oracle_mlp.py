"""Pins for the FP64 reference network of the learned form: the written-out
gradient against central finite differences, and Adam on a quadratic."""
import numpy as np

from oracle import mlp as M


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = M.init(3) + 0.01 * rng.standard_normal(M.N_PARAMS)
    X = rng.standard_normal((37, 8))
    T = rng.standard_normal((37, 2))
    C = rng.uniform(0.1, 1.0, (37, 2)) / 37
    g, L = M.grad(p, X, T, C)
    assert abs(L - M.loss(p, X, T, C)) < 1e-15 * max(1.0, L)
    idx = rng.choice(M.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(M.N_PARAMS)
        e[i] = h
        fd = (M.loss(p + e, X, T, C) - M.loss(p - e, X, T, C)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(g[i]), (i, fd, g[i])


def test_poisson_gradient_matches_finite_differences():
    """The log-link Poisson deviance e^y - T y, targets with many zeros."""
    rng = np.random.default_rng(2)
    p = M.init(5) + 0.01 * rng.standard_normal(M.N_PARAMS)
    X = rng.standard_normal((29, 8))
    T = np.where(rng.uniform(size=(29, 2)) < 0.6, 0.0, rng.exponential(2.0, (29, 2)))
    C = rng.uniform(0.1, 1.0, (29, 2)) / 29
    g, L = M.grad(p, X, T, C, kind=M.POISSON)
    assert abs(L - M.loss(p, X, T, C, kind=M.POISSON)) < 1e-14 * max(1.0, abs(L))
    h = 1e-6
    for i in rng.choice(M.N_PARAMS, 60, replace=False):
        e = np.zeros(M.N_PARAMS)
        e[i] = h
        fd = (M.loss(p + e, X, T, C, M.POISSON) - M.loss(p - e, X, T, C, M.POISSON)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(g[i]), (i, fd, g[i])


def test_poisson_minimiser_is_log_mean():
    """A bias-only output trained on zero-inflated targets goes to ln E[T]
    (the squared error on ln(T + floor) would not)."""
    rng = np.random.default_rng(3)
    T = np.where(rng.uniform(size=(4000, 1)) < 0.9, 0.0, rng.exponential(5.0, (4000, 1)))
    y = 0.0
    for _ in range(2000):
        y -= 0.5 * np.mean(np.exp(y) - T)
    assert abs(y - np.log(T.mean())) < 1e-9


def test_bf16_gradient_reduces_to_exact():
    """The BF16-operand gradient is the exact one when every operand is
    representable in BF16 (rounding is then the identity), and within the
    BF16 rounding (2^-8 relative per operand) of it otherwise."""
    rng = np.random.default_rng(4)
    p = M.bf16(M.init(6))
    X = np.zeros((1, 8))
    X[0, :6] = M.bf16(rng.standard_normal(6))
    T = rng.standard_normal((1, 2))
    C = np.ones((1, 2))
    g, L = M.grad(p, X, T, C)
    gb, Lb = M.grad_bf16(p, X, T, C)
    rel = np.linalg.norm(gb - g) / np.linalg.norm(g)
    assert 0 < rel < 2e-2
    # identity rounding: bitwise the exact code path
    g1, _ = M.grad(p, X, T, C, rnd=lambda a: a)
    np.testing.assert_array_equal(g1, g)


def test_parameter_layout():
    p = np.arange(M.N_PARAMS, dtype=float)
    d = M.unpack(p)
    assert M.N_PARAMS == 4738
    assert d["W1"][1, 0] == 64 and d["b1"][0] == 384 and d["W3"][0, 1] == 384 + 64 + 4096 + 64 + 1
    np.testing.assert_array_equal(M.pack(d), p)


def test_adam_minimises_a_quadratic():
    p = np.array([3.0, -2.0])
    m = v = np.zeros(2)
    for t in range(1, 3001):
        p, m, v = M.adam_step(p, m, v, 2 * p, t, 0.01)
    assert np.all(np.abs(p) < 1e-2)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.14159265])
    np.testing.assert_array_equal(M.bf16(x)[:3], [1.0, 1.0, 1.0 + 4 * 2 ** -8])
    assert abs(M.bf16(x)[3] + 3.140625) < 1e-12
