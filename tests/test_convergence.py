"""Host-side spectral error measure (eq:conv_parameter) and its bin mask."""
import numpy as np

from paper_2602_13198_amd import convergence as CV


def test_eps_err_known_values():
    ref = np.ones((3, 10))
    L = ref.copy()
    L[0] *= 1.02                     # 2 % everywhere in theta bin 0
    L[1, :5] *= 0.9                  # 10 % in half of theta bin 1
    mask = np.ones_like(ref, bool)
    mask[2] = False                  # theta bin 2 holds no masked bin
    assert abs(CV.eps_err(L, ref, mask) - (0.02 + 0.05) / 2) < 1e-12
    mask[1, 5:] = False              # only the perturbed half of bin 1
    assert abs(CV.eps_err(L, ref, mask) - (0.02 + 0.10) / 2) < 1e-12


def test_eps_err_scales_as_inverse_sqrt_n():
    rng = np.random.default_rng(0)
    ref = np.full((2, 50), 5.0)
    mask = np.ones_like(ref, bool)
    e = []
    for n in (100, 10000):
        L = ref * (1 + rng.standard_normal(ref.shape) / np.sqrt(n))
        e.append(CV.eps_err(L, ref, mask))
    assert 5 < e[0] / e[1] < 20


def test_error_mask():
    cnt = np.array([[500.0, 2000.0, 5000.0]])
    rse = np.array([[0.01, 0.2, 0.05]])
    np.testing.assert_array_equal(CV.error_mask(cnt, rse), [[False, False, True]])
