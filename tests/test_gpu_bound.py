"""The register-limited FP64 bound kernel: its chains are the exact IEEE
fused multiply-add sequences (checked bit for bit against libm's fma), and
its rate lies below the FP64 vector peak."""
import ctypes

import pytest

from paper_2602_13198_amd import gm

pytestmark = pytest.mark.gpu

_fma = ctypes.CDLL("libm.so.6").fma
_fma.restype = ctypes.c_double
_fma.argtypes = [ctypes.c_double] * 3


def chain_sum(t, chains, iters):
    s = 0.0
    for c in range(chains):
        x = (1.0 + 1e-9 * t) + 1e-3 * c
        for _ in range(iters):
            x = _fma(x, 0.9999999, 1e-7)
        s += x
    return s


@pytest.mark.parametrize("chains", [1, 2, 4])
def test_chain_values_exact(chains):
    c = gm.Context(0)
    try:
        ms, tf, out = c.fma_chain_bound(2, chains, 1000, n_out=257)
    finally:
        c.close()
    for t in (0, 1, 63, 64, 255, 256):
        assert out[t] == chain_sum(t, chains, 1000), (t, out[t])
    assert ms > 0.0 and 0.0 < tf < 78.6 * 1.02


@pytest.mark.parametrize("waves", [2, 3, 4])
def test_rate_below_peak_and_rises_with_chains(waves):
    c = gm.Context(0)
    try:
        rates = [c.fma_chain_bound(waves, ch, 20000)[1] for ch in (1, 8)]
    finally:
        c.close()
    assert all(0.0 < r < 78.6 * 1.02 for r in rates), rates
    assert rates[1] >= rates[0] * 0.95, rates
