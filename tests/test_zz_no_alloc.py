"""The allocation-free gradient entry point (gm_mlp_grad_noalloc, for callers
that cannot allocate) against gm_mlp_grad on the same inputs, through the
C ABI: two calls in a row, the second with fewer rows, each equal to the
allocating entry point's gradient and loss bit for bit (same kernels, same
block order); rows above the fixed scratch are refused."""
import numpy as np
import pytest

from oracle import mlp as OM

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_13198_amd import gm as _gm
    _gm.load_library()
    return _gm


def _case(seed, n):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, 8), np.float32)
    X[:, :6] = rng.standard_normal((n, 6))
    T = rng.standard_normal((n, 2)).astype(np.float32)
    C = (rng.uniform(0.5, 1.0, (n, 2)) / n).astype(np.float32)
    return X, T, C


@pytest.mark.parametrize("kind", [0, 1], ids=["squared", "poisson"])
def test_noalloc_gradient_equals_allocating_one(gm, kind):
    import torch
    c = gm.Context(0)
    c.mlp_set_params(OM.init(9).astype(np.float32))
    c.mlp_set_loss(kind)
    out = torch.empty(gm.MLP_PARAMS + 1, dtype=torch.float32, device="cuda")
    for n in (gm.MLP_NOALLOC_MAX_ROWS, 1000):           # the second call smaller
        X, T, C = _case(n, n)
        if kind == 1:
            T = np.abs(T)
        Xd, Td, Cd = (torch.as_tensor(a, device="cuda") for a in (X, T, C))
        out.fill_(float("nan"))
        c.mlp_grad_noalloc(Xd, Td, Cd, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        g, L = c.mlp_grad(X, T, C)
        assert np.all(np.isfinite(got))
        np.testing.assert_array_equal(got[:-1], g)
        assert got[-1] == np.float32(L)
    Xd = torch.zeros((gm.MLP_NOALLOC_MAX_ROWS + 1, 8), dtype=torch.float32, device="cuda")
    Td = torch.zeros((gm.MLP_NOALLOC_MAX_ROWS + 1, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(gm.GmError, match="exceed"):
        c.mlp_grad_noalloc(Xd, Td, Td, out)
    c.mlp_set_loss(0)
    c.close()
