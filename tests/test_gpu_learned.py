"""The learned form on the GPU: the matrix-core network kernels against the
FP64 oracle network (BF16 operand rounding emulated in the oracle), training
on the library's kernels, and the learned bias leaving the spectrum
unbiased."""
import math

import numpy as np
import pytest

from oracle import mlp as OM
from paper_2602_13198_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_13198_amd import gm as _gm
    _gm.load_library()
    return _gm


@pytest.fixture(scope="module")
def ctx(gm):
    c = gm.Context(0)
    yield c
    c.close()


def forward_bf16(p, X):
    """Oracle forward with the operands of every product rounded to BF16, as
    the matrix cores see them (accumulation and biases in full precision)."""
    Wd = OM.unpack(p)
    x = OM.bf16(X[:, :6])
    h1 = np.tanh(x @ OM.bf16(Wd["W1"]) + Wd["b1"])
    h2 = np.tanh(OM.bf16(h1) @ OM.bf16(Wd["W2"]) + Wd["b2"])
    return OM.bf16(h2) @ OM.bf16(Wd["W3"]) + Wd["b3"]


def _case(seed, n):
    rng = np.random.default_rng(seed)
    p = OM.init(seed)
    p[OM.N_PARAMS - 2:] = [0.3, -0.2]
    X = np.zeros((n, 8))
    X[:, :6] = rng.standard_normal((n, 6))
    T = rng.standard_normal((n, 2))
    C = rng.uniform(0.5, 1.0, (n, 2)) / n
    return p.astype(np.float32).astype(np.float64), X, T, C


@pytest.mark.parametrize("n", [1, 16, 1000, 4097])
def test_forward_matches_oracle(ctx, n):
    p, X, _, _ = _case(1, n)
    ctx.mlp_set_params(p)
    y = ctx.mlp_forward(X).cpu().numpy()
    ref = forward_bf16(p, X)
    assert np.all(np.abs(y - ref) <= 2e-2 * (np.abs(ref) + 0.1)), np.max(np.abs(y - ref))
    # and close to the exact FP64 network
    y64, _ = OM.forward(p, X)
    assert np.max(np.abs(y - y64)) < 0.1 * max(1.0, np.max(np.abs(y64)))


@pytest.mark.parametrize("kind", [0, 1], ids=["squared", "poisson"])
@pytest.mark.parametrize("n", [16, 333, 4096])
def test_gradient_matches_oracle(ctx, n, kind):
    """Gradient of the matrix-core kernels against the oracle's backward with
    the same BF16 operand rounding (within 1e-2 relative, by norm, overall
    and per weight matrix), and against the exact FP64 gradient within the
    BF16 rounding; two evaluations agree bit for bit."""
    p, X, T, C = _case(2, n)
    if kind == 1:
        T = np.where(np.random.default_rng(n).uniform(size=T.shape) < 0.7, 0.0, np.abs(T) * 3)
    ctx.mlp_set_loss(kind)
    ctx.mlp_set_params(p)
    g, L = ctx.mlp_grad(X, T, C)
    g2, L2 = ctx.mlp_grad(X, T, C)
    ctx.mlp_set_loss(0)
    assert np.array_equal(g, g2) and L == L2
    gb, Lb = OM.grad_bf16(p, X, T, C, kind)
    g64, L64 = OM.grad(p, X, T, C, kind)
    assert abs(L - Lb) <= 1e-2 * abs(Lb)
    rel = np.linalg.norm(g - gb) / np.linalg.norm(gb)
    rel64 = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    print("n=%d loss %d: gradient relative error %.3e vs BF16-operand oracle, %.3e vs exact FP64"
          % (n, kind, rel, rel64))
    assert rel <= 1e-2
    assert rel64 <= 5e-2
    for name, (a, b) in {"W1": (0, 384), "W2": (448, 4544), "W3": (4608, 4736)}.items():
        r = np.linalg.norm(g[a:b] - gb[a:b]) / np.linalg.norm(gb[a:b])
        assert r <= 1e-2, (name, r)


def test_training_reduces_loss(ctx):
    """A smooth regression target: 400 Adam steps on the library's kernels
    cut the loss by more than 10x; the oracle's FP64 Adam on the same data
    reaches a comparable loss."""
    import torch
    rng = np.random.default_rng(3)
    n = 4096
    X = np.zeros((n, 8), np.float32)
    X[:, :6] = rng.standard_normal((n, 6))
    T = np.stack([np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2], np.tanh(X[:, 3] - X[:, 4])], 1).astype(np.float32)
    C = np.full((n, 2), 1.0 / n, np.float32)
    p0 = OM.init(4)
    ctx.mlp_set_params(p0)
    Xd, Td, Cd = (torch.as_tensor(a, device="cuda") for a in (X, T, C))
    L0 = ctx.mlp_train_step(Xd, Td, Cd, 3e-3, want_loss=True)
    for _ in range(398):
        ctx.mlp_train_step(Xd, Td, Cd, 3e-3)
    L1 = ctx.mlp_train_step(Xd, Td, Cd, 3e-3, want_loss=True)
    assert L1 < 0.1 * L0, (L0, L1)
    p, m, v = p0.copy(), np.zeros(OM.N_PARAMS), np.zeros(OM.N_PARAMS)
    for t in range(1, 400):
        g, _ = OM.grad(p, X, T, C)
        p, m, v = OM.adam_step(p, m, v, g, t, 3e-3)
    Lo = OM.loss(p, X, T, C)
    print("loss: start %.4f  gpu after 399 steps %.4f  oracle %.4f" % (L0, L1, Lo))
    assert L1 < 3 * Lo + 1e-3


def test_train_steps_equal_single_steps(gm, ctx):
    """gm_mlp_train_steps: k Adam steps in one call (batches wrapping round
    the rows) leave the parameters bit for bit where the k single steps over
    the same batches with the same learning rates leave them, and report the
    same first and last losses; bad batch sizes or step counts give
    GM_EINVAL."""
    import torch
    n, b, k = 5000, 1024, 7                           # four batches a pass: the steps wrap
    p0, X, T, C = _case(11, n)
    T = np.abs(T)                                     # Poisson targets
    Xd, Td, Cd = (torch.as_tensor(a.astype(np.float32), device="cuda") for a in (X, T, C))
    ctx.mlp_set_loss(gm.MLP_POISSON)
    ctx.mlp_set_params(p0.astype(np.float32))
    L = ctx.mlp_train_steps(Xd, Td, Cd, b, k, 2e-3, 0.1, want_loss=True)
    pa = ctx.mlp_get_params()
    ctx.mlp_set_params(p0.astype(np.float32))         # also resets the Adam state
    lr0, dec = float(np.float32(2e-3)), float(np.float32(0.1))
    losses = []
    for s in range(k):
        j = s % (n // b)
        lr = float(np.float32(lr0 * dec ** (s / k)))
        ls = ctx.mlp_train_step(Xd[j * b:(j + 1) * b], Td[j * b:(j + 1) * b], Cd[j * b:(j + 1) * b], lr,
                                want_loss=s in (0, k - 1))
        if s in (0, k - 1):
            losses.append(ls)
    pb = ctx.mlp_get_params()
    ctx.mlp_set_loss(gm.MLP_SQUARED)
    assert np.array_equal(pa, pb) and not np.array_equal(pa, p0.astype(np.float32))
    assert L == tuple(losses)
    for bad in (dict(batch=0, steps=3), dict(batch=n + 1, steps=3), dict(batch=b, steps=0)):
        with pytest.raises(gm.GmError, match="error -1"):
            ctx.mlp_train_steps(Xd, Td, Cd, bad["batch"], bad["steps"], 2e-3, 0.1)


def test_learned_form_keeps_the_spectrum(gm, ctx):
    """Scattering sphere tau_T = 0.1: the learned form -- the network trained
    with the Poisson deviance on one pilot round's records, then the
    weight-window bias table and the defensive emission proposal it builds
    -- moves sampling effort only: over 24 rounds of each (different
    seeds), the total and each inclination's luminosity agree with the
    plain method's within 4 and 4.5 standard deviations of the rounds'
    spread, and of the bins holding >= 1e3 superphotons in both at most 2 %
    lie beyond 4 and none beyond 6; the training loss falls and at least
    one table is built."""
    from paper_2602_13198_amd import importance as IM
    wl = W.scattering_sphere(0.1, n_target=2e5, seed=0)
    c = gm.Context(0)
    c.load_zones(wl)
    n_s = wl.emit["n_target"]
    IM.pilot(c, wl, 0, 1, 300000, n_s, 4)
    info = IM.build_tables(c, wl, 0, wl.track["bias_value"], 1e3, n_s, "network", net_seed=1)
    c.set_event_log(0)
    print("learned form on the sphere: %s" % {k: v for k, v in info.items() if not k.endswith("_s")})
    assert info["loss_first_last"][1] < info["loss_first_last"][0]
    assert info["bias_table"] or info["emission_table"]

    def rounds(track, seeds):
        """Per-round spectra [rounds][n_theta][n_nu][3]."""
        out = []
        for s in seeds:
            c.make_superphotons(dict(wl.emit, seed=s))
            c.track_scatter(track)
            out.append(c.read_spectrum(0, reset=True)[0])
        return np.array(out)
    over = dict(bias_mode=gm.BIAS_WINDOW, bias_max=1e3) if info["bias_table"] else {}
    K = 24
    r_l = rounds(dict(wl.track, **over), range(2000, 2000 + K))
    c.set_emission_table(0, None)
    r_p = rounds(wl.track, range(1000, 1000 + K))
    c.close()

    # independent rounds: the spread of the round luminosities is each
    # mean's variance, whatever the correlations inside a root's family
    def z_of(Lp, Ll):
        return (Ll.mean(0) - Lp.mean(0)) / np.sqrt((Lp.var(0, ddof=1) + Ll.var(0, ddof=1)) / K)
    Lp, Ll = r_p[..., 0], r_l[..., 0]
    z_tot = z_of(Lp.sum((1, 2)), Ll.sum((1, 2)))
    z_th = z_of(Lp.sum(2), Ll.sum(2))
    use = (r_p[..., 2].sum(0) >= 1000) & (r_l[..., 2].sum(0) >= 1000)
    z = z_of(Lp[:, use], Ll[:, use])
    print("learned vs plain: total z %.2f, per inclination %s, %d bins: mean z^2 %.2f, max |z| %.2f, "
          "beyond 4 sigma %d" % (z_tot, np.round(z_th, 2), use.sum(), np.mean(z ** 2), np.abs(z).max(),
                                 (np.abs(z) > 4).sum()))
    # with the window bias the per-bin mean of z^2 sits near 1.65 (plain
    # against plain: 1.00) and stays there from 24 to 96 rounds, an excess
    # that does not grow with the rounds as a bias would: heavier-tailed
    # rounds, with neighbouring bins sharing photons; so the per-bin test
    # bounds the outliers' share rather than the mean of z^2
    assert use.sum() > 50
    assert abs(z_tot) < 4.0 and np.abs(z_th).max() < 4.5
    assert (np.abs(z) > 4).mean() < 0.02 and np.abs(z).max() < 6.0
