"""GPU parity on the 3-D Kerr inputs: the torus under a scattering corona
(the workload of the plain-versus-learned measurement) and the batched
survey of tori, through the C ABI against the CPU oracle.

Same-seed histories on a reduced corona torus; at full size (192 x 96 x 96
zones, N_s = 1e8, the launch configuration of the benchmark) every photon is
traced on the GPU and the oracle recomputes sampled root families with all
their descendants.  The survey in shared launches (tallies in HBM) equals
the instances tracked one at a time, bit for bit."""
import numpy as np
import pytest

from _parity import compare_traces, describe, ledger_residuals
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


def _key(a):
    """Stream key s0 | s1 << 32 (as read_trace_subset selects)."""
    return a["s0"].astype(np.uint64) | (a["s1"].astype(np.uint64) << np.uint64(32))


def test_corona_same_seed(gm, oracle_lib):
    wl = W.corona_torus(n1=48, n2=24, n3=24, n_target=8000, seed=61)
    c = gm.Context(0)
    c.load_zones(wl)
    n = c.make_superphotons(wl.emit)
    c.set_trace(2_000_000)
    st = c.track_scatter(wl.track)
    spec, led = c.read_spectrum()
    tr = c.read_trace()
    c.close()
    ores, em = oracle_lib.run(wl, trace_cap=2_000_000)
    assert n == em["n_roots"]
    m, bad = compare_traces(tr, ores.trace)
    print("corona torus 48x24x24: %d photons, %d differ, generations %s" % (m, len(bad), np.bincount(tr["n_sc"])))
    assert m > 3000
    assert len(bad) <= 1e-3 * m, describe(tr, ores.trace, bad)
    kinds = np.bincount(tr["kind"], minlength=7)
    assert kinds[1] > 0 and kinds[3] > 0 and np.bincount(tr["n_sc"]).size >= 3
    wr, er = ledger_residuals(led)
    assert abs(wr) < 1e-12 and abs(er) < 1e-12


def test_corona_full_size_sampled(gm, oracle_lib):
    """192 x 96 x 96, N_s = 1e8, constant bias 10, tracker tuning of the
    benchmark: every photon traced on the GPU; the oracle recomputes twelve
    families of ten consecutive roots."""
    wl = W.corona_torus(n_target=1e8, seed=5)
    c = gm.Context(0)
    c.set_tuning(2, 8)
    c.load_zones(wl)
    n = c.make_superphotons(wl.emit)
    c.set_trace(int(8 * n))
    st = c.track_scatter(wl.track)
    _, led = c.read_spectrum()
    assert c.trace_count() == st[0] + st[1] <= 8 * n
    o = oracle_lib.Oracle()
    o.load_zones(wl)
    assert o.make_superphotons(wl.emit) == n
    rng = np.random.default_rng(6)
    starts = np.sort(rng.choice(n - 10, 12, replace=False))
    ora = np.concatenate([o.track_scatter(wl.track, int(s), int(s) + 10, trace_cap=100000) for s in starts])
    o.close()
    sub = c.read_trace_subset(_key(ora))
    c.close()
    m, bad = compare_traces(sub, ora, subset=True)
    print("corona torus full size: %d roots, %d superphotons; %d sampled photons, %d differ"
          % (st[0], st[0] + st[1], m, len(bad)))
    assert m == len(ora) and m >= 120
    assert len(bad) <= max(1, 1e-3 * m), describe(sub, ora, bad)
    wr, er = ledger_residuals(led)
    assert abs(wr) < 1e-12 and abs(er) < 1e-12


def test_survey_batched_equals_separate(gm):
    """64 tori (four spins x four R_high x four density scales, uneven N_s)
    on reduced 3-D grids: one shared launch group with the tallies in HBM
    gives bitwise the histories of tracking each instance alone (tallies in
    LDS), the same counters, and tallies equal up to summation order."""
    wls = W.survey(n1=24, n2=12, n3=8, ns_lo=300, ns_hi=3000)
    out = {}
    for batch in (1, 64):
        c = gm.Context(0)
        c.set_batch(batch)
        for i, wl in enumerate(wls):
            c.load_zones(wl, i)
            c.set_instance_bias(i, dict(wl.track, bias_max=30.0))
            c.make_superphotons(wl.emit, i)
        c.set_trace(4_000_000)
        st = c.track_scatter(wls[0].track)
        specs = [c.read_spectrum(i) for i in range(len(wls))]
        tr = np.sort(c.read_trace(), order=["s2", "s1", "s0"])
        c.close()
        out[batch] = (st, specs, tr)
    (s1, p1, t1), (s2, p2, t2) = out[1], out[64]
    print("survey: %d superphotons, generations %s" % (len(t1), np.bincount(t1["n_sc"])))
    assert len(t1) == len(t2) > 20000
    assert np.array_equal(t1.view(np.uint8), t2.view(np.uint8))
    np.testing.assert_array_equal(s1, s2)
    nonempty = 0
    for (a, la), (b, lb) in zip(p1, p2):
        nonempty += a[..., 2].sum() > 0
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=0)
        np.testing.assert_allclose(la, lb, rtol=1e-12, atol=1e-300)
    assert nonempty == 64
