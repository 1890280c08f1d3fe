"""GPU parity of the bias modes beyond the constant one (generation-dependent,
table, weight window), the emission table, the event records with their
all-descendant scores, the HBM tallies and the error paths of the track
call: the HIP path through the C ABI against the CPU oracle on the same
seeds.

Histories must agree photon by photon (end kind, generation, tally bin and
step count exactly; weights and wavevectors within 1e-10), with the same
allowance for threshold flips as the other parity tests; event records by
the stream of the photon they created, scores within 1e-9 relative (both
sides sum them in different orders)."""
import math

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


def small_torus(**kw):
    kw.setdefault("step_h", 0.125)
    return W.torus(n1=64, n2=32, **kw)


def run_gpu(gm, wl, btab=None, blo=0.0, bhi=1.0, mtab=None, mlo=0.0, mhi=1.0, events=0, stride=0, sw=None,
            tally_mode=0, trace=2_000_000):
    c = gm.Context(0)
    c.load_zones(wl)
    if btab is not None:
        c.set_bias_table(0, btab, blo, bhi)
    if mtab is not None:
        c.set_emission_table(0, mtab, mlo, mhi)
    n = c.make_superphotons(wl.emit)
    em = c.read_emission()
    if events:
        c.set_event_log(events, stride)
    if sw is not None:
        c.set_score_weights(0, sw)
    c.set_tally_mode(tally_mode)
    if trace:
        c.set_trace(trace)
    st = c.track_scatter(wl.track)
    spec, led = c.read_spectrum()
    tr = c.read_trace() if trace else None
    ev = c.read_event_log() if events else None
    c.close()
    return dict(n=n, stats=st, spec=spec, ledger=led, trace=tr, emission=em, events=ev)


def run_oracle(oracle_lib, wl, btab=None, blo=0.0, bhi=1.0, mtab=None, mlo=0.0, mhi=1.0, events=0, stride=1,
               sw=None, trace=2_000_000):
    o = oracle_lib.Oracle()
    o.load_zones(wl)
    if btab is not None:
        o.set_bias_table(btab, blo, bhi)
    if mtab is not None:
        o.set_emission_table(mtab, mlo, mhi)
    n = o.make_superphotons(wl.emit)
    em = o.read_emission()
    if events:
        o.set_event_log(events, stride)
    if sw is not None:
        o.set_score_weights(sw)
    tr = o.track_scatter(wl.track, trace_cap=trace)
    res = o.read_spectrum()
    ev = o.read_event_log() if events else None
    o.close()
    return dict(n=n, stats=res.stats, spec=res.spectrum, ledger=res.ledger, trace=tr, emission=em, events=ev)


def _histories(g, o, max_bad_frac=1e-3, min_n=500):
    n, bad = compare_traces(g["trace"], o["trace"])
    assert n >= min_n, n
    print("%d photons compared, %d differ" % (n, len(bad)))
    assert len(bad) <= max(1, max_bad_frac * n), describe(g["trace"], o["trace"], bad)
    wr, er = ledger_residuals(g["ledger"])
    assert abs(wr) < 1e-12 and abs(er) < 1e-12
    if not bad:
        np.testing.assert_array_equal(g["spec"][..., 2], o["spec"][..., 2])
        np.testing.assert_allclose(g["spec"][..., 0], o["spec"][..., 0], rtol=1e-9, atol=1e-300)
    return n, bad


def _median_lnw(oracle_lib, wl):
    o = oracle_lib.Oracle()
    o.load_zones(wl)
    o.make_superphotons(wl.emit)
    lw = float(np.median(o.read_emission()["ln_w"]))
    o.close()
    return lw


LN_EPS = (math.log(1e-12), math.log(1e6))


def _bias_table(nz, n=7, base=math.log(10.0), amp=0.8, seed=3):
    rng = np.random.default_rng(seed)
    z = np.arange(nz)[:, None]
    k = np.arange(n)[None, :]
    return base + amp * np.sin(0.37 * z + 1.3 * k) + 0.1 * rng.standard_normal((nz, n))


def test_generation_bias_same_seed(gm, oracle_lib):
    """GEN2: b = (n_sc + 1)^2 / (n_e sigma_T bias_value ell) per generation."""
    wl = W.scattering_sphere(0.1, n_target=6000, seed=21).with_track(bias_mode=W.BIAS_GEN2, bias_value=1.0)
    g, o = run_gpu(gm, wl), run_oracle(oracle_lib, wl)
    _histories(g, o)
    gens = np.bincount(g["trace"]["n_sc"], minlength=5)
    assert gens[2] > 0 and gens[3] > 0


@pytest.mark.parametrize("mode", [W.BIAS_TABLE, W.BIAS_WINDOW], ids=["table", "window"])
def test_table_bias_same_seed_flat(gm, oracle_lib, mode):
    wl = W.scattering_sphere(0.1, n_target=6000, seed=22).with_track(bias_mode=mode, bias_max=200.0)
    base = math.log(10.0) if mode == W.BIAS_TABLE else math.log(10.0) - _median_lnw(oracle_lib, wl)
    tab = _bias_table(wl.n_zones, base=base)
    g = run_gpu(gm, wl, btab=tab, blo=LN_EPS[0], bhi=LN_EPS[1])
    o = run_oracle(oracle_lib, wl, btab=tab, blo=LN_EPS[0], bhi=LN_EPS[1])
    _histories(g, o)
    assert g["stats"][1] > 1000          # children


@pytest.mark.parametrize("mode", [W.BIAS_TABLE, W.BIAS_WINDOW], ids=["table", "window"])
def test_table_bias_same_seed_kerr(gm, oracle_lib, mode):
    wl = small_torus(n_target=1500, seed=23, bias_mode=mode, bias_max=1e3)
    base = math.log(300.0) if mode == W.BIAS_TABLE else math.log(300.0) - _median_lnw(oracle_lib, wl)
    tab = _bias_table(wl.n_zones, base=base, amp=1.0)
    g = run_gpu(gm, wl, btab=tab, blo=LN_EPS[0], bhi=LN_EPS[1])
    o = run_oracle(oracle_lib, wl, btab=tab, blo=LN_EPS[0], bhi=LN_EPS[1])
    _histories(g, o, max_bad_frac=1e-3)
    assert g["stats"][1] > 100


def test_paper_theta2_coefficient_kerr(gm, oracle_lib):
    """THETA2 at the coefficient of the paper's GRMHD run (b = 96e4 Theta_e^2)
    on a torus thin enough for it (M_unit lowered so that b tau_T ~ 1)."""
    wl = small_torus(n_target=1500, seed=24, M_unit=3e24, bias_value=96e4)
    g, o = run_gpu(gm, wl), run_oracle(oracle_lib, wl)
    _histories(g, o, max_bad_frac=1e-3)
    assert g["stats"][1] > 100


@pytest.mark.parametrize("kerr", [False, True], ids=["flat", "kerr"])
def test_emission_table_same_seed(gm, oracle_lib, kerr):
    """Per-zone emission modulation: counts, expected counts and bounds
    exactly as the oracle's, then the same histories."""
    wl = small_torus(n_target=4000, seed=25) if kerr else W.scattering_sphere(0.1, n_target=5000, seed=25)
    nz = wl.n_zones
    k = np.arange(6)[None, :]
    m = 0.7 * np.sin(0.3 * np.arange(nz)[:, None] + 0.9 * k)
    lo, hi = math.log(wl.emit["nu_min"]), math.log(wl.emit["nu_max"])
    g = run_gpu(gm, wl, mtab=m, mlo=lo, mhi=hi)
    o = run_oracle(oracle_lib, wl, mtab=m, mlo=lo, mhi=hi)
    assert g["n"] == o["n"]
    np.testing.assert_array_equal(g["emission"]["counts"], o["emission"]["counts"])
    np.testing.assert_allclose(g["emission"]["nbar"], o["emission"]["nbar"], rtol=1e-11, atol=0)
    np.testing.assert_allclose(g["emission"]["fmax"], o["emission"]["fmax"], rtol=1e-11, atol=0)
    _histories(g, o, max_bad_frac=1e-3)


def _key(ev):
    return {(int(r["s0"]), int(r["s1"]), int(r["s2"])): r for r in ev}


@pytest.mark.parametrize("kerr", [False, True], ids=["flat", "kerr"])
def test_event_records_and_scores(gm, oracle_lib, kerr):
    """Event records of scatterings and of every third root's emission, and
    their scores (score weights over the bins): the same records as the
    oracle's, each score the sum over the photon and its descendants."""
    if kerr:
        wl = small_torus(n_target=4000, seed=26, bias_value=3e3)
    else:
        wl = W.scattering_sphere(0.1, n_target=6000, seed=26)
    t = wl.track
    sw = np.random.default_rng(4).uniform(0.0, 2.0, (t["n_theta"], t["n_nu"]))
    g = run_gpu(gm, wl, events=2_000_000, stride=3, sw=sw)
    o = run_oracle(oracle_lib, wl, events=2_000_000, stride=3, sw=sw)
    n, bad = _histories(g, o, max_bad_frac=1e-3)
    ge, oe = g["events"], o["events"]
    assert len(oe) > 500
    assert (ge["gen"] == 0).sum() == (g["n"] + 2) // 3
    G, O = _key(ge), _key(oe)
    if not bad:
        assert set(G) == set(O)
    # records whose photon and every descendant agree: fields and scores
    flipped = set(bad)
    checked = 0
    for key, r in O.items():
        q = G.get(key)
        if q is None or key in flipped:
            continue
        assert (q["p0"], q["p1"], q["p2"], q["zone"], q["gen"]) == (r["p0"], r["p1"], r["p2"], r["zone"], r["gen"])
        assert q["eps"] == pytest.approx(r["eps"], rel=1e-10)
        assert q["w"] == pytest.approx(r["w"], rel=1e-10)
        np.testing.assert_allclose(q["x"], r["x"], rtol=0, atol=1e-10 * max(1.0, np.max(np.abs(r["x"]))))
        if not bad:
            assert q["score"] == pytest.approx(r["score"], rel=1e-9, abs=1e-300)
        checked += 1
    assert checked > 0.99 * len(O)
    # parent links: a scattering record's parent is the record of the photon that scattered
    sc = ge[(ge["gen"] > 0) & (ge["parent"] != gm.NO_EVENT)]
    par = ge[sc["parent"]]
    assert np.array_equal(par["s0"], sc["p0"]) and np.array_equal(par["s2"], sc["p2"])
    assert np.array_equal(par["gen"] + 1, sc["gen"])


def test_hbm_tally_equals_lds_tally(gm):
    """Tallies added to HBM directly equal the per-block LDS tallies up to
    the order of the FP64 sums."""
    wl = W.scattering_sphere(0.1, n_target=200000, seed=27)
    a = run_gpu(gm, wl, tally_mode=1, trace=0)
    b = run_gpu(gm, wl, tally_mode=2, trace=0)
    np.testing.assert_array_equal(a["spec"][..., 2], b["spec"][..., 2])
    np.testing.assert_allclose(a["spec"][..., :2], b["spec"][..., :2], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(a["ledger"], b["ledger"], rtol=1e-12, atol=1e-300)
    np.testing.assert_array_equal(a["stats"], b["stats"])


def test_single_root_overflow_leaves_state_unchanged(gm):
    """A single root whose cascade overflows the photon queue returns
    GM_ENOMEM with the tallies, ledger and trace count as before the call
    and the roots still pending: a second call with room gives the run of
    a fresh context."""
    wl = W.scattering_sphere(0.1, n_target=2000, seed=28).with_track(bias_value=200.0, n_sc_max=2)
    c = gm.Context(0)
    c.load_zones(wl)
    c.make_superphotons(wl.emit)
    c.set_trace(100000)
    c.set_queue_capacity(64)
    with pytest.raises(gm.GmError, match="error -2"):
        c.track_scatter(wl.track)
    spec, led = c.read_spectrum()
    assert not spec.any() and not led.any()
    assert len(c.read_trace()) == 0
    c.set_queue_capacity(0)
    c.track_scatter(wl.track)
    spec2, led2 = c.read_spectrum()
    c.close()
    ref = run_gpu(gm, wl, trace=0)
    np.testing.assert_array_equal(spec2[..., 2], ref["spec"][..., 2])
    np.testing.assert_allclose(spec2[..., 0], ref["spec"][..., 0], rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("field,value", [("n_e", float("nan")), ("theta_e", -1.0), ("ucon", 0.0)])
def test_device_zone_inputs_are_validated(gm, field, value):
    """Zones passed in device memory go through the same checks as host
    zones: a bad one is GM_EINVAL naming it, and nothing is loaded."""
    wl = W.scattering_sphere(0.1, n_target=100, seed=29, n=8)
    bad = dict(n_e=wl.n_e.copy(), theta_e=wl.theta_e.copy(), B=wl.B.copy(), ucon=wl.ucon.copy(), bcon=wl.bcon.copy())
    z = int(np.flatnonzero(wl.n_e > 0)[3])
    if field == "ucon":
        bad["ucon"][0, z] = value
    else:
        bad[field][z] = value
    c = gm.Context(0)
    with pytest.raises(gm.GmError, match="zone %d" % z):
        c.load_zones_device(wl.grid, **bad)
    with pytest.raises(gm.GmError, match="error -4"):
        c.make_superphotons(wl.emit)
    c.load_zones_device(wl.grid, n_e=wl.n_e, theta_e=wl.theta_e, B=wl.B, ucon=wl.ucon, bcon=wl.bcon)
    assert c.make_superphotons(wl.emit) > 0
    c.close()
