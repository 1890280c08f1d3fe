"""Integration pins for the oracle's transport: conservation ledgers, the
analytic sphere spectra of the paper's test section, Monte Carlo
convergence, the first-scattering fraction of a uniform sphere, and
determinism of photon histories."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

from paper_2602_13198_amd import workloads as W

ME, CL, HPL, EE, SIGT = 9.1093837015e-28, 2.99792458e10, 6.62607015e-27, 4.80320471e-10, 6.6524587321e-25


def ledger_residuals(res):
    L = res.ledger_dict()
    w_in = L["W_EMIT"] + L["W_ROUL"]
    w_out = L["W_ESC"] + L["W_OOB"] + L["W_ABS"] + L["W_CAPT"] + L["W_CAPLOSS"] + L["W_STUCK"]
    e_in = L["E_EMIT"] + L["E_ROUL"] + L["E_COMPTON"] + L["E_DRIFT"]
    e_out = L["E_ESC"] + L["E_OOB"] + L["E_ABS"] + L["E_CAPT"] + L["E_CAPLOSS"] + L["E_STUCK"]
    return w_in / w_out - 1, e_in / e_out - 1


def jnu_paper(ne, th, B, nu, c):
    s = math.sqrt(max(0.0, 1 - c * c))
    if s == 0:
        return 0.0
    nus = 2 / 9 * (EE * B / (2 * math.pi * ME * CL)) * th**2 * s
    X = nu / nus
    K2 = sp.kv(2, 1 / th)
    return math.sqrt(2) * math.pi * EE**2 * ne * nus / (3 * CL * K2) * \
        (X**0.5 + 2 ** (11 / 12) * X ** (1 / 6)) ** 2 * math.exp(-X ** (1 / 3))


def thin_expectation(wl, track):
    """E[S1] per (theta, nu) bin for an optically thin voxel sphere:
    V_eff * int_bin dnu int_thetabin j dOmega, V_eff = sum f_i dx^3 ell^3
    (eq:Lnu_analytic_thin_test on the voxel model), within the emission band."""
    m = wl.meta
    V = m["fill"].sum() * (2.0 / wl.grid["n"][0]) ** 3 * wl.grid["L_unit_cm"] ** 3
    nb, nt = track["n_nu"], track["n_theta"]
    edges = np.exp(np.linspace(math.log(track["nu_lo"]), math.log(track["nu_hi"]), nb + 1))
    th_edges = np.linspace(0, math.pi, nt + 1)
    E = np.zeros((nt, nb))
    for i in range(nb):
        lo, hi = max(edges[i], wl.emit["nu_min"]), min(edges[i + 1], wl.emit["nu_max"])
        if hi <= lo:
            continue
        for t in range(nt):
            c1, c0 = math.cos(th_edges[t]), math.cos(th_edges[t + 1])
            f = lambda c, lnnu: jnu_paper(m["n_e0"], m["theta_e"], m["B"], math.exp(lnnu), c) * math.exp(lnnu)
            E[t, i] = 2 * math.pi * V * si.dblquad(f, math.log(lo), math.log(hi), c0, c1,
                                                   epsabs=0, epsrel=1e-8)[0]
    return E


def test_ledgers_close(oracle_lib):
    for wl in (W.strictly_thin_sphere(n_target=3000), W.thin_sphere(n_target=3000),
               W.scattering_sphere(0.1, n_target=3000)):
        res, _ = oracle_lib.run(wl)
        wr, er = ledger_residuals(res)
        assert abs(wr) < 1e-12 and abs(er) < 1e-12, wl.name
        st = res.stats_dict()
        assert st["STUCK"] == 0


def test_emission_counts(oracle_lib):
    """Stochastic rounding gives floor or floor+1 per zone and an expected
    total of N_s when the weight floor never binds (band up to 1e12 Hz;
    above ~2e13 Hz the emissivity falls below 1e-30 of its peak and the
    floor removes those frequencies from the count)."""
    wl = W.strictly_thin_sphere(n_target=40000).with_emit(nu_max=1e12)
    o = oracle_lib.Oracle()
    o.load_zones(wl)
    n = o.make_superphotons(wl.emit)
    em = o.read_emission()
    fl = np.floor(em["nbar"])
    assert np.all((em["counts"] == fl) | (em["counts"] == fl + 1))
    assert em["counts"].sum() == n
    assert em["nbar"].sum() == pytest.approx(40000, rel=1e-9)
    assert abs(n - 40000) < 5 * math.sqrt(40000)


def test_thin_sphere_matches_analytic_spectrum(oracle_lib):
    """Optically thin sphere (eq:Lnu_analytic_thin_test): every (theta, nu)
    bin agrees with the analytic expectation within its Monte Carlo error.
    Four seeds pooled, ~600 bins: chi^2/dof has a spread of sqrt(2/600) =
    0.06 about 1, so the bound 1.2 is ~3.5 of those."""
    chi2, dof = 0.0, 0
    for seed in (1, 2, 3, 4):
        wl = W.strictly_thin_sphere(n_target=30000, seed=seed)
        tr = dict(wl.track, n_nu=48, nu_lo=1e8, nu_hi=1e14)
        res, _ = oracle_lib.run(wl.with_track(**tr))
        E = thin_expectation(wl, tr)
        S1, S2, N = res.spectrum[..., 0], res.spectrum[..., 1], res.spectrum[..., 2]
        use = N >= 30
        chi2 += ((S1[use] - E[use]) ** 2 / S2[use]).sum()
        dof += use.sum()
        assert S1.sum() == pytest.approx(E.sum(), rel=5 * math.sqrt(S2.sum()) / S1.sum())
    assert dof >= 480
    assert chi2 / dof < 1.2


def test_convergence_rate(oracle_lib):
    """eq:conv_parameter falls as N_s^-1/2 (thin sphere, theta-summed),
    within 0.05 of that slope."""
    # band kept below ~2e13 Hz, above which the weight floor leaves bins
    # with almost no superphotons at any of these N
    tr = dict(W.default_track(), n_nu=20, nu_lo=1e8, nu_hi=1e13, n_theta=1)
    wl0 = W.strictly_thin_sphere(n_target=1000)
    E = thin_expectation(wl0, tr)[0]
    logs, errs = [], []
    for N in (1000, 4000, 16000, 64000):
        e = []
        for seed in range(6):
            wl = W.strictly_thin_sphere(n_target=N, seed=100 + seed).with_track(**tr)
            res, _ = oracle_lib.run(wl)
            L = res.spectrum[0, :, 0]
            # eq:conv_parameter on bin centres: (1/span) sum |dL|/L dlog10(nu)
            e.append(np.mean(np.abs(E - L) / E))
        logs.append(math.log(N))
        errs.append(math.log(np.mean(e)))
    slope = np.polyfit(logs, errs, 1)[0]
    # six seeds per N: the slope scatters by ~0.015 between seed sets; the
    # emission's stratified counts per zone (floor or floor + 1) make it a
    # little steeper than -1/2 at these N (-0.52 over twelve seeds)
    assert -0.55 < slope < -0.45


def test_any_tau_sphere(oracle_lib):
    """Homogeneous sphere at any optical depth, per direction:
    dL/dOmega = B_nu pi R^2 [1 - (1 - (1 + 2 tau) e^-2tau)/(2 tau^2)],
    tau = R j(theta)/B_nu.  The voxel sphere differs by O(dx/R) where the
    sphere is thick."""
    wl = W.thin_sphere(n_target=80000, seed=2)
    tr = dict(wl.track, n_nu=24, nu_lo=1e8, nu_hi=1e14, n_theta=3)
    res, _ = oracle_lib.run(wl.with_track(**tr))
    R = wl.grid["L_unit_cm"]
    th = wl.meta["theta_e"]
    edges = np.exp(np.linspace(math.log(1e8), math.log(1e14), 25))
    th_edges = np.linspace(0, math.pi, 4)

    def dLdOm(nu, c):
        j = jnu_paper(wl.meta["n_e0"], th, 1.0, nu, c)
        x = HPL * nu / (ME * CL * CL * th)
        Bn = 2 * HPL * nu**3 / CL**2 / math.expm1(x)
        tau = R * j / Bn
        if tau < 1e-4:
            return 4 / 3 * math.pi * R**3 * j
        return Bn * math.pi * R * R * (1 - (1 - (1 + 2 * tau) * math.exp(-2 * tau)) / (2 * tau * tau))

    checked = thick = 0
    for t in range(3):
        for i in range(24):
            N = res.spectrum[t, i, 2]
            if N < 50:
                continue
            checked += 1
            thick += dLdOm(math.sqrt(edges[i] * edges[i + 1]), 0.0) < 0.5 * 4 / 3 * math.pi * R**3 * \
                jnu_paper(wl.meta["n_e0"], th, 1.0, math.sqrt(edges[i] * edges[i + 1]), 0.0)
            c0, c1 = math.cos(th_edges[t + 1]), math.cos(th_edges[t])
            f = lambda c, lnnu: dLdOm(math.exp(lnnu), c) * math.exp(lnnu)
            E = 2 * math.pi * si.dblquad(f, math.log(edges[i]), math.log(edges[i + 1]), c0, c1,
                                         epsrel=1e-6)[0]
            S1, S2 = res.spectrum[t, i, 0], res.spectrum[t, i, 1]
            assert abs(S1 / E - 1) < 0.08 + 5 * math.sqrt(S2) / S1, (t, i)
    assert checked >= 30 and thick >= 6


def test_first_scattering_fraction(oracle_lib):
    """Uniform sphere, Thomson regime, negligible absorption: the weight
    handed to first-generation children is 1 - P_esc(tau_T) of the emitted
    weight, P_esc = 3/(4 tau)[1 - 1/(2 tau^2) + (1/tau + 1/(2 tau^2)) e^-2tau]
    (mean escape probability from a uniform sphere, uniform sources)."""
    tau = 0.1
    # a narrow band keeps the superphoton weights nearly equal, so the
    # weighted fraction has Poisson-like error (~1 % here)
    wl = W.sphere(n=32, theta_e=4.0, n_e=tau / (SIGT * 1e14), B=1e-3, n_target=40000, seed=4,
                  nu_min=1e10, nu_max=1.2e10, scattering=1, bias_mode=W.BIAS_CONST,
                  bias_value=10.0, n_sc_max=1)
    res, _ = oracle_lib.run(wl, trace_cap=10**6)
    tr = res.trace
    child_w = tr["w_birth"][tr["n_sc"] == 1].sum()
    frac = child_w / res.ledger_dict()["W_EMIT"]
    pesc = 3 / (4 * tau) * (1 - 1 / (2 * tau**2) + (1 / tau + 1 / (2 * tau**2)) * math.exp(-2 * tau))
    assert res.ledger_dict()["W_ABS"] < 1e-6 * res.ledger_dict()["W_EMIT"]
    assert frac == pytest.approx(1 - pesc, rel=0.05)


def _sorted(tr):
    return np.sort(tr, order=["s2", "s1", "s0"])


def test_histories_independent_of_threads_and_subsets(oracle_lib):
    wl = W.scattering_sphere(0.1, n_target=1500, seed=3)
    o = oracle_lib.Oracle()
    o.load_zones(wl)
    n = o.make_superphotons(wl.emit)
    t1 = o.track_scatter(wl.track, n_threads=1, trace_cap=10**6)
    r1 = o.read_spectrum(reset=True)
    t4 = o.track_scatter(wl.track, n_threads=4, trace_cap=10**6)
    r4 = o.read_spectrum(reset=True)
    assert np.array_equal(_sorted(t1).view(np.uint8), _sorted(t4).view(np.uint8))
    np.testing.assert_allclose(r4.spectrum, r1.spectrum, rtol=1e-12, atol=0)
    ts = o.track_scatter(wl.track, root_begin=200, root_end=260, trace_cap=10**6)
    full = {r.tobytes() for r in t1}
    assert len(ts) > 60 and all(r.tobytes() in full for r in ts)


def test_corona_sphere_scatters_upward(oracle_lib):
    """The core-and-corona workload: only the magnetised core emits, the
    ledgers close, and each scattering generation escapes at a higher median
    frequency than the one before (inverse Compton in the hot shell), the
    first shift staying below the mean Thomson gain of the shell,
    1 + 4 Theta K3/K2 (Theta = 30)."""
    wl = W.corona_sphere(n_target=3000, seed=1)
    o = oracle_lib.Oracle()
    o.load_zones(wl)
    o.make_superphotons(wl.emit)
    counts = o.read_emission()["counts"]
    assert counts.sum() > 0 and counts[wl.B == 0].sum() == 0
    o.close()
    res, _ = oracle_lib.run(wl, trace_cap=10 ** 6)
    wr, er = ledger_residuals(res)
    assert abs(wr) < 1e-12 and abs(er) < 1e-12
    tr = res.trace
    esc = tr[tr["kind"] == 1]
    med = [np.median(esc["i_nu"][esc["n_sc"] == g]) for g in range(4)]
    assert all(b > a for a, b in zip(med, med[1:])), med
    th = 30.0
    gain = 1 + 4 * th * sp.kv(3, 1 / th) / sp.kv(2, 1 / th)
    dln = math.log10(wl.track["nu_hi"] / wl.track["nu_lo"]) / wl.track["n_nu"]
    assert (med[1] - med[0]) * dln < math.log10(gain), (med, gain)
