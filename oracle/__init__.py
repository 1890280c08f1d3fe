"""Plain CPU oracle for grmonty-style superphoton Monte Carlo transport.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with ``paper_2602_13198_amd`` and never imports it; both sides only take
inputs from :mod:`paper_2602_13198_amd.workloads` (seeded input generators
that hold none of the method's arithmetic).

The C sources (``gmo_*.c``) are compiled with gcc into ``liboracle.so`` next
to this file; this module is a thin ctypes wrapper around them.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ["gmo_physics.c", "gmo_spacetime.c", "gmo_transport.c"]
_HEADERS = ["gmo.h", "gmo_internal.h"]
LIB_PATH = os.path.join(_HERE, "liboracle.so")

SH_NT, SH_NE = 64, 256
L_N = 18
S_GEN0, MAX_GEN = 16, 16
S_N = S_GEN0 + MAX_GEN

LEDGER_NAMES = ["W_EMIT", "E_EMIT", "W_ESC", "E_ESC", "W_OOB", "E_OOB", "W_ABS", "E_ABS",
                "W_CAPT", "E_CAPT", "W_CAPLOSS", "E_CAPLOSS", "W_ROUL", "E_ROUL", "W_STUCK",
                "E_STUCK", "E_COMPTON", "E_DRIFT"]
STAT_NAMES = ["ROOTS", "CHILDREN", "STEPS", "VERLET_IT", "SCATTER", "ROUL_KILL",
              "ROUL_SURVIVE", "CAPTURED", "ESCAPED", "OOB", "STUCK", "OVERSHOOT",
              "NU_TRIALS", "DIR_TRIALS", "E_TRIALS", "ANG_TRIALS"]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (no fast-math, no FMA contraction)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    deps = srcs + [os.path.join(_HERE, h) for h in _HEADERS]
    if not force and os.path.exists(LIB_PATH):
        t = os.path.getmtime(LIB_PATH)
        if all(os.path.getmtime(d) <= t for d in deps):
            return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


# ---------------------------------------------------------------------------
# ctypes mirrors of gmo.h
# ---------------------------------------------------------------------------
class Grid(C.Structure):
    _fields_ = [("metric", C.c_int), ("n", C.c_int * 3), ("x_start", C.c_double * 3),
                ("dx", C.c_double * 3), ("a_spin", C.c_double), ("h_slope", C.c_double),
                ("L_unit_cm", C.c_double), ("r_record", C.c_double)]


class Dist(C.Structure):
    _fields_ = [("kind", C.c_int), ("p", C.c_double), ("g1", C.c_double), ("g2", C.c_double)]


def make_dist(el) -> Dist:
    """Electron distribution of a workload (None: thermal)."""
    if not el:
        return Dist(0, 0.0, 0.0, 0.0)
    return Dist(int(el["kind"]), float(el["p"]), float(el["gamma_min"]), float(el["gamma_max"]))


class Zones(C.Structure):
    _fields_ = [("n_e", C.c_void_p), ("theta_e", C.c_void_p), ("B", C.c_void_p),
                ("ucon", C.c_void_p), ("bcon", C.c_void_p), ("dist", Dist)]


class EmitParams(C.Structure):
    _fields_ = [("n_target", C.c_double), ("nu_min", C.c_double), ("nu_max", C.c_double),
                ("n_wnodes", C.c_int), ("w_floor_rel", C.c_double), ("seed", C.c_uint64),
                ("instance", C.c_int)]


class TrackParams(C.Structure):
    _fields_ = [("scattering", C.c_int), ("bias_mode", C.c_int), ("bias_value", C.c_double),
                ("bias_max", C.c_double), ("n_sc_max", C.c_int), ("step_h", C.c_double),
                ("verlet_tol", C.c_double), ("verlet_max_it", C.c_int),
                ("roulette_frac", C.c_double), ("roulette_p", C.c_double),
                ("horizon_eps", C.c_double), ("max_steps", C.c_int64), ("n_nu", C.c_int),
                ("nu_lo", C.c_double), ("nu_hi", C.c_double), ("n_theta", C.c_int),
                ("step_far", C.c_double), ("r_far", C.c_double)]


TRACE_DTYPE = np.dtype([("s0", "<u4"), ("s1", "<u4"), ("s2", "<u4"), ("n_sc", "<i4"),
                        ("kind", "<i4"), ("i_nu", "<i4"), ("i_theta", "<i4"),
                        ("n_steps", "<u4"), ("w_birth", "<f8"), ("w_end", "<f8"),
                        ("x", "<f8", 4), ("k", "<f8", 4)])
assert TRACE_DTYPE.itemsize == 112

EVENT_DTYPE = np.dtype([("s0", "<u4"), ("s1", "<u4"), ("s2", "<u4"), ("p0", "<u4"), ("p1", "<u4"),
                        ("p2", "<u4"), ("zone", "<i4"), ("gen", "<i4"), ("eps", "<f8"),
                        ("w", "<f8"), ("score", "<f8"), ("x", "<f8", 3)])
assert EVENT_DTYPE.itemsize == 80

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        d, i, u32p, u64 = C.c_double, C.c_int, C.POINTER(C.c_uint32), C.c_uint64
        dp = C.POINTER(C.c_double)
        sig = {
            "gmo_philox4x32_10": (None, [u32p, u32p, u32p]),
            "gmo_uniform_at": (d, [u64, u32p, C.c_uint32]),
            "gmo_child_stream": (None, [u64, u32p, C.c_uint32, u32p]),
            "gmo_k2": (d, [d]), "gmo_k2_of_theta": (d, [d]), "gmo_g_of_X": (d, [d]),
            "gmo_G_of_Xc": (d, [d]), "gmo_nu_c": (d, [d, d]), "gmo_A_coef": (d, [d, d, d]),
            "gmo_jnu": (d, [d, d, d, d, d]), "gmo_Jnu": (d, [d, d, d, d]),
            "gmo_planck": (d, [d, d]), "gmo_sigma_kn": (d, [d]),
            "gmo_sigma_hot_direct": (d, [d, d]), "gmo_sigma_hot_table": (None, [dp]),
            "gmo_sigma_hot_lookup": (d, [dp, d, d]),
            "gmo_sample_scatter_frame": (None, [u64, u32p, u32p, d, d, dp, dp, dp,
                                                C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
            "gmo_sample_electron": (None, [u64, u32p, u32p, d, d, dp, dp,
                                           C.POINTER(C.c_int64)]),
            "gmo_pl_jnu": (d, [C.POINTER(Dist), d, d, d, d]),
            "gmo_pl_Jnu": (d, [C.POINTER(Dist), d, d, d]),
            "gmo_pl_nualpha": (d, [C.POINTER(Dist), d, d, d, d]),
            "gmo_sigma_pl_direct": (d, [C.POINTER(Dist), d]),
            "gmo_sample_scatter_frame_dist": (None, [u64, u32p, u32p, C.POINTER(Dist), d, d, dp, dp, dp,
                                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
            "gmo_gcov": (None, [C.POINTER(Grid), dp, dp]),
            "gmo_gcon": (None, [C.POINTER(Grid), dp, dp]),
            "gmo_christoffel": (None, [C.POINTER(Grid), dp, dp]),
            "gmo_sqrt_neg_g": (d, [C.POINTER(Grid), dp]),
            "gmo_integrate_geodesic": (i, [C.POINTER(Grid), dp, dp, d, d, i, i, d, d, dp]),
            "gmo_create": (C.c_void_p, []), "gmo_destroy": (None, [C.c_void_p]),
            "gmo_load_zones": (i, [C.c_void_p, C.POINTER(Grid), C.POINTER(Zones)]),
            "gmo_make_superphotons": (i, [C.c_void_p, C.POINTER(EmitParams),
                                          C.POINTER(C.c_uint64)]),
            "gmo_read_emission": (i, [C.c_void_p, u32p, dp, dp, dp]),
            "gmo_track_scatter": (i, [C.c_void_p, C.POINTER(TrackParams), u64, u64, i,
                                      C.c_void_p, u64, C.POINTER(C.c_uint64)]),
            "gmo_read_spectrum": (i, [C.c_void_p, dp, dp, C.POINTER(C.c_int64), i]),
            "gmo_last_error": (C.c_char_p, []),
            "gmo_set_bias_table": (i, [C.c_void_p, dp, i, d, d]),
            "gmo_set_emission_table": (i, [C.c_void_p, dp, i, d, d]),
            "gmo_set_event_log": (i, [C.c_void_p, C.c_void_p, u64, u64]),
            "gmo_event_count": (i, [C.c_void_p, C.POINTER(C.c_uint64)]),
            "gmo_set_score_weights": (i, [C.c_void_p, dp, i]),
            "gmo_table_value": (d, [C.c_void_p, i, i, d]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _u32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    return a, a.ctypes.data_as(C.POINTER(C.c_uint32))


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle error %d: %s" % (rc, lib().gmo_last_error().decode()))


# ---------------------------------------------------------------------------
# primitives
# ---------------------------------------------------------------------------
def philox(ctr, key):
    c, cp = _u32(ctr)
    k, kp = _u32(key)
    o = np.zeros(4, np.uint32)
    lib().gmo_philox4x32_10(cp, kp, o.ctypes.data_as(C.POINTER(C.c_uint32)))
    return o


def uniform_at(seed, stream, block):
    s, sp = _u32(stream)
    return lib().gmo_uniform_at(seed, sp, block)


def child_stream(seed, parent, block):
    s, sp = _u32(parent)
    o = np.zeros(3, np.uint32)
    lib().gmo_child_stream(seed, sp, block, o.ctypes.data_as(C.POINTER(C.c_uint32)))
    return o


def k2(x): return lib().gmo_k2(x)
def k2_of_theta(t): return lib().gmo_k2_of_theta(t)
def g_of_X(X): return lib().gmo_g_of_X(X)
def G_of_Xc(X): return lib().gmo_G_of_Xc(X)
def nu_c(t, B): return lib().gmo_nu_c(t, B)
def A_coef(n, t, B): return lib().gmo_A_coef(n, t, B)
def jnu(n, t, B, nu, c): return lib().gmo_jnu(n, t, B, nu, c)
def Jnu(n, t, B, nu): return lib().gmo_Jnu(n, t, B, nu)
def planck(nu, t): return lib().gmo_planck(nu, t)
def sigma_kn(e): return lib().gmo_sigma_kn(e)
def sigma_hot_direct(t, e): return lib().gmo_sigma_hot_direct(t, e)


def sigma_hot_table() -> np.ndarray:
    t = np.zeros((SH_NT, SH_NE))
    lib().gmo_sigma_hot_table(_dp(t))
    return t


def sigma_hot_lookup(table, theta, eps):
    t = np.ascontiguousarray(table, dtype=np.float64)
    return lib().gmo_sigma_hot_lookup(_dp(t), theta, eps)


def sample_scatter_frame(seed, stream, block, theta, eps):
    """One scattering of a photon of fluid-frame energy eps along +x.
    Returns (gamma, mu, k_out[4], next_block, e_trials, ang_trials)."""
    s, sp = _u32(stream)
    b = np.array([block], np.uint32)
    g, m = C.c_double(), C.c_double()
    k = np.zeros(4)
    et, at = C.c_int64(0), C.c_int64(0)
    lib().gmo_sample_scatter_frame(seed, sp, b.ctypes.data_as(C.POINTER(C.c_uint32)), theta,
                                   eps, C.byref(g), C.byref(m), _dp(k), C.byref(et), C.byref(at))
    return g.value, m.value, k, int(b[0]), et.value, at.value


def pl_jnu(el, n, B, nu, c): return lib().gmo_pl_jnu(C.byref(make_dist(el)), n, B, nu, c)
def pl_Jnu(el, n, B, nu): return lib().gmo_pl_Jnu(C.byref(make_dist(el)), n, B, nu)
def pl_nualpha(el, n, B, nu, c): return lib().gmo_pl_nualpha(C.byref(make_dist(el)), n, B, nu, c)
def sigma_pl_direct(el, e): return lib().gmo_sigma_pl_direct(C.byref(make_dist(el)), e)


def sample_scatter_frame_dist(seed, stream, block, el, theta, eps):
    """sample_scatter_frame with the electrons of el (None: thermal)."""
    s, sp = _u32(stream)
    b = np.array([block], np.uint32)
    g, m = C.c_double(), C.c_double()
    k = np.zeros(4)
    et, at = C.c_int64(0), C.c_int64(0)
    D = make_dist(el)
    lib().gmo_sample_scatter_frame_dist(seed, sp, b.ctypes.data_as(C.POINTER(C.c_uint32)), C.byref(D), theta,
                                        eps, C.byref(g), C.byref(m), _dp(k), C.byref(et), C.byref(at))
    return g.value, m.value, k, int(b[0]), et.value, at.value


def sample_electron(seed, stream, block, theta, eps):
    s, sp = _u32(stream)
    b = np.array([block], np.uint32)
    g, m = C.c_double(), C.c_double()
    t = C.c_int64(0)
    lib().gmo_sample_electron(seed, sp, b.ctypes.data_as(C.POINTER(C.c_uint32)), theta, eps,
                              C.byref(g), C.byref(m), C.byref(t))
    return g.value, m.value, int(b[0]), t.value


def make_grid(g: dict) -> Grid:
    G = Grid()
    G.metric = int(g["metric"])
    for j in range(3):
        G.n[j] = int(g["n"][j])
        G.x_start[j] = float(g["x_start"][j])
        G.dx[j] = float(g["dx"][j])
    G.a_spin = float(g.get("a_spin", 0.0))
    G.h_slope = float(g.get("h_slope", 0.0))
    G.L_unit_cm = float(g["L_unit_cm"])
    G.r_record = float(g.get("r_record", 0.0))
    return G


def gcov(grid: dict, x):
    G = make_grid(grid)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros((4, 4))
    lib().gmo_gcov(C.byref(G), _dp(xx), _dp(out))
    return out


def gcon(grid: dict, x):
    G = make_grid(grid)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros((4, 4))
    lib().gmo_gcon(C.byref(G), _dp(xx), _dp(out))
    return out


def christoffel(grid: dict, x):
    G = make_grid(grid)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros((4, 4, 4))
    lib().gmo_christoffel(C.byref(G), _dp(xx), _dp(out))
    return out


def sqrt_neg_g(grid: dict, x):
    G = make_grid(grid)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    return lib().gmo_sqrt_neg_g(C.byref(G), _dp(xx))


def integrate_geodesic(grid: dict, x0, k0, h=0.5, tol=1e-3, max_it=8, n=10000, r_min=0.0,
                       r_max=1e300):
    """States (x, k) after each step: array [steps, 8]."""
    G = make_grid(grid)
    x = np.ascontiguousarray(x0, dtype=np.float64)
    k = np.ascontiguousarray(k0, dtype=np.float64)
    out = np.zeros((n, 8))
    m = lib().gmo_integrate_geodesic(C.byref(G), _dp(x), _dp(k), h, tol, max_it, n, r_min, r_max,
                                     _dp(out))
    return out[:m]


# ---------------------------------------------------------------------------
# the method
# ---------------------------------------------------------------------------
@dataclass
class Result:
    spectrum: np.ndarray        # [n_theta, n_nu, 3]
    ledger: np.ndarray          # [L_N]
    stats: np.ndarray           # [S_N] int64
    trace: np.ndarray | None    # TRACE_DTYPE records

    def ledger_dict(self):
        return dict(zip(LEDGER_NAMES, self.ledger))

    def stats_dict(self):
        d = dict(zip(STAT_NAMES, self.stats[:len(STAT_NAMES)]))
        d["GEN"] = self.stats[S_GEN0:S_GEN0 + MAX_GEN]
        return d


class Oracle:
    """One oracle context holding one loaded workload."""

    def __init__(self):
        self._c = lib().gmo_create()
        self._keep = []

    def close(self):
        if self._c:
            lib().gmo_destroy(self._c)
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_zones(self, wl):
        G = make_grid(wl.grid)
        arrs = [np.ascontiguousarray(a, dtype=np.float64)
                for a in (wl.n_e, wl.theta_e, wl.B, wl.ucon, wl.bcon)]
        Z = Zones(*[a.ctypes.data for a in arrs], make_dist(getattr(wl, "electrons", None)))
        _check(lib().gmo_load_zones(self._c, C.byref(G), C.byref(Z)))
        self.nz = int(np.prod(wl.grid["n"]))
        self.grid = wl.grid

    def make_superphotons(self, emit: dict) -> int:
        P = EmitParams(float(emit["n_target"]), float(emit["nu_min"]), float(emit["nu_max"]),
                       int(emit.get("n_wnodes", 257)), float(emit.get("w_floor_rel", 1e-30)),
                       int(emit.get("seed", 0)), int(emit.get("instance", 0)))
        self.n_wnodes = P.n_wnodes
        n = C.c_uint64(0)
        _check(lib().gmo_make_superphotons(self._c, C.byref(P), C.byref(n)))
        self.n_roots = int(n.value)
        return self.n_roots

    def read_emission(self):
        counts = np.zeros(self.nz, np.uint32)
        nbar, fmax = np.zeros(self.nz), np.zeros(self.nz)
        lnw = np.zeros(self.n_wnodes)
        _check(lib().gmo_read_emission(self._c, counts.ctypes.data_as(C.POINTER(C.c_uint32)),
                                       _dp(nbar), _dp(fmax), _dp(lnw)))
        return dict(counts=counts, nbar=nbar, fmax=fmax, ln_w=lnw)

    def track_scatter(self, track: dict, root_begin=0, root_end=None, n_threads=0,
                      trace_cap=0):
        T = track_params(track)
        self.n_nu, self.n_theta = T.n_nu, T.n_theta
        if root_end is None:
            root_end = self.n_roots
        tr = np.zeros(trace_cap, TRACE_DTYPE) if trace_cap else None
        tn = C.c_uint64(0)
        _check(lib().gmo_track_scatter(self._c, C.byref(T), int(root_begin), int(root_end),
                                       int(n_threads), tr.ctypes.data if tr is not None else None,
                                       int(trace_cap), C.byref(tn)))
        return tr[:tn.value] if tr is not None else None

    def set_bias_table(self, table, lo, hi):
        """Per-zone table [nz][n] in ln eps for the TABLE and WINDOW bias
        modes (None removes it)."""
        if table is None:
            _check(lib().gmo_set_bias_table(self._c, None, 0, 0.0, 0.0))
            return
        t = np.ascontiguousarray(table, dtype=np.float64)
        self._btab = t
        _check(lib().gmo_set_bias_table(self._c, _dp(t), int(t.shape[1]), float(lo), float(hi)))

    def set_emission_table(self, table, lo, hi):
        """Per-zone modulation [nz][n] in ln nu of the emission weights
        (None removes it); takes effect at the next make."""
        if table is None:
            _check(lib().gmo_set_emission_table(self._c, None, 0, 0.0, 0.0))
            return
        t = np.ascontiguousarray(table, dtype=np.float64)
        _check(lib().gmo_set_emission_table(self._c, _dp(t), int(t.shape[1]), float(lo), float(hi)))

    def table_value(self, which, zone, v):
        return lib().gmo_table_value(self._c, int(which), int(zone), float(v))

    def set_event_log(self, capacity, root_stride=1):
        if capacity <= 0:
            self._ev = None
            _check(lib().gmo_set_event_log(self._c, None, 0, 0))
            return
        self._ev = np.zeros(int(capacity), EVENT_DTYPE)
        _check(lib().gmo_set_event_log(self._c, self._ev.ctypes.data, int(capacity), int(root_stride)))

    def read_event_log(self):
        n = C.c_uint64(0)
        _check(lib().gmo_event_count(self._c, C.byref(n)))
        return self._ev[:min(int(n.value), len(self._ev))].copy()

    def set_score_weights(self, sw):
        if sw is None:
            _check(lib().gmo_set_score_weights(self._c, None, 0))
            return
        a = np.ascontiguousarray(sw, dtype=np.float64).reshape(-1)
        _check(lib().gmo_set_score_weights(self._c, _dp(a), int(a.size)))

    def read_spectrum(self, reset=False) -> Result:
        spec = np.zeros((self.n_theta, self.n_nu, 3))
        led = np.zeros(L_N)
        st = np.zeros(S_N, np.int64)
        _check(lib().gmo_read_spectrum(self._c, _dp(spec), _dp(led),
                                       st.ctypes.data_as(C.POINTER(C.c_int64)), int(reset)))
        return Result(spec, led, st, None)


def track_params(track: dict) -> TrackParams:
    T = TrackParams()
    T.scattering = int(track.get("scattering", 0))
    T.bias_mode = int(track.get("bias_mode", 0))
    T.bias_value = float(track.get("bias_value", 1.0))
    T.bias_max = float(track.get("bias_max", 1e6))
    T.n_sc_max = int(track.get("n_sc_max", 4))
    T.step_h = float(track.get("step_h", 0.25))
    T.step_far = float(track.get("step_far", 0.0))
    T.r_far = float(track.get("r_far", 0.0))
    T.verlet_tol = float(track.get("verlet_tol", 1e-3))
    T.verlet_max_it = int(track.get("verlet_max_it", 8))
    T.roulette_frac = float(track.get("roulette_frac", 1e-4))
    T.roulette_p = float(track.get("roulette_p", 0.1))
    T.horizon_eps = float(track.get("horizon_eps", 1e-2))
    T.max_steps = int(track.get("max_steps", 1000000))
    T.n_nu = int(track["n_nu"])
    T.nu_lo = float(track["nu_lo"])
    T.nu_hi = float(track["nu_hi"])
    T.n_theta = int(track["n_theta"])
    return T


def run(wl, root_begin=0, root_end=None, n_threads=0, trace_cap=0):
    """Load, make, track and read one workload.  Returns (Result, emission dict)."""
    o = Oracle()
    o.load_zones(wl)
    o.make_superphotons(wl.emit)
    em = o.read_emission()
    tr = o.track_scatter(wl.track, root_begin, root_end, n_threads, trace_cap)
    res = o.read_spectrum()
    res.trace = tr
    em["n_roots"] = o.n_roots
    o.close()
    return res, em
