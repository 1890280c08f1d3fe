"""ctypes binding of ``include/gm.h`` (argument marshalling only).

Every step of the transport runs in the HIP kernels of ``libgm.so``; this
module converts Python/numpy/torch arguments to the C structs and pointers of
the ABI and back.  Importing it imports torch first so that the library binds
to the same HIP runtime as torch.  It raises if the library is missing: there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime that libgm.so must share)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libgm.so")

GM_MAX_INSTANCES = 64
L_N = 18
S_GEN0 = 16
S_COEF_EVALS = S_GEN0 + 16
S_N = S_GEN0 + 17
LEDGER_NAMES = ["W_EMIT", "E_EMIT", "W_ESC", "E_ESC", "W_OOB", "E_OOB", "W_ABS", "E_ABS",
                "W_CAPT", "E_CAPT", "W_CAPLOSS", "E_CAPLOSS", "W_ROUL", "E_ROUL", "W_STUCK",
                "E_STUCK", "E_COMPTON", "E_DRIFT"]
STAT_NAMES = ["ROOTS", "CHILDREN", "STEPS", "VERLET_IT", "SCATTER", "ROUL_KILL",
              "ROUL_SURVIVE", "CAPTURED", "ESCAPED", "OOB", "STUCK", "OVERSHOOT",
              "NU_TRIALS", "DIR_TRIALS", "E_TRIALS", "ANG_TRIALS"]

TRACE_DTYPE = np.dtype([("s0", "<u4"), ("s1", "<u4"), ("s2", "<u4"), ("n_sc", "<i4"),
                        ("kind", "<i4"), ("i_nu", "<i4"), ("i_theta", "<i4"),
                        ("n_steps", "<u4"), ("w_birth", "<f8"), ("w_end", "<f8"),
                        ("x", "<f8", 4), ("k", "<f8", 4)])
TRACE_BYTES = 112

EVENT_DTYPE = np.dtype([("s0", "<u4"), ("s1", "<u4"), ("s2", "<u4"), ("p0", "<u4"), ("p1", "<u4"),
                        ("p2", "<u4"), ("zone", "<i4"), ("gen", "<i4"), ("parent", "<u4"), ("pad", "<u4"),
                        ("eps", "<f8"), ("w", "<f8"), ("score", "<f8"), ("x", "<f8", 3)])
EVENT_BYTES = 88
assert EVENT_DTYPE.itemsize == EVENT_BYTES
NO_EVENT = 0xFFFFFFFF
MLP_PARAMS = 4738
BIAS_CONST, BIAS_THETA2, BIAS_GEN2, BIAS_TABLE, BIAS_WINDOW = 0, 1, 2, 3, 4
BIAS_LEARNED = BIAS_TABLE
PRECISION_F64, PRECISION_F32_EMISSIVITY = 0, 1
MLP_SQUARED, MLP_POISSON = 0, 1
MLP_NOALLOC_MAX_ROWS = 56640

# Every function the header declares (checked by the CPU symbol test).
EXPORTS = ["gm_create", "gm_destroy", "gm_last_error", "gm_load_zones", "gm_make_superphotons",
           "gm_track_scatter", "gm_read_spectrum", "gm_read_emission", "gm_set_trace",
           "gm_trace_count", "gm_sigma_hot_table", "gm_eval_G", "gm_set_timing",
           "gm_read_timing", "gm_set_tuning", "gm_mlp_set_params", "gm_mlp_get_params",
           "gm_mlp_forward", "gm_mlp_grad", "gm_mlp_train_step", "gm_mlp_train_steps", "gm_set_bias_table",
           "gm_set_event_log", "gm_event_count", "gm_event_band", "gm_set_batch",
           "gm_set_instance_bias", "gm_fma_chain_bound", "gm_set_queue_capacity",
           "gm_queue_stats", "gm_set_emission_table", "gm_set_score_weights", "gm_set_tally_mode",
           "gm_mlp_set_loss", "gm_unload_zones", "gm_mlp_grad_noalloc", "gm_mlp_fill_table",
           "gm_cells_accumulate", "gm_cells_fill_table", "gm_remap_table", "gm_expected_roots", "gm_read_table",
           "gm_set_graph"]


class GmGrid(C.Structure):
    _fields_ = [("metric", C.c_int), ("n", C.c_int * 3), ("x_start", C.c_double * 3),
                ("dx", C.c_double * 3), ("a_spin", C.c_double), ("h_slope", C.c_double),
                ("L_unit_cm", C.c_double), ("r_record", C.c_double)]


class GmElectrons(C.Structure):
    _fields_ = [("kind", C.c_int), ("p", C.c_double), ("gamma_min", C.c_double), ("gamma_max", C.c_double)]


def electrons_struct(el) -> GmElectrons:
    """gm_electrons of a workload's electrons (None: thermal)."""
    if not el:
        return GmElectrons(0, 0.0, 0.0, 0.0)
    return GmElectrons(int(el["kind"]), float(el["p"]), float(el["gamma_min"]), float(el["gamma_max"]))


class GmZones(C.Structure):
    _fields_ = [("on_device", C.c_int), ("n_e", C.c_void_p), ("theta_e", C.c_void_p),
                ("B", C.c_void_p), ("ucon", C.c_void_p), ("bcon", C.c_void_p), ("electrons", GmElectrons)]


class GmEmitParams(C.Structure):
    _fields_ = [("n_target", C.c_double), ("nu_min", C.c_double), ("nu_max", C.c_double),
                ("n_wnodes", C.c_int), ("w_floor_rel", C.c_double), ("seed", C.c_uint64)]


class GmImportanceMap(C.Structure):
    _fields_ = [("table", C.c_int), ("n_nodes", C.c_int), ("lo", C.c_double), ("hi", C.c_double),
                ("kind", C.c_int), ("a", C.c_double), ("b", C.c_double), ("alpha", C.c_double),
                ("shift", C.c_double), ("per_photon", C.c_int)]


TABLE_BIAS, TABLE_EMISSION = 0, 1
IMP_LINEAR, IMP_MIXTURE = 0, 1


class GmTrackParams(C.Structure):
    _fields_ = [("scattering", C.c_int), ("bias_mode", C.c_int), ("bias_value", C.c_double),
                ("bias_max", C.c_double), ("n_sc_max", C.c_int), ("step_h", C.c_double),
                ("verlet_tol", C.c_double), ("verlet_max_it", C.c_int),
                ("roulette_frac", C.c_double), ("roulette_p", C.c_double),
                ("horizon_eps", C.c_double), ("max_steps", C.c_int64), ("n_nu", C.c_int),
                ("nu_lo", C.c_double), ("nu_hi", C.c_double), ("n_theta", C.c_int),
                ("precision", C.c_int), ("step_far", C.c_double), ("r_far", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libgm.so; raises FileNotFoundError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError("libgm.so is not built (%s); run __graft_entry__.build()" % path)
    L = C.CDLL(path)
    vp, i, u64, dp = C.c_void_p, C.c_int, C.c_uint64, C.POINTER(C.c_double)
    sig = {
        "gm_create": (i, [C.POINTER(C.c_void_p), i, vp]),
        "gm_destroy": (i, [vp]),
        "gm_last_error": (C.c_char_p, []),
        "gm_load_zones": (i, [vp, i, C.POINTER(GmGrid), C.POINTER(GmZones)]),
        "gm_make_superphotons": (i, [vp, i, C.POINTER(GmEmitParams), C.POINTER(C.c_uint64)]),
        "gm_track_scatter": (i, [vp, C.POINTER(GmTrackParams), C.POINTER(C.c_int64)]),
        "gm_read_spectrum": (i, [vp, i, vp, i, dp, i]),
        "gm_read_emission": (i, [vp, i, C.POINTER(C.c_uint32), dp, dp, dp]),
        "gm_set_trace": (i, [vp, vp, u64]),
        "gm_trace_count": (i, [vp, C.POINTER(C.c_uint64)]),
        "gm_sigma_hot_table": (i, [vp, dp]),
        "gm_eval_G": (i, [vp, dp, dp, i]),
        "gm_set_timing": (i, [vp, i]),
        "gm_read_timing": (i, [vp, dp, C.POINTER(C.c_uint64)]),
        "gm_set_tuning": (i, [vp, i, i]),
        "gm_mlp_set_params": (i, [vp, vp]),
        "gm_mlp_get_params": (i, [vp, vp]),
        "gm_mlp_forward": (i, [vp, vp, C.c_int64, vp]),
        "gm_mlp_grad": (i, [vp, vp, vp, vp, C.c_int64, vp, vp]),
        "gm_mlp_train_step": (i, [vp, vp, vp, vp, C.c_int64, C.c_float, vp]),
        "gm_mlp_train_steps": (i, [vp, vp, vp, vp, C.c_int64, C.c_int64, i, C.c_float, C.c_float, vp]),
        "gm_set_bias_table": (i, [vp, i, dp, i, C.c_double, C.c_double]),
        "gm_set_event_log": (i, [vp, vp, u64, u64]),
        "gm_event_band": (i, [vp, dp, dp]),
        "gm_set_emission_table": (i, [vp, i, dp, i, C.c_double, C.c_double]),
        "gm_set_score_weights": (i, [vp, i, dp, i]),
        "gm_set_tally_mode": (i, [vp, i]),
        "gm_mlp_set_loss": (i, [vp, i]),
        "gm_unload_zones": (i, [vp, i]),
        "gm_mlp_grad_noalloc": (i, [vp, vp, vp, vp, C.c_int64, vp]),
        "gm_mlp_fill_table": (i, [vp, i, C.POINTER(GmImportanceMap), i, vp, vp]),
        "gm_cells_accumulate": (i, [vp, i, C.POINTER(GmImportanceMap), C.POINTER(C.c_int), dp]),
        "gm_cells_fill_table": (i, [vp, i, C.POINTER(GmImportanceMap), C.c_double]),
        "gm_remap_table": (i, [vp, i, C.POINTER(GmImportanceMap)]),
        "gm_expected_roots": (i, [vp, i, C.POINTER(GmEmitParams), dp]),
        "gm_read_table": (i, [vp, i, i, dp, C.c_int64, C.POINTER(C.c_int)]),
        "gm_set_graph": (i, [vp, i, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
        "gm_event_count": (i, [vp, C.POINTER(C.c_uint64)]),
        "gm_set_batch": (i, [vp, i]),
        "gm_set_instance_bias": (i, [vp, i, i, C.c_double, C.c_double]),
        "gm_fma_chain_bound": (i, [vp, i, i, C.c_int64, dp, dp, dp, i]),
        "gm_set_queue_capacity": (i, [vp, u64]),
        "gm_queue_stats": (i, [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class GmError(RuntimeError):
    pass


def _check(rc: int):
    if rc != 0:
        raise GmError("gm error %d: %s" % (rc, load_library().gm_last_error().decode()))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def grid_struct(g: dict) -> GmGrid:
    G = GmGrid()
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


def emit_struct(e: dict) -> GmEmitParams:
    return GmEmitParams(float(e["n_target"]), float(e["nu_min"]), float(e["nu_max"]),
                        int(e.get("n_wnodes", 257)), float(e.get("w_floor_rel", 1e-30)),
                        int(e.get("seed", 0)))


def track_struct(t: dict) -> GmTrackParams:
    T = GmTrackParams()
    T.scattering = int(t.get("scattering", 0))
    T.bias_mode = int(t.get("bias_mode", 0))
    T.bias_value = float(t.get("bias_value", 1.0))
    T.bias_max = float(t.get("bias_max", 1e6))
    T.n_sc_max = int(t.get("n_sc_max", 4))
    T.step_h = float(t.get("step_h", 0.25))
    T.step_far = float(t.get("step_far", 0.0))
    T.r_far = float(t.get("r_far", 0.0))
    T.verlet_tol = float(t.get("verlet_tol", 1e-3))
    T.verlet_max_it = int(t.get("verlet_max_it", 8))
    T.roulette_frac = float(t.get("roulette_frac", 1e-4))
    T.roulette_p = float(t.get("roulette_p", 0.1))
    T.horizon_eps = float(t.get("horizon_eps", 1e-2))
    T.max_steps = int(t.get("max_steps", 1000000))
    T.n_nu = int(t["n_nu"])
    T.nu_lo = float(t["nu_lo"])
    T.nu_hi = float(t["nu_hi"])
    T.n_theta = int(t["n_theta"])
    T.precision = int(t.get("precision", 0))
    return T


class Context:
    """A gm_ctx on one device, queuing on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        L = load_library()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        _check(L.gm_create(C.byref(h), int(device), C.c_void_p(stream.cuda_stream)))
        self._h = h
        self.device = device
        self._trace = None
        self.shapes = {}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().gm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the four calls of the hot path ------------------------------------
    def load_zones(self, wl, instance: int = 0):
        arrs = [np.ascontiguousarray(a, dtype=np.float64)
                for a in (wl.n_e, wl.theta_e, wl.B, wl.ucon, wl.bcon)]
        Z = GmZones(0, *[a.ctypes.data for a in arrs], electrons_struct(getattr(wl, "electrons", None)))
        G = grid_struct(wl.grid)
        _check(load_library().gm_load_zones(self._h, int(instance), C.byref(G), C.byref(Z)))
        self.shapes[instance] = int(np.prod(wl.grid["n"]))

    def load_zones_device(self, grid: dict, n_e, theta_e, B, ucon, bcon, instance: int = 0, electrons=None):
        """gm_load_zones with the zone arrays in device memory (copied to
        float64 cuda tensors first when given as host arrays)."""
        dev = "cuda:%d" % self.device
        ts = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(dev) if not torch.is_tensor(a)
              else a.to(device=dev, dtype=torch.float64).contiguous()
              for a in (n_e, theta_e, B, ucon, bcon)]
        Z = GmZones(1, *[t.data_ptr() for t in ts], electrons_struct(electrons))
        G = grid_struct(grid)
        _check(load_library().gm_load_zones(self._h, int(instance), C.byref(G), C.byref(Z)))
        self.shapes[instance] = int(np.prod(grid["n"]))

    def expected_roots(self, emit: dict, instance: int = 0) -> float:
        """Expected roots of a make with these parameters (nothing drawn)."""
        P = emit_struct(emit)
        v = C.c_double(0.0)
        _check(load_library().gm_expected_roots(self._h, int(instance), C.byref(P), C.byref(v)))
        return v.value

    def unload(self, instance: int = 0):
        """Free an instance's device memory."""
        _check(load_library().gm_unload_zones(self._h, int(instance)))
        self.shapes.pop(instance, None)

    def make_superphotons(self, emit: dict, instance: int = 0, sync: bool = True) -> int | None:
        P = emit_struct(emit)
        self.n_wnodes = P.n_wnodes
        n = C.c_uint64(0)
        _check(load_library().gm_make_superphotons(self._h, int(instance), C.byref(P),
                                                   C.byref(n) if sync else None))
        return int(n.value) if sync else None

    def track_scatter(self, track: dict, stats: bool = True):
        T = track_struct(track)
        self.n_nu, self.n_theta = T.n_nu, T.n_theta
        st = np.zeros(S_N, np.int64)
        _check(load_library().gm_track_scatter(
            self._h, C.byref(T), st.ctypes.data_as(C.POINTER(C.c_int64)) if stats else None))
        return st if stats else None

    def read_spectrum(self, instance: int = 0, reset: bool = False, out=None):
        """Host numpy [n_theta, n_nu, 3] (or a device torch tensor `out`) and the ledger."""
        led = np.zeros(L_N)
        if out is None:
            spec = np.zeros((self.n_theta, self.n_nu, 3))
            _check(load_library().gm_read_spectrum(self._h, int(instance), C.c_void_p(spec.ctypes.data),
                                                   0, _dp(led), int(reset)))
            return spec, led
        assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
        assert out.numel() == self.n_theta * self.n_nu * 3
        _check(load_library().gm_read_spectrum(self._h, int(instance), C.c_void_p(out.data_ptr()),
                                               1, _dp(led), int(reset)))
        return out, led

    def reset_spectrum(self, instance: int = 0):
        """Clear an instance's tally and ledger; an instance never tracked
        has none, and nothing is done."""
        if not hasattr(self, "n_theta"):
            return
        try:
            self.read_spectrum(instance, reset=True)
        except GmError as exc:
            if "error -4" not in str(exc):
                raise

    # -- inspection ---------------------------------------------------------
    def read_emission(self, instance: int = 0):
        nz = self.shapes[instance]
        counts = np.zeros(nz, np.uint32)
        nbar, fmax = np.zeros(nz), np.zeros(nz)
        lnw = np.zeros(self.n_wnodes)
        _check(load_library().gm_read_emission(self._h, int(instance),
                                               counts.ctypes.data_as(C.POINTER(C.c_uint32)),
                                               _dp(nbar), _dp(fmax), _dp(lnw)))
        return dict(counts=counts, nbar=nbar, fmax=fmax, ln_w=lnw)

    def set_trace(self, capacity: int):
        if capacity <= 0:
            self._trace = None
            _check(load_library().gm_set_trace(self._h, None, 0))
            return
        self._trace = torch.empty(capacity * TRACE_BYTES, dtype=torch.uint8,
                                  device="cuda:%d" % self.device)
        _check(load_library().gm_set_trace(self._h, C.c_void_p(self._trace.data_ptr()), int(capacity)))

    def trace_count(self) -> int:
        """Finished photons counted by the trace (also those past its capacity)."""
        n = C.c_uint64(0)
        _check(load_library().gm_trace_count(self._h, C.byref(n)))
        return int(n.value)

    def read_trace_subset(self, keys) -> np.ndarray:
        """Trace records whose stream (s0 | s1 << 32) is in `keys`, selected
        on the device (for traces too large to copy whole)."""
        cap = self._trace.numel() // TRACE_BYTES
        m = min(self.trace_count(), cap)
        rec = self._trace[: m * TRACE_BYTES].view(m, TRACE_BYTES)
        w = rec.view(torch.int32)[:, :2].to(torch.int64)
        k = (w[:, 0] & 0xFFFFFFFF) | (w[:, 1] << 32)
        want = torch.as_tensor(np.asarray(keys, dtype=np.uint64).view(np.int64), device=rec.device)
        sel = rec[torch.isin(k, want)]
        return sel.cpu().numpy().reshape(-1).view(TRACE_DTYPE).copy()

    def read_trace(self) -> np.ndarray:
        n = C.c_uint64(0)
        _check(load_library().gm_trace_count(self._h, C.byref(n)))
        cap = self._trace.numel() // TRACE_BYTES
        m = min(int(n.value), cap)
        raw = self._trace[: m * TRACE_BYTES].cpu().numpy()
        return raw.view(TRACE_DTYPE).copy()

    def set_event_log(self, capacity: int, root_stride: int = 0):
        """Event records of scatterings, and of the emission of every
        root_stride-th root (0: none), into a device buffer of `capacity`."""
        if capacity <= 0:
            self._evlog = None
            _check(load_library().gm_set_event_log(self._h, None, 0, 0))
            return
        self._evlog = torch.empty(capacity * EVENT_BYTES, dtype=torch.uint8,
                                  device="cuda:%d" % self.device)
        _check(load_library().gm_set_event_log(self._h, C.c_void_p(self._evlog.data_ptr()), int(capacity),
                                               int(root_stride)))

    def read_event_log(self) -> np.ndarray:
        n = C.c_uint64(0)
        _check(load_library().gm_event_count(self._h, C.byref(n)))
        cap = self._evlog.numel() // EVENT_BYTES
        m = min(int(n.value), cap)
        raw = self._evlog[: m * EVENT_BYTES].cpu().numpy()       # a fresh host copy
        return raw.view(EVENT_DTYPE)

    def event_band(self):
        """(eps_min, eps_max) of the event log's emission records, m_e c^2."""
        lo, hi = C.c_double(0.0), C.c_double(0.0)
        _check(load_library().gm_event_band(self._h, C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    # ---- learned form: the network ----
    def mlp_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_PARAMS
        _check(load_library().gm_mlp_set_params(self._h, C.c_void_p(p.ctypes.data)))

    def mlp_set_loss(self, kind: int):
        """0: weighted squared error; 1: log-link Poisson deviance."""
        _check(load_library().gm_mlp_set_loss(self._h, int(kind)))

    def mlp_get_params(self) -> np.ndarray:
        p = np.zeros(MLP_PARAMS, np.float32)
        _check(load_library().gm_mlp_get_params(self._h, C.c_void_p(p.ctypes.data)))
        return p

    @staticmethod
    def _dev_rows(a, width):
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)) if not torch.is_tensor(a) else a
        t = t.to(device="cuda", dtype=torch.float32).contiguous()
        assert t.dim() == 2 and t.shape[1] == width
        return t

    def mlp_forward(self, X):
        """X: [n][8] (numpy or torch); returns a device tensor [n][2]."""
        Xd = self._dev_rows(X, 8)
        Y = torch.empty((Xd.shape[0], 2), dtype=torch.float32, device=Xd.device)
        _check(load_library().gm_mlp_forward(self._h, C.c_void_p(Xd.data_ptr()), int(Xd.shape[0]),
                                             C.c_void_p(Y.data_ptr())))
        return Y

    def mlp_grad(self, X, T, Cw):
        Xd, Td, Cd = self._dev_rows(X, 8), self._dev_rows(T, 2), self._dev_rows(Cw, 2)
        g = np.zeros(MLP_PARAMS, np.float32)
        L = np.zeros(1, np.float32)
        _check(load_library().gm_mlp_grad(self._h, C.c_void_p(Xd.data_ptr()), C.c_void_p(Td.data_ptr()),
                                          C.c_void_p(Cd.data_ptr()), int(Xd.shape[0]),
                                          C.c_void_p(g.ctypes.data), C.c_void_p(L.ctypes.data)))
        return g, float(L[0])

    def mlp_grad_noalloc(self, Xd, Td, Cd, out):
        """gm_mlp_grad_noalloc on device tensors: `out` (float32, device,
        MLP_PARAMS + 1 entries) receives the gradient and the loss; nothing
        is allocated and nothing synchronised."""
        assert out.is_cuda and out.dtype == torch.float32 and out.numel() == MLP_PARAMS + 1 and out.is_contiguous()
        _check(load_library().gm_mlp_grad_noalloc(self._h, C.c_void_p(Xd.data_ptr()), C.c_void_p(Td.data_ptr()),
                                                  C.c_void_p(Cd.data_ptr()), int(Xd.shape[0]),
                                                  C.c_void_p(out.data_ptr())))
        return out

    def mlp_train_step(self, Xd, Td, Cd, lr: float, want_loss: bool = False):
        """One Adam step on device tensors (see _dev_rows); returns the loss
        before the step when asked (synchronises then)."""
        L = np.zeros(1, np.float32)
        _check(load_library().gm_mlp_train_step(self._h, C.c_void_p(Xd.data_ptr()), C.c_void_p(Td.data_ptr()),
                                                C.c_void_p(Cd.data_ptr()), int(Xd.shape[0]), float(lr),
                                                C.c_void_p(L.ctypes.data) if want_loss else None))
        return float(L[0]) if want_loss else None

    def mlp_train_steps(self, Xd, Td, Cd, batch: int, steps: int, lr0: float, decay: float,
                        want_loss: bool = False):
        """`steps` Adam steps in one library call over consecutive batches of
        the rows as given; returns (loss before the first, before the last
        step) when asked (synchronises then)."""
        L = np.zeros(2, np.float32)
        _check(load_library().gm_mlp_train_steps(self._h, C.c_void_p(Xd.data_ptr()), C.c_void_p(Td.data_ptr()),
                                                 C.c_void_p(Cd.data_ptr()), int(Xd.shape[0]), int(batch),
                                                 int(steps), float(lr0), float(decay),
                                                 C.c_void_p(L.ctypes.data) if want_loss else None))
        return (float(L[0]), float(L[1])) if want_loss else None

    def set_bias_table(self, instance: int, ln_b, ln_eps_lo: float, ln_eps_hi: float):
        t = np.ascontiguousarray(ln_b, dtype=np.float64)
        _check(load_library().gm_set_bias_table(self._h, int(instance), _dp(t), int(t.shape[1]),
                                                float(ln_eps_lo), float(ln_eps_hi)))

    def set_emission_table(self, instance: int, table, ln_nu_lo: float = 0.0, ln_nu_hi: float = 1.0):
        """Per-zone emission modulation [nz][n] in ln nu (None removes it)."""
        if table is None:
            _check(load_library().gm_set_emission_table(self._h, int(instance), None, 0, 0.0, 0.0))
            return
        t = np.ascontiguousarray(table, dtype=np.float64)
        _check(load_library().gm_set_emission_table(self._h, int(instance), _dp(t), int(t.shape[1]),
                                                    float(ln_nu_lo), float(ln_nu_hi)))

    def set_score_weights(self, instance: int, sw):
        """Score weights [n_theta][n_nu] of the event records (None: 1)."""
        if sw is None:
            _check(load_library().gm_set_score_weights(self._h, int(instance), None, 0))
            return
        a = np.ascontiguousarray(sw, dtype=np.float64).reshape(-1)
        _check(load_library().gm_set_score_weights(self._h, int(instance), _dp(a), int(a.size)))

    def set_tally_mode(self, mode: int):
        """0 automatic, 1 per-block LDS tallies, 2 direct HBM tallies."""
        _check(load_library().gm_set_tally_mode(self._h, int(mode)))

    @staticmethod
    def importance_map(table, n_nodes, lo, hi, kind=IMP_LINEAR, a=1.0, b=0.0, alpha=0.0, shift=0.0,
                       per_photon=0):
        return GmImportanceMap(int(table), int(n_nodes), float(lo), float(hi), int(kind), float(a), float(b),
                               float(alpha), float(shift), int(per_photon))

    def mlp_fill_table(self, instance, imap, output, mu, sd):
        m = np.ascontiguousarray(mu, dtype=np.float32)
        s = np.ascontiguousarray(sd, dtype=np.float32)
        _check(load_library().gm_mlp_fill_table(self._h, int(instance), C.byref(imap), int(output),
                                                C.c_void_p(m.ctypes.data), C.c_void_p(s.ctypes.data)))

    def cells_accumulate(self, instance, imap, blocks=(8, 8, 8)):
        """(sum score, sum weight, records) of the event log's records for the map's table."""
        b = (C.c_int * 3)(*[int(x) for x in blocks])
        tot = np.zeros(3)
        _check(load_library().gm_cells_accumulate(self._h, int(instance), C.byref(imap), b, _dp(tot)))
        return tot

    def read_table(self, instance, table):
        """The instance's bias (0) or emission (1) table, [nz][nodes]."""
        nz = self.shapes[instance]
        nn = C.c_int(0)
        _check(load_library().gm_read_table(self._h, int(instance), int(table), None, 0, C.byref(nn)))
        buf = np.zeros(nz * nn.value)
        _check(load_library().gm_read_table(self._h, int(instance), int(table), _dp(buf), buf.size, None))
        return buf.reshape(nz, nn.value)

    def remap_table(self, instance, imap):
        """The instance's table (imap.table) mapped in place, values taken as ln I."""
        _check(load_library().gm_remap_table(self._h, int(instance), C.byref(imap)))

    def cells_fill_table(self, instance, imap, prior=20.0):
        _check(load_library().gm_cells_fill_table(self._h, int(instance), C.byref(imap), float(prior)))

    def sigma_hot_table(self) -> np.ndarray:
        t = np.zeros((64, 256))
        _check(load_library().gm_sigma_hot_table(self._h, _dp(t)))
        return t

    def set_tuning(self, track_waves: int = 2, refill_min: int = 8):
        _check(load_library().gm_set_tuning(self._h, int(track_waves), int(refill_min)))

    def set_instance_bias(self, instance: int, track: dict | None):
        """Per-instance bias from a track dict (bias_mode, bias_value,
        bias_max); None removes the override."""
        if track is None:
            _check(load_library().gm_set_instance_bias(self._h, int(instance), -1, 0.0, 0.0))
            return
        _check(load_library().gm_set_instance_bias(self._h, int(instance), int(track.get("bias_mode", 0)),
                                                   float(track.get("bias_value", 1.0)),
                                                   float(track.get("bias_max", 1e6))))

    def set_graph(self, enable: int):
        """1: launch each root chunk as a captured HIP graph; 0: directly;
        -1: no change.  Returns (graph launches, instantiations) so far."""
        a, b = C.c_uint64(0), C.c_uint64(0)
        _check(load_library().gm_set_graph(self._h, int(enable), C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def set_batch(self, max_instances: int):
        _check(load_library().gm_set_batch(self._h, int(max_instances)))

    def set_timing(self, enable: bool = True):
        _check(load_library().gm_set_timing(self._h, int(enable)))

    def read_timing(self):
        """(summed tracking-kernel event time in ms, number of launches)."""
        ms, n = C.c_double(0.0), C.c_uint64(0)
        _check(load_library().gm_read_timing(self._h, C.byref(ms), C.byref(n)))
        return ms.value, int(n.value)

    def set_queue_capacity(self, entries: int = 0):
        """Fix the photon-queue capacity (entries; 0 = automatic)."""
        _check(load_library().gm_set_queue_capacity(self._h, int(entries)))

    def queue_stats(self):
        """(capacity of the last track call, chunks redone after an overflow)."""
        cap, n = C.c_uint64(0), C.c_uint64(0)
        _check(load_library().gm_queue_stats(self._h, C.byref(cap), C.byref(n)))
        return int(cap.value), int(n.value)

    def fma_chain_bound(self, waves: int, chains: int, iters: int, n_out: int = 0):
        """(ms, TFLOP/s, sums of the first n_out lanes) of the FP64 FMA-chain
        kernel at `waves` waves per SIMD with `chains` chains per lane."""
        ms, tf = C.c_double(0.0), C.c_double(0.0)
        out = np.zeros(max(n_out, 1))
        _check(load_library().gm_fma_chain_bound(self._h, int(waves), int(chains), int(iters), C.byref(ms),
                                                 C.byref(tf), _dp(out) if n_out else None, int(n_out)))
        return ms.value, tf.value, out[:n_out]

    def eval_G(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        _check(load_library().gm_eval_G(self._h, _dp(x), _dp(y), int(x.size)))
        return y
