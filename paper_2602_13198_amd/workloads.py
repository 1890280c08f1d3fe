"""Seeded synthetic inputs for the superphoton transport.

This module is the only code that both the HIP path and the CPU oracle use.
It builds plasma on a zone grid (density, temperature, field strength, fluid
velocity and field direction) and the parameter dictionaries of a run.  It
holds none of the method's arithmetic: no emissivity, opacity, weights,
sampling or transport.

Workloads
---------
* ``sphere`` -- a uniform synchrotron sphere in flat spacetime on a Cartesian
  voxel grid with partial cells (the paper's test section: optically thin
  sphere, and the scattering sphere).  Boundary cells are subdivided and the
  density is scaled by the fraction of sub-cells inside the sphere; the paper
  does this with 5x5 sub-cells on a 2-D grid, here 5x5x5 on a 3-D grid.
* ``torus`` -- a Fishbone-Moncrief torus around a Kerr black hole on a
  modified Kerr-Schild grid, standing in for the GRMHD snapshot of the paper's
  GRMHD test section (that snapshot is not available): log-normal density and
  internal-energy perturbations, a poloidal single-loop field at a fixed
  gas-to-magnetic pressure ratio, and R-beta electron temperatures.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SIGMA_T = 6.6524587321e-25     # cm^2, for setting a density from a Thomson depth
M_SUN = 1.98847e33
G_NEWTON = 6.6743e-8
C_LIGHT = 2.99792458e10
M_P = 1.67262192369e-24
M_E = 9.1093837015e-28

METRIC_MINKOWSKI_CART = 0
METRIC_KS_MKS = 1

BIAS_CONST, BIAS_THETA2, BIAS_GEN2, BIAS_LEARNED = 0, 1, 2, 3


@dataclass
class Workload:
    name: str
    grid: dict
    n_e: np.ndarray
    theta_e: np.ndarray
    B: np.ndarray
    ucon: np.ndarray          # [4, nz]
    bcon: np.ndarray          # [4, nz]
    emit: dict
    track: dict
    meta: dict = field(default_factory=dict)

    @property
    def n_zones(self) -> int:
        return int(np.prod(self.grid["n"]))

    def with_emit(self, **kw) -> "Workload":
        e = dict(self.emit)
        e.update(kw)
        return Workload(self.name, self.grid, self.n_e, self.theta_e, self.B, self.ucon,
                        self.bcon, e, self.track, dict(self.meta))

    def with_track(self, **kw) -> "Workload":
        t = dict(self.track)
        t.update(kw)
        return Workload(self.name, self.grid, self.n_e, self.theta_e, self.B, self.ucon,
                        self.bcon, self.emit, t, dict(self.meta))


def default_track(**kw) -> dict:
    t = dict(scattering=0, bias_mode=BIAS_CONST, bias_value=1.0, bias_max=1e6, n_sc_max=4,
             step_h=0.25, verlet_tol=1e-3, verlet_max_it=8, roulette_frac=1e-4,
             roulette_p=0.1, horizon_eps=1e-2, max_steps=1000000,
             n_nu=128, nu_lo=1e8, nu_hi=1e24, n_theta=6)
    t.update(kw)
    return t


def sphere_fill(n: int, sub: int = 5) -> np.ndarray:
    """Fraction of each cell of an n^3 grid on [-1,1]^3 inside the unit
    sphere, from sub^3 sub-cell centres.  Returned in row-major zone order."""
    dx = 2.0 / n
    c = -1.0 + (np.arange(n) + 0.5) * dx
    o = (np.arange(sub) + 0.5) / sub - 0.5
    s = (c[:, None] + o[None, :] * dx).reshape(-1)           # n*sub sub-centres
    r2x = s * s
    inside = (r2x[:, None, None] + r2x[None, :, None] + r2x[None, None, :]) < 1.0
    frac = inside.reshape(n, sub, n, sub, n, sub).mean(axis=(1, 3, 5))
    return frac.reshape(-1)


def sphere(n: int = 32, R_cm: float = 1e14, theta_e: float = 10.0, n_e: float = 1e6,
           B: float = 1.0, n_target: float = 1e5, seed: int = 0, nu_min: float = 1e8,
           nu_max: float = 1e14, name: str = "sphere", **track_kw) -> Workload:
    """Uniform synchrotron sphere of radius R filling [-R, R]^3 (ell = R)."""
    f = sphere_fill(n)
    nz = n ** 3
    ne = n_e * f
    th = np.full(nz, float(theta_e))
    Bz = np.full(nz, float(B))
    ucon = np.zeros((4, nz))
    ucon[0] = 1.0
    bcon = np.zeros((4, nz))
    bcon[3] = 1.0
    grid = dict(metric=METRIC_MINKOWSKI_CART, n=[n, n, n], x_start=[-1.0, -1.0, -1.0],
                dx=[2.0 / n] * 3, a_spin=0.0, h_slope=0.0, L_unit_cm=float(R_cm), r_record=0.0)
    emit = dict(n_target=float(n_target), nu_min=nu_min, nu_max=nu_max, n_wnodes=257,
                w_floor_rel=1e-30, seed=int(seed), instance=0)
    return Workload(name, grid, ne, th, Bz, ucon, bcon, emit, default_track(**track_kw),
                    meta=dict(R_cm=R_cm, fill=f, n_e0=n_e, theta_e=theta_e, B=B))


def thin_sphere(n_target=1e5, seed=0, n=32) -> Workload:
    """Optically thin synchrotron sphere: R = 1e14 cm, Theta_e = 10,
    n_e = 1e6 cm^-3, B = 1 G along z, no scattering."""
    return sphere(n=n, theta_e=10.0, n_e=1e6, B=1.0, n_target=n_target, seed=seed,
                  name="thin_sphere")


def strictly_thin_sphere(n_target=1e5, seed=0, n=32) -> Workload:
    """The same sphere with n_e = 1e-6 cm^-3 so that absorption is below
    1e-5 at every frequency (the exactly-thin analytic check)."""
    return sphere(n=n, theta_e=10.0, n_e=1e-6, B=1.0, n_target=n_target, seed=seed,
                  name="strictly_thin_sphere")


def scattering_sphere(tau_T: float = 0.1, n_target=1e6, seed=0, n=32, instance=0) -> Workload:
    """Scattering synchrotron sphere: Theta_e = 4, n_e = tau_T/(sigma_T R),
    B = 1 G, thermal Compton with constant bias b = 1/tau_T, up to four
    scattering generations."""
    R = 1e14
    wl = sphere(n=n, theta_e=4.0, n_e=tau_T / (SIGMA_T * R), B=1.0, n_target=n_target,
                seed=seed, name="scattering_sphere_tau%g" % tau_T, scattering=1,
                bias_mode=BIAS_CONST, bias_value=1.0 / tau_T, n_sc_max=4)
    wl.emit["instance"] = int(instance)
    wl.meta["tau_T"] = tau_T
    return wl
