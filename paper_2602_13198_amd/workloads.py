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
* ``corona_torus`` -- the torus on a 3-D grid under a hot, field-free
  scattering corona (n_e falling as 1/r, radial Thomson depth 0.1).
* ``survey`` -- many 3-D tori differing in spin, electron-temperature ratio,
  density scale and superphoton count (batched runs of the paper's
  implementation section).
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
METRIC_FLAT_SPH = 2

BIAS_CONST, BIAS_THETA2, BIAS_GEN2, BIAS_TABLE, BIAS_WINDOW = 0, 1, 2, 3, 4
DIST_THERMAL, DIST_POWERLAW = 0, 1
BIAS_LEARNED = BIAS_TABLE


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
    # electrons of every zone: None (thermal at theta_e) or a power law
    # dict(kind=DIST_POWERLAW, p=..., gamma_min=..., gamma_max=...)
    electrons: dict | None = None

    @property
    def n_zones(self) -> int:
        return int(np.prod(self.grid["n"]))

    def outer_plasma_radius(self) -> float:
        """Outer radius of the outermost first-axis zone holding plasma
        (spherical grids, x1 = ln r); the least r_far the far-field step
        rule accepts on this grid (with 4 M)."""
        n1 = self.grid["n"][0]
        rows = np.flatnonzero(self.n_e.reshape(n1, -1).max(axis=1) > 0.0)
        i1 = int(rows[-1]) if len(rows) else -1
        return float(np.exp(self.grid["x_start"][0] + (i1 + 1) * self.grid["dx"][0]))

    def with_far_steps(self, factor: float) -> "Workload":
        """Outgoing photons beyond the plasma (and 4 M) step `factor` times
        further."""
        return self.with_track(step_far=float(factor), r_far=max(self.outer_plasma_radius(), 4.0))

    def with_emit(self, **kw) -> "Workload":
        e = dict(self.emit)
        e.update(kw)
        return Workload(self.name, self.grid, self.n_e, self.theta_e, self.B, self.ucon,
                        self.bcon, e, self.track, dict(self.meta), self.electrons)

    def with_track(self, **kw) -> "Workload":
        t = dict(self.track)
        t.update(kw)
        return Workload(self.name, self.grid, self.n_e, self.theta_e, self.B, self.ucon,
                        self.bcon, self.emit, t, dict(self.meta), self.electrons)


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


def log_r_sphere(n1=8192, n2=128, R_cm=1.0, r_in=1e-2, r_out=1e4, r_record=3000.0, theta_e=100.0,
                 n_e=1e13, B=1.0, n_target=1e5, seed=0, nu_min=1e8, nu_max=None, n_nu=2500, dln_nu=0.01,
                 n_theta=6, sub=5, step_h=2.0, name="log_r_sphere", **track_kw) -> Workload:
    """Uniform synchrotron sphere of radius R on the flat spherical grid of
    the paper's sphere tests: coordinates (t, ln r, theta, phi), n1 x n2 x 1
    zones over r in [r_in, r_out] (cm; ell = 1 cm) and theta uniform in
    [0, pi]; static plasma, vertical field B^z = B, i.e. B^r = B cos theta,
    B^theta = -B sin theta / r; photons recorded at r_record; n_nu bins of
    width dln_nu in ln nu from nu_min (2500 x 0.01 by default) and emission
    over the same band.  Cells that straddle r = R hold n_e times the
    fraction of their sub x sub sub-cells (in x1, x2) whose centres lie
    inside.  The step factor is in zone widths: 2 keeps a step within
    0.34 % of r and 0.05 rad of theta on the 8192 x 128 grid (8 lets the
    polar steps reach 0.2 rad, and photons passing near the axis then miss
    the polar inclination bins by a quarter)."""
    x1a, x1b = math.log(r_in), math.log(r_out)
    dx = [(x1b - x1a) / n1, 1.0 / n2, 2.0 * math.pi]
    if nu_max is None:
        nu_max = nu_min * math.exp(n_nu * dln_nu)
    # fraction of sub-cells inside the sphere, per radial zone
    o = (np.arange(sub) + 0.5) / sub
    r_sub = np.exp(x1a + (np.arange(n1)[:, None] + o[None, :]) * dx[0])
    frac = (r_sub < R_cm).mean(axis=1)
    x2c = (np.arange(n2) + 0.5) * dx[1]
    th = math.pi * x2c
    r_c = np.exp(x1a + (np.arange(n1) + 0.5) * dx[0])
    nz = n1 * n2
    ne = np.repeat(n_e * frac, n2)
    the = np.where(ne > 0, float(theta_e), 0.0)
    Bf = np.where(ne > 0, float(B), 0.0)
    ucon = np.zeros((4, nz))
    ucon[0] = 1.0
    bcon = np.zeros((4, nz))
    # coordinate components in (ln r, x2): b^1 = B^r / r, b^2 = B^theta / (dtheta/dx2)
    bcon[1] = (np.cos(th)[None, :] / r_c[:, None]).reshape(-1)
    bcon[2] = (-np.sin(th)[None, :] / (r_c[:, None] * math.pi)).reshape(-1)
    grid = dict(metric=METRIC_FLAT_SPH, n=[n1, n2, 1], x_start=[x1a, 0.0, 0.0], dx=dx, a_spin=0.0,
                h_slope=1.0, L_unit_cm=1.0, r_record=float(r_record))
    emit = dict(n_target=float(n_target), nu_min=nu_min, nu_max=nu_max, n_wnodes=257,
                w_floor_rel=1e-30, seed=int(seed), instance=0)
    tk = dict(step_h=step_h, n_nu=n_nu, nu_lo=nu_min, nu_hi=nu_min * math.exp(n_nu * dln_nu),
              n_theta=n_theta)
    tk.update(track_kw)
    vol = (4.0 * math.pi / 3.0) * np.sum(frac * (np.exp(x1a + (np.arange(n1) + 1) * dx[0]) ** 3
                                                 - np.exp(x1a + np.arange(n1) * dx[0]) ** 3))
    return Workload(name, grid, ne, the, Bf, ucon, bcon, emit, default_track(**tk),
                    meta=dict(R_cm=R_cm, n_e0=n_e, theta_e=theta_e, B=B, frac=frac, V_eff=vol))


def paper_thin_sphere(n1=8192, n2=128, n_target=1e5, seed=0, **kw) -> Workload:
    """The optically thin synchrotron sphere of the paper's tests: R = 1 cm,
    Theta_e = 100, n_e = 1e13 cm^-3, B = 1 G, 8192 x 128 x 1 log-r grid out
    to 1e4 cm, record at 3000 cm, 2500 bins of 0.01 in ln nu, no scattering."""
    return log_r_sphere(n1=n1, n2=n2, n_target=n_target, seed=seed, name="paper_thin_sphere", **kw)


def paper_scattering_sphere(n1=8192, n2=128, n_target=1e5, seed=0, n_sc_max=4, **kw) -> Workload:
    """The scattering sphere of the paper's tests: the same cloud with
    n_e = 1e18 cm^-3 and Theta_e = 3, thermal Compton with the generation
    bias b = (n_sc + 1)^2 / (n_e sigma_T R) (the printed product inverted,
    so that b >= 1), up to n_sc_max scatterings."""
    R = 1.0
    tau = 1e18 * SIGMA_T * R
    return log_r_sphere(n1=n1, n2=n2, theta_e=3.0, n_e=1e18, n_target=n_target, seed=seed,
                        name="paper_scattering_sphere", scattering=1, bias_mode=BIAS_GEN2,
                        bias_value=R, n_sc_max=n_sc_max, **kw)


def power_law_sphere(n=32, R_cm=1e14, n_e=1.0, B=1.0, p=3.0, gamma_min=10.0, gamma_max=1e5, tau_T=0.0,
                     n_target=1e5, seed=0, nu_min=1e9, nu_max=1e16, bias_value=None, name="power_law_sphere",
                     **track_kw) -> Workload:
    """Uniform sphere of non-thermal electrons (isotropic power law of index
    p on [gamma_min, gamma_max], the same in every zone) on the 32^3
    Cartesian grid of the flat spheres, B along z, static plasma; emission
    over [nu_min, nu_max], inside nu_c(gamma_min) << nu << nu_c(gamma_max)
    where the power law's asymptotic synchrotron forms hold.  tau_T > 0 sets
    n_e = tau_T / (sigma_T R) and turns on Compton scattering off the same
    electrons with a constant bias (1 / tau_T unless given), four
    generations.  Theta_e is set to 1 (unused by a power law except by the
    Theta_e^2 bias)."""
    if tau_T > 0.0:
        n_e = tau_T / (SIGMA_T * R_cm)
        track_kw = dict(dict(scattering=1, bias_mode=BIAS_CONST,
                             bias_value=bias_value if bias_value else 1.0 / tau_T, n_sc_max=4), **track_kw)
    wl = sphere(n=n, R_cm=R_cm, theta_e=1.0, n_e=n_e, B=B, n_target=n_target, seed=seed, nu_min=nu_min,
                nu_max=nu_max, name=name, **track_kw)
    wl.electrons = dict(kind=DIST_POWERLAW, p=float(p), gamma_min=float(gamma_min), gamma_max=float(gamma_max))
    wl.meta.update(p=p, gamma_min=gamma_min, gamma_max=gamma_max, tau_T=tau_T)
    return wl


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


def corona_sphere(n_target=1e6, seed=0, n=32, instance=0, r_core=0.3, theta_core=4.0,
                  tau_core=0.1, B_core=1.0, theta_shell=30.0, tau_shell=0.1, bias_value=10.0) -> Workload:
    """Synchrotron core inside a hot scattering shell (a flat stand-in for an
    accretion flow under a corona): zones whose centre lies within r_core R
    hold the core (Theta_e = theta_core, radial Thomson depth tau_core,
    field B_core along z); zones out to R hold the shell (Theta_e =
    theta_shell, radial Thomson depth tau_shell over its thickness, no
    field, so no emission); beyond R is vacuum.  Static plasma; thermal
    Compton with a constant bias, up to four generations.  The shell's
    inverse-Compton photons populate frequencies the core does not reach."""
    R = 1e14
    wl = sphere(n=n, theta_e=theta_core, n_e=1.0, B=B_core, n_target=n_target, seed=seed,
                name="corona_sphere", scattering=1, bias_mode=BIAS_CONST, bias_value=bias_value,
                n_sc_max=4)
    c = (np.arange(n) + 0.5) * (2.0 / n) - 1.0
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2).reshape(-1)
    core = r < r_core
    shell = (r >= r_core) & (r < 1.0)
    ne = np.zeros(n ** 3)
    ne[core] = tau_core / (SIGMA_T * R * r_core)
    ne[shell] = tau_shell / (SIGMA_T * R * (1.0 - r_core))
    th = np.where(shell, float(theta_shell), float(theta_core))
    Bf = np.where(core, float(B_core), 0.0)
    wl = Workload(wl.name, wl.grid, ne, th, Bf, wl.ucon, wl.bcon, wl.emit, wl.track,
                  meta=dict(R_cm=R, r_core=r_core, theta_core=theta_core, theta_shell=theta_shell,
                            tau_core=tau_core, tau_shell=tau_shell))
    wl.emit["instance"] = int(instance)
    return wl


# ---------------------------------------------------------------------------
# Kerr accretion torus (stands in for the GRMHD snapshot of the paper's GRMHD
# test section)
# ---------------------------------------------------------------------------
def _fm_lnh(r, th, a, l):
    """Fishbone-Moncrief enthalpy of a constant-angular-momentum torus
    (Boyer-Lindquist r, theta; up to an additive constant)."""
    s2 = np.sin(th) ** 2
    S = r * r + a * a * np.cos(th) ** 2
    D = r * r - 2 * r + a * a
    A = (r * r + a * a) ** 2 - D * a * a * s2
    q = np.sqrt(1 + 4 * l * l * S * S * D / (A * A * s2))
    return 0.5 * np.log((1 + q) / (S * D / A)) - 0.5 * q - 2 * a * r * l / A


def _fm_angular_momentum(a, r_max):
    """The l that puts the pressure maximum at r_max on the equator."""
    def dlnh(l, h=1e-4):
        return (_fm_lnh(r_max + h, np.pi / 2, a, l) - _fm_lnh(r_max - h, np.pi / 2, a, l)) / (2 * h)
    lo, hi = 1.0, 20.0
    flo = dlnh(lo)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        fm = dlnh(mid)
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def torus(n1=256, n2=128, n3=1, a=0.9375, h_slope=0.3, r_in=6.0, r_max=12.0, gamma_ad=13.0 / 9.0,
          beta=100.0, R_high=40.0, R_low=1.0, M_bh_sun=6.5e9, M_unit=1e27, perturb=0.05,
          perturb_seed=1, n_target=1e7, seed=3, nu_min=1e8, nu_max=1e16, r_record=1000.0,
          theta_floor=1e-2, name="kerr_torus", **track_kw) -> Workload:
    """Fishbone-Moncrief-shaped torus on a modified Kerr-Schild grid
    (x1 = ln r over [ln(0.9 r_h), ln r_record], theta = pi x2 +
    (1-h)/2 sin(2 pi x2), n3 azimuthal zones).

    Density and internal energy follow the FM enthalpy (polytrope
    p = K rho^gamma, both normalised to the density maximum) times seeded
    log-normal factors exp(s Z - s^2/2).  The fluid rotates on circles with
    angular velocity 1/(R^1.5 + a), R = r sin(theta); ucon gives only the
    direction (1, 0, 0, Omega) and each consumer normalises it with its own
    metric.  The field direction follows a single poloidal loop
    A_phi ~ max(rho/rho_max - 0.2, 0); its strength is set from a uniform
    plasma beta: B^2/(8 pi) = p_gas / beta.  Electron temperature from the
    R-beta prescription Theta_e = (m_p/m_e)(gamma-1)(u/rho)/(1 + R),
    R = (R_high beta^2 + R_low)/(1 + beta^2), floored at theta_floor.  Units: ell = r_g = G M/c^2,
    rho_unit = M_unit / ell^3.

    Transport defaults: scattering bias b = 1e3 Theta_e^2 (the paper's
    Theta_e^2 form; its coefficient 96e4 belongs to a hotter, thinner
    snapshot and here would give b tau_T ~ 300, an exponential cascade of
    generations) and a step factor of half a zone, meant for the full
    256x128 grid: on coarser test grids scale step_h down in proportion."""
    rh = 1.0 + math.sqrt(1.0 - a * a)
    x1a, x1b = math.log(0.9 * rh), math.log(r_record)
    dx = [(x1b - x1a) / n1, 1.0 / n2, 2.0 * math.pi / n3]
    x1 = x1a + (np.arange(n1) + 0.5) * dx[0]
    x2 = (np.arange(n2) + 0.5) * dx[1]
    r = np.exp(x1)[:, None]
    th = (np.pi * x2 + 0.5 * (1 - h_slope) * np.sin(2 * np.pi * x2))[None, :]
    l = _fm_angular_momentum(a, r_max)
    with np.errstate(invalid="ignore", divide="ignore"):      # no torus inside the horizon
        lnh = _fm_lnh(r, th, a, l) - _fm_lnh(r_in, np.pi / 2, a, l)
    lnh = np.nan_to_num(lnh, nan=-1.0)
    inside = (lnh > 0) & (r >= r_in)
    hh = np.where(inside, np.exp(np.where(inside, lnh, 0.0)), 1.0)
    kappa = 1e-3
    rho = np.where(inside, ((hh - 1) * (gamma_ad - 1) / (kappa * gamma_ad)) ** (1 / (gamma_ad - 1)), 0.0)
    uu = kappa * rho ** gamma_ad / (gamma_ad - 1)
    rmax = rho.max()
    rho, uu = rho / rmax, uu / rmax
    # vector potential and poloidal field direction (finite differences in code coordinates)
    Aphi = np.maximum(rho - 0.2, 0.0)
    dA1 = np.gradient(Aphi, dx[0], axis=0)
    dA2 = np.gradient(Aphi, dx[1], axis=1)
    rng = np.random.Generator(np.random.Philox(perturb_seed))
    shape = (n1, n2, n3)
    rho3 = np.repeat(rho[:, :, None], n3, axis=2) * np.exp(perturb * rng.standard_normal(shape) - perturb ** 2 / 2)
    uu3 = np.repeat(uu[:, :, None], n3, axis=2) * np.exp(perturb * rng.standard_normal(shape) - perturb ** 2 / 2)
    L = G_NEWTON * M_bh_sun * M_SUN / C_LIGHT ** 2
    rho_unit = M_unit / L ** 3
    n_e = rho3 * rho_unit / M_P
    p_gas = (gamma_ad - 1) * uu3 * rho_unit * C_LIGHT ** 2
    B = np.sqrt(8 * math.pi * p_gas / beta)
    R = (R_high * beta ** 2 + R_low) / (1 + beta ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        theta_e = np.where(rho3 > 0, (M_P / M_E) * (gamma_ad - 1) * uu3 / rho3 / (1 + R), 0.0)
    # floor: below ~1e-3 the thermal normalisation K2(1/Theta) underflows
    theta_e = np.where(rho3 > 0, np.maximum(theta_e, theta_floor), 0.0)
    has_field = (np.repeat((np.abs(dA1) + np.abs(dA2))[:, :, None], n3, axis=2) > 0)
    B = np.where(has_field, B, 0.0)
    Rc = r * np.sin(th)
    Omega = 1.0 / (Rc ** 1.5 + a)
    nz = n1 * n2 * n3
    ucon = np.zeros((4, nz))
    ucon[0] = 1.0
    ucon[3] = np.repeat(Omega[:, :, None], n3, axis=2).reshape(-1)
    bcon = np.zeros((4, nz))
    bcon[1] = np.repeat(-dA2[:, :, None], n3, axis=2).reshape(-1)
    bcon[2] = np.repeat(dA1[:, :, None], n3, axis=2).reshape(-1)
    grid = dict(metric=METRIC_KS_MKS, n=[n1, n2, n3], x_start=[x1a, 0.0, 0.0], dx=dx, a_spin=a,
                h_slope=h_slope, L_unit_cm=L, r_record=r_record)
    emit = dict(n_target=float(n_target), nu_min=nu_min, nu_max=nu_max, n_wnodes=257,
                w_floor_rel=1e-30, seed=int(seed), instance=0)
    tk = dict(scattering=1, bias_mode=BIAS_THETA2, bias_value=1e3, bias_max=1e6, n_sc_max=4,
              step_h=0.5, n_nu=200, nu_lo=1e8, nu_hi=1e24, n_theta=6)
    tk.update(track_kw)
    return Workload(name, grid, n_e.reshape(-1), theta_e.reshape(-1), B.reshape(-1), ucon, bcon,
                    emit, default_track(**tk),
                    meta=dict(l=l, rho_unit=rho_unit, M_unit=M_unit, r_h=rh, R_high=R_high))


def normal_observer(grid: dict):
    """Direction of the normal observer's 4-velocity in every zone of a
    modified Kerr-Schild grid: u^mu proportional to -g^{mu t} =
    (1 + 2r/Sigma, -2/Sigma, 0, 0) in (t, ln r, x2, phi), Sigma = r^2 +
    a^2 cos^2 theta -- timelike everywhere, inside the ergosphere too
    (consumers normalise it with their own metric)."""
    n1, n2, n3 = grid["n"]
    a, hs = grid["a_spin"], grid["h_slope"]
    x1 = grid["x_start"][0] + (np.arange(n1) + 0.5) * grid["dx"][0]
    x2 = grid["x_start"][1] + (np.arange(n2) + 0.5) * grid["dx"][1]
    r = np.exp(x1)[:, None]
    th = (np.pi * x2 + 0.5 * (1 - hs) * np.sin(2 * np.pi * x2))[None, :]
    sig = r * r + a * a * np.cos(th) ** 2
    u0 = np.repeat((1.0 + 2.0 * r / sig)[:, :, None], n3, axis=2).reshape(-1)
    u1 = np.repeat((-2.0 / sig)[:, :, None], n3, axis=2).reshape(-1)
    return u0, u1


def corona_torus(n1=192, n2=96, n3=96, a=0.9375, R_high=40.0, tau_corona=0.1, theta_corona=1.0,
                 r_corona=40.0, n_target=1e8, seed=5, bias_value=10.0, name="corona_torus", **kw) -> Workload:
    """The 3-D torus (3-D log-normal perturbations) under a scattering
    corona: every zone the torus leaves empty with r_h < r < r_corona holds
    electrons at n_e = n_0 r_g / r, Theta_e = theta_corona, no field (a pure
    scatterer, no emission), moving with the normal observer; n_0 sets the
    radial Thomson depth, n_0 sigma_T r_g ln(r_corona / r_h) = tau_corona.
    The torus emits synchrotron photons that the corona Compton-scatters
    into bands the torus does not reach.  Transport: constant bias b =
    bias_value (1 / tau_corona), four scattering generations."""
    kw.setdefault("step_h", 0.5)
    wl = torus(n1=n1, n2=n2, n3=n3, a=a, R_high=R_high, n_target=n_target, seed=seed, name=name,
               bias_mode=BIAS_CONST, bias_value=bias_value, **kw)
    g = wl.grid
    rh = wl.meta["r_h"]
    L = g["L_unit_cm"]
    x1 = g["x_start"][0] + (np.arange(n1) + 0.5) * g["dx"][0]
    r = np.repeat(np.exp(x1), n2 * n3)
    n0 = tau_corona / (SIGMA_T * L * math.log(r_corona / rh))
    cor = (wl.n_e <= 0.0) & (r > rh) & (r < r_corona)
    n_e = np.where(cor, n0 / r, wl.n_e)
    theta_e = np.where(cor, float(theta_corona), wl.theta_e)
    B = np.where(cor, 0.0, wl.B)
    u0, u1 = normal_observer(g)
    ucon = wl.ucon.copy()
    ucon[0] = np.where(cor, u0, ucon[0])
    ucon[1] = np.where(cor, u1, ucon[1])
    ucon[3] = np.where(cor, 0.0, ucon[3])
    meta = dict(wl.meta, n0=n0, r_corona=r_corona, tau_corona=tau_corona, theta_corona=theta_corona,
                corona=cor)
    return Workload(name, g, n_e, theta_e, B, ucon, wl.bcon, wl.emit, wl.track, meta)


SURVEY_SPINS = (-0.5, 0.0, 0.5, 0.9375)
SURVEY_R_HIGH = (1.0, 10.0, 40.0, 160.0)
# torus radii (r_in, r_max) per spin: with r_in = 6 a retrograde a = -0.5
# torus is empty (its ISCO lies at 7.6)
SURVEY_RADII = {-0.5: (10.0, 20.0), 0.0: (8.0, 16.0), 0.5: (7.0, 14.0), 0.9375: (6.0, 12.0)}


def survey(n1=192, n2=96, n3=96, n_draw=4, M_c=1e27, ns_lo=1e5, ns_hi=1e7, seed=4, step_h=0.5,
           bias_c=1e4, **track_kw):
    """Batched survey: for every spin in SURVEY_SPINS and R_high in
    SURVEY_R_HIGH, n_draw density scales M_unit log-uniform on
    [M_c / 10, 10 M_c] (4 x 4 x 4 = 64 instances by default), each with its
    own N_s log-uniform on [ns_lo, ns_hi] and its own emission seed.  One
    torus structure per spin (shared perturbations); R_high and M_unit only
    rescale it (Theta_e through R-beta, n_e by M_unit, B by sqrt(M_unit)),
    so the instances are built without recomputing the torus.  The
    coefficient c of the bias b = c Theta_e^2 is bias_c (M_c / M_unit)
    ((1 + R) / (1 + R(40)))^2 per instance, which keeps b tau_T where the
    torus is densest and hottest at the value of the R_high = 40,
    M_unit = M_c torus with c = bias_c, so every instance scatters about
    as much (a fixed c would give the hot R_high = 1 tori about a thousand
    scattered superphotons per root, an exponential cascade over the
    generations).  Returns the list of workloads, instance i at emit["instance"] = i."""
    rng = np.random.Generator(np.random.Philox(seed))
    out = []
    i = 0
    for a in SURVEY_SPINS:
        rin, rmax = SURVEY_RADII[a]
        base = torus(n1=n1, n2=n2, n3=n3, a=a, r_in=rin, r_max=rmax, R_high=1.0, M_unit=1.0,
                     step_h=step_h, **track_kw)
        beta = 100.0
        R40 = (40.0 * beta ** 2 + 1.0) / (1 + beta ** 2)
        for rh_ in SURVEY_R_HIGH:
            Rf = (rh_ * beta ** 2 + 1.0) / (1 + beta ** 2)
            R1 = (1.0 * beta ** 2 + 1.0) / (1 + beta ** 2)
            # Theta_e scales as 1/(1 + R) before the floor; the floor is re-applied
            th_raw = np.where(base.n_e > 0, base.theta_e * (1 + R1) / (1 + Rf), 0.0)
            theta_e = np.where(base.n_e > 0, np.maximum(th_raw, 1e-2), 0.0)
            for _ in range(n_draw):
                Mu = M_c * 10.0 ** rng.uniform(-1.0, 1.0)
                ns = 10.0 ** rng.uniform(math.log10(ns_lo), math.log10(ns_hi))
                emit = dict(base.emit, n_target=float(ns), seed=int(1000 + i), instance=i)
                tk = dict(base.track, bias_value=bias_c * (M_c / Mu) * ((1 + Rf) / (1 + R40)) ** 2)
                wl = Workload("survey_%d" % i, base.grid, base.n_e * Mu, theta_e, base.B * math.sqrt(Mu),
                              base.ucon, base.bcon, emit, tk,
                              meta=dict(a=a, R_high=rh_, M_unit=Mu, N_s=ns, r_h=base.meta["r_h"]))
                out.append(wl)
                i += 1
    return out
