"""Seeded synthetic workloads for the transport step.

This module only builds INPUTS: grid edges, the background fluid/metric state,
opacities, equilibrium occupations and initial occupations, drawn from a
SplitMix64 stream.  It contains none of the transport method's arithmetic (no
quadrature, geometry, remap, flux or collision code); both the GPU library and
the CPU reference receive exactly these arrays.

The five recipes stand in for the paper's analytic tests and its core-collapse
application (which needs a progenitor, a hydro code and opacity tables that
are not available): power-law density, temperature and infall profiles with a
seeded shock and seeded angular perturbations, in the momentum-space
resolutions the paper uses (12-24 logarithmic energy groups, Gauss-Lobatto mu
nodes times uniform Phi bins).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED = 20030245

GEOM_COLUMN, GEOM_AXISYM2D, GEOM_PLANAR = 0, 1, 2
BC_REFLECT, BC_OUTFLOW, BC_EQUIL = 0, 1, 2
PHI_SIN, PHI_LINEAR = 0, 1
THETA_AXIS, THETA_DISK = 0, 1
PREC_FP64, PREC_MIXED = 0, 1


class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood 2014) with 53-bit uniform doubles."""

    MASK = (1 << 64) - 1

    def __init__(self, seed: int):
        self.state = seed & self.MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & self.MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & self.MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & self.MASK
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def integer(self, lo: int, hi: int) -> int:
        """uniform integer in [lo, hi]"""
        return lo + int(self.uniform() * (hi - lo + 1)) if hi > lo else lo


@dataclass
class Workload:
    name: str
    geometry: int
    n_r: int
    n_theta: int
    n_eps: int
    n_mu: int
    n_phi: int
    n_species: int
    mu_rule: str                 # "legendre" or "lobatto"
    r_edges: np.ndarray
    theta_edges: np.ndarray
    dphi: float
    eps_edges: np.ndarray
    v_r: np.ndarray              # [zone]
    v_theta: np.ndarray          # [zone]
    alpha: np.ndarray            # [zone]
    psi: np.ndarray              # [zone]
    kappa_a: np.ndarray          # [zone][species][eps]
    kappa_s: np.ndarray
    f_eq: np.ndarray
    f0: np.ndarray               # [zone][species][eps][dir]
    n_steps: int
    precision: int = PREC_FP64
    cfl: float = 0.4
    inner_bc: int = BC_REFLECT
    outer_bc: int = BC_OUTFLOW
    phi_rule: int = PHI_SIN
    theta_bc: int = THETA_AXIS
    disk_radius: float = 0.0
    n_phi_zones: int = 1             # > 1: 3D, phi zones of width dphi, periodic
    v_phi: Optional[np.ndarray] = None   # [zone] azimuthal fluid velocity (None: 0)
    meta: dict = field(default_factory=dict)

    @property
    def n_zones(self) -> int:
        return self.n_r * self.n_theta * self.n_phi_zones

    @property
    def n_dir(self) -> int:
        return self.n_mu * self.n_phi

    @property
    def block(self) -> int:
        return self.n_species * self.n_eps * self.n_dir

    @property
    def n_values(self) -> int:
        return self.n_zones * self.block


def fermi_dirac(eps, T, eta=0.0):
    return 1.0 / (np.exp(eps / T - eta) + 1.0)


def log_edges(lo, hi, n):
    return lo * (hi / lo) ** (np.arange(n + 1) / n)


def _centres(edges):
    return 0.5 * (edges[:-1] + edges[1:])


def _group_energies(eps_edges):
    # background quantities are sampled at the geometric group centre
    return np.sqrt(eps_edges[:-1] * eps_edges[1:])


def _assemble(name, geometry, r_edges, theta_edges, dphi, eps_edges, n_mu, n_phi,
              mu_rule, v_r, v_th, alpha, psi, ka, ks, feq, f0_iso, n_steps, precision,
              **kw):
    n_r = len(r_edges) - 1
    n_theta = len(theta_edges) - 1 if geometry == GEOM_AXISYM2D else 1
    n_eps = len(eps_edges) - 1
    n_species = ka.shape[1]
    n_dir = n_mu * n_phi
    nz = n_r * n_theta
    if f0_iso:
        f0 = np.repeat(feq[:, :, :, None], n_dir, axis=3).copy()
    else:
        f0 = np.zeros((nz, n_species, n_eps, n_dir))
    return Workload(name=name, geometry=geometry, n_r=n_r, n_theta=n_theta, n_eps=n_eps,
                    n_mu=n_mu, n_phi=n_phi, n_species=n_species, mu_rule=mu_rule,
                    r_edges=np.asarray(r_edges, float), theta_edges=np.asarray(theta_edges, float),
                    dphi=float(dphi), eps_edges=np.asarray(eps_edges, float),
                    v_r=np.ascontiguousarray(v_r, float), v_theta=np.ascontiguousarray(v_th, float),
                    alpha=np.ascontiguousarray(alpha, float), psi=np.ascontiguousarray(psi, float),
                    kappa_a=np.ascontiguousarray(ka, float), kappa_s=np.ascontiguousarray(ks, float),
                    f_eq=np.ascontiguousarray(feq, float), f0=np.ascontiguousarray(f0, float),
                    n_steps=n_steps, precision=precision, **kw)


# --------------------------------------------------------------------------
# 1: homogeneous radiating sphere (Sec. 4.1 analogue), spherical symmetry
# --------------------------------------------------------------------------
def radiating_sphere(n_r=64, n_eps=8, n_mu=16, n_phi=4, r_max=3.0, R=1.0, kappa=10.0,
                     T=5.0, n_steps=200, mu_rule="legendre"):
    r_edges = np.linspace(0.0, r_max, n_r + 1)
    eps_edges = log_edges(1.0, 100.0, n_eps)
    e = _group_energies(eps_edges)
    rc = _centres(r_edges)
    inside = rc < R
    ka = np.where(inside[:, None, None], kappa, 0.0) * np.ones((n_r, 1, n_eps))
    feq = np.where(inside[:, None, None], fermi_dirac(e, T)[None, None, :], 0.0)
    z = np.zeros(n_r)
    return _assemble("radiating_sphere", GEOM_COLUMN, r_edges, np.array([0.0, math.pi]), 0.0,
                     eps_edges, n_mu, n_phi, mu_rule, z, z, np.ones(n_r), np.ones(n_r),
                     ka, np.zeros_like(ka), feq, False, n_steps, PREC_FP64,
                     meta={"R": R, "kappa_a": kappa, "T": T})


def radiating_sphere_2d(n_r=100, n_theta=32, n_mu=16, n_phi=8, r_min=0.02, r_max=4.0, R=1.0,
                        kappa=10.0, mu_rule="lobatto"):
    """The homogeneous radiating sphere on the axisymmetric grid (Sec. 4.5.1):
    one group, f_eq = 1 and kappa_a = kappa inside R, vacuum outside, static
    flat background, logarithmic radial zones from r_min (specular inner
    boundary), uniform theta zones over [0, pi]."""
    r_edges = log_edges(r_min, r_max, n_r)
    theta_edges = np.linspace(0.0, math.pi, n_theta + 1)
    rc = np.tile(_centres(r_edges), n_theta)
    nz = n_r * n_theta
    inside = (rc < R)[:, None, None]
    ka = np.where(inside, kappa, 0.0) * np.ones((nz, 1, 1))
    feq = np.where(inside, 1.0, 0.0) * np.ones((nz, 1, 1))
    z = np.zeros(nz)
    return _assemble("radiating_sphere_2d", GEOM_AXISYM2D, r_edges, theta_edges, math.pi / n_theta,
                     np.array([1.0, 2.0]), n_mu, n_phi, mu_rule, z, z, np.ones(nz), np.ones(nz),
                     ka, np.zeros_like(ka), feq, False, 0, PREC_FP64,
                     meta={"R": R, "kappa_a": kappa})


def radiating_disk(n_r=100, n_theta=32, n_mu=16, n_phi=8, r_min=0.05, r_max=4.0, R=1.0,
                   mu_rule="lobatto"):
    """A geometrically thin, optically thick disk radiating into vacuum (Sec.
    4.5.2): theta over [0, pi/2], the equatorial plane an isotropic f_eq = 1
    emitter inside R and empty outside, kappa = 0 everywhere, one group,
    static flat background, logarithmic radial zones from r_min."""
    r_edges = log_edges(r_min, r_max, n_r)
    theta_edges = np.linspace(0.0, 0.5 * math.pi, n_theta + 1)
    nz = n_r * n_theta
    zero = np.zeros((nz, 1, 1))
    z = np.zeros(nz)
    w = _assemble("radiating_disk", GEOM_AXISYM2D, r_edges, theta_edges, 0.5 * math.pi / n_theta,
                  np.array([1.0, 2.0]), n_mu, n_phi, mu_rule, z, z, np.ones(nz), np.ones(nz),
                  zero, zero.copy(), np.ones((nz, 1, 1)), False, 0, PREC_FP64, meta={"R": R})
    w.theta_bc = THETA_DISK
    w.disk_radius = float(R)
    return w


def radial_slab(w, a0, n):
    """radial zones a0 .. a0+n-1 of every theta row (and phi zone) of a
    workload, as a workload of its own: the share of one GPU of a radially
    decomposed grid, its two-zone halos included.  Pure data slicing."""
    import copy as _copy
    v = _copy.copy(w)
    nz_row = w.n_r
    keep = np.array([z for z in range(w.n_zones) if a0 <= z % nz_row < a0 + n])
    for name in ("v_r", "v_theta", "alpha", "psi", "kappa_a", "kappa_s", "f_eq", "f0"):
        setattr(v, name, np.ascontiguousarray(getattr(w, name)[keep]))
    if w.v_phi is not None:
        v.v_phi = np.ascontiguousarray(w.v_phi[keep])
    v.r_edges = np.ascontiguousarray(w.r_edges[a0:a0 + n + 1])
    v.n_r = n
    v.name = w.name + f"_slab{a0}+{n}"
    return v


def extrude_phi(w, n_phi_zones):
    """The 3D grid of n_phi_zones copies of an axisymmetric workload's wedge
    around the axis (phi zones of the wedge's width, periodic): every
    per-zone array repeated for each phi zone, zone index (c n_theta + b) n_r + a."""
    import copy as _copy
    assert w.geometry == GEOM_AXISYM2D and w.n_phi_zones == 1
    v = _copy.copy(w)
    rep = lambda a: np.ascontiguousarray(np.concatenate([a] * n_phi_zones, axis=0))
    for name in ("v_r", "v_theta", "alpha", "psi", "kappa_a", "kappa_s", "f_eq", "f0"):
        setattr(v, name, rep(getattr(w, name)))
    v.v_phi = rep(w.v_phi) if w.v_phi is not None else np.zeros(w.n_zones * n_phi_zones)
    v.n_phi_zones = int(n_phi_zones)
    v.name = w.name + f"_3d{n_phi_zones}"
    return v


# --------------------------------------------------------------------------
# 2/3/5: axisymmetric CCSN-like profiles
# --------------------------------------------------------------------------
def _ccsn_background(rc, thc, e, n_theta, rng, species_scale, shock=None, modes=None,
                     v_pert=0.05):
    """rho, T, v_r, alpha for zones (theta-major) of an axisymmetric grid"""
    n_r = len(rc)
    u_b = np.array([rng.uniform(-1.0, 1.0) for _ in range(n_theta)])
    R = np.tile(rc, n_theta)
    TH = np.repeat(thc, n_r)
    rho = 1e14 * (R / 10.0) ** -3
    v = -0.1 * (R / 100.0) ** -0.5
    if shock is not None:
        D, J, r_s = shock
        out = R >= r_s
        rho = np.where(out, rho / D, rho)
        v = np.where(out, v * J, v * 0.25)
    if modes is not None:
        a = np.asarray(modes)
        pl = np.polynomial.legendre.legval(np.cos(TH), np.concatenate([[0.0], a]))
        rho = rho * (1.0 + 0.1 * pl / np.sum(np.abs(a)))
    v = v * (1.0 + v_pert * np.repeat(u_b, n_r))
    T = 10.0 * (R / 10.0) ** -0.5
    alpha = 1.0 - 0.2 * (10.0 / R)
    psi = alpha ** -0.5
    base = 1e-3 * (rho / 1e12)[:, None] * (e[None, :] / 10.0) ** 2
    sc = np.asarray(species_scale, float)
    ka = base[:, None, :] * sc[None, :, None]
    ks = 2.0 * ka
    feq = np.repeat(fermi_dirac(e[None, :], T[:, None])[:, None, :], len(sc), axis=1)
    return v, alpha, psi, ka, ks, feq


def axisym_2d(n_r=256, n_theta=64, n_eps=16, n_mu=8, n_phi=8, n_steps=100, seed_offset=1,
              r_min=10.0, r_max=1000.0, e_min=2.0, e_max=200.0):
    rng = SplitMix64(SEED + seed_offset)
    r_edges = log_edges(r_min, r_max, n_r)
    theta_edges = np.linspace(0.0, math.pi, n_theta + 1)
    eps_edges = log_edges(e_min, e_max, n_eps)
    e = _group_energies(eps_edges)
    v, alpha, psi, ka, ks, feq = _ccsn_background(_centres(r_edges), _centres(theta_edges), e,
                                                  n_theta, rng, [1.0])
    return _assemble("axisym_2d", GEOM_AXISYM2D, r_edges, theta_edges, math.pi / n_theta,
                     eps_edges, n_mu, n_phi, "lobatto", v, np.zeros_like(v), alpha, psi, ka, ks,
                     feq, True, n_steps, PREC_FP64)


def shock_2d(n_r=550, n_theta=128, n_eps=21, n_mu=10, n_phi=8, n_steps=100, seed_offset=2,
             precision=PREC_MIXED, modes=False, name="shock_2d", e_max=300.0):
    rng = SplitMix64(SEED + seed_offset)
    r_edges = log_edges(10.0, 1000.0, n_r)
    theta_edges = np.linspace(0.0, math.pi, n_theta + 1)
    eps_edges = log_edges(2.0, e_max, n_eps)
    e = _group_energies(eps_edges)
    D = rng.uniform(4.0, 10.0)
    J = rng.uniform(1.5, 2.5)
    a = [rng.uniform(-1.0, 1.0) for _ in range(8)] if modes else None
    v, alpha, psi, ka, ks, feq = _ccsn_background(_centres(r_edges), _centres(theta_edges), e,
                                                  n_theta, rng, [1.0, 0.7, 0.3],
                                                  shock=(D, J, 150.0), modes=a)
    return _assemble(name, GEOM_AXISYM2D, r_edges, theta_edges, math.pi / n_theta,
                     eps_edges, n_mu, n_phi, "lobatto", v, np.zeros_like(v), alpha, psi, ka, ks,
                     feq, True, n_steps, precision,
                     meta={"shock_D": D, "shock_J": J, "modes": a})


def hires_2d(n_r=600, n_theta=256, n_eps=24, n_mu=12, n_phi=8, n_steps=50, precision=PREC_MIXED):
    return shock_2d(n_r=n_r, n_theta=n_theta, n_eps=n_eps, n_mu=n_mu, n_phi=n_phi,
                    n_steps=n_steps, seed_offset=5, precision=precision, modes=True,
                    name="hires_2d")


# --------------------------------------------------------------------------
# 4: batch of independent spherically symmetric models of uneven sizes
# --------------------------------------------------------------------------
def batch_models(n_models=64, n_steps=100, size_scale=1.0, seed_offset=4):
    rng = SplitMix64(SEED + seed_offset)
    models = []
    for m in range(n_models):
        n_r = max(4, int(round(rng.integer(100, 600) * size_scale)))
        n_eps = rng.integer(12, 24)
        n_dir = 16 + 4 * rng.integer(0, 8)
        n_phi = 4
        n_mu = n_dir // n_phi
        p = rng.uniform(2.5, 3.5)
        q = rng.uniform(0.3, 0.7)
        v0 = 0.2 * (1.0 - rng.uniform())          # (0, 0.2]
        r_edges = log_edges(10.0, 1000.0, n_r)
        eps_edges = log_edges(2.0, 200.0, n_eps)
        e = _group_energies(eps_edges)
        rc = _centres(r_edges)
        rho = 1e14 * (rc / 10.0) ** -p
        T = 10.0 * (rc / 10.0) ** -q
        v = -v0 * (rc / 10.0) ** -0.5
        alpha = 1.0 - 0.2 * (10.0 / rc)
        psi = alpha ** -0.5
        ka = (1e-3 * (rho / 1e12)[:, None] * (e[None, :] / 10.0) ** 2)[:, None, :]
        ks = 2.0 * ka
        feq = fermi_dirac(e[None, :], T[:, None])[:, None, :]
        models.append(_assemble(f"batch_{m}", GEOM_COLUMN, r_edges, np.array([0.0, math.pi]), 0.0,
                                eps_edges, n_mu, n_phi, "lobatto", v, np.zeros_like(v), alpha,
                                psi, ka, ks, feq, True, n_steps, PREC_MIXED,
                                meta={"p": p, "q": q, "v0": v0}))
    return models


def planar(n_z=100, z_min=-1.0, z_max=1.0, n_eps=1, n_mu=8, n_phi=1, kappa_a=0.0, kappa_s=0.0,
           f_eq=0.0, n_steps=10, mu_rule="legendre", inner_bc=BC_OUTFLOW, outer_bc=BC_OUTFLOW,
           v=0.0, alpha=1.0):
    """slab geometry (tests only): the paper's planar diffusion wave set-up"""
    z_edges = np.linspace(z_min, z_max, n_z + 1)
    eps_edges = log_edges(1.0, 2.0, n_eps) if n_eps > 1 else np.array([1.0, 2.0])
    ka = np.full((n_z, 1, n_eps), float(kappa_a))
    ks = np.full((n_z, 1, n_eps), float(kappa_s))
    feq = np.full((n_z, 1, n_eps), float(f_eq))
    vv = np.full(n_z, float(v))
    al = np.full(n_z, float(alpha))
    return _assemble("planar", GEOM_PLANAR, z_edges, np.array([0.0, math.pi]), 0.0, eps_edges,
                     n_mu, n_phi, mu_rule, vv, np.zeros(n_z), al, al ** -0.5, ka, ks, feq,
                     f_eq != 0.0, n_steps, PREC_FP64, inner_bc=inner_bc, outer_bc=outer_bc,
                     phi_rule=PHI_LINEAR if n_phi < 3 else PHI_SIN)


# --------------------------------------------------------------------------
# relativistic radiating spheres (boost, redshift, both), spherical symmetry
# --------------------------------------------------------------------------
def relativistic_sphere(test, params, n_inner=8, n_outer=56, r_max=600.0, n_mu=8, n_phi=4,
                        kappa=100.0, T=10.0):
    """Column grid: uniform radial zones inside the sphere, logarithmic outside.
    test 1: shock-like infall profile, flat metric; test 2: static fluid in a
    lapse well; test 3: both, opaque in the top energy group only.  params: the
    printed set-up (sphere radius, velocity and lapse laws, energy grid)."""
    R = params["sphere_radius_km"]
    eg = params["combined_test_energy_grid"]
    r_in = np.linspace(0.0, R, n_inner + 1)
    r_out = R * (r_max / R) ** (np.arange(1, n_outer + 1) / n_outer)
    r_edges = np.concatenate([r_in, r_out])
    rc = _centres(r_edges)
    n_r = len(rc)
    eps_edges = log_edges(eg["eps_min_MeV"], eg["eps_max_MeV"], eg["n_eps"])
    e = _group_energies(eps_edges)
    vp, lp = params["velocity_profile"], params["lapse_profile"]
    v = np.zeros(n_r)
    alpha = np.ones(n_r)
    if test in (1, 3):
        r0, r1, vmax = vp["r0_km"], vp["r1_km"], vp["vmax"]
        v = np.where(rc < r0, 0.0, np.where(rc <= r1, -vmax * (rc - r0) / (r1 - r0),
                                              -vmax * (r1 / rc) ** 2))
    if test in (2, 3):
        a0, rk = lp["a0"], lp["rk_km"]
        alpha = np.where(rc < rk, a0, a0 + (1.0 - a0) * (1.0 - rk / rc))
    psi = alpha ** -0.5
    inside = rc < R
    ka = np.zeros((n_r, 1, len(e)))
    if test == 3:
        ka[inside, 0, -1] = params["combined_test_opacity"]["kappa_a"]
    else:
        ka[inside, 0, :] = kappa
    feq = np.where(inside[:, None, None], fermi_dirac(e, T)[None, None, :], 0.0)
    return _assemble(f"relativistic_sphere_{test}", GEOM_COLUMN, r_edges, np.array([0.0, math.pi]), 0.0,
                     eps_edges, n_mu, n_phi, "lobatto", v, np.zeros(n_r), alpha, psi, ka,
                     np.zeros_like(ka), feq, False, 0, PREC_FP64, meta={"R": R, "test": test})


CONFIGS = {
    "radiating_sphere": radiating_sphere,
    "axisym_2d": axisym_2d,
    "shock_2d": shock_2d,
    "batch_models": batch_models,
    "hires_2d": hires_2d,
}
