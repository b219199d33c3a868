"""P-14, spherical (Sec. 4.3): the diffusion wave on the spherical grid, a
1D column from r = 0 with Delta r = 0.01, pure isotropic scattering, started
from the exact diffusion solution
    E = (k/t)^{3/2} exp(-3 k r^2 / 4t),  F = r E / 2t,
(E = 4 pi J, F = 4 pi H) with f = (E + 3 mu F)/4pi, and compared with it at
the paper's sample times: k = 1e2 (Pe = 1) from t = 1 to t = 2, 4, 5 and
k = 1e5 (Pe = 1000) from t = 200 to t = 240 (t = 300 and 400 run on the GPU
path, which the parity tests tie to this reference).

The paper leaves the column's angular width free and recommends faces of
similar area (Sec. 3.3.4).  Here it is 0.4 rad, at which the lateral and
radial faces of the innermost zones are of similar area; the default width,
set by the outermost zone (0.01 rad here), lets content pile up in the apex
zone (2.4 times the exact density at t = 2; test below) and takes a 40 times
smaller time step.  The paper finds acceptable agreement with a small error
next to r = 0; the bounds are 10% of the largest E (all zones) and |F|
(beyond five zones from the centre) for Pe = 1, and 2% for Pe = 1000."""
import math

import numpy as np
import pytest

from paper_2003_02845_amd import workloads as W

WIDTH = 0.4


def wave_column(ks, t0, dr=0.01, r_max=1.0, n_mu=8, n_phi=4, width=WIDTH):
    n = int(round(r_max / dr))
    w = W.radiating_sphere(n_r=n, n_eps=1, n_mu=n_mu, n_phi=n_phi, r_max=r_max, kappa=0.0,
                           mu_rule="lobatto")
    w.dphi = width
    w.kappa_a = np.zeros((n, 1, 1))
    w.kappa_s = np.full((n, 1, 1), ks)
    w.f_eq = np.zeros((n, 1, 1))
    rc = 0.5 * (w.r_edges[1:] + w.r_edges[:-1])
    mu = np.repeat(W_quad_mu(n_mu), n_phi)

    def EF(t):
        E = (ks / t) ** 1.5 * np.exp(-3 * ks * rc ** 2 / (4 * t))
        return E, rc / (2 * t) * E

    E0, F0 = EF(t0)
    w.f0 = ((E0[:, None] + 3 * mu[None, :] * F0[:, None]) / (4 * math.pi))[:, None, None, :].copy()
    return w, rc, mu, EF


def W_quad_mu(n):
    """Gauss-Lobatto nodes (closed forms are pinned in test_oracle_pins)"""
    P = np.polynomial.legendre.Legendre.basis(n - 1)
    return np.concatenate([[-1.0], np.sort(P.deriv().roots().real), [1.0]])


def moments_EF(f, wmu, n_phi, mu):
    dOm = np.repeat(wmu, n_phi) * 2 * math.pi / n_phi
    return f @ dOm, f @ (dOm * mu)


def evolve(oracle_mod, ks, t0, times, **kw):
    w, rc, mu, EF = wave_column(ks, t0, **kw)
    o = oracle_mod.Oracle(w)
    dt = o.max_dt(0.4)
    t, out = t0, []
    for ts in times:
        n = int(math.ceil((ts - t) / dt))
        o.step((ts - t) / n, n)
        t = ts
        E, F = moments_EF(o.state()[:, 0, 0, :], o.wmu, w.n_phi, mu)
        out.append((ts, E, F) + EF(ts))
    return rc, out


def test_spherical_diffusion_wave_pe1(oracle_mod):
    rc, out = evolve(oracle_mod, 100.0, 1.0, (2.0, 4.0, 5.0))
    far = rc > 0.05
    for ts, E, F, Ex, Fx in out:
        assert np.max(np.abs(E - Ex)) < 0.10 * Ex.max(), ts
        assert np.max(np.abs(F - Fx)[far]) < 0.10 * np.abs(Fx).max(), ts


@pytest.mark.slow
def test_spherical_diffusion_wave_pe1000(oracle_mod):
    rc, out = evolve(oracle_mod, 1e5, 200.0, (240.0,), r_max=0.4, n_mu=6)
    far = rc > 0.05
    for ts, E, F, Ex, Fx in out:
        assert np.max(np.abs(E - Ex)) < 0.02 * Ex.max(), ts
        assert np.max(np.abs(F - Fx)[far]) < 0.02 * np.abs(Fx).max(), ts


def test_narrow_column_piles_up_at_the_apex(oracle_mod):
    """the reason for the width above: with the default width (the outermost
    zone's, 0.01 rad) the apex zone holds far more than the exact solution,
    with 0.4 rad it is within a few per cent (short run, Delta r = 0.02)"""
    dens = {}
    for width in (0.0, WIDTH):
        rc, out = evolve(oracle_mod, 100.0, 1.0, (1.2,), dr=0.02, width=width)
        _, E, F, Ex, Fx = out[0]
        dens[width] = E[0] / Ex[0]
    assert dens[0.0] > 1.5 and abs(dens[WIDTH] - 1.0) < 0.1, dens
