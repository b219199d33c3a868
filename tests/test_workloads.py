"""The seeded synthetic inputs: the generator, the grids and the profile
recipe of the benchmark configurations (CPU only, no method arithmetic)."""
import math

import numpy as np

from paper_2003_02845_amd import workloads as W


def test_splitmix64_reference_outputs():
    """the first outputs of SplitMix64 from state 0, as published with the
    generator, and uniforms in [0, 1) with 53 bits"""
    r = W.SplitMix64(0)
    assert [r.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                 0x06C45D188009454F]
    r = W.SplitMix64(20030245)
    u = [r.uniform() for _ in range(1000)]
    assert min(u) >= 0.0 and max(u) < 1.0
    assert all(x * 2.0 ** 53 == int(x * 2.0 ** 53) for x in u)


def test_inputs_are_reproducible():
    a = W.shock_2d(n_r=20, n_theta=6, n_eps=5, n_mu=4, n_phi=4, modes=True)
    b = W.shock_2d(n_r=20, n_theta=6, n_eps=5, n_mu=4, n_phi=4, modes=True)
    for name in ("v_r", "alpha", "psi", "kappa_a", "kappa_s", "f_eq", "f0"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name
    ms = [(w.n_r, w.n_eps, w.n_dir) for w in W.batch_models()]
    assert ms == [(w.n_r, w.n_eps, w.n_dir) for w in W.batch_models()]


def test_benchmark_grid_shape():
    """600 r x 256 theta zones, 3 species, 24 log groups over 2-300 MeV,
    12 mu x 8 Phi directions: 1,061,683,200 values (built here at 8 theta rows)"""
    w = W.hires_2d(n_theta=8)
    assert (w.n_r, w.n_species, w.n_eps, w.n_mu, w.n_phi) == (600, 3, 24, 12, 8)
    assert w.n_r * 256 * w.n_species * w.n_eps * w.n_mu * w.n_phi == 1_061_683_200
    e = np.asarray(w.eps_edges)
    assert math.isclose(e[0], 2.0) and math.isclose(e[-1], 300.0)
    ratio = e[1:] / e[:-1]
    assert np.allclose(ratio, ratio[0])
    r = np.asarray(w.r_edges)
    assert math.isclose(r[0], 10.0) and math.isclose(r[-1], 1000.0)
    assert np.allclose(r[1:] / r[:-1], r[1] / r[0])


def test_profile_recipe():
    """alpha = 1 - 0.2 (10 km / r), psi = alpha^-1/2, ks = 2 ka, species
    opacities in the ratio 1 : 0.7 : 0.3, ka growing as eps^2, and the
    equilibrium a Fermi-Dirac occupation at zero degeneracy (below 1/2)"""
    w = W.shock_2d(n_r=30, n_theta=4, n_eps=6, n_mu=4, n_phi=4)
    rc = np.sqrt(np.asarray(w.r_edges)[1:] * np.asarray(w.r_edges)[:-1])
    R = np.tile(rc, w.n_theta)
    assert np.allclose(w.alpha, 1.0 - 0.2 * 10.0 / R, rtol=0.02)
    assert np.allclose(w.psi, w.alpha ** -0.5)
    assert np.allclose(w.kappa_s, 2.0 * w.kappa_a)
    assert np.allclose(w.kappa_a[:, 1, :] / w.kappa_a[:, 0, :], 0.7)
    assert np.allclose(w.kappa_a[:, 2, :] / w.kappa_a[:, 0, :], 0.3)
    e = np.sqrt(np.asarray(w.eps_edges)[1:] * np.asarray(w.eps_edges)[:-1])
    assert np.allclose(w.kappa_a[:, 0, 1:] / w.kappa_a[:, 0, :-1], (e[1:] / e[:-1]) ** 2)
    assert np.all(w.f_eq > 0.0) and np.all(w.f_eq < 0.5)
    assert np.all(w.v_r < 0.0)                       # infall


def test_batch_model_ranges():
    """64 spherically symmetric models: 100-600 radial zones, 12-24 groups,
    16-48 directions, infall up to 0.2 c"""
    ws = W.batch_models()
    assert len(ws) == 64
    for w in ws:
        assert 100 <= w.n_r <= 600 and 12 <= w.n_eps <= 24 and 16 <= w.n_dir <= 48
        assert w.geometry == W.GEOM_COLUMN
        assert np.all(np.abs(w.v_r) <= 0.2 + 1e-12)
