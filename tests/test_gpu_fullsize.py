"""GPU parity at the full sizes of the benchmark configurations, at their
stated lengths.

- The radiating sphere (64 radial zones, 8 groups, 16 x 4 directions): its 200
  steps against the FP64 reference (full f), and its own grid run to a steady
  state with time levels against the exact sphere (Sec. 4.1).
- The FP64 axisymmetric profile (256 x 64 zones, 16 groups, 64 directions): 100
  steps against the reference, full f.
- The shock profile (550 x 128 zones, 3 species, 21 groups, 80 directions),
  mixed precision: 10 steps against the reference (per-zone number and J;
  the largest deviation of f reported), and 100 steps against the FP64 GPU run.
- The high-resolution profile (600 x 256 zones, 3 species, 24 groups, 96
  directions): one step in the benchmark's launch configuration on sampled
  zones that the reference computes one by one (the four grid corners, the
  axis rows, the radial boundaries and seeded random zones), and its 50 steps
  in mixed precision against the FP64 GPU run.

Bounds: FP64 <= 1e-12 relative to the largest value; mixed <= 1e-5 relative
to the block maximum per value, and <= 1e-5 in the per-zone moments where J >
1e-8 of its maximum.
"""
import sys

import numpy as np
import pytest

from paper_2003_02845_amd import workloads as W

pytestmark = pytest.mark.gpu


def _btx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_02845_amd import btx
    return btx


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sample_zones(w, n_random, seed):
    nr, nth = w.n_r, w.n_theta
    fixed = [0, nr - 1, (nth - 1) * nr, nth * nr - 1,            # corners
             nr // 2, (nth - 1) * nr + nr // 2,                    # axis rows
             (nth // 2) * nr, (nth // 2) * nr + nr - 1]            # inner / outer boundary
    rng = np.random.default_rng(seed)
    extra = rng.choice(w.n_zones, n_random, replace=False)
    return np.unique(np.concatenate([np.array(fixed), extra])).astype(np.int32)


def _zone_moments(w, f):
    """per (zone, species): sum of f G dOmega and of f eps G dOmega (number-like and energy-like)"""
    from oracle import oracle  # quadrature only
    mu, wmu = oracle.quadrature(w.mu_rule, w.n_mu)
    dOm = np.repeat(wmu * 2.0 * np.pi / w.n_phi, w.n_phi)
    e = w.eps_edges
    G = (e[1:] ** 3 - e[:-1] ** 3) / 3.0
    eps = np.sqrt(e[1:] * e[:-1])
    n = np.einsum("zsid,i,d->zs", f, G, dOm)
    en = np.einsum("zsid,i,d->zs", f, G * eps, dOm)
    return n, en


def _perturbed(w, seed):
    rng = np.random.default_rng(seed)
    w.f0 = w.f0 * (1.0 + 0.2 * rng.random(w.f0.shape))
    return w


def _full_fp64(w, steps, oracle_mod):
    btx = _btx()
    o = oracle_mod.Oracle(w)
    dt = o.max_dt(w.cfl)
    ctx = btx.Context(w, precision=W.PREC_FP64)
    ctx.set_background()
    ctx.set_state(w.f0)
    ctx.step(dt, steps)
    o.step(dt, steps)
    got, ref = ctx.get_state(), o.state()
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    zg, tg = ctx.moments()
    zr, tr = o.moments()
    ctx.close()
    return err, zg, zr, tg, tr


def test_radiating_sphere_full_200_steps(oracle_mod):
    w = W.radiating_sphere()
    _say(f"[gpu] radiating sphere, {w.n_zones} zones x {w.block}, {w.n_steps} steps, FP64")
    err, zg, zr, tg, tr = _full_fp64(w, w.n_steps, oracle_mod)
    _say(f"[gpu]   rel err {err:.3e}")
    assert err <= 1e-12
    m = np.abs(zr[..., 1]).max()
    assert np.max(np.abs(zg[..., 1] - zr[..., 1])) <= 1e-12 * m
    assert np.allclose(tg, tr, rtol=1e-12, atol=1e-12 * np.abs(tr).max())


def test_radiating_sphere_own_grid_steady_state():
    """The sphere's own grid (uniform from r = 0, the default column width)
    stepped with time levels up to 6 to t = 7 R/c, a stationary state: the
    exact H/J and K/J of the homogeneous sphere (f = f_eq (1 - exp(-ka s)),
    Sec. 4.1, with the path-length reading s = r mu + R g inside) within 0.03
    at radii inside and outside the sphere."""
    import torch
    btx = _btx()
    w = W.radiating_sphere()
    ctx = btx.Context(w, precision=W.PREC_FP64, stream=torch.cuda.current_stream().cuda_stream)
    ctx.set_background()
    ctx.set_state(w.f0)
    dt = ctx.max_dt(w.cfl)
    lev = ctx.time_levels(6)
    L = int(lev.max())
    ctx.set_time_levels(lev)
    n = int(round(7.0 / (dt * 2 ** L)))
    _say(f"[gpu] radiating sphere own grid: levels up to {L}, {n} steps of {2 ** L} substeps")
    ctx.step(dt, n)
    zm, _ = ctx.moments()
    ctx.close()
    rc = 0.5 * (w.r_edges[1:] + w.r_edges[:-1])
    J, H, K = zm[:, 0, 1], zm[:, 0, 2], zm[:, 0, 3]
    mu = np.linspace(-1, 1, 200001)
    mu = 0.5 * (mu[1:] + mu[:-1])
    kap = w.meta["kappa_a"]
    for x in (0.3, 0.5, 0.8, 1.2, 1.5, 2.0, 2.5):
        g = np.sqrt(np.maximum(0, 1 - x ** 2 * (1 - mu ** 2)))
        s = x * mu + g if x < 1 else np.where(mu >= np.sqrt(1 - 1 / x ** 2), 2 * g, 0.0)
        fe = 1 - np.exp(-kap * s)
        hj, kj = np.mean(fe * mu) / np.mean(fe), np.mean(fe * mu * mu) / np.mean(fe)
        dh, dk = np.interp(x, rc, H / J) - hj, np.interp(x, rc, K / J) - kj
        _say(f"[gpu]   r = {x}: H/J {dh:+.4f}, K/J {dk:+.4f}")
        assert abs(dh) < 0.03 and abs(dk) < 0.03, (x, dh, dk)


def test_axisym_fp64_100_steps(oracle_mod):
    w = _perturbed(W.axisym_2d(), 11)
    _say(f"[gpu] axisymmetric FP64, {w.n_zones} zones x {w.block}, 100 steps")
    err, zg, zr, tg, tr = _full_fp64(w, 100, oracle_mod)
    _say(f"[gpu]   rel err {err:.3e}")
    assert err <= 1e-12
    assert np.allclose(tg, tr, rtol=1e-12, atol=1e-12 * np.abs(tr).max())


def _moment_err(zg, zr):
    """largest relative deviation of the per-zone number and J where J > 1e-8 of its maximum"""
    J = zr[..., 1]
    m = np.abs(J) > 1e-8 * np.abs(J).max()
    eN = np.max(np.abs(zg[..., 0] - zr[..., 0])[m] / np.abs(zr[..., 0][m]))
    eJ = np.max(np.abs(zg[..., 1] - J)[m] / np.abs(J[m]))
    return float(eN), float(eJ)


def _gpu_run(btx, w, prec, dt, steps, want_f=True):
    import torch
    ctx = btx.Context(w, precision=prec, stream=torch.cuda.current_stream().cuda_stream)
    ctx.set_background()
    ctx.set_state(w.f0)
    ctx.step(dt, steps)
    torch.cuda.synchronize()
    f = ctx.get_state() if want_f else None
    zm, tot = ctx.moments()
    ctx.close()
    return f, zm, tot


def test_shock_mixed_10_steps_and_fp64_gpu_100(oracle_mod):
    btx = _btx()
    w = _perturbed(W.shock_2d(), 14)
    _say(f"[gpu] shock profile {w.n_zones} zones x {w.block}: 10 steps mixed and FP64 against the reference")
    o = oracle_mod.Oracle(w)
    dt = o.max_dt(w.cfl)
    o.step(dt, 10)
    ref = o.state()
    zr, tr = o.moments()
    del o
    f32, z32, t32 = _gpu_run(btx, w, W.PREC_MIXED, dt, 10)
    ef = float(np.max(np.abs(f32 - ref)) / np.max(np.abs(ref)))
    eN, eJ = _moment_err(z32, zr)
    _say(f"[gpu]   mixed: N {eN:.2e}, J {eJ:.2e}, max |f - f_ref| / max f_ref {ef:.2e}")
    assert eN <= 1e-5 and eJ <= 1e-5
    del f32
    f64, z64, _ = _gpu_run(btx, w, W.PREC_FP64, dt, 10)
    e64 = float(np.max(np.abs(f64 - ref)) / np.max(np.abs(ref)))
    _say(f"[gpu]   FP64: {e64:.2e}")
    assert e64 <= 1e-12
    del f64, ref
    _, z32, t32 = _gpu_run(btx, w, W.PREC_MIXED, dt, 100, want_f=False)
    _, z64, t64 = _gpu_run(btx, w, W.PREC_FP64, dt, 100, want_f=False)
    eN, eJ = _moment_err(z32, z64)
    drift = float(np.max(np.abs(t32[:, 0] + t32[:, 1] - t64[:, 0] - t64[:, 1]) / t64[:, 0]))
    _say(f"[gpu]   100 steps mixed against FP64 GPU: N {eN:.2e}, J {eJ:.2e}, number {drift:.2e}")
    assert eN <= 1e-5 and eJ <= 1e-5


def test_hires_mixed_50_steps_against_fp64_gpu():
    btx = _btx()
    w = W.hires_2d()
    dt = None
    import torch
    ctx = btx.Context(w, precision=W.PREC_FP64, stream=torch.cuda.current_stream().cuda_stream)
    dt = ctx.max_dt(w.cfl)
    ctx.close()
    _say(f"[gpu] high-resolution profile {w.n_zones} zones x {w.block}: 50 steps mixed against FP64 GPU")
    _, z32, t32 = _gpu_run(btx, w, W.PREC_MIXED, dt, 50, want_f=False)
    _, z64, t64 = _gpu_run(btx, w, W.PREC_FP64, dt, 50, want_f=False)
    eN, eJ = _moment_err(z32, z64)
    drift = float(np.max(np.abs(t32[:, 0] + t32[:, 1] - t64[:, 0] - t64[:, 1]) / t64[:, 0]))
    _say(f"[gpu]   N {eN:.2e}, J {eJ:.2e}, number {drift:.2e}")
    assert eN <= 1e-5 and eJ <= 1e-5


@pytest.mark.parametrize("maker", ["shock_2d", "hires_2d"])
def test_mixed_sampled_full_size(maker, oracle_mod):
    btx = _btx()
    import torch
    w = _perturbed(getattr(W, maker)(), 12)
    zones = _sample_zones(w, 40, 13)
    _say(f"[gpu] {maker} full size: {w.n_zones} zones x {w.block} = {w.n_values:.3g} values, "
         f"{len(zones)} sampled zones")
    o = oracle_mod.Oracle(w)
    dt = o.max_dt(w.cfl)
    ref = o.step_sample(dt, zones)
    del o
    res = {}
    for prec in (W.PREC_MIXED, W.PREC_FP64):
        ctx = btx.Context(w, precision=prec, stream=torch.cuda.current_stream().cuda_stream)
        assert abs(ctx.max_dt(w.cfl) - dt) <= 1e-13 * dt
        ctx.set_background()
        ctx.set_state(w.f0)
        ctx.step(dt, 1)
        torch.cuda.synchronize()
        res[prec] = ctx.get_state()[zones].astype(np.float64)
        ctx.close()
    scale = np.abs(ref).reshape(len(zones), -1).max(axis=1)[:, None, None, None]
    e64 = float(np.max(np.abs(res[W.PREC_FP64] - ref) / scale))
    e32 = float(np.max(np.abs(res[W.PREC_MIXED] - ref) / scale))
    _say(f"[gpu]   fp64 rel err {e64:.3e}, mixed rel err {e32:.3e}")
    assert e64 <= 1e-12
    assert e32 <= 1e-5
    nr_, er_ = _zone_moments(w, ref)
    ng_, eg_ = _zone_moments(w, res[W.PREC_MIXED])
    assert np.max(np.abs(ng_ - nr_) / np.abs(nr_)) <= 1e-5
    assert np.max(np.abs(eg_ - er_) / np.abs(er_)) <= 1e-5
