"""Multi-dimensional end-to-end checks on the GPU path (Sec. 4.5, tests in
axisymmetry).

Radiating disk: theta over [0, pi/2] with the equatorial disk boundary; a
thick f = 1 disk of radius 1 radiates into vacuum. The stationary mean
intensity is compared with the exact solid-angle integral away from the
plane itself (z > 0.1) and from the inner boundary (r > 2.5 r_min), in three
regions whose bounds come from a study of
the disk on the CPU reference (N_theta 8-32, N_mu 8-16, N_Phi 4-16, both Phi
splits, inner radius 0.1 and 0.2):
  * the theta rows within 8.4 degrees of the pole: the axis artefact the
    paper reports; reported, not bounded (it grows with N_theta and with
    N_Phi at fixed N_mu, and is larger with the linear Phi split);
  * off the axis rows, within 4 inner radii: the specular inner boundary
    returns radiation that would pass through the centre; its error falls
    with N_mu (0.10 -> 0.05 for N_mu 8 -> 16) and grows with N_Phi at fixed
    N_mu (0.10 -> 0.18 for N_Phi 8 -> 16) and with N_theta (0.10 -> 0.24 for
    16 -> 32 rows); bounded by 0.25, above the study's largest (0.24);
  * the rest: ray effects, falling with N_Phi (0.15, 0.05-0.07, 0.04-0.06
    for N_Phi = 4, 8, 16 at 16 rows), largest where the two other regions
    meet (0.097 at 32 rows, N_mu = 8); bounded by 0.1, and by 0.03 in the
    mean (the study's means: 0.021-0.025).
The GPU runs take 16 or 17 mu nodes, which the study shows lowers the
errors near the axis and the inner boundary.

The homogeneous radiating sphere (kappa_a R = 10) is run on the axisymmetric
grid to a stationary state in FP64. Along rays near the pole, at 45 degrees
and at the equator, H/J and K/J are compared with the exact solution
f(r, mu) = f_eq (1 - exp(-kappa s)) of the classical sphere (Sec. 4.1). The
rays must also agree with each other, since the problem is spherically
symmetric and only the cell shapes change with theta. The paper's grid has
17 x 32 directions; the kernels hold at most 128, so this runs 16 Lobatto mu
x 8 Phi (the paper reports agreement in a figure, not a number).
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


def _pins():
    sys.path.insert(0, __import__("os").path.dirname(__file__))
    import test_oracle_pins
    return test_oracle_pins


def _disk_regions(w, zm):
    """|J - exact| of the radiating disk in the three regions of the module
    docstring: {name: errors}, with the zones' (x, z) for reports"""
    rc = np.tile(0.5 * (w.r_edges[1:] + w.r_edges[:-1]), w.n_theta)
    thc = np.repeat(0.5 * (w.theta_edges[1:] + w.theta_edges[:-1]), w.n_r)
    J = zm[:, 0, 1] / (np.sqrt(2.0) * 7.0 / 3.0)
    x, z = rc * np.sin(thc), rc * np.cos(thc)
    sel = (z > 0.1) & (rc < 2.5) & (rc > 2.5 * w.r_edges[0])
    exact = np.array([_pins()._disk_exact(a, b) for a, b in zip(x[sel], z[sel])])
    err = np.abs(J[sel] - exact)
    axis = np.degrees(thc[sel]) < 8.44
    inner = ~axis & (rc[sel] < 4.0 * w.r_edges[0])
    rest = ~axis & ~inner
    out = {}
    for name, m in (("axis rows", axis), ("2.5-4 r_min", inner), ("rest", rest)):
        e = err[m]
        q = int(np.argmax(e))
        _say(f"[gpu]   {name}: |J - exact| max {e.max():.4f} at x={x[sel][m][q]:.3f} z={z[sel][m][q]:.3f}, "
             f"mean {e.mean():.4f} ({m.sum()} zones)")
        out[name] = e
    return out


def _sphere_exact(x, kappa):
    mu = np.linspace(-1, 1, 20001)
    mu = 0.5 * (mu[1:] + mu[:-1])
    g = np.sqrt(np.maximum(0, 1 - x ** 2 * (1 - mu ** 2)))
    s = x * mu + g if x < 1 else np.where(mu >= np.sqrt(1 - 1 / x ** 2), 2 * g, 0.0)
    fe = 1 - np.exp(-kappa * s)
    return np.mean(fe * mu) / np.mean(fe), np.mean(fe * mu * mu) / np.mean(fe)


def test_radiating_sphere_2d():
    btx = _btx()
    w = W.radiating_sphere_2d(n_r=100, n_theta=32, n_mu=16, n_phi=8, r_min=0.05)
    ctx = btx.Context(w, precision=W.PREC_FP64)
    ctx.set_background()
    ctx.set_state(w.f0)
    dt = ctx.max_dt(0.4)
    steps = int(7.0 / dt)
    _say(f"[gpu] 2D radiating sphere: {w.n_r} x {w.n_theta} zones x {w.n_dir} directions, {steps} steps")
    ctx.step(dt, steps)
    zm, _ = ctx.moments()
    ctx.close()
    J, H, K = (zm[:, 0, k].reshape(w.n_theta, w.n_r) for k in (1, 2, 3))
    rc = 0.5 * (w.r_edges[1:] + w.r_edges[:-1])
    rays = {"pole": 1, "45deg": w.n_theta // 4, "equator": w.n_theta // 2}
    worst = {}
    for r in [0.5, 0.8, 1.2, 1.5, 2.0, 3.0]:
        a = int(np.argmin(abs(rc - r)))
        hj, kj = _sphere_exact(rc[a], 10.0)
        vals = []
        for name, b in rays.items():
            h, k = H[b, a] / J[b, a], K[b, a] / J[b, a]
            vals.append((h, k))
            worst[name] = max(worst.get(name, 0.0), abs(h - hj), abs(k - kj))
            _say(f"[gpu]   r={rc[a]:.3f} {name:8s} H/J {h:.4f} ({hj:.4f})  K/J {k:.4f} ({kj:.4f})")
        vals = np.array(vals)
        assert np.max(np.abs(vals - vals[-1])) < 0.03     # rays agree with the equator's
    _say(f"[gpu]   worst deviation from the exact solution per ray: {worst}")
    assert worst["equator"] < 0.03 and worst["45deg"] < 0.03
    assert worst["pole"] < 0.05


def test_radiating_disk_2d():
    btx = _btx()
    w = W.radiating_disk(n_r=100, n_theta=32, n_mu=16, n_phi=8, r_min=0.1, r_max=4.0)
    ctx = btx.Context(w, precision=W.PREC_FP64)
    ctx.set_background()
    ctx.set_state(w.f0)
    dt = ctx.max_dt(0.4)
    steps = int(4.5 / dt)
    _say(f"[gpu] radiating disk: {w.n_r} x {w.n_theta} zones x {w.n_dir} directions, {steps} steps")
    ctx.step(dt, steps)
    zm, tot = ctx.moments()
    ctx.close()
    e = _disk_regions(w, zm)
    assert e["rest"].max() < 0.1 and e["rest"].mean() < 0.03
    assert e["2.5-4 r_min"].max() < 0.25


def test_3d_symmetric_equals_axisymmetric_gpu():
    """a 3D grid of four copies of the wedge around the axis, with data
    independent of phi, steps like the axisymmetric wedge on the GPU.  Not bit
    for bit: the wedge's periodic self-face reuses the zone's own slope,
    while a 3D phi face limits each side's slope in its own frame (the same
    value up to rounding).  FP64 to 1e-13, mixed to 1e-5, relative to the
    block maximum; the phi momentum source term vanishes to the same level."""
    btx = _btx()
    w2 = W.shock_2d(n_r=16, n_theta=8, n_eps=8, n_mu=6, n_phi=4, precision=W.PREC_FP64)
    w2.f0 = w2.f0 * (1.0 + 0.3 * np.random.default_rng(3).random(w2.f0.shape))
    w3 = W.extrude_phi(w2, 4)
    _say(f"[gpu] 3D (4 phi zones) against the axisymmetric wedge, {w2.n_zones} zones per wedge")
    for prec, tol in ((W.PREC_FP64, 1e-13), (W.PREC_MIXED, 1e-5)):
        out = []
        for w in (w2, w3):
            ctx = btx.Context(w, precision=prec)
            ctx.set_background()
            ctx.set_state(w.f0)
            ctx.step(ctx.max_dt(0.4), 3)
            out.append((ctx.get_state().astype(np.float64), ctx.source_terms()))
            ctx.close()
        ref = out[0][0]
        s3 = out[1][0].reshape((4,) + ref.shape)
        errs = [float(np.max(np.abs(s3[c] - ref)) / np.max(np.abs(ref))) for c in range(4)]
        q2, q3 = out[0][1], out[1][1].reshape(4, w2.n_zones, 5)
        qerr = float(np.max(np.abs(q3 - q2[None])) / np.max(np.abs(q2)))
        _say(f"[gpu]   precision {prec}: state {max(errs):.3e}, source terms {qerr:.3e}")
        assert max(errs) <= tol and qerr <= 10 * tol


def test_radiating_sphere_2d_time_levels():
    """the 2D radiating sphere with local time stepping (levels up to 5)
    reaches the same stationary H/J and K/J as the global step: within 0.03
    of the exact solution on the three rays (the global step: 0.011)"""
    btx = _btx()
    w = W.radiating_sphere_2d(n_r=100, n_theta=32, n_mu=16, n_phi=8, r_min=0.05)
    ctx = btx.Context(w, precision=W.PREC_FP64)
    ctx.set_background()
    ctx.set_state(w.f0)
    dt = ctx.max_dt(0.4)
    lev = ctx.time_levels(5)
    L = int(lev.max())
    ctx.set_time_levels(lev)
    steps = int(7.0 / (dt * 2 ** L))
    frac = float(np.sum(2.0 ** (L - lev))) / (w.n_zones * 2 ** L)
    _say(f"[gpu] 2D radiating sphere with time levels up to {L}: {steps} steps of {2 ** L} substeps, "
         f"zone updates {frac:.3f} of the global step's")
    ctx.step(dt, steps)
    zm, _ = ctx.moments()
    ctx.close()
    J, H, K = (zm[:, 0, k].reshape(w.n_theta, w.n_r) for k in (1, 2, 3))
    rc = 0.5 * (w.r_edges[1:] + w.r_edges[:-1])
    worst = 0.0
    for r in [0.5, 0.8, 1.2, 1.5, 2.0, 3.0]:
        a = int(np.argmin(abs(rc - r)))
        hj, kj = _sphere_exact(rc[a], 10.0)
        for b in (1, w.n_theta // 4, w.n_theta // 2):
            worst = max(worst, abs(H[b, a] / J[b, a] - hj), abs(K[b, a] / J[b, a] - kj))
    _say(f"[gpu]   worst deviation from the exact solution {worst:.4f}")
    assert worst < 0.03 and frac < 0.5


def _levels_run(btx, w, t_end, max_level=5):
    ctx = btx.Context(w, precision=W.PREC_FP64)
    ctx.set_background()
    ctx.set_state(w.f0)
    dt = ctx.max_dt(0.4)
    lev = ctx.time_levels(max_level)
    L = int(lev.max())
    ctx.set_time_levels(lev)
    steps = int(t_end / (dt * 2 ** L))
    ctx.step(dt, steps)
    zm, tot = ctx.moments()
    ctx.close()
    return zm, tot, steps, L


def test_radiating_sphere_2d_paper_resolution():
    """the 2D radiating sphere at the paper's resolution: 100 x 32 zones, 17
    Gauss-Legendre mu x 32 Phi = 544 directions (remap tables through the
    caches), with time levels up to 5: H/J and K/J on the three rays within
    0.03 of the exact solution and of each other"""
    btx = _btx()
    w = W.radiating_sphere_2d(n_r=100, n_theta=32, n_mu=17, n_phi=32, r_min=0.05, mu_rule="legendre")
    _say(f"[gpu] 2D radiating sphere, {w.n_zones} zones x {w.n_dir} directions")
    zm, _, steps, L = _levels_run(btx, w, 7.0)
    J, H, K = (zm[:, 0, k].reshape(w.n_theta, w.n_r) for k in (1, 2, 3))
    rc = 0.5 * (w.r_edges[1:] + w.r_edges[:-1])
    worst = {}
    for r in [0.5, 0.8, 1.2, 1.5, 2.0, 3.0]:
        a = int(np.argmin(abs(rc - r)))
        hj, kj = _sphere_exact(rc[a], 10.0)
        vals = []
        for name, b in (("pole", 1), ("45deg", w.n_theta // 4), ("equator", w.n_theta // 2)):
            h, k = H[b, a] / J[b, a], K[b, a] / J[b, a]
            vals.append((h, k))
            worst[name] = max(worst.get(name, 0.0), abs(h - hj), abs(k - kj))
        vals = np.array(vals)
        assert np.max(np.abs(vals - vals[-1])) < 0.03
    _say(f"[gpu]   {steps} steps of {2 ** L} substeps; worst deviation per ray {worst}")
    assert max(worst.values()) < 0.03


def test_radiating_disk_paper_resolution():
    """the radiating disk at the paper's resolution (100 x 32 zones, 17 x 32
    directions) with time levels up to 5, against the exact solid-angle
    integral, in the regions and with the bounds of the module docstring"""
    btx = _btx()
    w = W.radiating_disk(n_r=100, n_theta=32, n_mu=17, n_phi=32, r_min=0.1, r_max=4.0,
                         mu_rule="legendre")
    _say(f"[gpu] radiating disk, {w.n_zones} zones x {w.n_dir} directions")
    zm, tot, steps, L = _levels_run(btx, w, 4.5)
    _say(f"[gpu]   {steps} steps of {2 ** L} substeps")
    e = _disk_regions(w, zm)
    assert e["rest"].max() < 0.1 and e["rest"].mean() < 0.03
    assert e["2.5-4 r_min"].max() < 0.25