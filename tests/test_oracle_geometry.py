"""Pins of the reference's flat-faced cell geometry (Sec. 3.1): the spherical
polar grid has planar quadrilateral faces through the grid vertices, so every
cell is a polyhedron with six (possibly degenerate) flat faces.

For every zone the test builds the eight vertices itself, takes each face's
area vector as the sum of its two triangles' area vectors (not the diagonal
cross product the reference uses), checks that the outward area vectors of
the cell sum to zero (a closed surface; this pins the test's own vertex
bookkeeping), and then checks the reference against two facts of solid
geometry:
  * its cell volume equals (1/3) sum_s A_s . x_s over the six faces (the
    divergence theorem for the position vector, x_s any point of face s);
  * its face areas equal the magnitudes of those area vectors.
A shell volume (r1^3 - r0^3)/3 * solid angle in place of the flat-faced one,
a swapped vertex order, or wrong edge or column angles fail these."""
import math

import numpy as np
import pytest

from paper_2003_02845_amd import workloads as W


def vertex(r, th, ph):
    return np.array([r * math.sin(th) * math.cos(ph), r * math.sin(th) * math.sin(ph), r * math.cos(th)])


def area_vector(P):
    """sum of the area vectors of the triangles (P0, P1, P2) and (P0, P2, P3)"""
    return 0.5 * (np.cross(P[1] - P[0], P[2] - P[0]) + np.cross(P[2] - P[0], P[3] - P[0]))


def cell_faces(r0, r1, t0, t1, p0, p1):
    """the six faces of a cell as (key, vertices): r-, r+, theta-, theta+, phi-, phi+"""
    V = {(i, j, k): vertex((r0, r1)[i], (t0, t1)[j], (p0, p1)[k])
         for i in (0, 1) for j in (0, 1) for k in (0, 1)}
    return [
        ("r-", [V[0, 0, 0], V[0, 1, 0], V[0, 1, 1], V[0, 0, 1]]),
        ("r+", [V[1, 0, 0], V[1, 1, 0], V[1, 1, 1], V[1, 0, 1]]),
        ("t-", [V[0, 0, 0], V[1, 0, 0], V[1, 0, 1], V[0, 0, 1]]),
        ("t+", [V[0, 1, 0], V[1, 1, 0], V[1, 1, 1], V[0, 1, 1]]),
        ("p-", [V[0, 0, 0], V[1, 0, 0], V[1, 1, 0], V[0, 1, 0]]),
        ("p+", [V[0, 0, 1], V[1, 0, 1], V[1, 1, 1], V[0, 1, 1]]),
    ]


def cell_geometry(r0, r1, t0, t1, p0, p1):
    """outward area vectors of the six faces, the closure residual and the
    divergence-theorem volume"""
    faces = cell_faces(r0, r1, t0, t1, p0, p1)
    centre = np.mean([v for _, P in faces for v in P], axis=0)
    out, total, vol = {}, np.zeros(3), 0.0
    for key, P in faces:
        A = area_vector(P)
        fc = np.mean(P, axis=0)
        if np.dot(A, fc - centre) < 0.0:
            A = -A
        out[key] = A
        total += A
        vol += np.dot(A, P[0]) / 3.0
    return out, total, vol


def zone_angles(w, z, delta):
    """(a, theta range, phi range) of zone z in its own frame (the wedge, or
    a 3D phi zone, centred on phi = 0; the column at the equator)"""
    a = z % w.n_r
    if w.geometry == W.GEOM_AXISYM2D:
        b = (z // w.n_r) % w.n_theta
        return a, w.theta_edges[b], w.theta_edges[b + 1], -0.5 * w.dphi, 0.5 * w.dphi
    return a, 0.5 * math.pi - 0.5 * delta, 0.5 * math.pi + 0.5 * delta, -0.5 * delta, 0.5 * delta


def grids():
    col = W.radiating_sphere(n_r=12, n_eps=2, n_mu=4, n_phi=4)                    # from r = 0
    logcol = W.batch_models(n_models=1, size_scale=0.05)[0]                     # log radii from 10 km
    ax = W.shock_2d(n_r=9, n_theta=7, n_eps=3, n_mu=4, n_phi=4)                  # axis at both ends
    disk = W.radiating_disk(n_r=8, n_theta=5, n_mu=4, n_phi=4)                   # [0, pi/2]
    d3 = W.extrude_phi(W.shock_2d(n_r=6, n_theta=5, n_eps=2, n_mu=4, n_phi=4), 3)
    return {"column": col, "log_column": logcol, "axisym": ax, "disk": disk, "3d": d3}


@pytest.mark.parametrize("name", ["column", "log_column", "axisym", "disk", "3d"])
def test_flat_faced_cells(oracle_mod, name):
    w = grids()[name]
    o = oracle_mod.Oracle(w, background=False, state=False)
    vol, rc, thc = o.geometry()
    re = np.asarray(w.r_edges, float)
    delta = (re[-1] - re[-2]) / re[-1]
    cells = {}
    for z in range(w.n_zones):
        a, t0, t1, p0, p1 = zone_angles(w, z, delta)
        A, total, V = cell_geometry(re[a], re[a + 1], t0, t1, p0, p1)
        amax = max(np.linalg.norm(v) for v in A.values())
        assert np.linalg.norm(total) <= 1e-14 * amax, (z, total)          # closed surface
        assert abs(vol[z] - V) <= 1e-13 * V, (z, vol[z], V)
        assert abs(rc[z] - 0.5 * (re[a] + re[a + 1])) <= 1e-15 * rc[z]
        cells[z] = A
    # every face of the reference against the area vector of an adjacent cell
    key_of = {(0, "L"): "r+", (0, "R"): "r-", (1, "L"): "t+", (1, "R"): "t-", (2, "L"): "p+", (2, "R"): "p-"}
    seen = {0: 0, 1: 0, 2: 0}
    for fid in range(o.n_faces()):
        zL, zR, axis, area, active = o.face_geom(fid)
        if not active:
            assert zL < 0 and zR < 0 and area == 0.0
            continue
        side, z = ("L", zL) if zL >= 0 else ("R", zR)
        ref = np.linalg.norm(cells[z][key_of[axis, side]])
        assert abs(area - ref) <= 1e-13 * ref, (fid, axis, area, ref)
        seen[axis] += 1
    assert seen[0] > 0 and seen[2] > 0 and (seen[1] > 0)


def test_flat_faced_volume_is_not_the_shell_volume(oracle_mod):
    """the pin distinguishes the flat-faced cell from the spherical shell
    sector of the same angles (the reading the flat faces replace)"""
    w = W.shock_2d(n_r=4, n_theta=3, n_eps=2, n_mu=4, n_phi=4)
    o = oracle_mod.Oracle(w, background=False, state=False)
    vol, _, _ = o.geometry()
    re = w.r_edges
    t0, t1 = w.theta_edges[0], w.theta_edges[1]
    shell = (re[1] ** 3 - re[0] ** 3) / 3.0 * (math.cos(t0) - math.cos(t1)) * w.dphi
    assert abs(vol[0] - shell) > 1e-4 * shell


def test_planar_cells(oracle_mod):
    """slab geometry: unit face areas and cell volumes equal to the widths"""
    w = W.planar(n_z=7, z_min=-1.0, z_max=0.4, n_mu=4)
    o = oracle_mod.Oracle(w, background=False, state=False)
    vol, _, _ = o.geometry()
    assert np.allclose(vol, np.diff(w.r_edges), rtol=1e-15, atol=0.0)
    for fid in range(o.n_faces()):
        _, _, axis, area, active = o.face_geom(fid)
        assert active and axis == 0 and area == 1.0
