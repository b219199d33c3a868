"""ctypes front end of the FP64 CPU reference (btx_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the CPU-baseline leg of the benchmark.  The GPU library never imports it.

Gauss quadrature nodes and weights are taken from numpy (a library primitive);
everything else is in btx_oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "btx_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def build(force: bool = True) -> str:
    """compile the reference with gcc (plain IEEE FP64, no contraction)"""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Desc(C.Structure):
    _fields_ = [("n_r", C.c_int), ("n_theta", C.c_int), ("n_eps", C.c_int), ("n_mu", C.c_int),
                ("n_phi", C.c_int), ("n_species", C.c_int), ("geometry", C.c_int),
                ("phi_rule", C.c_int), ("inner_bc", C.c_int), ("outer_bc", C.c_int),
                ("r_edges", _dp), ("theta_edges", _dp), ("dphi", C.c_double),
                ("eps_edges", _dp), ("mu_nodes", _dp), ("mu_weights", _dp),
                ("theta_bc", C.c_int), ("disk_radius", C.c_double), ("n_phi_zones", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Desc)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_background.argtypes = [C.c_void_p] + [_dp] * 8
        L.orc_update_background.argtypes = [C.c_void_p] + [_dp] * 8
        L.orc_source_terms.argtypes = [C.c_void_p, _dp]
        L.orc_time_levels.argtypes = [C.c_void_p, C.c_int, _ip]
        L.orc_set_levels.argtypes = [C.c_void_p, _ip]
        L.orc_set_state.argtypes = [C.c_void_p, _dp]
        L.orc_get_state.argtypes = [C.c_void_p, _dp]
        L.orc_max_dt.restype = C.c_double
        L.orc_max_dt.argtypes = [C.c_void_p, C.c_double]
        L.orc_step.argtypes = [C.c_void_p, C.c_double, C.c_int]
        L.orc_step_sample.argtypes = [C.c_void_p, C.c_double, C.c_int, _ip, _dp]
        L.orc_moments.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_set_blend_mode.argtypes = [C.c_void_p, C.c_int]
        L.orc_n_faces.argtypes = [C.c_void_p]
        L.orc_geometry.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_face_debug.argtypes = [C.c_void_p, C.c_int, C.c_double, _dp, _dp, _dp, _dp]
        L.orc_face_geom.argtypes = [C.c_void_p, C.c_int, _ip, _dp]
        L.orc_chain.argtypes = [_dp, _dp, C.c_int, C.c_int, _dp, _dp]
        L.orc_chain.restype = None
        L.orc_remap_block.argtypes = [C.c_void_p, _dp, _dp, C.c_int, C.c_int, C.c_int, C.c_int,
                                      _dp, _dp]
        L.orc_collide.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                  C.c_double, _dp, _dp]
        L.orc_collide.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def gauss_legendre(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def gauss_lobatto(n):
    """nodes: +-1 and the roots of P'_{n-1}; weights 2/(n(n-1) P_{n-1}(x)^2)"""
    P = np.polynomial.legendre.Legendre.basis(n - 1)
    inner = np.sort(P.deriv().roots().real)
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (n * (n - 1) * P(x) ** 2)
    return x, w


def quadrature(rule, n):
    return gauss_legendre(n) if rule == "legendre" else gauss_lobatto(n)


def chain(S, D, axis, rotate, u):
    out = np.zeros(4)
    lib().orc_chain(_p(_c(S)), _p(_c(D)), axis, rotate, _p(_c(u)), _p(out))
    return out


def collide(f, dJ, tau, ka, ks, feq, dOm):
    f = _c(f)
    out = np.zeros_like(f)
    dj = _c(dJ) if dJ is not None else None
    lib().orc_collide(len(f), _p(f), _p(dj) if dj is not None else None, tau, ka, ks, feq,
                      _p(_c(dOm)), _p(out))
    return out


class Oracle:
    """FP64 reference stepper for one Workload (see paper_2003_02845_amd.workloads)"""

    def __init__(self, w, background=True, state=True):
        self.w = w
        self.mu, self.wmu = quadrature(w.mu_rule, w.n_mu)
        self._keep = [_c(w.r_edges), _c(w.theta_edges), _c(w.eps_edges), _c(self.mu),
                      _c(self.wmu)]
        d = _Desc(w.n_r, w.n_theta, w.n_eps, w.n_mu, w.n_phi, w.n_species, w.geometry,
                  w.phi_rule, w.inner_bc, w.outer_bc, _p(self._keep[0]), _p(self._keep[1]),
                  w.dphi, _p(self._keep[2]), _p(self._keep[3]), _p(self._keep[4]),
                  w.theta_bc, w.disk_radius, w.n_phi_zones)
        self.ctx = lib().orc_create(C.byref(d))
        if not self.ctx:
            raise ValueError("oracle rejected the grid description")
        self.shape = (w.n_zones, w.n_species, w.n_eps, w.n_dir)
        if background:
            self.set_background(w)
        if state:
            self.set_state(w.f0)

    def __del__(self):
        if getattr(self, "ctx", None):
            lib().orc_destroy(self.ctx)
            self.ctx = None

    @staticmethod
    def _bg(w):
        vph = getattr(w, "v_phi", None)
        return [_c(w.v_r), _c(w.v_theta), _c(vph if vph is not None else np.zeros_like(w.v_r)),
                _c(w.alpha), _c(w.psi), _c(w.kappa_a), _c(w.kappa_s), _c(w.f_eq)]

    def set_background(self, w):
        arrs = self._bg(w)
        rc = lib().orc_set_background(self.ctx, *[_p(a) for a in arrs])
        assert rc == 0

    def update_background(self, w):
        """new background: the state is remapped to the new comoving frames (forward in time)"""
        arrs = self._bg(w)
        rc = lib().orc_update_background(self.ctx, *[_p(a) for a in arrs])
        assert rc == 0

    def set_state(self, f):
        f = _c(f).reshape(-1)
        assert f.size == np.prod(self.shape)
        assert lib().orc_set_state(self.ctx, _p(f)) == 0

    def state(self):
        out = np.zeros(self.shape)
        lib().orc_get_state(self.ctx, _p(out))
        return out

    def max_dt(self, cfl=None):
        return lib().orc_max_dt(self.ctx, self.w.cfl if cfl is None else cfl)

    def step(self, dt, n=1):
        rc = lib().orc_step(self.ctx, dt, n)
        if rc:
            raise RuntimeError(f"orc_step failed ({rc})")

    def step_sample(self, dt, zones):
        zones = np.ascontiguousarray(zones, dtype=np.int32)
        out = np.zeros((len(zones),) + self.shape[1:])
        rc = lib().orc_step_sample(self.ctx, dt, len(zones), zones.ctypes.data_as(_ip), _p(out))
        if rc:
            raise RuntimeError(f"orc_step_sample failed ({rc})")
        return out

    def time_levels(self, max_level):
        lev = np.zeros(self.w.n_zones, dtype=np.int32)
        assert lib().orc_time_levels(self.ctx, max_level, lev.ctypes.data_as(_ip)) == 0
        return lev

    def set_levels(self, levels):
        """per-zone time levels for local time stepping (None: global step)"""
        if levels is None:
            assert lib().orc_set_levels(self.ctx, None) == 0
            return
        self._lev = np.ascontiguousarray(levels, dtype=np.int32)
        assert lib().orc_set_levels(self.ctx, self._lev.ctypes.data_as(_ip)) == 0

    def source_terms(self):
        """[zone][5]: Q_Ye, Q_E, Q_M,r, Q_M,theta, Q_M,phi of the last full step"""
        q = np.zeros((self.w.n_zones, 5))
        assert lib().orc_source_terms(self.ctx, _p(q)) == 0
        return q

    def moments(self):
        zm = np.zeros((self.w.n_zones, self.w.n_species, 5))
        tot = np.zeros((self.w.n_species, 3))
        assert lib().orc_moments(self.ctx, _p(zm), _p(tot)) == 0
        return zm, tot

    def set_blend_mode(self, mode):
        lib().orc_set_blend_mode(self.ctx, mode)

    def n_faces(self):
        return lib().orc_n_faces(self.ctx)

    def geometry(self):
        nz = self.w.n_zones
        vol, rc, thc = np.zeros(nz), np.zeros(nz), np.zeros(nz)
        lib().orc_geometry(self.ctx, _p(vol), _p(rc), _p(thc))
        return vol, rc, thc

    def face_geom(self, fid):
        """(zone on the L side, zone on the R side (-1: ghost or inactive), axis, area, active)"""
        z = np.zeros(2, dtype=np.int32)
        info = np.zeros(3)
        assert lib().orc_face_geom(self.ctx, fid, z.ctypes.data_as(_ip), _p(info)) == 0
        return int(z[0]), int(z[1]), int(info[0]), float(info[1]), bool(info[2])

    def face_debug(self, fid, dt):
        blk = self.shape[1:]
        flw, flux, info = np.zeros(blk), np.zeros(blk), np.zeros(8)
        dN = np.zeros((2,) + blk)
        assert lib().orc_face_debug(self.ctx, fid, dt, _p(flw), _p(flux), _p(dN), _p(info)) == 0
        return flw, flux, dN, info

    def remap_block(self, S, D, axis, rotate, density, X, general=False):
        X = _c(X)
        Y = np.zeros_like(X)
        lib().orc_remap_block(self.ctx, _p(_c(S)), _p(_c(D)), axis, rotate, density,
                              int(general), _p(X), _p(Y))
        return Y
