"""Thin ctypes binding of libbtx (include/btx.h).

Argument marshalling only: every step of the transport update runs in the HIP
kernels of libbtx.so.  torch is imported first so that the library shares
torch's HIP runtime (streams and device pointers are exchanged with it).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:                                   # share torch's HIP runtime when it is present
    import torch                       # noqa: F401
except Exception:                      # pragma: no cover - torch is part of the image
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbtx.so")

BTX_OK, BTX_E_INVAL, BTX_E_NOMEM, BTX_E_DEVICE, BTX_E_CFL, BTX_E_STATE, BTX_E_UNSUPPORTED = range(7)
PREC_FP64, PREC_MIXED = 0, 1
MU_LEGENDRE, MU_LOBATTO = 0, 1
GEOM_COLUMN, GEOM_AXISYM2D, GEOM_PLANAR = 0, 1, 2      # btx_geometry
ABI_SYMBOLS = ["btx_create", "btx_set_background", "btx_max_dt", "btx_set_state",
               "btx_get_state", "btx_step", "btx_moments", "btx_timing", "btx_destroy",
               "btx_last_error", "btx_update_background", "btx_batch_create",
               "btx_batch_set_background", "btx_batch_update_background",
               "btx_update_background_device", "btx_batch_update_background_device",
               "btx_batch_max_dt", "btx_batch_set_state", "btx_batch_get_state", "btx_batch_step",
               "btx_batch_use_graph", "btx_batch_shape", "btx_batch_moments", "btx_batch_destroy",
               "btx_batch_time_levels", "btx_batch_set_time_levels",
               "btx_source_terms", "btx_batch_source_terms", "btx_time_levels",
               "btx_set_time_levels", "btx_moments_device"]

_dp = C.POINTER(C.c_double)


class BtxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libbtx status {status}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_theta", C.c_int32), ("n_eps", C.c_int32),
                ("n_mu", C.c_int32), ("n_phi", C.c_int32), ("n_species", C.c_int32),
                ("geometry", C.c_int32), ("mu_rule", C.c_int32), ("phi_rule", C.c_int32),
                ("inner_bc", C.c_int32), ("outer_bc", C.c_int32), ("precision", C.c_int32),
                ("r_edges", _dp), ("theta_edges", _dp), ("dphi", C.c_double),
                ("eps_edges", _dp), ("fp64_threshold", C.c_double),
                ("theta_bc", C.c_int32), ("disk_radius", C.c_double), ("n_phi_zones", C.c_int32)]


class Background(C.Structure):
    _fields_ = [(n, _dp) for n in ("v_r", "v_theta", "alpha", "psi", "kappa_a", "kappa_s", "f_eq",
                                   "v_phi")]


_lib = None


def lib():
    """load libbtx.so; raises if it has not been built (no fallback exists)"""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.btx_create.argtypes = [C.POINTER(GridDesc), C.c_int, vp, C.POINTER(vp)]
        L.btx_set_background.argtypes = [vp, C.POINTER(Background)]
        L.btx_update_background.argtypes = [vp, C.POINTER(Background)]
        L.btx_batch_update_background.argtypes = [vp, C.c_int32, C.POINTER(Background)]
        L.btx_update_background_device.argtypes = [vp, C.POINTER(Background)]
        L.btx_batch_update_background_device.argtypes = [vp, C.c_int32, C.POINTER(Background)]
        L.btx_max_dt.argtypes = [vp, C.c_double, _dp]
        L.btx_set_state.argtypes = [vp, vp, C.c_int]
        L.btx_get_state.argtypes = [vp, vp, C.c_int]
        L.btx_step.argtypes = [vp, C.c_double, C.c_int32]
        L.btx_moments.argtypes = [vp, _dp, _dp]
        L.btx_timing.argtypes = [vp, C.c_int, _dp, C.POINTER(C.c_int64), C.c_int]
        L.btx_destroy.argtypes = [vp]
        L.btx_batch_create.argtypes = [C.POINTER(GridDesc), C.c_int32, C.c_int, vp, C.c_char_p,
                                       C.POINTER(vp)]
        L.btx_batch_set_background.argtypes = [vp, C.c_int32, C.POINTER(Background)]
        L.btx_batch_max_dt.argtypes = [vp, C.c_int32, C.c_double, _dp]
        L.btx_batch_set_state.argtypes = [vp, C.c_int32, vp, C.c_int]
        L.btx_batch_get_state.argtypes = [vp, C.c_int32, vp, C.c_int]
        L.btx_batch_step.argtypes = [vp, _dp, C.c_int32]
        L.btx_batch_use_graph.argtypes = [vp, C.c_int]
        L.btx_batch_shape.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.btx_batch_moments.argtypes = [vp, C.c_int32, _dp, _dp]
        L.btx_source_terms.argtypes = [vp, _dp]
        L.btx_moments_device.argtypes = [vp, vp, vp]
        L.btx_time_levels.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
        L.btx_set_time_levels.argtypes = [vp, C.POINTER(C.c_int32)]
        L.btx_batch_source_terms.argtypes = [vp, C.c_int32, _dp]
        L.btx_batch_time_levels.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
        L.btx_batch_set_time_levels.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
        L.btx_batch_destroy.argtypes = [vp]
        L.btx_last_error.restype = C.c_char_p
        for name in ABI_SYMBOLS:
            if name != "btx_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status):
    if status != BTX_OK:
        raise BtxError(status, lib().btx_last_error().decode())


def _p(a):
    return a.ctypes.data_as(_dp)


def _need(ok, msg, exc=ValueError):
    if not ok:
        raise exc(msg)


def _desc(w, precision, fp64_threshold):
    keep = [np.ascontiguousarray(w.r_edges, float).reshape(-1),
            np.ascontiguousarray(w.theta_edges, float).reshape(-1),
            np.ascontiguousarray(w.eps_edges, float).reshape(-1)]
    # the library reads as many edges as the counts say
    _need(keep[0].size >= w.n_r + 1, f"r_edges needs {w.n_r + 1} values")
    _need(w.geometry != GEOM_AXISYM2D or keep[1].size >= w.n_theta + 1,
          f"theta_edges needs {w.n_theta + 1} values")
    _need(keep[2].size >= w.n_eps + 1, f"eps_edges needs {w.n_eps + 1} values")
    d = GridDesc(w.n_r, w.n_theta, w.n_eps, w.n_mu, w.n_phi, w.n_species, w.geometry,
                 MU_LEGENDRE if w.mu_rule == "legendre" else MU_LOBATTO, w.phi_rule,
                 w.inner_bc, w.outer_bc, precision, _p(keep[0]), _p(keep[1]),
                 float(w.dphi), _p(keep[2]), float(fp64_threshold), int(w.theta_bc),
                 float(w.disk_radius), int(w.n_phi_zones))
    return d, keep


def _background(w, grid):
    """the background arrays of w, checked against the sizes of grid (the
    workload the context or model was created from)"""
    nz, nk = grid.n_zones, grid.n_zones * grid.n_species * grid.n_eps
    arrs = [np.ascontiguousarray(a, float).reshape(-1) for a in
            (w.v_r, w.v_theta, w.alpha, w.psi, w.kappa_a, w.kappa_s, w.f_eq)]
    for name, a, n in zip(("v_r", "v_theta", "alpha", "psi", "kappa_a", "kappa_s", "f_eq"), arrs,
                          (nz, nz, nz, nz, nk, nk, nk)):
        _need(a.size == n, f"{name} has {a.size} values, the grid needs {n}")
    vph = getattr(w, "v_phi", None)
    if vph is not None:
        arrs.append(np.ascontiguousarray(vph, float).reshape(-1))
        _need(arrs[-1].size == nz, f"v_phi has {arrs[-1].size} values, the grid needs {nz}")
    return Background(*[_p(a) for a in arrs]), arrs


def _background_device(bg, grid, device):
    """a Background of device pointers from a mapping of contiguous FP64 GPU
    tensors (v_r, v_theta, alpha, psi, kappa_a, kappa_s, f_eq, optional
    v_phi), checked against the sizes of grid"""
    import torch
    nz, nk = grid.n_zones, grid.n_zones * grid.n_species * grid.n_eps
    names = ("v_r", "v_theta", "alpha", "psi", "kappa_a", "kappa_s", "f_eq")
    ts = []
    for name, n in zip(names, (nz, nz, nz, nz, nk, nk, nk)):
        t = bg[name]
        _device_tensor(t, n, torch.float64, device)
        ts.append(t)
    vph = bg.get("v_phi")
    if vph is not None:
        _device_tensor(vph, nz, torch.float64, device)
        ts.append(vph)
    return Background(*[C.cast(C.c_void_p(t.data_ptr()), _dp) for t in ts]), ts


def _device_tensor(t, n, dtype, device):
    """a GPU tensor the library may read or write n values of dtype through"""
    _need(t.is_cuda and t.is_contiguous(), "the tensor must be a contiguous GPU tensor")
    _need(t.device.index == device, f"the tensor is on GPU {t.device.index}, the context on {device}")
    _need(t.numel() == n, f"the tensor has {t.numel()} values, the state {n}")
    _need(t.dtype == dtype, f"the tensor is {t.dtype}, the state {dtype}", TypeError)


class Context:
    """one transport grid on one GPU (btx_create ... btx_destroy)"""

    def __init__(self, w, device=0, stream=None, precision=None, fp64_threshold=1.0):
        self.w = w
        self.precision = w.precision if precision is None else precision
        self.dtype = np.float64 if self.precision == PREC_FP64 else np.float32
        d, self._keep = _desc(w, self.precision, fp64_threshold)
        h = C.c_void_p()
        _check(lib().btx_create(C.byref(d), device, C.c_void_p(stream or 0), C.byref(h)))
        self.h = h
        self.device = device
        self.shape = (w.n_zones, w.n_species, w.n_eps, w.n_dir)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().btx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_background(self, w=None):
        bg, keep = _background(w or self.w, self.w)
        _check(lib().btx_set_background(self.h, C.byref(bg)))

    def update_background(self, w):
        """evolve the background: the state is remapped into the new comoving frames"""
        bg, keep = _background(w, self.w)
        _check(lib().btx_update_background(self.h, C.byref(bg)))

    def update_background_device(self, bg):
        """update_background from FP64 GPU tensors already on this context's device
        (a mapping: v_r, v_theta, alpha, psi, kappa_a, kappa_s, f_eq, optional v_phi)"""
        b, keep = _background_device(bg, self.w, self.device)
        _check(lib().btx_update_background_device(self.h, C.byref(b)))

    def max_dt(self, cfl=None):
        out = C.c_double()
        _check(lib().btx_max_dt(self.h, self.w.cfl if cfl is None else cfl, C.byref(out)))
        return out.value

    def set_state(self, f):
        """f: numpy array (host) or torch tensor on the GPU, dtype of the precision"""
        n = int(np.prod(self.shape))
        if torch is not None and isinstance(f, torch.Tensor):
            _device_tensor(f, n, torch.float64 if self.dtype == np.float64 else torch.float32, self.device)
            _check(lib().btx_set_state(self.h, C.c_void_p(f.data_ptr()), 1))
        else:
            a = np.ascontiguousarray(f, dtype=self.dtype).reshape(-1)
            _need(a.size == n, f"the state has {n} values, not {a.size}")
            _check(lib().btx_set_state(self.h, C.c_void_p(a.ctypes.data), 0))

    def get_state(self, out=None):
        """the state as a numpy array, or into out (a GPU tensor of the state's size and dtype)"""
        if out is not None:
            _need(torch is not None and isinstance(out, torch.Tensor), "out must be a torch tensor", TypeError)
            _device_tensor(out, int(np.prod(self.shape)),
                           torch.float64 if self.dtype == np.float64 else torch.float32, self.device)
            _check(lib().btx_get_state(self.h, C.c_void_p(out.data_ptr()), 1))
            return out
        a = np.empty(self.shape, dtype=self.dtype)
        _check(lib().btx_get_state(self.h, C.c_void_p(a.ctypes.data), 0))
        return a

    def step(self, dt, n=1):
        _check(lib().btx_step(self.h, float(dt), int(n)))

    def moments(self):
        zm = np.zeros((self.w.n_zones, self.w.n_species, 5))
        tot = np.zeros((self.w.n_species, 3))
        _check(lib().btx_moments(self.h, _p(zm), _p(tot)))
        return zm, tot

    def moments_device(self, zone_moments=None, totals=None):
        """btx_moments_device: moments into float64 GPU tensors ([zone][species][5],
        [species][3]; either may be None), enqueued on the context's stream"""
        ptrs = []
        for t, n in ((zone_moments, self.w.n_zones * self.w.n_species * 5), (totals, self.w.n_species * 3)):
            if t is None:
                ptrs.append(None)
                continue
            _need(torch is not None and isinstance(t, torch.Tensor), "outputs must be torch tensors", TypeError)
            _device_tensor(t, n, torch.float64, self.device)
            ptrs.append(C.c_void_p(t.data_ptr()))
        _check(lib().btx_moments_device(self.h, ptrs[0], ptrs[1]))
        return zone_moments, totals

    def time_levels(self, max_level):
        """the library's proposal of a time level per zone (local time stepping)"""
        lev = np.zeros(self.w.n_zones, dtype=np.int32)
        _check(lib().btx_time_levels(self.h, int(max_level), lev.ctypes.data_as(C.POINTER(C.c_int32))))
        return lev

    def set_time_levels(self, levels):
        """adopt per-zone time levels (None: the global step); one step is then
        2^max(levels) substeps of dt"""
        if levels is None:
            _check(lib().btx_set_time_levels(self.h, None))
            return
        self._lev = np.ascontiguousarray(levels, dtype=np.int32)
        _check(lib().btx_set_time_levels(self.h, self._lev.ctypes.data_as(C.POINTER(C.c_int32))))

    def source_terms(self):
        """[zone][5]: Q_Ye, Q_E, Q_M,r, Q_M,theta, Q_M,phi of the last step"""
        q = np.zeros((self.w.n_zones, 5))
        _check(lib().btx_source_terms(self.h, _p(q)))
        return q

    def timing(self, enable=True, reset=False):
        ms = np.zeros(2)
        n = (C.c_int64 * 2)()
        _check(lib().btx_timing(self.h, int(enable), _p(ms), n, int(reset)))
        return ms, np.array([n[0], n[1]])


class Batch:
    """independent models stepped together (btx_batch_create ... btx_batch_destroy)"""

    def __init__(self, workloads, device=0, stream=None, precision=None, tune_cache=None,
                 fp64_threshold=1.0):
        self.ws = list(workloads)
        self.device = device
        self.precision = self.ws[0].precision if precision is None else precision
        self.dtype = np.float64 if self.precision == PREC_FP64 else np.float32
        descs = (GridDesc * len(self.ws))()
        self._keep = []
        for k, w in enumerate(self.ws):
            d, keep = _desc(w, self.precision, fp64_threshold)
            descs[k] = d
            self._keep.append(keep)
        h = C.c_void_p()
        path = None if tune_cache is None else str(tune_cache).encode()
        _check(lib().btx_batch_create(descs, len(self.ws), device, C.c_void_p(stream or 0), path,
                                      C.byref(h)))
        self.h = h
        self.shapes = [(w.n_zones, w.n_species, w.n_eps, w.n_dir) for w in self.ws]

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().btx_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_background(self, m, w=None):
        bg, keep = _background(w or self.ws[m], self.ws[m])
        _check(lib().btx_batch_set_background(self.h, m, C.byref(bg)))

    def update_background(self, m, w):
        bg, keep = _background(w, self.ws[m])
        _check(lib().btx_batch_update_background(self.h, m, C.byref(bg)))

    def update_background_device(self, m, bg):
        b, keep = _background_device(bg, self.ws[m], self.device)
        _check(lib().btx_batch_update_background_device(self.h, m, C.byref(b)))

    def max_dt(self, m, cfl=None):
        out = C.c_double()
        _check(lib().btx_batch_max_dt(self.h, m, self.ws[m].cfl if cfl is None else cfl, C.byref(out)))
        return out.value

    def set_state(self, m, f):
        a = np.ascontiguousarray(f, dtype=self.dtype).reshape(-1)
        _need(a.size == int(np.prod(self.shapes[m])), f"model {m}'s state has {int(np.prod(self.shapes[m]))} values")
        _check(lib().btx_batch_set_state(self.h, m, C.c_void_p(a.ctypes.data), 0))

    def get_state(self, m):
        a = np.empty(self.shapes[m], dtype=self.dtype)
        _check(lib().btx_batch_get_state(self.h, m, C.c_void_p(a.ctypes.data), 0))
        return a

    def step(self, dts, n=1):
        d = np.ascontiguousarray(dts, dtype=np.float64).reshape(-1)
        _need(d.size == len(self.ws), f"one dt per model ({len(self.ws)})")
        _check(lib().btx_batch_step(self.h, _p(d), int(n)))

    def use_graph(self, enable):
        _check(lib().btx_batch_use_graph(self.h, int(enable)))

    def shape(self, m):
        a, b = C.c_int32(), C.c_int32()
        _check(lib().btx_batch_shape(self.h, m, C.byref(a), C.byref(b)))
        return a.value, b.value

    def moments(self, m):
        w = self.ws[m]
        zm = np.zeros((w.n_zones, w.n_species, 5))
        tot = np.zeros((w.n_species, 3))
        _check(lib().btx_batch_moments(self.h, m, _p(zm), _p(tot)))
        return zm, tot

    def time_levels(self, m, max_level):
        """the library's proposal of a time level per zone of model m"""
        lev = np.zeros(self.ws[m].n_zones, dtype=np.int32)
        _check(lib().btx_batch_time_levels(self.h, m, int(max_level), lev.ctypes.data_as(C.POINTER(C.c_int32))))
        return lev

    def set_time_levels(self, m, levels):
        """levels of model m (None: all zones at level 0); the batch then steps in place"""
        if levels is None:
            _check(lib().btx_batch_set_time_levels(self.h, m, None))
            return
        lev = np.ascontiguousarray(levels, dtype=np.int32).reshape(-1)
        _need(lev.size == self.ws[m].n_zones, f"model {m} has {self.ws[m].n_zones} zones")
        _check(lib().btx_batch_set_time_levels(self.h, m, lev.ctypes.data_as(C.POINTER(C.c_int32))))

    def source_terms(self, m):
        """[zone][5]: Q_Ye, Q_E, Q_M,r, Q_M,theta, Q_M,phi of model m's last step"""
        q = np.zeros((self.ws[m].n_zones, 5))
        _check(lib().btx_batch_source_terms(self.h, m, _p(q)))
        return q
