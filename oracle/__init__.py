"""ctypes front end of the plain FP64 CPU oracle (oracle/sphref.c).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg use it to check and time the GPU library.
It imports nothing from the GPU package; its inputs come from the seeded
generator, never from the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class Geometry(C.Structure):
    _fields_ = [("dim", C.c_int32), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("n_holes", C.c_int32), ("holes", C.POINTER(C.c_double)),
                ("domain", C.c_int32), ("phi", C.POINTER(C.c_double)),
                ("phi_n", C.c_int32 * 3), ("phi_lo", C.c_double * 3), ("phi_hi", C.c_double * 3),
                ("n_curves", C.c_int32), ("curve_off", C.POINTER(C.c_int32)),
                ("curve_pts", C.POINTER(C.c_double)), ("curve_ends", C.POINTER(C.c_int32)),
                ("n_corners", C.c_int32), ("corners", C.POINTER(C.c_double)),
                ("n_patches", C.c_int32), ("curve_patches", C.POINTER(C.c_int32))]


class Sizing(C.Structure):
    _fields_ = [("kind", C.c_int32), ("h0", C.c_double), ("grad", C.c_double),
                ("dcap", C.c_double), ("point", C.c_double * 3),
                ("grid", C.POINTER(C.c_double)), ("grid_n", C.c_int32 * 3),
                ("grid_lo", C.c_double * 3), ("grid_hi", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [("p0", C.c_double), ("eps_damp", C.c_double), ("tol", C.c_double),
                ("dt_max", C.c_double), ("boundary_weighting", C.c_int32),
                ("reset_period", C.c_int32), ("sample_every", C.c_int32),
                ("window_samples", C.c_int32), ("ramp_steps", C.c_int32),
                ("ramp_halving", C.c_int32), ("phase2_steps", C.c_int32),
                ("max_phase1_steps", C.c_int32), ("sum_order", C.c_int32),
                ("kernel_support", C.c_double), ("boundary_scale", C.c_double)]


F_H, F_AP, F_A, F_VT, F_GAMMA, F_VMID = range(6)

_dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


_lib_omp = None


def lib(openmp=False):
    """The oracle library; openmp=True loads the build whose per-particle
    loops run on OpenMP threads (bit-identical results, for timing)."""
    global _lib, _lib_omp
    if openmp:
        if _lib_omp is None:
            _lib_omp = _load(_build.LIB_OMP, openmp=True)
        return _lib_omp
    if _lib is None:
        _lib = _load(_build.LIB, openmp=False)
    return _lib


def _load(path, openmp):
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(
            os.path.join(_build.HERE, "sphref.c")):
        _build.build(openmp=openmp)
    if True:
        L = C.CDLL(path)
        L.sphref_W.restype = C.c_double
        L.sphref_W.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.sphref_dWdr.restype = C.c_double
        L.sphref_dWdr.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.sphref_h_at.restype = C.c_double
        L.sphref_h_at.argtypes = [C.POINTER(Geometry), C.POINTER(Sizing), _dp]
        L.sphref_project.argtypes = [C.POINTER(Geometry), C.c_int32, _dp]
        L.sphref_n_features.argtypes = [C.POINTER(Geometry)]
        L.sphref_feature_type.argtypes = [C.POINTER(Geometry), C.c_int32]
        L.sphref_boundary_normal.argtypes = [C.POINTER(Geometry), C.c_int32, C.c_int32, _dp, _dp]
        L.sphref_boundary_normal_at.argtypes = [C.POINTER(Geometry), C.c_int32, C.c_int32, _dp,
                                                _dp, _dp]
        _ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.sphref_tags.argtypes = [C.POINTER(Geometry), _ip, _ip, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32), C.c_void_p]
        L.sphref_create.argtypes = [C.POINTER(Geometry), C.POINTER(Sizing), C.POINTER(Params),
                                    C.c_int64, _dp, np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS"),
                                    C.POINTER(C.c_void_p)]
        L.sphref_destroy.argtypes = [C.c_void_p]
        L.sphref_destroy.restype = None
        L.sphref_step.argtypes = [C.c_void_p, C.c_int32]
        L.sphref_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.sphref_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.sphref_get_field.argtypes = [C.c_void_p, C.c_int32, _dp]
        L.sphref_neighbors.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                       C.POINTER(C.c_int64)]
        L.sphref_error.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.sphref_group_state.argtypes = [C.c_void_p, C.c_int32, _dp]
        L.sphref_counters.argtypes = [C.c_void_p, _dp]
        L.sphref_control_replay.argtypes = [C.POINTER(Params), C.c_int32, _dp, _dp,
                                            np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS"),
                                            np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS"), _dp]
        L.sphref_sample.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.sphref_last_error.restype = C.c_char_p
    return L


def _err():
    return lib().sphref_last_error().decode()


def make_geometry(dim, lo, hi, holes, domain=0, level=None):
    holes = np.ascontiguousarray(np.asarray(holes, np.float64).reshape(-1, 15))
    g = Geometry()
    g.dim = dim
    for a in range(3):
        g.lo[a] = float(lo[a]) if a < len(lo) else 0.0
        g.hi[a] = float(hi[a]) if a < len(hi) else 0.0
    g.n_holes = holes.shape[0]
    g.holes = holes.ctypes.data_as(C.POINTER(C.c_double)) if holes.size else None
    g.domain = int(domain)
    g._keep = holes
    if level is not None:
        ph = np.ascontiguousarray(np.asarray(level["phi"], np.float64).ravel())
        g.phi = ph.ctypes.data_as(C.POINTER(C.c_double))
        g._keep_phi = ph
        for a in range(3):
            g.phi_n[a] = int(level["n"][a])
            g.phi_lo[a] = float(level["lo"][a])
            g.phi_hi[a] = float(level["hi"][a])
        if level.get("curves"):
            cv = level["curves"]
            off = np.ascontiguousarray(np.asarray(cv["off"], np.int32))
            pts = np.ascontiguousarray(np.asarray(cv["pts"], np.float64).reshape(-1, 3))
            ends = np.ascontiguousarray(np.asarray(cv["ends"], np.int32).reshape(-1, 2))
            cor = np.ascontiguousarray(np.asarray(cv["corners"], np.float64).reshape(-1, 3))
            g.n_curves = len(off) - 1
            g.curve_off = off.ctypes.data_as(C.POINTER(C.c_int32))
            g.curve_pts = pts.ctypes.data_as(C.POINTER(C.c_double))
            g.curve_ends = ends.ctypes.data_as(C.POINTER(C.c_int32))
            g.n_corners = cor.shape[0]
            g.corners = cor.ctypes.data_as(C.POINTER(C.c_double))
            g._keep_curves = (off, pts, ends, cor)
            if "patches" in cv:
                cp = np.ascontiguousarray(np.asarray(cv["patches"], np.int32).reshape(-1, 2))
                g.n_patches = int(cv["n_patches"])
                g.curve_patches = cp.ctypes.data_as(C.POINTER(C.c_int32))
                g._keep_patches = cp
    return g


def tags(geom, n_curves=0):
    """The cell tag system of a level-set geometry: (ctype, cindex) per grid
    cell (x fastest), the volume and patch counts, and the two patches
    beside each curve."""
    L = lib()
    nc = [max(int(geom.phi_n[a]) - 1, 1) for a in range(3)]
    if geom.dim == 2:
        nc[2] = 1
    ncell = nc[0] * nc[1] * nc[2]
    ct = np.empty(ncell, np.int32)
    ci = np.empty(ncell, np.int32)
    nv, npch = C.c_int32(), C.c_int32()
    cp = np.full(2 * max(n_curves, 1), -1, np.int32)
    rc = L.sphref_tags(C.byref(geom), ct, ci, C.byref(nv), C.byref(npch), cp.ctypes.data)
    if rc:
        raise RuntimeError("sphref_tags: " + L.sphref_last_error().decode())
    shape = (nc[2], nc[1], nc[0])
    return ct.reshape(shape), ci.reshape(shape), nv.value, npch.value, cp[:2 * n_curves].reshape(-1, 2)


def make_sizing(sz):
    s = Sizing()
    s.kind = int(sz["kind"])
    s.h0 = float(sz["h0"])
    s.grad = float(sz.get("grad", 0.0))
    s.dcap = float(sz.get("dcap", np.inf))
    for a in range(3):
        s.point[a] = float(sz.get("point", [0, 0, 0])[a])
    if "grid" in sz:
        g = np.ascontiguousarray(np.asarray(sz["grid"], np.float64).ravel())
        s.grid = g.ctypes.data_as(C.POINTER(C.c_double))
        s._keep = g
        for a in range(3):
            s.grid_n[a] = int(sz["grid_n"][a])
            s.grid_lo[a] = float(sz["grid_lo"][a])
            s.grid_hi[a] = float(sz["grid_hi"][a])
    return s


def make_params(p):
    q = Params()
    for name, _ in Params._fields_:
        setattr(q, name, type(getattr(q, name))(p.get(name, 0)))
    return q


def W(k, r, h):
    return lib().sphref_W(k, r, h)


def dWdr(k, r, h):
    return lib().sphref_dWdr(k, r, h)


class RefJob:
    """One relaxation job on the CPU oracle."""

    def __init__(self, wl, xyz=None, feature=None, params=None, openmp=False):
        L = self.L = lib(openmp)
        self.dim = wl.dim
        self.geom = make_geometry(wl.dim, wl.lo, wl.hi, wl.holes, wl.domain, wl.level)
        self.sizing = make_sizing(wl.sizing)
        self.params = make_params(params if params is not None else wl.params)
        xyz = np.ascontiguousarray(wl.xyz if xyz is None else xyz, dtype=np.float64)
        feature = np.ascontiguousarray(wl.feature if feature is None else feature, dtype=np.int32)
        self.n = xyz.shape[0]
        h = C.c_void_p()
        rc = L.sphref_create(C.byref(self.geom), C.byref(self.sizing), C.byref(self.params),
                             self.n, xyz, feature, C.byref(h))
        if rc:
            raise RuntimeError("sphref_create: " + L.sphref_last_error().decode())
        self.h = h
        self.feature = feature

    def __del__(self):
        if getattr(self, "h", None):
            self.L.sphref_destroy(self.h)
            self.h = None

    def step(self, n=1):
        rc = self.L.sphref_step(self.h, n)
        if rc:
            raise RuntimeError("sphref_step: " + self.L.sphref_last_error().decode())

    def set_state(self, xyz=None, vel=None):
        x = None if xyz is None else np.ascontiguousarray(xyz, np.float64)
        v = None if vel is None else np.ascontiguousarray(vel, np.float64)
        self.L.sphref_set_state(self.h, None if x is None else x.ctypes.data,
                               None if v is None else v.ctypes.data)

    def state(self):
        x = np.zeros((self.n, 3))
        v = np.zeros((self.n, 3))
        self.L.sphref_get_state(self.h, x.ctypes.data, v.ctypes.data)
        return x, v

    def field(self, which):
        shape = (self.n, 3) if which in (F_AP, F_A, F_VMID) else (self.n,)
        out = np.zeros(shape)
        if self.L.sphref_get_field(self.h, which, out):
            raise RuntimeError(self.L.sphref_last_error().decode())
        return out

    def neighbors(self):
        """CSR (offsets, ids, rel) of the current positions, ids ascending."""
        L = self.L
        npairs = C.c_int64()
        off = np.zeros(self.n + 1, np.int64)
        if L.sphref_neighbors(self.h, off.ctypes.data, None, None, 0, C.byref(npairs)):
            raise RuntimeError(self.L.sphref_last_error().decode())
        ids = np.zeros(max(npairs.value, 1), np.int32)
        rel = np.zeros(max(npairs.value, 1), np.int8)
        if L.sphref_neighbors(self.h, off.ctypes.data, ids.ctypes.data, rel.ctypes.data,
                              ids.size, C.byref(npairs)):
            raise RuntimeError(self.L.sphref_last_error().decode())
        return off, ids[:npairs.value], rel[:npairs.value]

    def sample(self, idx, cap_per=256):
        """Brute-force lists and sweep-A quantities of the particles idx at
        the current positions (any job size)."""
        idx = np.ascontiguousarray(idx, np.int64)
        m = idx.size
        cap = cap_per * max(m, 1)
        off = np.zeros(m + 1, np.int64)
        ids = np.zeros(cap, np.int32)
        rel = np.zeros(cap, np.int8)
        ap = np.zeros((m, 3))
        vt = np.zeros(m)
        gam = np.zeros(m)
        if self.L.sphref_sample(self.h, m, idx.ctypes.data, off.ctypes.data, ids.ctypes.data,
                               rel.ctypes.data, cap, ap.ctypes.data, vt.ctypes.data,
                               gam.ctypes.data):
            raise RuntimeError(self.L.sphref_last_error().decode())
        return off, ids[:off[-1]], rel[:off[-1]], ap, vt, gam

    def error(self):
        e = C.c_double()
        ph = C.c_int32()
        conv = C.c_int32()
        st = C.c_int64()
        self.L.sphref_error(self.h, C.byref(e), C.byref(ph), C.byref(conv), C.byref(st))
        return dict(e_sys=e.value, phase=ph.value, converged=bool(conv.value), step=st.value)

    def group_state(self, f):
        out = np.zeros(10)
        self.L.sphref_group_state(self.h, f, out)
        keys = ["phase", "n_ph", "e_sys", "dt1", "dt", "vbar", "reset_next", "a_last", "a_prev", "n_windows"]
        return dict(zip(keys, out.tolist()))

    def counters(self):
        out = np.zeros(4)
        self.L.sphref_counters(self.h, out)
        return dict(steps=int(out[0]), escaped=int(out[1]), interactions=int(out[2]),
                    interactions_last=int(out[3]))


def control_replay(params, vbar, dt):
    p = make_params(params)
    vbar = np.ascontiguousarray(vbar, np.float64)
    dt = np.ascontiguousarray(dt, np.float64)
    n = vbar.size
    ph = np.zeros(n, np.int32)
    rs = np.zeros(n, np.int32)
    es = np.zeros(n)
    lib().sphref_control_replay(C.byref(p), n, vbar, dt, ph, rs, es)
    return ph, rs, es
