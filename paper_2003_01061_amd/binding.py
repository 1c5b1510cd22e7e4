"""ctypes binding of libsphmesh.so (include/sph_mesh.h): argument marshalling
only, every step of the relaxation runs in the library's HIP kernels.

Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsphmesh.so")

SPH_FP64, SPH_FP32_MIXED, SPH_FP32_COMPENSATED = 0, 1, 2
FIELD_H, FIELD_AP, FIELD_A, FIELD_VT, FIELD_GAMMA, FIELD_VMID = range(6)


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
                ("max_phase1_steps", C.c_int32), ("precision", C.c_int32),
                ("max_neighbors", C.c_int32), ("cell_factor", C.c_double),
                ("scan_tile", C.c_int32), ("cell_levels", C.c_int32),
                ("kernel_support", C.c_double), ("boundary_scale", C.c_double),
                ("use_graph", C.c_int32),
                ("debug_fields", C.c_int32), ("stream", C.c_void_p),
                ("n_particles", C.c_int64), ("seed", C.c_uint64), ("init", C.c_int32),
                ("mass_res", C.c_int32), ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p),
                ("alloc_ctx", C.c_void_p), ("verlet_skin", C.c_double)]

# device allocator callbacks (void *alloc(size_t, void *ctx), void free(void *, void *ctx))
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
SPH_INIT_DENSITY, SPH_INIT_UNIFORM = 0, 1


class BatchParams(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("max_particles", C.c_int64),
                ("max_cells", C.c_int64), ("max_jobs", C.c_int32), ("max_neighbors", C.c_int32),
                ("scan_tile", C.c_int32), ("use_graph", C.c_int32), ("debug_fields", C.c_int32), ("stream", C.c_void_p),
                ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p), ("alloc_ctx", C.c_void_p),
                ("verlet_skin", C.c_double)]


class SphError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} -> status {status}: {msg}")
        self.status = status


_lib = None
_dp = C.POINTER(C.c_double)


def lib():
    """Load libsphmesh.so; raise if it is missing (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python paper_2003_01061_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.sph_mesh_create_with_particles.argtypes = [C.POINTER(Geometry), C.POINTER(Sizing),
                                                     C.POINTER(Params), C.c_int64, vp, vp,
                                                     C.POINTER(vp)]
        L.sph_mesh_create.argtypes = [C.POINTER(Geometry), C.POINTER(Sizing), C.POINTER(Params),
                                      C.POINTER(vp)]
        L.sph_mesh_setup_info.argtypes = [vp, C.POINTER(C.c_double), vp, C.c_int32,
                                          C.POINTER(C.c_int32)]
        L.sph_job_setup.argtypes = [C.POINTER(Geometry), C.POINTER(Sizing), C.POINTER(Params),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), vp, C.c_int32, C.POINTER(C.c_int32),
                                    vp, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.sph_tags.argtypes = [C.POINTER(Geometry), vp, vp, C.POINTER(C.c_int32),
                               C.POINTER(C.c_int32), vp]
        L.sph_mesh_step.argtypes = [vp, C.c_int32]
        L.sph_mesh_positions.argtypes = [vp, vp, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.sph_mesh_error.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.sph_mesh_destroy.argtypes = [vp]
        L.sph_mesh_destroy.restype = None
        L.sph_mesh_last_error.restype = C.c_char_p
        L.sph_mesh_set_state.argtypes = [vp, vp, vp]
        L.sph_mesh_velocities.argtypes = [vp, vp]
        L.sph_mesh_neighbors.argtypes = [vp, vp, vp, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.sph_mesh_neighbors_of.argtypes = [vp, C.c_int32, vp, vp, vp, vp, C.c_int64,
                                            C.POINTER(C.c_int64)]
        L.sph_mesh_field.argtypes = [vp, C.c_int32, vp]
        L.sph_mesh_group_state.argtypes = [vp, C.c_int32, vp]
        L.sph_mesh_counters.argtypes = [vp, vp]
        L.sph_mesh_control_replay.argtypes = [C.POINTER(Params), C.c_int32, vp, vp, vp, vp, vp]
        L.sph_mesh_control_replay_noalloc.argtypes = [C.POINTER(Params), C.c_int32, vp, vp, vp,
                                                      vp, vp, vp]
        L.sph_mesh_profile.argtypes = [vp, C.c_int32]
        L.sph_mesh_kernel_stats.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.sph_mesh_kernel_count.restype = C.c_int32
        L.sph_mesh_kernel_name.argtypes = [C.c_int32]
        L.sph_mesh_kernel_name.restype = C.c_char_p
        L.sph_mesh_sync.argtypes = [vp]
        L.sph_mesh_device_bytes.argtypes = [vp]
        L.sph_mesh_device_bytes.restype = C.c_int64
        bpp = C.POINTER(BatchParams)
        L.sph_batch_footprint.argtypes = [bpp]
        L.sph_batch_footprint.restype = C.c_int64
        L.sph_job_cells.argtypes = [C.POINTER(Geometry), C.POINTER(Sizing), C.POINTER(Params)]
        L.sph_job_cells.restype = C.c_int64
        L.sph_batch_create.argtypes = [bpp, C.POINTER(vp)]
        L.sph_batch_add.argtypes = [vp, C.POINTER(Geometry), C.POINTER(Sizing), C.POINTER(Params),
                                    C.c_int64, vp, vp, C.POINTER(C.c_int32)]
        L.sph_batch_remove.argtypes = [vp, C.c_int32]
        L.sph_batch_step.argtypes = [vp, C.c_int32]
        L.sph_batch_sync.argtypes = [vp]
        L.sph_batch_status.argtypes = [vp, vp, vp, vp, C.c_int32]
        L.sph_batch_positions.argtypes = [vp, C.c_int32, vp, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.sph_batch_error.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.sph_batch_counters.argtypes = [vp, C.c_int32, vp]
        L.sph_batch_destroy.argtypes = [vp]
        L.sph_batch_destroy.restype = None
        _lib = L
    return _lib


def _check(fn, status):
    if status != 0:
        raise SphError(fn, status, lib().sph_mesh_last_error().decode())


def make_geometry(dim, lo, hi, holes, domain=0, level=None):
    holes = np.ascontiguousarray(np.asarray(holes, np.float64).reshape(-1, 15))
    g = Geometry()
    g.dim = dim
    for a in range(3):
        g.lo[a] = float(lo[a]) if a < len(lo) else 0.0
        g.hi[a] = float(hi[a]) if a < len(hi) else 0.0
    g.n_holes = holes.shape[0]
    g.holes = holes.ctypes.data_as(_dp) if holes.size else None
    g.domain = int(domain)
    g._keep = holes
    if level is not None:
        ph = np.ascontiguousarray(np.asarray(level["phi"], np.float64).ravel())
        g.phi = ph.ctypes.data_as(_dp)
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


_POINTERS = ("stream", "dev_alloc", "dev_free", "alloc_ctx")


def make_params(p, stream=None, allocator=None):
    """sph_params from a dict; allocator = (ALLOC_FN, FREE_FN) callbacks kept
    alive by the caller, or None for hipMalloc / hipFree."""
    q = Params()
    for name, typ in Params._fields_:
        if name in _POINTERS:
            continue
        setattr(q, name, typ(p.get(name, 0)).value)
    q.stream = stream
    if allocator is not None:
        q.dev_alloc = C.cast(allocator[0], C.c_void_p)
        q.dev_free = C.cast(allocator[1], C.c_void_p)
    return q


def torch_allocator():
    """Callbacks that take device memory from PyTorch's caching allocator on
    the current device and stream (keep the returned pair alive while the
    handle that uses it exists)."""
    import torch

    def alloc(nbytes, ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes)))
        except Exception:
            return None

    def free(ptr, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    return ALLOC_FN(alloc), FREE_FN(free)


def current_torch_stream():
    """The raw hipStream_t of PyTorch's current stream (None if unavailable)."""
    try:
        import torch
        if torch.cuda.is_available():
            h = torch.cuda.current_stream().cuda_stream
            return h or None
    except Exception:
        pass
    return None


class SphMesh:
    """One relaxation job on the GPU (libsphmesh.so handle)."""

    def __init__(self, wl, params=None, xyz=None, feature=None, stream=None, allocator=None,
                 **over):
        L = lib()
        p = dict(wl.params if params is None else params)
        p.update(over)
        self.dim = wl.dim
        self._geom = make_geometry(wl.dim, wl.lo, wl.hi, wl.holes, wl.domain, wl.level)
        self._sizing = make_sizing(wl.sizing)
        self._alloc = allocator
        self._params = make_params(p, stream, allocator)
        xyz = np.ascontiguousarray(wl.xyz if xyz is None else xyz, np.float64)
        feature = np.ascontiguousarray(wl.feature if feature is None else feature, np.int32)
        self.n = int(xyz.shape[0])
        h = C.c_void_p()
        _check("sph_mesh_create_with_particles", L.sph_mesh_create_with_particles(
            C.byref(self._geom), C.byref(self._sizing), C.byref(self._params), self.n,
            xyz.ctypes.data, feature.ctypes.data, C.byref(h)))
        self.h = h

    @classmethod
    def from_problem(cls, dim, lo, hi, holes, sizing, params, domain=0, stream=None,
                     allocator=None):
        """sph_mesh_create: the particles are placed by the library from the
        problem statement (params["n_particles"], "seed", "init",
        "mass_res")."""
        L = lib()
        self = cls.__new__(cls)
        self.dim = dim
        self._geom = make_geometry(dim, lo, hi, holes, domain, None)
        self._sizing = make_sizing(sizing)
        self._alloc = allocator
        self._params = make_params(params, stream, allocator)
        h = C.c_void_p()
        _check("sph_mesh_create", L.sph_mesh_create(C.byref(self._geom), C.byref(self._sizing),
                                                    C.byref(self._params), C.byref(h)))
        self.h = h
        info = self.setup_info()
        self.n = int(sum(info["counts"]))
        return self

    def setup_info(self):
        L = lib()
        s = C.c_double()
        nf = C.c_int32()
        _check("sph_mesh_setup_info", L.sph_mesh_setup_info(self.h, C.byref(s), None, 0, C.byref(nf)))
        counts = np.zeros(max(nf.value, 1), np.int64)
        _check("sph_mesh_setup_info", L.sph_mesh_setup_info(self.h, C.byref(s), counts.ctypes.data,
                                                            counts.size, C.byref(nf)))
        return dict(h_scale=s.value, counts=counts[:nf.value].tolist())

    def close(self):
        if getattr(self, "h", None):
            lib().sph_mesh_destroy(self.h)
            self.h = None

    __del__ = close

    def step(self, n=1):
        _check("sph_mesh_step", lib().sph_mesh_step(self.h, int(n)))

    def sync(self):
        _check("sph_mesh_sync", lib().sph_mesh_sync(self.h))

    def positions(self, with_feature=False):
        x = np.zeros((self.n, 3))
        f = np.zeros(self.n, np.int32) if with_feature else None
        nout = C.c_int64()
        _check("sph_mesh_positions", lib().sph_mesh_positions(
            self.h, x.ctypes.data, None if f is None else f.ctypes.data, self.n, C.byref(nout)))
        return (x, f) if with_feature else x

    def velocities(self):
        v = np.zeros((self.n, 3))
        _check("sph_mesh_velocities", lib().sph_mesh_velocities(self.h, v.ctypes.data))
        return v

    def state(self):
        return self.positions(), self.velocities()

    def set_state(self, xyz=None, vel=None):
        x = None if xyz is None else np.ascontiguousarray(xyz, np.float64)
        v = None if vel is None else np.ascontiguousarray(vel, np.float64)
        _check("sph_mesh_set_state", lib().sph_mesh_set_state(
            self.h, None if x is None else x.ctypes.data, None if v is None else v.ctypes.data))

    def neighbors(self):
        L = lib()
        off = np.zeros(self.n + 1, np.int64)
        npairs = C.c_int64()
        _check("sph_mesh_neighbors", L.sph_mesh_neighbors(self.h, off.ctypes.data, None, None, 0,
                                                          C.byref(npairs)))
        ids = np.zeros(max(npairs.value, 1), np.int32)
        rel = np.zeros(max(npairs.value, 1), np.int8)
        _check("sph_mesh_neighbors", L.sph_mesh_neighbors(self.h, off.ctypes.data, ids.ctypes.data,
                                                          rel.ctypes.data, ids.size,
                                                          C.byref(npairs)))
        return off, ids[:npairs.value], rel[:npairs.value]

    def neighbors_of(self, idx):
        """Lists of the particles idx only (caller ids), as neighbors() gives
        them: offsets into ids / rel per requested particle."""
        L = lib()
        idx = np.ascontiguousarray(idx, np.int64)
        off = np.zeros(idx.size + 1, np.int64)
        npairs = C.c_int64()
        _check("sph_mesh_neighbors_of", L.sph_mesh_neighbors_of(
            self.h, idx.size, idx.ctypes.data, off.ctypes.data, None, None, 0, C.byref(npairs)))
        ids = np.zeros(max(npairs.value, 1), np.int32)
        rel = np.zeros(max(npairs.value, 1), np.int8)
        _check("sph_mesh_neighbors_of", L.sph_mesh_neighbors_of(
            self.h, idx.size, idx.ctypes.data, off.ctypes.data, ids.ctypes.data, rel.ctypes.data,
            ids.size, C.byref(npairs)))
        return off, ids[:npairs.value], rel[:npairs.value]

    def field(self, which):
        shape = (self.n, 3) if which in (FIELD_AP, FIELD_A, FIELD_VMID) else (self.n,)
        out = np.zeros(shape)
        _check("sph_mesh_field", lib().sph_mesh_field(self.h, which, out.ctypes.data))
        return out

    def error(self):
        e = C.c_double()
        ph = C.c_int32()
        conv = C.c_int32()
        st = C.c_int64()
        _check("sph_mesh_error", lib().sph_mesh_error(self.h, C.byref(e), C.byref(ph),
                                                      C.byref(conv), C.byref(st)))
        return dict(e_sys=e.value, phase=ph.value, converged=bool(conv.value), step=st.value)

    def group_state(self, f):
        out = np.zeros(10)
        _check("sph_mesh_group_state", lib().sph_mesh_group_state(self.h, f, out.ctypes.data))
        keys = ["phase", "n_ph", "e_sys", "dt1", "dt", "vbar", "reset_next", "a_last", "a_prev",
                "n_windows"]
        return dict(zip(keys, out.tolist()))

    def counters(self):
        out = np.zeros(4)
        _check("sph_mesh_counters", lib().sph_mesh_counters(self.h, out.ctypes.data))
        return dict(steps=int(out[0]), escaped=int(out[1]), interactions=int(out[2]),
                    interactions_last=int(out[3]))

    def list_builds(self):
        """Verlet candidate lists built so far (0 without a skin)."""
        v = C.c_int64()
        _check("sph_mesh_list_builds", lib().sph_mesh_list_builds(self.h, C.byref(v)))
        return int(v.value)

    def profile(self, enable=True):
        _check("sph_mesh_profile", lib().sph_mesh_profile(self.h, 1 if enable else 0))

    def kernel_stats(self):
        L = lib()
        out = {}
        for k in range(L.sph_mesh_kernel_count()):
            ms = C.c_double()
            cnt = C.c_int64()
            _check("sph_mesh_kernel_stats", L.sph_mesh_kernel_stats(self.h, k, C.byref(ms),
                                                                    C.byref(cnt)))
            out[L.sph_mesh_kernel_name(k).decode()] = (ms.value, cnt.value)
        return out

    def device_bytes(self):
        return int(lib().sph_mesh_device_bytes(self.h))


class JobSpec:
    """Marshalled description of one job (geometry, sizing, parameters,
    particles) for sph_batch_add / sph_job_cells."""

    def __init__(self, wl, params=None, xyz=None, feature=None, **over):
        p = dict(wl.params if params is None else params)
        p.update(over)
        self.dim = wl.dim
        self.geom = make_geometry(wl.dim, wl.lo, wl.hi, wl.holes, wl.domain, wl.level)
        self.sizing = make_sizing(wl.sizing)
        self.params = make_params(p)
        self.xyz = np.ascontiguousarray(wl.xyz if xyz is None else xyz, np.float64)
        self.feature = np.ascontiguousarray(wl.feature if feature is None else feature, np.int32)
        self.n = int(self.xyz.shape[0])

    def cells(self):
        return int(lib().sph_job_cells(C.byref(self.geom), C.byref(self.sizing),
                                       C.byref(self.params)))


def batch_params(dim, precision=SPH_FP64, max_particles=0, max_cells=1, max_jobs=1,
                 max_neighbors=0, use_graph=1, debug_fields=0, stream=None, scan_tile=0,
                 allocator=None, verlet_skin=0.0):
    bp = BatchParams()
    bp.dim, bp.precision = dim, precision
    bp.verlet_skin = float(verlet_skin)
    bp.max_particles, bp.max_cells, bp.max_jobs = max_particles, max_cells, max_jobs
    bp.max_neighbors, bp.use_graph, bp.debug_fields = max_neighbors, use_graph, debug_fields
    bp.scan_tile = scan_tile
    bp.stream = stream
    if allocator is not None:
        bp.dev_alloc = C.cast(allocator[0], C.c_void_p)
        bp.dev_free = C.cast(allocator[1], C.c_void_p)
    return bp


def job_setup(dim, lo, hi, holes, sizing, params, domain=0, particles=True):
    """sph_job_setup (host only): the split of params["n_particles"] over the
    features, the scale of h and, if particles, the initial particles."""
    L = lib()
    g = make_geometry(dim, lo, hi, holes, domain, None)
    sz = make_sizing(sizing)
    p = make_params(params)
    s, h0, gr = C.c_double(), C.c_double(), C.c_double()
    nf, n = C.c_int32(), C.c_int64()
    counts = np.zeros(256, np.int64)
    _check("sph_job_setup", L.sph_job_setup(C.byref(g), C.byref(sz), C.byref(p), C.byref(s),
                                            C.byref(h0), C.byref(gr), counts.ctypes.data,
                                            counts.size, C.byref(nf), None, None, 0, C.byref(n)))
    out = dict(h_scale=s.value, h0=h0.value, grad=gr.value, counts=counts[:nf.value].tolist(),
               n=int(n.value))
    if particles:
        xyz = np.zeros((n.value, 3))
        feat = np.zeros(n.value, np.int32)
        _check("sph_job_setup", L.sph_job_setup(C.byref(g), C.byref(sz), C.byref(p), None, None,
                                                None, None, 0, None, xyz.ctypes.data,
                                                feat.ctypes.data, n.value, None))
        out.update(xyz=xyz, feature=feat)
    return out


def tags(dim, level):
    """sph_tags (host only): the cell tag system of a level-set domain with
    the description level (phi, n, lo, hi and optional curves): per cell
    (z, y, x) its type and feature index, the volume and patch counts and
    the two patches beside each curve."""
    L = lib()
    g = make_geometry(dim, [0, 0, 0], [1, 1, 1], np.zeros((0, 15)), 2, level)
    nc = [int(level["n"][a]) - 1 if a < dim else 1 for a in range(3)]
    ct = np.empty(nc[0] * nc[1] * nc[2], np.int32)
    ci = np.empty_like(ct)
    ncv = int(g.n_curves)
    cp = np.full(2 * max(ncv, 1), -1, np.int32)
    nv, npch = C.c_int32(), C.c_int32()
    _check("sph_tags", L.sph_tags(C.byref(g), ct.ctypes.data, ci.ctypes.data, C.byref(nv),
                                  C.byref(npch), cp.ctypes.data))
    shape = (nc[2], nc[1], nc[0])
    return ct.reshape(shape), ci.reshape(shape), nv.value, npch.value, cp[:2 * ncv].reshape(-1, 2)


def batch_footprint(**kw):
    """Device bytes of a batch with these capacities (-1 if invalid)."""
    bp = batch_params(**kw)
    return int(lib().sph_batch_footprint(C.byref(bp)))


class SphBatch:
    """Many relaxation jobs sharing one set of device arrays and one launch
    sequence per step (libsphmesh.so batch handle)."""

    def __init__(self, dim, precision=SPH_FP64, max_particles=0, max_cells=1, max_jobs=1,
                 max_neighbors=0, use_graph=1, stream=None, scan_tile=0, allocator=None,
                 verlet_skin=0.0):
        self._alloc = allocator
        self.bp = batch_params(dim, precision, max_particles, max_cells, max_jobs,
                               max_neighbors, use_graph, 0, stream, scan_tile, allocator,
                               verlet_skin)
        self.max_jobs = max_jobs
        h = C.c_void_p()
        _check("sph_batch_create", lib().sph_batch_create(C.byref(self.bp), C.byref(h)))
        self.h = h
        self.n_of = {}

    def close(self):
        if getattr(self, "h", None):
            lib().sph_batch_destroy(self.h)
            self.h = None

    __del__ = close

    def add(self, spec):
        j = C.c_int32()
        _check("sph_batch_add", lib().sph_batch_add(
            self.h, C.byref(spec.geom), C.byref(spec.sizing), C.byref(spec.params), spec.n,
            spec.xyz.ctypes.data, spec.feature.ctypes.data, C.byref(j)))
        self.n_of[j.value] = spec.n
        return j.value

    def remove(self, job):
        _check("sph_batch_remove", lib().sph_batch_remove(self.h, int(job)))
        self.n_of.pop(int(job), None)

    def step(self, n=1):
        _check("sph_batch_step", lib().sph_batch_step(self.h, int(n)))

    def sync(self):
        _check("sph_batch_sync", lib().sph_batch_sync(self.h))

    def status(self):
        m = self.max_jobs
        live = np.zeros(m, np.int32)
        conv = np.zeros(m, np.int32)
        steps = np.zeros(m, np.int64)
        _check("sph_batch_status", lib().sph_batch_status(
            self.h, live.ctypes.data, conv.ctypes.data, steps.ctypes.data, m))
        return live.astype(bool), conv.astype(bool), steps

    def positions(self, job, with_feature=False):
        n = self.n_of[job]
        x = np.zeros((n, 3))
        f = np.zeros(n, np.int32) if with_feature else None
        nout = C.c_int64()
        _check("sph_batch_positions", lib().sph_batch_positions(
            self.h, int(job), x.ctypes.data, None if f is None else f.ctypes.data, n,
            C.byref(nout)))
        return (x, f) if with_feature else x

    def error(self, job):
        e = C.c_double()
        ph = C.c_int32()
        conv = C.c_int32()
        st = C.c_int64()
        _check("sph_batch_error", lib().sph_batch_error(self.h, int(job), C.byref(e),
                                                        C.byref(ph), C.byref(conv), C.byref(st)))
        return dict(e_sys=e.value, phase=ph.value, converged=bool(conv.value), step=st.value)

    def list_builds(self):
        v = C.c_int64()
        _check("sph_batch_list_builds", lib().sph_batch_list_builds(self.h, C.byref(v)))
        return int(v.value)

    def counters(self, job):
        out = np.zeros(4)
        _check("sph_batch_counters", lib().sph_batch_counters(self.h, int(job), out.ctypes.data))
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
    _check("sph_mesh_control_replay", lib().sph_mesh_control_replay(
        C.byref(p), n, vbar.ctypes.data, dt.ctypes.data, ph.ctypes.data, rs.ctypes.data,
        es.ctypes.data))
    return ph, rs, es


def control_replay_noalloc(params, n, vbar, dt, phase, reset, e_sys, stream=None):
    """sph_mesh_control_replay_noalloc: every array argument is a DEVICE
    address (an int, e.g. a torch tensor's data_ptr()); enqueued on stream
    (a hipStream_t handle as an int; None = the null stream)."""
    p = make_params(params)
    _check("sph_mesh_control_replay_noalloc", lib().sph_mesh_control_replay_noalloc(
        C.byref(p), int(n), vbar, dt, phase, reset, e_sys, stream))


def exported_symbols():
    """Names the header declares (checked by the CPU test of the ABI)."""
    return ["sph_mesh_create", "sph_mesh_create_with_particles", "sph_mesh_setup_info",
            "sph_job_setup", "sph_tags",
            "sph_mesh_step", "sph_mesh_positions", "sph_mesh_error",
            "sph_mesh_destroy", "sph_mesh_last_error", "sph_mesh_set_state", "sph_mesh_velocities",
            "sph_mesh_neighbors", "sph_mesh_neighbors_of", "sph_mesh_field", "sph_mesh_group_state", "sph_mesh_counters",
            "sph_mesh_control_replay", "sph_mesh_control_replay_noalloc", "sph_mesh_profile", "sph_mesh_kernel_stats",
            "sph_mesh_kernel_count", "sph_mesh_kernel_name", "sph_mesh_sync",
            "sph_mesh_device_bytes", "sph_batch_footprint", "sph_job_cells", "sph_batch_create",
            "sph_batch_add", "sph_batch_remove", "sph_batch_step", "sph_batch_status",
            "sph_batch_positions", "sph_batch_error", "sph_batch_counters", "sph_batch_destroy",
            "sph_batch_sync", "sph_mesh_list_builds", "sph_batch_list_builds"]
