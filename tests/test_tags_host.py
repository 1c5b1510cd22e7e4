"""The library's tag system (sph_tags, host code behind the C-ABI, sec. 3.2)
against the oracle's, bit for bit: cell types, feature indices, counts and
the patches beside each curve, on the level-set domains of the workloads
and on random fields; and its error paths."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2003_01061_amd import binding as bd
from paper_2003_01061_amd import workload as wk


def _both(dim, level):
    g = oracle.make_geometry(dim, [0, 0, 0], [1, 1, 1], np.zeros((0, 15)), 2, level)
    ncv = int(g.n_curves)
    return oracle.tags(g, ncv), bd.tags(dim, level)


@pytest.mark.parametrize("name", ["level_cube_sharp", "level_cylinder", "zalesak_disc",
                                  "level_peanut", "level_torus"])
def test_tags_equal_the_oracle(name):
    wl = getattr(wk, name)()
    a, b = _both(wl.dim, wl.level)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("dim,seed", [(2, 4), (3, 5)])
def test_tags_of_random_fields_with_curves(dim, seed):
    """random phi with random polylines and corners: curve marks, corner
    marks and their precedence, patch components and curve-patch pairs"""
    rng = np.random.default_rng(seed)
    n = [17, 14, 11 if dim == 3 else 1]
    phi = rng.normal(0.1, 1.0, n[0] * n[1] * n[2])
    polys = [rng.uniform(0.05, 0.95, (rng.integers(2, 6), 3)) for _ in range(4)]
    for p in polys:
        if dim == 2:
            p[:, 2] = 0.0
    off = np.cumsum([0] + [len(p) for p in polys]).astype(np.int32)
    cor = np.array([polys[0][0], polys[1][-1], polys[2][0]])
    ends = np.array([[0, -1], [-1, 1], [2, -1], [-1, -1]], np.int32)
    level = dict(phi=phi, n=n, lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0],
                 curves=dict(off=off, pts=np.concatenate(polys), ends=ends, corners=cor))
    a, b = _both(dim, level)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.count_nonzero(a[0] == 3) > 0 and np.count_nonzero(a[0] == 4) > 0


def test_tags_errors():
    L = bd.lib()
    g = bd.make_geometry(2, [0, 0, 0], [1, 1, 0], np.zeros((0, 15)), 0)
    buf = np.zeros(16, np.int32)
    nv, npch = C.c_int32(), C.c_int32()
    assert L.sph_tags(C.byref(g), buf.ctypes.data, buf.ctypes.data, C.byref(nv), C.byref(npch),
                      None) == 1                       # not a level-set domain
    wl = wk.level_peanut(n_total=400, res=64)
    g = bd.make_geometry(2, wl.lo, wl.hi, wl.holes, 2, wl.level)
    assert L.sph_tags(C.byref(g), None, buf.ctypes.data, C.byref(nv), C.byref(npch), None) == 1
    assert b"NULL" in L.sph_mesh_last_error()
