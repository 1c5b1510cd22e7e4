"""Pins of the oracle's gridded sizing: h_t sampled at the nodes of a
Cartesian background grid and interpolated multilinearly (sec. 2.2 keeps
h_t on the background mesh).  Checks against what the interpolant must
reproduce exactly, independent of the oracle:

* a field linear in x, y, z, and the bilinear x*y, everywhere in the grid;
* the node values at the nodes;
* clamping: outside the grid box, the value at the nearest point of the box;
* the Lipschitz bound against finite differences;
* the neighbour lists of a gridded workload against brute force, and the
  lazily evaluated sample lists against the full lists.
"""
import numpy as np
import pytest

import oracle
from paper_2003_01061_amd import workload as wk


def _sizing(dim, n, lo, hi, f):
    gn = [n[0], n[1], n[2] if dim == 3 else 1]
    ax = [lo[a] + np.arange(gn[a]) * (hi[a] - lo[a]) / (gn[a] - 1) if gn[a] > 1 else np.zeros(1)
          for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    vals = f(X.ravel(), Y.ravel(), Z.ravel())
    return dict(kind=wk.H_GRID, h0=float(vals.min()), grad=0.0, dcap=0.0, point=[0, 0, 0],
                grid=vals, grid_n=gn, grid_lo=list(lo), grid_hi=list(hi))


def _h(dim, sz, x):
    lo = sz["grid_lo"]
    hi = [sz["grid_hi"][a] if a < dim else 0.0 for a in range(3)]
    g = oracle.make_geometry(dim, lo, hi, np.zeros((0, 15)))
    s = oracle.make_sizing(sz)
    return oracle.lib().sphref_h_at(g, s, np.ascontiguousarray(x, float))


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_and_bilinear_fields_are_reproduced(dim):
    lo, hi = [0.2, -0.5, 1.0], [1.7, 0.9, 2.5]
    rng = np.random.default_rng(4)
    lin = lambda x, y, z: 0.3 + 0.05 * x + 0.02 * y + (0.04 * z if dim == 3 else 0.0)
    bil = lambda x, y, z: 0.5 + 0.1 * (x - 0.2) * (y + 0.5)
    for f in (lin, bil):
        sz = _sizing(dim, [7, 5, 6], lo, hi, f)
        for t in range(200):
            x = np.zeros(3)
            x[:dim] = [rng.uniform(lo[a], hi[a]) for a in range(dim)]
            want = f(x[0], x[1], x[2])
            assert abs(_h(dim, sz, x) - want) <= 4e-16 * abs(want), (x, want)


def test_node_values_and_clamping():
    lo, hi = [0.0, 0.0, 0.0], [1.0, 2.0, 0.0]
    rng = np.random.default_rng(5)
    vals = rng.uniform(0.01, 0.02, 6 * 9)
    sz = dict(kind=wk.H_GRID, h0=vals.min(), grad=0.0, dcap=0.0, point=[0, 0, 0], grid=vals,
              grid_n=[6, 9, 1], grid_lo=lo, grid_hi=[1.0, 2.0, 1.0])
    g = vals.reshape(9, 6)
    for j in range(8):          # nodes of the lower-left cells: t = 0 exactly
        for i in range(5):
            x = np.array([i / 5.0, j * 2.0 / 8.0, 0.0])
            if not (x[0] * 5.0 == i and x[1] * 4.0 == j):
                continue
            assert _h(2, sz, x) == g[j, i]
    # outside the box: the value at the nearest point of the box
    assert _h(2, sz, np.array([-3.0, 0.0, 0.0])) == _h(2, sz, np.array([0.0, 0.0, 0.0]))
    assert _h(2, sz, np.array([0.4, 9.0, 0.0])) == _h(2, sz, np.array([0.4, 2.0, 0.0]))


def test_lipschitz_bound_covers_finite_differences():
    wl = wk.with_grid_sizing(wk.paper_square(), 17)
    sz = wl.sizing
    L = wk._lipschitz(sz)
    rng = np.random.default_rng(6)
    worst = 0.0
    for t in range(400):
        a = np.zeros(3); b = np.zeros(3)
        a[:2] = rng.uniform(0, 100, 2)
        b[:2] = a[:2] + rng.normal(0, 3.0, 2)
        b[:2] = np.clip(b[:2], 0, 100)
        d = np.linalg.norm(a - b)
        if d == 0:
            continue
        worst = max(worst, abs(_h(2, sz, a) - _h(2, sz, b)) / d)
    assert 0 < worst <= L * (1 + 1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_lists_of_a_gridded_workload_match_brute_force(dim):
    base = wk.paper_square(n_total=1500) if dim == 2 else wk.paper_cube(n_total=2500, res=32)
    wl = wk.with_grid_sizing(base, 9)
    ref = oracle.RefJob(wl)
    off, ids, rel = ref.neighbors()
    h = np.array([_h(dim, wl.sizing, wl.xyz[i]) for i in range(wl.n)])
    assert np.array_equal(ref.field(oracle.F_H), h)
    c = wl.params["kernel_support"]
    x = wl.xyz
    for i in range(0, wl.n, 3):
        if wl.ftype[wl.feature[i]] == wk.SI:
            continue
        d2 = np.zeros(wl.n)
        for a in range(dim):
            d2 = d2 + (x[i, a] - x[:, a]) ** 2
        m = np.maximum(h[i], h)
        cand = np.nonzero(d2 < (c * c) * (m * m))[0]
        cand = cand[cand != i]
        got = ids[off[i]:off[i + 1]]
        assert np.all(np.isin(got, cand)), i
        same = cand[wl.feature[cand] == wl.feature[i]]
        assert np.all(np.isin(same, got)), i
    idx = np.arange(0, wl.n, 11)
    so, si, sr, _, _, _ = ref.sample(idx, cap_per=2048)
    for t, i in enumerate(idx):
        assert np.array_equal(si[so[t]:so[t + 1]], ids[off[i]:off[i + 1]]), i
