"""Pins of the oracle's imported sharp features (sec. 2.1: feature curves as
polylines and singular points, on a level-set domain), on Zalesak's slotted
disc.  Independent checks:

* projection: the result lies on the particle's own polyline and is no
  farther than any of a dense sample of that polyline;
* normals: the volume's normal at a curve particle is perpendicular to the
  closest segment and points to decreasing phi; at the slot's bottom corners
  it is the closed-form diagonal; a curve's normal at its end corner runs
  along its end segment, away from the curve;
* lists against brute force with the boundary relation (a curve sees only
  its two end corners);
* steps keep curve particles on their polylines, moving along them, and the
  corners fixed.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2003_01061_amd import workload as wk


@pytest.fixture(scope="module")
def wl():
    return wk.zalesak_disc(n_total=1500)


def _geom(wl):
    return oracle.make_geometry(2, wl.lo, wl.hi, wl.holes, 2, wl.level)


def _poly(wl, c):
    cv = wl.level["curves"]
    return np.asarray(cv["pts"], float)[cv["off"][c]:cv["off"][c + 1]]


def _dist_to_poly(P, x):
    best = np.inf
    for k in range(len(P) - 1):
        a, b = P[k, :2], P[k + 1, :2]
        t = np.clip(np.dot(x[:2] - a, b - a) / np.dot(b - a, b - a), 0, 1)
        best = min(best, np.linalg.norm(x[:2] - (a + t * (b - a))))
    return best


def test_features_and_projection(wl):
    g = _geom(wl)
    L = oracle.lib()
    assert L.sphref_n_features(g) == 9
    assert [L.sphref_feature_type(g, f) for f in range(9)] == [wk.VOL] + [wk.CURVE] * 4 + [wk.SI] * 4
    rng = np.random.default_rng(7)
    for c in range(4):
        P = _poly(wl, c)
        dense = np.concatenate([P[k] + np.linspace(0, 1, 400, endpoint=False)[:, None] * (P[k + 1] - P[k])
                                for k in range(len(P) - 1)] + [P[-1:]])
        for t in range(25):
            x = np.zeros(3)
            x[:2] = dense[rng.integers(len(dense)), :2] + rng.normal(0, 0.02, 2)
            q = x.copy()
            L.sphref_project(g, 1 + c, q)
            assert _dist_to_poly(P, q) <= 1e-15
            dq = np.linalg.norm(q[:2] - x[:2])
            assert dq <= np.min(np.linalg.norm(dense[:, :2] - x[:2], axis=1)) + 1e-15
    cor = np.asarray(wl.level["curves"]["corners"], float)
    for m in range(4):
        q = np.array([0.3, 0.2, 0.0])
        L.sphref_project(g, 5 + m, q)
        assert np.array_equal(q, cor[m])


def test_normals(wl):
    g = _geom(wl)
    L = oracle.lib()
    rng = np.random.default_rng(8)
    phi = lambda x: wk._level_eval(wl.level, 2, np.atleast_2d(x))[0][0]
    for c in range(4):
        P = _poly(wl, c)
        for t in range(10):
            k = rng.integers(len(P) - 1)
            u = rng.uniform(0.1, 0.9)
            xb = np.zeros(3)
            xb[:2] = P[k, :2] + u * (P[k + 1, :2] - P[k, :2])
            n = np.zeros(3)
            assert L.sphref_boundary_normal(g, 0, 1 + c, xb, n) == 1
            seg = P[k + 1, :2] - P[k, :2]
            assert abs(np.linalg.norm(n) - 1) <= 1e-15 and abs(n[:2] @ seg) <= 1e-15
            assert phi(xb + 2e-3 * n) < phi(xb - 2e-3 * n)
    cor = np.asarray(wl.level["curves"]["corners"], float)
    r = 1 / math.sqrt(2)
    n = np.zeros(3)
    assert L.sphref_boundary_normal(g, 0, 6, cor[1], n) == 1       # B: slot bottom-left
    assert np.allclose(n[:2], [r, r], atol=1e-15)
    assert L.sphref_boundary_normal(g, 0, 7, cor[2], n) == 1       # C: slot bottom-right
    assert np.allclose(n[:2], [-r, r], atol=1e-15)
    # curve 2 runs C -> B: at B (its last point) the normal continues past B
    assert L.sphref_boundary_normal(g, 3, 6, cor[1], n) == 1
    assert np.allclose(n[:2], [-1.0, 0.0], atol=1e-15)
    # ... and at C (its first point) it points back beyond C
    assert L.sphref_boundary_normal(g, 3, 7, cor[2], n) == 1
    assert np.allclose(n[:2], [1.0, 0.0], atol=1e-15)
    # a curve is not bounded by a corner it does not end at
    assert L.sphref_boundary_normal(g, 3, 5, cor[0], n) == 0


def test_lists_match_brute_force(wl):
    ref = oracle.RefJob(wl)
    off, ids, rel = ref.neighbors()
    h = ref.field(oracle.F_H)
    c = wl.params["kernel_support"]
    x = wl.xyz
    ends = np.asarray(wl.level["curves"]["ends"]).reshape(-1, 2)
    for i in range(wl.n):
        fi = wl.feature[i]
        got = ids[off[i]:off[i + 1]]
        if fi >= 5:
            assert got.size == 0
            continue
        d2 = (x[i, 0] - x[:, 0]) ** 2 + (x[i, 1] - x[:, 1]) ** 2
        cand = np.nonzero(d2 < (c * c) * np.maximum(h[i], h) ** 2)[0]
        cand = cand[cand != i]
        fj = wl.feature[cand]
        if fi == 0:
            want = cand
        else:
            want = cand[(fj == fi) | np.isin(fj, 5 + ends[fi - 1])]
        assert np.array_equal(got, want), i


def test_steps_keep_curves_on_polylines_and_corners_fixed(wl):
    ref = oracle.RefJob(wl)
    ref.step(10)
    x, v = ref.state()
    cor = np.asarray(wl.level["curves"]["corners"], float)
    for c in range(4):
        P = _poly(wl, c)
        sel = np.nonzero(wl.feature == 1 + c)[0]
        for i in sel:
            assert _dist_to_poly(P, x[i]) <= 1e-14
    sel = np.nonzero(wl.feature >= 5)[0]
    assert np.array_equal(x[sel], cor[wl.feature[sel] - 5])
    assert np.all(v[sel] == 0)
    assert np.abs(v[wl.feature == 2]).max() > 0 or np.abs(v[wl.feature == 1]).max() > 0
    # the slot's walls are vertical and its bottom horizontal: motion along them only
    assert np.all(v[wl.feature == 2, 0] == 0) and np.all(v[wl.feature == 4, 0] == 0)
    assert np.all(v[wl.feature == 3, 1] == 0)
