"""Pins of the oracle's ball domain (the paper's sphere cases, sec. 4): the
volume inside a ball (disc) bounded by one sphere (circle) feature, and the
sizing graded both ways from an interior sphere.  Each check is against a
closed form or an invariant the oracle does not compute itself:

* h of the two-sided sizing at points of known radius;
* the closest-point projection onto the sphere (radial, |x - c| = R);
* the boundary normal of the volume at the sphere: the unit radial vector,
  pointing out of the ball;
* the tangent projection of a sphere particle's velocity (no radial part);
* the neighbour lists against brute force with h from the sizing formula;
* a few steps: sphere particles stay on the sphere and move tangentially,
  volume particles stay inside.
"""
import numpy as np
import pytest

import oracle
from paper_2003_01061_amd import workload as wk


def _ball_geom(dim, lo, hi):
    return oracle.make_geometry(dim, lo, hi, np.zeros((0, 15)), domain=1)


def test_shell_sizing_closed_form():
    g = _ball_geom(3, [-1, -1, -1], [1, 1, 1])
    s = oracle.make_sizing(dict(kind=wk.H_SHELL, h0=0.025, grad=0.2, dcap=0.5, point=[0, 0, 0]))
    L = oracle.lib()
    rng = np.random.default_rng(1)
    for r in (0.0, 0.1, 0.5, 0.73, 1.0):
        u = rng.standard_normal(3)
        x = np.ascontiguousarray(r * u / np.linalg.norm(u))
        assert abs(L.sphref_h_at(g, s, x) - (0.025 + 0.2 * abs(r - 0.5))) <= 1e-16


@pytest.mark.parametrize("dim", [2, 3])
def test_projection_normal_and_tangent_on_the_sphere(dim):
    lo, hi = [0.0, 0.0, 0.0], [2.0, 2.0, 2.0 if dim == 3 else 0.0]
    c, R = np.array([1.0, 1.0, 1.0 if dim == 3 else 0.0]), 1.0
    g = _ball_geom(dim, lo, hi)
    L = oracle.lib()
    assert L.sphref_n_features(g) == 2
    assert L.sphref_feature_type(g, 0) == wk.VOL
    assert L.sphref_feature_type(g, 1) == (wk.CURVE if dim == 2 else wk.SURF)
    rng = np.random.default_rng(2)
    for t in range(40):
        u = np.zeros(3)
        u[:dim] = rng.standard_normal(dim)
        u /= np.linalg.norm(u)
        x = c + rng.uniform(0.9, 1.1) * R * u
        q = x.copy()
        L.sphref_project(g, 1, q)
        assert abs(np.linalg.norm(q - c) - R) <= 1e-15
        assert np.abs(q - (c + R * u)).max() <= 1e-15       # radial: the closest point
        n = np.zeros(3)
        assert L.sphref_boundary_normal(g, 0, 1, q, n) == 1
        assert np.abs(n - u).max() <= 1e-15                 # unit, radial, outwards


def _lists_vs_brute(wl):
    g = oracle.make_geometry(wl.dim, wl.lo, wl.hi, wl.holes, wl.domain)
    s = oracle.make_sizing(wl.sizing)
    L = oracle.lib()
    x = wl.xyz
    h = np.array([L.sphref_h_at(g, s, np.ascontiguousarray(x[i])) for i in range(wl.n)])
    p = wl.sizing
    hf = p["h0"] + p["grad"] * np.linalg.norm(x[:, :wl.dim] - np.asarray(p["point"][:wl.dim]), axis=1)
    assert np.allclose(h, hf, rtol=1e-15, atol=0)
    ref = oracle.RefJob(wl)
    off, ids, rel = ref.neighbors()
    c = wl.params["kernel_support"]
    for i in range(wl.n):
        d2 = np.zeros(wl.n)
        for a in range(wl.dim):
            d2 = d2 + (x[i, a] - x[:, a]) ** 2
        m = np.maximum(h[i], h)
        cand = np.nonzero(d2 < (c * c) * (m * m))[0]
        cand = cand[cand != i]
        fi = wl.feature[i]
        # the volume sees the sphere as its boundary; the sphere sees only itself
        want = cand if fi == 0 else cand[wl.feature[cand] == fi]
        got = ids[off[i]:off[i + 1]]
        assert np.array_equal(np.sort(got), want), i
        r = rel[off[i]:off[i + 1]]
        assert np.array_equal(r, np.where(wl.feature[got] == fi, 1, 2)), i


def test_lists_match_brute_force_disc():
    _lists_vs_brute(wk.graded_disc(n_total=1200, res=128))


def test_lists_match_brute_force_sphere():
    _lists_vs_brute(wk.paper_sphere01(n_total=1500, res=32))


@pytest.mark.parametrize("dim", [2, 3])
def test_steps_keep_sphere_particles_on_it_and_volume_inside(dim):
    wl = wk.graded_disc(n_total=1200, res=128) if dim == 2 else wk.paper_sphere01(n_total=1500, res=32)
    c = 0.5 * (wl.lo + wl.hi)
    R = 0.5 * (wl.hi[0] - wl.lo[0])
    ref = oracle.RefJob(wl)
    ref.step(8)
    x, v = ref.state()
    on = wl.feature == 1
    r = np.linalg.norm(x[:, :dim] - c[:dim], axis=1)
    assert np.abs(r[on] - R).max() <= 1e-13 * R
    radial = np.sum((x[on, :dim] - c[:dim]) * v[on, :dim], axis=1) / r[on]
    assert np.abs(radial).max() <= 1e-12 * max(np.abs(v[on]).max(), 1e-300)
    assert np.abs(v[on]).max() > 0
    assert np.all(r[~on] < R)
