"""Pins of the oracle's ellipsoidal holes.

Sec. 2.1 describes the geometry by a level set; for an ellipsoid that level
set is the quadric sum_k (y_k / a_k)^2 = 1 in the hole's own frame.  What
these tests pin, each against something the oracle does not compute itself:

* the distance to the surface (the sizing field of sec. 2.2): closed form on
  the principal axes, and a minimisation over the surface's parametrisation
  (scipy) everywhere else;
* the closest-point projection of surface particles (a fixed number of
  Newton steps): on the surface to 1e-14 and equal to the
  parametric minimiser;
* the boundary normal of the volume at the hole: unit length, perpendicular
  to the surface's tangents (finite differences of the parametrisation),
  pointing out of the domain;
* h inside a hole (distance zero) and the tangency of surface velocities
  after a step;
* the neighbour lists of an ellipsoid workload against brute force with h
  from the pinned sizing function, and the lazily evaluated sample lists
  against the full lists.
"""
import math

import numpy as np
import pytest
from scipy import optimize
from scipy.spatial.transform import Rotation

import oracle
from paper_2003_01061_amd import workload as wk

C3 = np.array([0.5, 0.48, 0.53])
A3 = np.array([0.21, 0.13, 0.07])
C2 = np.array([0.5, 0.46, 0.0])
A2 = np.array([0.23, 0.09])


def _rot(dim, seed):
    if dim == 3:
        return Rotation.random(random_state=seed).as_matrix()
    t = 0.3 + seed
    return np.array([[math.cos(t), math.sin(t), 0.0], [-math.sin(t), math.cos(t), 0.0],
                     [0.0, 0.0, 1.0]])


def _hole(dim, seed=7):
    c, a = (C3, A3) if dim == 3 else (C2, A2)
    R = _rot(dim, seed)
    rec = np.zeros(15)
    rec[:3] = c
    rec[3:3 + dim] = a
    if dim == 2:
        rec[5] = a[0]
    rec[6:] = R.ravel()
    return rec, c, a, R


def _geom(dim, rec):
    hi = [1.0, 1.0, 1.0 if dim == 3 else 0.0]
    return oracle.make_geometry(dim, [0.0, 0.0, 0.0], hi, rec[None, :])


def _surface_point(dim, c, a, R, p):
    """point of the surface at parameters p (angle; or polar, azimuth)"""
    if dim == 2:
        y = np.array([a[0] * math.cos(p[0]), a[1] * math.sin(p[0])])
    else:
        y = np.array([a[0] * math.sin(p[0]) * math.cos(p[1]),
                      a[1] * math.sin(p[0]) * math.sin(p[1]), a[2] * math.cos(p[0])])
    x = np.zeros(3)
    x[:dim] = c[:dim] + R[:dim, :dim].T @ y
    return x


def _closest_by_search(dim, c, a, R, x):
    """global minimiser of |x - s(p)| over the parametrisation: a dense grid,
    then a local refinement from the best grid point"""
    if dim == 2:
        th = np.linspace(0, 2 * np.pi, 4001)[:-1]
        cand = [(t,) for t in th]
    else:
        th = np.linspace(0, np.pi, 181)
        ph = np.linspace(0, 2 * np.pi, 361)[:-1]
        cand = [(t, p) for t in th for p in ph]
    P = np.array([_surface_point(dim, c, a, R, p) for p in cand])
    k = int(np.argmin(np.linalg.norm(P - x, axis=1)))

    def f(p):
        d = _surface_point(dim, c, a, R, p) - x
        return float(d @ d)
    r = optimize.minimize(f, np.array(cand[k], float), method="Nelder-Mead",
                          options=dict(xatol=1e-13, fatol=1e-30, maxiter=20000, maxfev=40000))
    return _surface_point(dim, c, a, R, r.x), math.sqrt(r.fun)


def _level(rec, dim, x):
    R = rec[6:].reshape(3, 3)[:dim, :dim]
    y = R @ (x[:dim] - rec[:dim])
    return float(np.sum((y / rec[3:3 + dim]) ** 2))


def _sizing_d():
    """h = 1 + d: the oracle's h_t gives the distance as h - 1"""
    return oracle.make_sizing(dict(kind=wk.H_GRADED_TO_HOLES, h0=1.0, grad=1.0, dcap=np.inf))


@pytest.mark.parametrize("dim", [2, 3])
def test_distance_on_the_principal_axes(dim):
    rec, c, a, R = _hole(dim)
    g = _geom(dim, rec)
    s = _sizing_d()
    L = oracle.lib()
    for k in range(dim):
        for sign in (1.0, -1.0):
            for delta in (1e-4, 0.03, 0.11):
                y = np.zeros(dim)
                y[k] = sign * (a[k] + delta)
                x = np.zeros(3)
                x[:dim] = c[:dim] + R[:dim, :dim].T @ y
                d = L.sphref_h_at(g, s, x) - 1.0
                assert abs(d - delta) <= 2e-15, (k, sign, delta, d)


@pytest.mark.parametrize("dim", [2, 3])
def test_distance_matches_parametric_minimum(dim):
    rec, c, a, R = _hole(dim)
    g = _geom(dim, rec)
    s = _sizing_d()
    L = oracle.lib()
    rng = np.random.default_rng(3)
    n = 0
    while n < (12 if dim == 3 else 25):
        x = np.zeros(3)
        x[:dim] = rng.uniform(0.02, 0.98, dim)
        if _level(rec, dim, x) <= 1.0:
            continue
        n += 1
        d = L.sphref_h_at(g, s, x) - 1.0
        _, dref = _closest_by_search(dim, c, a, R, x)
        assert abs(d - dref) <= 1e-11, (x, d, dref)


@pytest.mark.parametrize("dim", [2, 3])
def test_h_inside_a_hole_is_h0(dim):
    rec, c, a, R = _hole(dim)
    g = _geom(dim, rec)
    s = oracle.make_sizing(dict(kind=wk.H_GRADED_TO_HOLES, h0=0.01, grad=4.0, dcap=np.inf))
    L = oracle.lib()
    for f in (0.0, 0.5, 0.999):
        for k in range(dim):
            y = np.zeros(dim)
            y[k] = f * a[k]
            x = np.zeros(3)
            x[:dim] = c[:dim] + R[:dim, :dim].T @ y
            assert L.sphref_h_at(g, s, x) == 0.01


@pytest.mark.parametrize("dim", [2, 3])
def test_projection_lands_on_the_closest_surface_point(dim):
    rec, c, a, R = _hole(dim)
    g = _geom(dim, rec)
    L = oracle.lib()
    hole_feature = 5 if dim == 2 else 7
    rng = np.random.default_rng(11)
    for t in range(30 if dim == 2 else 16):
        p = rng.uniform(0, 2 * np.pi, dim - 1)
        if dim == 3:
            p[0] = math.acos(rng.uniform(-1, 1))
        q0 = _surface_point(dim, c, a, R, p)
        off = np.zeros(3)
        off[:dim] = rng.standard_normal(dim)
        off *= rng.uniform(-3e-3, 3e-3) * a.min() / np.linalg.norm(off)
        x = q0 + off
        q = x.copy()
        L.sphref_project(g, hole_feature, q)
        assert abs(_level(rec, dim, q) - 1.0) <= 1e-14
        qref, _ = _closest_by_search(dim, c, a, R, x)
        assert np.abs(q - qref).max() <= 1e-9, (q, qref)


@pytest.mark.parametrize("dim", [2, 3])
def test_boundary_normal_is_the_unit_normal_out_of_the_domain(dim):
    rec, c, a, R = _hole(dim)
    g = _geom(dim, rec)
    L = oracle.lib()
    hole_feature = 5 if dim == 2 else 7
    rng = np.random.default_rng(5)
    eps = 1e-5
    for t in range(40):
        p = rng.uniform(0.2, 2 * np.pi - 0.2, dim - 1)
        if dim == 3:
            p[0] = rng.uniform(0.2, np.pi - 0.2)
        xb = _surface_point(dim, c, a, R, p)
        n = np.zeros(3)
        assert L.sphref_boundary_normal(g, 0, hole_feature, xb, n) == 1
        assert abs(np.linalg.norm(n) - 1.0) <= 1e-15
        for k in range(dim - 1):
            dp = np.zeros(dim - 1)
            dp[k] = eps
            tng = _surface_point(dim, c, a, R, p + dp) - _surface_point(dim, c, a, R, p - dp)
            assert abs(n @ tng) <= 1e-8 * np.linalg.norm(tng)
        # the hole is convex and holds its centre: out of the domain is towards it
        assert n @ (xb - c) < 0


def _inclusion_workload(dim, n, seed):
    if dim == 3:
        return wk.ellipsoid_inclusions(n_total=n, seed=seed, dim=3, n_incl=3, amin=0.08,
                                       amax=0.16, cmin=0.25, cmax=0.75, ratio=4.0, ramp=0.2,
                                       res=24, envelope_grid=16)
    return wk.ellipsoid_inclusions(n_total=n, seed=seed, dim=2, n_incl=3, amin=0.06,
                                   amax=0.16, cmin=0.25, cmax=0.75, ratio=4.0, ramp=0.2,
                                   res=128, envelope_grid=64)


@pytest.mark.parametrize("dim,n", [(2, 1500), (3, 2500)])
def test_lists_match_brute_force_and_lazy_samples(dim, n):
    wl = _inclusion_workload(dim, n, seed=31)
    g = oracle.make_geometry(dim, wl.lo, wl.hi, wl.holes)
    s = oracle.make_sizing(wl.sizing)
    L = oracle.lib()
    x = wl.xyz
    h = np.array([L.sphref_h_at(g, s, np.ascontiguousarray(x[i])) for i in range(wl.n)])
    ref = oracle.RefJob(wl)
    off, ids, rel = ref.neighbors()
    nonempty = 0
    for i in range(wl.n):
        got = ids[off[i]:off[i + 1]]
        if wl.ftype[wl.feature[i]] == wk.SI:
            assert got.size == 0
            continue
        acc = np.zeros(wl.n)
        for a in range(dim):
            d = x[i, a] - x[:, a]
            acc = acc + d * d
        m = np.maximum(h[i], h)
        c = wl.params["kernel_support"]
        cand = np.nonzero(acc < (c * c) * (m * m))[0]
        cand = cand[cand != i]
        # the relation filter only drops candidates; every kept id is a candidate
        assert np.all(np.isin(got, cand)), i
        same = cand[wl.feature[cand] == wl.feature[i]]
        assert np.all(np.isin(same, got)), i
        nonempty += got.size > 0
    assert nonempty > 0.9 * wl.n - 16
    idx = np.arange(0, wl.n, 7)
    so, si, sr, _, _, _ = ref.sample(idx)
    for t, i in enumerate(idx):
        assert np.array_equal(si[so[t]:so[t + 1]], ids[off[i]:off[i + 1]]), i
        assert np.array_equal(sr[so[t]:so[t + 1]], rel[off[i]:off[i + 1]]), i


@pytest.mark.parametrize("dim,n", [(2, 1500), (3, 2500)])
def test_surface_particles_stay_on_their_ellipsoid_and_move_tangentially(dim, n):
    wl = _inclusion_workload(dim, n, seed=32)
    ref = oracle.RefJob(wl)
    ref.step(6)
    x, v = ref.state()
    first_hole = 5 if dim == 2 else 7
    moved = 0
    for q, rec in enumerate(wl.holes):
        sel = np.nonzero(wl.feature == first_hole + q)[0]
        Rq = rec[6:].reshape(3, 3)[:dim, :dim]
        for i in sel:
            assert abs(_level(rec, dim, x[i]) - 1.0) <= 1e-14
            y = Rq @ (x[i, :dim] - rec[:dim])
            nrm = Rq.T @ (y / rec[3:3 + dim] ** 2)          # gradient of the level
            nrm /= np.linalg.norm(nrm)
            sp = np.linalg.norm(v[i, :dim])
            assert abs(nrm @ v[i, :dim]) <= 1e-12 * max(sp, 1e-300)
            moved += sp > 0
    assert moved > 0
