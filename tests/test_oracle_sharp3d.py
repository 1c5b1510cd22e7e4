"""Pins of the oracle's 3D imported sharp features and of the cell tag system
(sec. 2.1: feature curves on a level set; sec. 3.2: the background grid's
cell types and feature indices), on two level-set domains: a cube with its
twelve edges and eight vertices imported, and a cylinder with its two rims.
Independent checks:

* tags: cells that no curve or corner marks take the type the signs of phi
  at their nodes give; positive and surface components agree with
  scipy.ndimage.label (face connectivity) on random fields; the cube's
  zero set splits into exactly its six faces, each edge between the two
  faces that meet there, and the cylinder's into two discs and a side;
* features: on the cube, the boundary relation of every feature pair and the
  outward normal of every bounding pair equal those of the box domain (an
  independent code path of the oracle); on the cylinder, the normal of a
  disc or of the side at a rim is the closed-form conormal;
* projections: onto a 3D polyline, the closest point beats a dense sample;
  onto a patch, |phi| <= 1e-14;
* lists against brute force with the patch-curve-vertex relations;
* steps keep edge and rim particles on their polylines, patch particles on
  phi = 0 and vertices fixed.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2003_01061_amd import workload as wk


@pytest.fixture(scope="module")
def cube():
    return wk.level_cube_sharp(n_total=4000)


@pytest.fixture(scope="module")
def cyl():
    return wk.level_cylinder(n_total=5000)


def _geom(wl):
    return oracle.make_geometry(3, wl.lo, wl.hi, wl.holes, 2, wl.level)


def _poly(wl, c):
    cv = wl.level["curves"]
    return np.asarray(cv["pts"], float)[cv["off"][c]:cv["off"][c + 1]]


def _dist_to_poly(P, x):
    best = np.inf
    for k in range(len(P) - 1):
        a, b = P[k], P[k + 1]
        t = np.clip(np.dot(x - a, b - a) / np.dot(b - a, b - a), 0, 1)
        best = min(best, np.linalg.norm(x - (a + t * (b - a))))
    return best


def _node_types(level, dim):
    """cell types from the signs of phi at the cell's nodes: 1 all positive,
    0 all negative, 2 otherwise"""
    n = level["n"]
    phi = np.asarray(level["phi"], float).reshape(n[2], n[1], n[0]) if dim == 3 else \
        np.asarray(level["phi"], float).reshape(1, n[1], n[0])
    if dim == 3:
        nodes = [phi[dz:dz + n[2] - 1, dy:dy + n[1] - 1, dx:dx + n[0] - 1]
                 for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
    else:
        nodes = [phi[:, dy:dy + n[1] - 1, dx:dx + n[0] - 1] for dy in (0, 1) for dx in (0, 1)]
    pos = np.all([v > 0 for v in nodes], axis=0)
    neg = np.all([v < 0 for v in nodes], axis=0)
    return np.where(pos, 1, np.where(neg, 0, 2))


# ---------------------------------------------------------------------------
# the tag system
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,seed", [(2, 1), (3, 2), (3, 3)])
def test_tags_of_random_fields_match_label(dim, seed):
    rng = np.random.default_rng(seed)
    n = [13, 11, 9 if dim == 3 else 1]
    phi = rng.normal(0.2, 1.0, n[0] * n[1] * n[2])
    level = dict(phi=phi, n=n, lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0])
    g = oracle.make_geometry(dim, [0, 0, 0], [1, 1, 1], np.zeros((0, 15)), 2, level)
    ct, ci, nv, npch, _ = oracle.tags(g)
    want = _node_types(level, dim)
    assert np.array_equal(ct, want)
    st = ndimage.generate_binary_structure(3, 1)          # face neighbours
    for t, count in ((1, nv), (2, npch)):
        lab, _ = ndimage.label(want == t, structure=st)
        order = {}
        for v in lab.ravel():
            if v and v not in order:
                order[v] = len(order)
        exp = np.full(lab.shape, -1)
        for v, k in order.items():
            exp[lab == v] = k
        assert count == len(order)
        assert np.array_equal(np.where(want == t, ci, -1), exp)
    assert np.all(ci[want == 0] == -1)


def test_tags_of_a_hand_grid():
    """2D, 5 x 3 nodes (4 x 2 cells): phi > 0 on the two left node columns
    and on the right one, negative between: cells 0 (positive), 1, 2
    (mixed: one surface component), 3 (mixed), in both rows"""
    row = [1.0, 1.0, -1.0, -1.0, 1.0]
    phi = np.array(row * 3)
    level = dict(phi=phi, n=[5, 3, 1], lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0])
    g = oracle.make_geometry(2, [0, 0, 0], [1, 1, 1], np.zeros((0, 15)), 2, level)
    ct, ci, nv, npch, _ = oracle.tags(g)
    assert ct[0].tolist() == [[1, 2, 0, 2], [1, 2, 0, 2]]
    assert ci[0].tolist() == [[0, 0, -1, 1], [0, 0, -1, 1]]
    assert (nv, npch) == (1, 2)


def _mark_checks(wl, ct, ci):
    """cells that no curve or vertex marks keep their node-sign type; a
    curve cell lies within a cell diagonal plus a side of its curve, a vertex
    cell within the vertex's cell neighbourhood"""
    want = _node_types(wl.level, 3)
    free = ct <= 2
    assert np.array_equal(ct[free], want[free])
    n = wl.level["n"]
    side = 1.0 / (n[0] - 1)
    kk, jj, ii = np.nonzero(ct == 3)
    for k, j, i in zip(kk[::7], jj[::7], ii[::7]):
        c = np.array([i + 0.5, j + 0.5, k + 0.5]) * side
        assert _dist_to_poly(_poly(wl, ci[k, j, i]), c) <= side * (0.5 * math.sqrt(3) + 1) + 1e-12
    cor = np.asarray(wl.level["curves"]["corners"], float)
    kk, jj, ii = np.nonzero(ct == 4)
    for k, j, i in zip(kk, jj, ii):
        own = np.floor(cor[ci[k, j, i]] / side)
        assert np.max(np.abs(own - [i, j, k])) <= 1


def test_tags_split_the_cube_into_its_faces(cube):
    g = _geom(cube)
    ct, ci, nv, npch, cp = oracle.tags(g, 12)
    assert (nv, npch) == (1, 6)
    assert np.array_equal(cp, cube.level["curves"]["patches"])
    # each face's centre cell is a surface cell of that face's patch
    a0, a1 = 0.2125, 0.7875
    side = 1.0 / 40
    order = [(2, 0), (1, 0), (0, 0), (0, 1), (1, 1), (2, 1)]
    for p, (axis, sd) in enumerate(order):
        x = np.full(3, 0.5)
        x[axis] = a1 if sd else a0
        i, j, k = np.floor(x / side).astype(int)
        assert (ct[k, j, i], ci[k, j, i]) == (2, p)
    assert np.count_nonzero(ct == 4) == 8 * 27
    _mark_checks(cube, ct, ci)


def test_tags_split_the_cylinder(cyl):
    g = _geom(cyl)
    ct, ci, nv, npch, cp = oracle.tags(g, 2)
    assert (nv, npch) == (1, 3)
    assert cp.tolist() == [[0, 1], [1, 2]]
    side = 1.0 / 32
    for x, p in (([0.5, 0.5, 0.2], 0), ([0.8, 0.5, 0.5], 1), ([0.5, 0.5, 0.8], 2)):
        i, j, k = np.floor(np.array(x) / side).astype(int)
        assert (ct[k, j, i], ci[k, j, i]) == (2, p)
    i, j, k = np.floor(np.array([0.5, 0.5, 0.5]) / side).astype(int)
    assert (ct[k, j, i], ci[k, j, i]) == (1, 0)
    i, j, k = np.floor(np.array([0.8, 0.5, 0.2]) / side).astype(int)   # on the bottom rim
    assert (ct[k, j, i], ci[k, j, i]) == (3, 0)
    _mark_checks(cyl, ct, ci)


# ---------------------------------------------------------------------------
# features, relations and normals
# ---------------------------------------------------------------------------
def _box_feature(f):
    """the box domain's feature for a feature of the level-set cube"""
    if 1 <= f <= 6:
        axis, sd = [(2, 0), (1, 0), (0, 0), (0, 1), (1, 1), (2, 1)][f - 1]
        return 1 + 2 * axis + sd
    return f


def _point_on(cube, f, rng):
    """a point of feature f of the cube away from the other features"""
    a0, a1 = 0.2125, 0.7875
    cv = cube.level["curves"]
    if f == 0:
        return np.full(3, 0.5)
    if 1 <= f <= 6:
        axis, sd = [(2, 0), (1, 0), (0, 0), (0, 1), (1, 1), (2, 1)][f - 1]
        x = rng.uniform(0.35, 0.65, 3)
        x[axis] = a1 if sd else a0
        return x
    if f <= 18:
        P = _poly(cube, f - 7)
        return P[0] + rng.uniform(0.3, 0.7) * (P[1] - P[0])
    return np.asarray(cv["corners"], float)[f - 19].copy()


def test_cube_relations_and_normals_equal_the_box_domain(cube):
    L = oracle.lib()
    g = _geom(cube)
    a0, a1 = 0.2125, 0.7875
    gb = oracle.make_geometry(3, [a0, a0, a0], [a1, a1, a1], np.zeros((0, 15)), 0)
    assert L.sphref_n_features(g) == 27 and L.sphref_n_features(gb) == 27
    assert [L.sphref_feature_type(g, f) for f in range(27)] == \
        [L.sphref_feature_type(gb, _box_feature(f)) for f in range(27)]
    rng = np.random.default_rng(5)
    n, nb = np.zeros(3), np.zeros(3)
    checked = 0
    for fi in range(27):
        for fb in range(27):
            xb = _point_on(cube, fb, rng)
            xi = _point_on(cube, fi, rng)
            if 1 <= fi <= 6 and fb >= 19:
                # a face seen from a vertex: take x_i on the face's diagonal
                # through that vertex, where the box's constant normal holds
                axis = [2, 1, 0, 0, 1, 2][fi - 1]
                xi = xb + 0.25 * (np.full(3, 0.5) - xb)
                xi[axis] = xb[axis]
            r = L.sphref_boundary_normal_at(g, fi, fb, xb, xi, n)
            rb = L.sphref_boundary_normal(gb, _box_feature(fi), _box_feature(fb), xb, nb)
            assert r == rb, (fi, fb)
            if r == 1:
                assert np.allclose(n, nb, rtol=0, atol=1e-12), (fi, fb, n, nb)
                checked += 1
    # the volume sees 26 features; each face 4 edges and 4 vertices; each
    # edge 2 vertices
    assert checked == 26 + 6 * 8 + 12 * 2


def test_patch_normal_needs_the_particle(cube):
    L = oracle.lib()
    g = _geom(cube)
    n = np.zeros(3)
    xb = _poly(cube, 0)[0] + 0.5 * (_poly(cube, 0)[1] - _poly(cube, 0)[0])
    with pytest.raises(Exception):
        L.sphref_boundary_normal_at(g, 1, 7, xb, None, n)
    assert L.sphref_boundary_normal(g, 1, 7, xb, n) == -1


def test_cylinder_conormals(cyl):
    """at the midpoint of a rim segment, seen from a point of a disc on the
    same radius or of the side on the same vertical line, the normal is the
    radial direction (discs) or the axis (side), outwards"""
    L = oracle.lib()
    g = _geom(cyl)
    n = np.zeros(3)
    R, c = 0.3, 0.5
    rng = np.random.default_rng(3)
    for rim, zc in ((0, 0.2), (1, 0.8)):
        P = _poly(cyl, rim)
        for k in rng.integers(0, len(P) - 1, 6):
            xb = 0.5 * (P[k] + P[k + 1])
            u = np.array([xb[0] - c, xb[1] - c, 0.0])
            u /= np.linalg.norm(u)
            disc = 1 + 2 * rim                      # patch 0 bottom, 2 top
            xi = np.array([c, c, zc]) + 0.15 * u
            assert L.sphref_boundary_normal_at(g, disc, 4 + rim, xb, xi, n) == 1
            assert np.allclose(n, u, atol=1e-12)
            # the side's normal at x_i comes from the interpolated phi, off the
            # radial direction by an angle delta, which tilts n by at most
            # about delta
            xi = np.array([c + R * u[0], c + R * u[1], 0.5])
            gr = wk._level_eval(cyl.level, 3, xi[None])[1][0]
            delta = math.acos(min(1.0, -np.dot(gr, u) / np.linalg.norm(gr)))
            assert L.sphref_boundary_normal_at(g, 2, 4 + rim, xb, xi, n) == 1
            assert np.linalg.norm(n - [0, 0, -1 if rim == 0 else 1]) <= 2 * delta + 1e-12
            # the volume: a unit vector out of the domain at the rim
            assert L.sphref_boundary_normal(g, 0, 4 + rim, xb, n) == 1
            assert abs(np.linalg.norm(n) - 1) < 1e-14
            assert np.dot(n, u) > 0.3 and n[2] * (1 if rim else -1) > 0.3
    # a disc does not see the other rim; the rims do not see each other
    xb = _poly(cyl, 1)[0]
    assert L.sphref_boundary_normal_at(g, 1, 5, xb, np.array([0.5, 0.5, 0.2]), n) == 0
    assert L.sphref_boundary_normal(g, 4, 5, xb, n) == 0


def test_projections(cube, cyl):
    L = oracle.lib()
    rng = np.random.default_rng(9)
    for wl, curves, first_curve in ((cube, 12, 7), (cyl, 2, 4)):
        g = _geom(wl)
        for c in range(curves):
            P = _poly(wl, c)
            dense = np.concatenate([P[k] + np.linspace(0, 1, 200, endpoint=False)[:, None] * (P[k + 1] - P[k])
                                    for k in range(len(P) - 1)] + [P[-1:]])
            for t in range(8):
                x = dense[rng.integers(len(dense))] + rng.normal(0, 0.02, 3)
                q = x.copy()
                L.sphref_project(g, first_curve + c, q)
                assert _dist_to_poly(P, q) <= 1e-15
                assert np.linalg.norm(q - x) <= np.min(np.linalg.norm(dense - x, axis=1)) + 1e-15
        for p in range(1, first_curve):
            for t in range(10):
                x = rng.uniform(0.15, 0.85, 3)
                L.sphref_project(g, p, x)
                assert abs(wk._level_eval(wl.level, 3, x[None])[0][0]) <= 1e-14


# ---------------------------------------------------------------------------
# lists and steps
# ---------------------------------------------------------------------------
def _bounding(wl):
    """bound[fi] = the features that bound fi, from the geometry description"""
    cv = wl.level["curves"]
    npch, ncv = int(cv["n_patches"]), len(cv["off"]) - 1
    pat = np.asarray(cv["patches"]).reshape(-1, 2)
    ends = np.asarray(cv["ends"]).reshape(-1, 2)
    nf = 1 + npch + ncv + len(cv["corners"])
    bound = {0: set(range(1, nf))}
    for p in range(npch):
        cs = [c for c in range(ncv) if p in pat[c]]
        bound[1 + p] = {1 + npch + c for c in cs} | {1 + npch + ncv + m for c in cs for m in ends[c] if m >= 0}
    for c in range(ncv):
        bound[1 + npch + c] = {1 + npch + ncv + m for m in ends[c] if m >= 0}
    for m in range(len(cv["corners"])):
        bound[1 + npch + ncv + m] = set()
    return bound


@pytest.mark.parametrize("name", ["cube", "cyl"])
def test_lists_match_brute_force(name, cube, cyl):
    wl = {"cube": cube, "cyl": cyl}[name]
    ref = oracle.RefJob(wl)
    off, ids, rel = ref.neighbors()
    h = ref.field(oracle.F_H)
    c = wl.params["kernel_support"]
    x = wl.xyz
    bound = _bounding(wl)
    for i in range(0, wl.n, 3):
        fi = wl.feature[i]
        got = ids[off[i]:off[i + 1]]
        if wl.ftype[fi] == wk.SI:
            assert got.size == 0
            continue
        d2 = np.sum((x[i] - x) ** 2, axis=1)
        cand = np.nonzero(d2 < (c * c) * np.maximum(h[i], h) ** 2)[0]
        cand = cand[cand != i]
        fj = wl.feature[cand]
        keep = (fj == fi) | np.isin(fj, sorted(bound[fi]))
        assert np.array_equal(got, cand[keep]), i
        assert np.array_equal(rel[off[i]:off[i + 1]], np.where(fj[keep] == fi, 1, 2))


@pytest.mark.parametrize("name", ["cube", "cyl"])
def test_steps_keep_particles_on_their_features(name, cube, cyl):
    wl = {"cube": cube, "cyl": cyl}[name]
    ref = oracle.RefJob(wl)
    ref.step(6)
    x, v = ref.state()
    cv = wl.level["curves"]
    npch, ncv = int(cv["n_patches"]), len(cv["off"]) - 1
    f = wl.feature
    surf = (f >= 1) & (f <= npch)
    assert np.abs(wk._level_eval(wl.level, 3, x[surf])[0]).max() <= 1e-13
    for c in range(ncv):
        P = _poly(wl, c)
        for i in np.nonzero(f == 1 + npch + c)[0]:
            assert _dist_to_poly(P, x[i]) <= 1e-15
    vc = f > npch + ncv
    cor = np.asarray(cv["corners"], float)
    assert np.array_equal(x[vc], cor[f[vc] - 1 - npch - ncv]) and np.all(v[vc] == 0)
    assert np.abs(v[surf]).max() > 0
    if name == "cube":
        # an edge particle moves along its edge only; a face particle in its plane
        for c in range(12):
            axis = c // 4
            sel = f == 7 + c
            others = [a for a in range(3) if a != axis]
            assert np.all(v[sel][:, others] == 0)
        assert np.all(np.isfinite(x))
