"""Pins of the mesh-quality measures (sec. 4's definitions) on shapes whose
values are known in closed form, and of the element filter.  CPU only."""
import math

import numpy as np

from paper_2003_01061_amd import quality as q


def test_equilateral_triangle_has_unit_G_and_sixty_degrees():
    P = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, math.sqrt(3) / 2]])
    G, ang = q.triangle_quality(P, np.array([[0, 1, 2]]))
    assert abs(G[0] - 1.0) < 1e-15
    assert np.allclose(ang, 60.0, atol=1e-12)


def test_right_isosceles_triangle():
    # S = 1/2, half-perimeter (2 + sqrt 2) / 2, longest edge sqrt 2:
    # G = 2 sqrt 3 (1/2) / ((1 + sqrt 2 / 2) sqrt 2) = sqrt 3 / (sqrt 2 + 1)
    P = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    G, ang = q.triangle_quality(P, np.array([[0, 1, 2]]))
    assert abs(G[0] - math.sqrt(3) / (math.sqrt(2) + 1)) < 1e-15
    assert np.allclose(sorted(ang[0]), [45.0, 45.0, 90.0], atol=1e-12)
    s = q.summarize_triangles(G, ang)
    assert s["theta_min"] == s["theta_min_avg"] and s["n_theta_below_30"] == 0


def test_regular_tetrahedron():
    P = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    g, dih = q.tet_quality(P, np.array([[0, 1, 2, 3]]))
    assert abs(g[0] - 1.0) < 1e-14
    assert np.allclose(dih, math.degrees(math.acos(1.0 / 3.0)), atol=1e-12)


def test_corner_tetrahedron_angles_and_ratio():
    # the tetrahedron (0, e1, e2, e3): three right dihedral angles at the
    # origin's edges, three of arccos(1/sqrt 3) at the slanted face;
    # r_in = 1 / (3 + sqrt 3), r_circ = sqrt 3 / 2
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    g, dih = q.tet_quality(P, np.array([[0, 1, 2, 3]]))
    d = sorted(dih[0])
    assert np.allclose(d[:3], math.degrees(math.acos(1 / math.sqrt(3))), atol=1e-12)
    assert np.allclose(d[3:], 90.0, atol=1e-12)
    assert abs(g[0] - 3 * (1 / (3 + math.sqrt(3))) / (math.sqrt(3) / 2)) < 1e-14


def test_sliver_is_counted():
    # four points nearly on a plane (a flattened square): tiny volume
    P = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 1e-3], [0, 1, 0]], float)
    g, dih = q.tet_quality(P, np.array([[0, 1, 2, 3]]))
    s = q.summarize_tets(g, dih)
    assert g[0] < 0.01
    assert s["slivers"]["10"] == 1


def test_hexagonal_lattice_mesh_is_equilateral():
    h = 0.02
    pts = []
    for j in range(60):
        for i in range(60):
            pts.append([0.1 + i * h + (j % 2) * h / 2, 0.1 + j * h * math.sqrt(3) / 2])
    P = np.array(pts)
    xyz = np.zeros((len(P), 3))
    xyz[:, :2] = P
    # away from the staggered rows' ragged hull, every triangle is equilateral
    s = q.mesh_quality(xyz, 2, [0, 0, 0], [1, 1, 0], np.zeros((0, 15)),
                       region=([0.2, 0.2, 0.0], [1.1, 1.0, 0.0]))
    assert s["n_elements"] > 3000
    assert s["G_min"] > 1 - 1e-9 and abs(s["theta_min"] - 60) < 1e-6


def test_elements_in_holes_are_dropped():
    rng = np.random.default_rng(0)
    xyz = np.zeros((4000, 3))
    xyz[:, :2] = rng.random((4000, 2))
    hole = np.zeros(15)
    hole[:3] = [0.5, 0.5, 0.0]
    hole[3:6] = [0.3, 0.15, 0.3]
    hole[6:] = np.eye(3).ravel()
    keep = q.inside_domain(xyz, 2, [0, 0, 0], [1, 1, 0], hole[None])
    # the points inside the ellipse are not in the domain
    y = xyz[:, :2] - 0.5
    assert np.array_equal(keep, (y[:, 0] / 0.3) ** 2 + (y[:, 1] / 0.15) ** 2 > 1)
    from scipy.spatial import Delaunay
    tri = Delaunay(xyz[keep, :2]).simplices
    full = q.mesh_quality(xyz[keep], 2, [0, 0, 0], [1, 1, 0], np.zeros((0, 15)))
    cut = q.mesh_quality(xyz[keep], 2, [0, 0, 0], [1, 1, 0], hole[None])
    assert full["n_elements"] == len(tri)
    assert cut["n_elements"] < full["n_elements"]


def test_region_sample_matches_the_whole_mesh_inside_it():
    rng = np.random.default_rng(1)
    xyz = rng.random((3000, 3))
    whole = q.mesh_quality(xyz, 3, [0, 0, 0], [1, 1, 1], np.zeros((0, 15)))
    part = q.mesh_quality(xyz, 3, [0, 0, 0], [1, 1, 1], np.zeros((0, 15)),
                          region=([0.3, 0.3, 0.3], [0.7, 0.7, 0.7]))
    assert 0 < part["n_elements"] < whole["n_elements"]
    assert part["gamma_min"] >= whole["gamma_min"]


def test_ball_domain_filter():
    """domain 1: strictly inside the ball inscribed in the box"""
    rng = np.random.default_rng(3)
    xyz = rng.uniform(0.0, 2.0, (5000, 3))
    keep = q.inside_domain(xyz, 3, [0, 0, 0], [2, 2, 2], np.zeros((0, 15)), domain=1)
    assert np.array_equal(keep, np.sum((xyz - 1.0) ** 2, axis=1) < 1.0)
    keep2 = q.inside_domain(xyz, 2, [0, 0, 0], [2, 2, 0], np.zeros((0, 15)), domain=1)
    assert np.array_equal(keep2, np.sum((xyz[:, :2] - 1.0) ** 2, axis=1) < 1.0)


def test_level_set_domain_filter():
    """domain 2: inside the box where the interpolated level set is positive"""
    from paper_2003_01061_amd import workload as wk
    wl = wk.zalesak_disc(n_total=800)
    rng = np.random.default_rng(4)
    xyz = np.zeros((4000, 3))
    xyz[:, :2] = rng.random((4000, 2))
    keep = q.inside_domain(xyz, 2, wl.lo, wl.hi, wl.holes, domain=2, level=wl.level)
    assert np.array_equal(keep, wk._level_eval(wl.level, 2, xyz)[0] > 0)
    # the slot is outside: points in its middle are dropped
    slot = np.array([[0.5, 0.6, 0.0], [0.5, 0.75, 0.0]])
    assert not np.any(q.inside_domain(slot, 2, wl.lo, wl.hi, wl.holes, domain=2, level=wl.level))
