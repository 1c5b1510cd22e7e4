"""Mesh quality of a relaxed particle set (host post-processing).

The particles are the mesh vertices.  As in the paper's sec. 4, connectivity
is built only after the run, to measure quality: here a Delaunay
triangulation / tetrahedralisation of the final positions (scipy, Qhull),
keeping the elements whose centroid lies in the domain (the box minus its
holes, the ball inscribed in the box, or the positive phase of a gridded
level set).  The relaxation never uses it.

Triangles (sec. 4): G = 2 sqrt(3) S / (P H), with S the area, P the
half-perimeter and H the longest edge (G = 1 for an equilateral triangle),
and the interior angles.  Reported: G_avg, G_min, theta_max, theta_min, the
average over triangles of their smallest angle (theta_min#) and the number
of triangles with an angle below 30 degrees.

Tetrahedra (sec. 4): the dihedral angles and the radius ratio
gamma = 3 r_in / r_circ (1 for a regular tetrahedron).  Reported: gamma_avg,
gamma_min, theta_min, theta_max, the average smallest dihedral angle
(theta_min#) and the sliver counts: tetrahedra whose smallest dihedral angle
is below 10, 20, 30 and 40 degrees.
"""
from __future__ import annotations

import numpy as np


def inside_domain(pts, dim, lo, hi, holes, domain=0, level=None):
    """Strictly inside the box [lo, hi]^dim and outside every hole (hole
    records: centre[3], semi-axes[3], rotation[9] row-major with local
    coordinates y = rot (x - centre); the hole is sum (y_k / a_k)^2 <= 1);
    for domain 1, strictly inside the ball inscribed in the box; for domain
    2, inside the box where the gridded level set `level` is positive."""
    pts = np.asarray(pts, float)
    if domain == 2:
        from .workload import _level_eval
        ok = np.all((pts[:, :dim] > np.asarray(lo)[:dim]) & (pts[:, :dim] < np.asarray(hi)[:dim]), axis=1)
        return ok & (_level_eval(level, dim, pts)[0] > 0)
    if domain == 1:
        c = 0.5 * (np.asarray(lo, float)[:dim] + np.asarray(hi, float)[:dim])
        R = 0.5 * (float(hi[0]) - float(lo[0]))
        return np.sum((pts[:, :dim] - c) ** 2, axis=1) < R * R
    ok = np.all((pts[:, :dim] > np.asarray(lo)[:dim]) & (pts[:, :dim] < np.asarray(hi)[:dim]), axis=1)
    for rec in np.asarray(holes, float).reshape(-1, 15):
        R = rec[6:15].reshape(3, 3)[:dim, :dim]
        y = (pts[:, :dim] - rec[:dim]) @ R.T
        ok &= np.sum((y / rec[3:3 + dim]) ** 2, axis=1) > 1.0
    return ok


def triangle_quality(P, tris):
    """Per-triangle G and angles (degrees) of triangles tris (m x 3) over
    points P (n x 2)."""
    a, b, c = P[tris[:, 0]], P[tris[:, 1]], P[tris[:, 2]]
    la = np.linalg.norm(b - c, axis=1)          # edge opposite a
    lb = np.linalg.norm(c - a, axis=1)
    lc = np.linalg.norm(a - b, axis=1)
    u, v = b - a, c - a
    S = 0.5 * np.abs(u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0])
    Ph = 0.5 * (la + lb + lc)
    H = np.maximum(np.maximum(la, lb), lc)
    G = 2.0 * np.sqrt(3.0) * S / (Ph * H)

    def angle(opp, s1, s2):                      # law of cosines
        cs = (s1 * s1 + s2 * s2 - opp * opp) / (2.0 * s1 * s2)
        return np.degrees(np.arccos(np.clip(cs, -1.0, 1.0)))
    ang = np.stack([angle(la, lb, lc), angle(lb, lc, la), angle(lc, la, lb)], 1)
    return G, ang


def tet_quality(P, tets):
    """Per-tetrahedron radius ratio and the six dihedral angles (degrees)."""
    p = [P[tets[:, k]] for k in range(4)]
    u, v, w = p[1] - p[0], p[2] - p[0], p[3] - p[0]
    det = np.einsum("ij,ij->i", u, np.cross(v, w))
    vol = np.abs(det) / 6.0
    faces = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]
    area = sum(0.5 * np.linalg.norm(np.cross(p[j] - p[i], p[k] - p[i]), axis=1)
               for i, j, k in faces)
    r_in = 3.0 * vol / area
    # circumcentre relative to p0: (|u|^2 v x w + |v|^2 w x u + |w|^2 u x v) / (2 u . (v x w))
    num = (np.sum(u * u, 1)[:, None] * np.cross(v, w) + np.sum(v * v, 1)[:, None] * np.cross(w, u)
           + np.sum(w * w, 1)[:, None] * np.cross(u, v))
    with np.errstate(divide="ignore", invalid="ignore"):
        r_circ = np.linalg.norm(num, axis=1) / np.abs(2.0 * det)
        gamma = np.where(r_circ > 0, 3.0 * r_in / r_circ, 0.0)
    dih = []
    for i, j in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)):
        k, l = [m for m in range(4) if m not in (i, j)]
        e = p[j] - p[i]
        e = e / np.linalg.norm(e, axis=1, keepdims=True)
        # the other two vertices projected onto the plane normal to the edge
        a = p[k] - p[i]
        b = p[l] - p[i]
        a = a - np.sum(a * e, 1)[:, None] * e
        b = b - np.sum(b * e, 1)[:, None] * e
        cs = np.sum(a * b, 1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
        dih.append(np.degrees(np.arccos(np.clip(cs, -1.0, 1.0))))
    return np.nan_to_num(gamma), np.stack(dih, 1)


def summarize_triangles(G, ang):
    if len(G) == 0:
        return dict(n_elements=0)
    amin = ang.min(1)
    return dict(n_elements=int(len(G)), G_avg=float(G.mean()), G_min=float(G.min()),
                theta_max=float(ang.max()), theta_min=float(amin.min()),
                theta_min_avg=float(amin.mean()), n_theta_below_30=int(np.sum(amin < 30.0)))


def summarize_tets(gamma, dih):
    if len(gamma) == 0:
        return dict(n_elements=0)
    dmin = dih.min(1)
    return dict(n_elements=int(len(gamma)), gamma_avg=float(gamma.mean()),
                gamma_min=float(gamma.min()), theta_min=float(dmin.min()),
                theta_max=float(dih.max()), theta_min_avg=float(dmin.mean()),
                slivers={str(t): int(np.sum(dmin < t)) for t in (10, 20, 30, 40)})


def mesh_quality(xyz, dim, lo, hi, holes, region=None, domain=0, level=None):
    """Delaunay mesh of the positions xyz (n x 3) and its quality summary.
    region = (rlo, rhi) restricts the measure to elements whose centroid lies
    in that sub-box (a sample of a mesh too large to tetrahedralise whole:
    the points within the sub-box grown by a margin are triangulated)."""
    from scipy.spatial import Delaunay
    P = np.asarray(xyz, float)[:, :dim]
    if region is not None:
        rlo, rhi = (np.asarray(r, float)[:dim] for r in region)
        m = 0.1 * float(np.max(rhi - rlo))
        keep = np.all((P > rlo - m) & (P < rhi + m), axis=1)
        P = P[keep]
    simp = Delaunay(P).simplices
    cen = np.zeros((len(simp), 3))
    cen[:, :dim] = P[simp].mean(1)
    ok = inside_domain(cen, dim, lo, hi, holes, domain, level)
    if region is not None:
        ok &= np.all((cen[:, :dim] > rlo) & (cen[:, :dim] < rhi), axis=1)
    simp = simp[ok]
    if dim == 2:
        return summarize_triangles(*triangle_quality(P, simp))
    return summarize_tets(*tet_quality(P, simp))
