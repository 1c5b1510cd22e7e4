"""Pins of the oracle's level-set domain (sec. 2.1: the geometry is the
positive phase of a level set phi kept on a Cartesian background mesh).
phi is interpolated multilinearly from grid nodes; the zero level set is
one surface (curve) feature.  Checked against closed forms and against the
input generator's own evaluation of the interpolated phi:

* a plane: phi linear, so interpolation and gradient are exact, one Newton
  step lands on the plane, and the normal out of the domain is -grad/|grad|;
* the 2D peanut: projected points satisfy phi = 0; the lists match brute
  force; after a few steps the curve particles still sit on phi = 0 and
  move tangentially, the volume particles stay where phi > 0.
"""
import numpy as np
import pytest

import oracle
from paper_2003_01061_amd import workload as wk


def _plane_level(dim, n):
    lo, hi = [0.0, 0.0, 0.0], [1.0, 1.0, 1.0 if dim == 3 else 0.0]
    k = np.array([0.6, -0.3, 0.5 if dim == 3 else 0.0])
    gn = [n, n + 2, n + 1 if dim == 3 else 1]
    ax = [np.arange(gn[a]) / (gn[a] - 1) if gn[a] > 1 else np.zeros(1) for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    phi = 0.1 + k[0] * X.ravel() + k[1] * Y.ravel() + k[2] * Z.ravel()
    level = dict(phi=phi, n=gn, lo=lo, hi=[1.0, 1.0, 1.0])
    return lo, hi, k, level


@pytest.mark.parametrize("dim", [2, 3])
def test_plane_level_set(dim):
    lo, hi, k, level = _plane_level(dim, 9)
    g = oracle.make_geometry(dim, lo, hi, np.zeros((0, 15)), domain=2, level=level)
    L = oracle.lib()
    assert L.sphref_n_features(g) == 2
    rng = np.random.default_rng(3)
    kn = k[:dim] / np.linalg.norm(k[:dim])
    done = 0
    while done < 50:
        x = np.zeros(3)
        x[:dim] = rng.uniform(0.1, 0.9, dim)
        # only where the plane's closest point lies inside the grid box
        star = x[:dim] - (0.1 + k[:dim] @ x[:dim]) / (k[:dim] @ k[:dim]) * k[:dim]
        if not np.all((star > 0.02) & (star < 0.98)):
            continue
        done += 1
        q = x.copy()
        L.sphref_project(g, 1, q)
        val = 0.1 + k[:dim] @ q[:dim]
        assert abs(val) <= 1e-15
        # the closest point of a plane: x moved along the normal only
        dx = q[:dim] - x[:dim]
        assert np.linalg.norm(dx - (dx @ kn) * kn) <= 1e-14
        n = np.zeros(3)
        assert L.sphref_boundary_normal(g, 0, 1, q, n) == 1
        assert np.abs(n[:dim] + kn).max() <= 1e-15


def _phi(wl, x):
    return wk._level_eval(wl.level, wl.dim, np.atleast_2d(x))


def test_peanut_projection_lands_on_the_zero_set():
    wl = wk.level_peanut(n_total=800)
    g = oracle.make_geometry(2, wl.lo, wl.hi, wl.holes, 2, wl.level)
    L = oracle.lib()
    rng = np.random.default_rng(4)
    for t in range(60):
        x = np.array([rng.uniform(0.05, 0.95), rng.uniform(0.15, 0.85), 0.0])
        f, _ = _phi(wl, x)
        if abs(f[0]) > 0.04:
            continue
        q = x.copy()
        L.sphref_project(g, 1, q)
        fq, _ = _phi(wl, q)
        assert abs(fq[0]) <= 1e-14, (x, q, fq)


def test_peanut_lists_match_brute_force():
    wl = wk.level_peanut(n_total=1200)
    ref = oracle.RefJob(wl)
    off, ids, rel = ref.neighbors()
    h = ref.field(oracle.F_H)
    c = wl.params["kernel_support"]
    x = wl.xyz
    for i in range(wl.n):
        d2 = (x[i, 0] - x[:, 0]) ** 2 + (x[i, 1] - x[:, 1]) ** 2
        m = np.maximum(h[i], h)
        cand = np.nonzero(d2 < (c * c) * (m * m))[0]
        cand = cand[cand != i]
        fi = wl.feature[i]
        want = cand if fi == 0 else cand[wl.feature[cand] == fi]
        assert np.array_equal(ids[off[i]:off[i + 1]], want), i


def test_peanut_steps_keep_particles_on_and_inside():
    wl = wk.level_peanut(n_total=1200)
    ref = oracle.RefJob(wl)
    ref.step(10)
    x, v = ref.state()
    f, gr = _phi(wl, x)
    on = wl.feature == 1
    assert np.abs(f[on]).max() <= 1e-13
    nrm = gr[on] / np.linalg.norm(gr[on], axis=1, keepdims=True)
    vn = np.sum(nrm * v[on, :2], axis=1)
    assert np.abs(vn).max() <= 1e-12 * max(np.abs(v[on]).max(), 1e-300)
    assert np.abs(v[on]).max() > 0
    assert np.all(f[~on] > 0)
