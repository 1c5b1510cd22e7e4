"""Verlet candidate lists (Algorithm 1's Verlet neighbour list, built with a
skin and filtered every step): the filtered lists are the cut-off lists, so
the trajectory follows the oracle (which scans every step) to the FP64 bar,
the interaction counts are equal step for step, and the particles are
re-sorted only when some particle has moved as far as the skin allows."""
import numpy as np
import pytest

import oracle
from paper_2003_01061_amd import binding
from paper_2003_01061_amd import workload as wk

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5

CASES = {
    "square64": (lambda: wk.square_lattice(), 200),
    "hole2d_20011": (lambda: wk.scaled_hole_2d(20011, seed=21, res=512), 60),
    "paper_square": (lambda: wk.paper_square(), 150),
    "ball3d_30011": (lambda: wk.scaled_ball_3d(30011, seed=22, res=96), 25),
    "ell3d_30011": (lambda: wk.ellipsoid_inclusions(n_total=30011, seed=24, dim=3, n_incl=16,
                                                    ratio=4.0, res=32, envelope_grid=24), 20),
    "zalesak_disc": (lambda: wk.zalesak_disc(), 60),
    "level_cube_sharp": (lambda: wk.level_cube_sharp(), 12),
}
_cache = {}


def case(name):
    if name not in _cache:
        mk, K = CASES[name]
        wl = mk()
        ref = oracle.RefJob(wl)
        per_step = []
        for _ in range(K):
            ref.step(1)
            per_step.append(ref.counters()["interactions_last"])
        _cache[name] = (wl, K, ref.state()[0], ref.counters(), per_step)
    return _cache[name]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(gpu):
    return gpu


def domain(wl):
    return float(np.max(wl.hi[:wl.dim] - wl.lo[:wl.dim]))


@pytest.mark.parametrize("skin", [0.3, 1.0])
@pytest.mark.parametrize("name", list(CASES))
def test_verlet_lists_follow_the_oracle(name, skin):
    wl, K, xr, cr, per_step = case(name)
    gpu = binding.SphMesh(wl, use_graph=1, verlet_skin=skin)
    got = []
    for _ in range(K // 2):              # graph pairs, with the count of each step
        gpu.step(2)
        got.append(gpu.counters()["interactions_last"])
    if K % 2:
        gpu.step(1)
    err = np.abs(gpu.positions() - xr).max() / domain(wl)
    assert err <= TOL64, err
    c = gpu.counters()
    assert c["interactions"] == cr["interactions"]
    assert c["escaped"] == cr["escaped"]
    assert got == per_step[1::2][:len(got)]
    builds = gpu.list_builds()
    assert 1 <= builds < K, builds       # the skin spares some sorts and scans


def test_verlet_fp32_mixed_follows_the_oracle():
    wl, K, xr, cr, _ = case("hole2d_20011")
    gpu = binding.SphMesh(wl, precision=binding.SPH_FP32_MIXED, use_graph=1, verlet_skin=0.3)
    gpu.step(K)
    err = np.abs(gpu.positions() - xr).max() / domain(wl)
    assert err <= TOL32, err


def test_verlet_eager_and_graph_steps_agree():
    wl, K, xr, _, _ = case("square64")
    a = binding.SphMesh(wl, use_graph=1, verlet_skin=0.3)
    b = binding.SphMesh(wl, use_graph=0, verlet_skin=0.3)
    a.step(K)
    b.step(K)
    assert np.array_equal(a.positions(), b.positions())
    assert a.list_builds() == b.list_builds()


def test_verlet_state_change_and_list_query_force_a_rebuild():
    """set_state and a neighbour query re-sort the particles, so the next step
    starts from fresh lists; the trajectory still follows the oracle"""
    wl, _, _, _, _ = case("hole2d_20011")
    ref = oracle.RefJob(wl)
    gpu = binding.SphMesh(wl, use_graph=1, verlet_skin=0.3)
    ref.step(7)
    gpu.step(7)
    x, v = ref.state()
    x2 = x.copy()
    x2[wl.feature == 0] += 1e-4 * np.sin(np.arange(3 * np.count_nonzero(wl.feature == 0))).reshape(-1, 3) * \
        np.array([1, 1, 0])
    # keep the moved volume particles inside: only the interior ones
    inner = (wl.feature == 0) & (np.abs(x[:, 0] - 0.5) < 0.4) & (np.abs(x[:, 1] - 0.5) < 0.4) & \
        (np.hypot(x[:, 0] - 0.5, x[:, 1] - 0.5) > 0.3)
    x3 = np.where(inner[:, None], x2, x)
    ref.set_state(x3, v)
    gpu.set_state(x3, v)
    b0 = gpu.list_builds()
    off_g, ids_g, rel_g = gpu.neighbors()
    off_r, ids_r, rel_r = ref.neighbors()
    assert np.array_equal(off_g, off_r) and np.array_equal(ids_g, ids_r)
    ref.step(9)
    gpu.step(9)
    assert gpu.list_builds() >= b0 + 1
    err = np.abs(gpu.positions() - ref.state()[0]).max()
    assert err <= TOL64, err


def test_verlet_batch_jobs_follow_the_oracle():
    """a batch with Verlet lists: a rebuild is due for every job once any
    job's particle has moved far enough; jobs joining and leaving force one"""
    wls = [wk.scaled_hole_2d(3001, seed=31), wk.square_lattice(n_side=32, seed=5),
           wk.scaled_hole_2d(7001, seed=34, centre=(0.45, 0.55), radius=0.2)]
    specs = [binding.JobSpec(w) for w in wls]
    b = binding.SphBatch(2, binding.SPH_FP64, max_particles=sum(s.n for s in specs),
                         max_cells=sum(s.cells() for s in specs), max_jobs=3, verlet_skin=0.3)
    A = b.add(specs[0])
    B = b.add(specs[1])
    b.step(12)
    C = b.add(specs[2])
    b.step(9)
    b.remove(A)
    b.step(6)
    for job, wl, K in ((B, wls[1], 27), (C, wls[2], 15)):
        ref = oracle.RefJob(wl)
        ref.step(K)
        err = np.abs(b.positions(job) - ref.state()[0]).max()
        assert err <= TOL64, (job, err)
        assert b.counters(job)["interactions"] == ref.counters()["interactions"]
    assert 3 <= b.list_builds() < 27


def test_verlet_skin_is_validated():
    wl = wk.square_lattice(n_side=16)
    with pytest.raises(binding.SphError):
        binding.SphMesh(wl, verlet_skin=-0.1)
    with pytest.raises(binding.SphError):
        binding.SphMesh(wl, verlet_skin=2.5)
    assert binding.SphMesh(wl).list_builds() == 0
