"""Autotuning knobs on the GPU: the scan tile never changes a result, the
cell size changes only the rounding of the sums (lists stay bit-exact), and
a tuned configuration stays within the oracle tolerance."""
import numpy as np
import pytest

import oracle
from paper_2003_01061_amd import autotune, binding
from paper_2003_01061_amd import workload as wk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(gpu):
    return gpu


@pytest.mark.parametrize("make", [lambda: wk.scaled_hole_2d(6007, seed=61),
                                  lambda: wk.scaled_ball_3d(8009, seed=62, res=48)])
def test_scan_tile_is_bit_exact(make):
    wl = make()
    runs = []
    for tile in (2, 4, 8):
        g = binding.SphMesh(wl, precision=binding.SPH_FP32_MIXED, use_graph=1, scan_tile=tile)
        g.step(15)
        runs.append((g.positions(), g.counters()))
    for x, c in runs[1:]:
        assert np.array_equal(x, runs[0][0]) and c == runs[0][1]


@pytest.mark.parametrize("cf", [0.75, 1.25, 2.0])
def test_cell_factor_keeps_lists_exact_and_positions_in_tolerance(cf):
    wl = wk.scaled_hole_2d(6007, seed=61)
    ref = oracle.RefJob(wl)
    off_r, ids_r, rel_r = ref.neighbors()
    g = binding.SphMesh(wl, use_graph=1, cell_factor=cf)
    off, ids, rel = g.neighbors()
    assert np.array_equal(off, off_r) and np.array_equal(ids, ids_r)
    assert np.array_equal(rel, rel_r)
    ref.step(30)
    g.step(30)
    assert np.abs(g.positions() - ref.state()[0]).max() <= 1e-12


def test_tuned_configuration_runs_and_matches_the_oracle():
    wl = wk.scaled_hole_2d(20011, seed=63)
    spec = binding.JobSpec(wl)
    r = autotune.tune([spec], 2, binding.SPH_FP64, steps=6, warmup=2)
    n_grid = len(autotune.CELL_FACTORS) * len(autotune.SCAN_TILES)
    assert len(r.table) == n_grid + len(autotune.SKINS) * len(autotune.SCAN_TILES)
    assert all(t["ms_per_step"] > 0 for t in r.table)
    best = r.best
    g = binding.SphMesh(wl, use_graph=1, **best)
    g.step(20)
    ref = oracle.RefJob(wl)
    ref.step(20)
    assert np.abs(g.positions() - ref.state()[0]).max() <= 1e-12
