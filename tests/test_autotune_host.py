"""Selection logic of the autotuner with an injected timing (no GPU)."""
import pytest

from paper_2003_01061_amd import autotune


class Spec:
    n = 1000


def test_picks_the_fastest_configuration():
    times = {(1.0, 4): 3.0, (0.75, 2): 2.0, (1.25, 8): 2.5}
    r = autotune.tune([Spec()], 2, 1, measure=lambda cf, t: times.get((cf, t), 9.0))
    assert r.best == {"cell_factor": 0.75, "scan_tile": 2, "verlet_skin": 0.0}
    assert len(r.table) == len(autotune.CELL_FACTORS) * len(autotune.SCAN_TILES)
    assert r.speedup_over_default() == pytest.approx(1.5)


def test_ties_keep_the_default_and_the_grid_always_holds_it():
    r = autotune.tune([Spec()], 3, 1, cell_factors=(0.5, 0.75), scan_tiles=(2,),
                      measure=lambda cf, t: 1.0)
    assert r.table[0]["cell_factor"] == 1.0 and r.table[0]["scan_tile"] == 4
    assert r.best == autotune.DEFAULT


def test_needs_a_job():
    with pytest.raises(ValueError):
        autotune.tune([], 2, 1, measure=lambda cf, t: 1.0)


def test_a_gain_within_the_noise_keeps_the_default():
    times = {(1.0, 4): 1.00, (0.75, 2): 0.99}
    r = autotune.tune([Spec()], 2, 1, measure=lambda cf, t: times.get((cf, t), 9.0))
    assert r.best == autotune.DEFAULT
    r = autotune.tune([Spec()], 2, 1, measure=lambda cf, t: times.get((cf, t), 9.0), min_gain=0.0)
    assert r.best == {"cell_factor": 0.75, "scan_tile": 2, "verlet_skin": 0.0}


def test_skins_are_timed_at_the_best_pair_and_kept_only_when_faster():
    times = {(1.0, 4): 3.0, (0.75, 2): 2.0}
    seen = []

    def skin_time(cf, t, sk):
        seen.append((cf, t, sk))
        return {0.3: 1.9, 0.5: 1.5, 0.8: 1.7}[sk] + (0.0 if t == 8 else 0.1)
    r = autotune.tune([Spec()], 3, 1, measure=lambda cf, t: times.get((cf, t), 9.0),
                      measure_skin=skin_time)
    assert seen == [(0.75, t, sk) for sk in autotune.SKINS for t in autotune.SCAN_TILES]
    assert r.best == {"cell_factor": 0.75, "scan_tile": 8, "verlet_skin": 0.5}
    assert r.speedup_over_default() == pytest.approx(2.0)
    # a skin within the noise of the best pair is not taken
    r = autotune.tune([Spec()], 3, 1, measure=lambda cf, t: times.get((cf, t), 9.0),
                      measure_skin=lambda cf, t, sk: 1.99)
    assert r.best["verlet_skin"] == 0.0


def test_at_a_skin_a_tile_within_the_noise_keeps_the_best_pairs_tile():
    times = {(1.0, 4): 3.0}

    def skin_time(cf, t, sk):
        # skin 0.8 is the fastest; at it tile 8 is 1% faster than tile 4
        return {0.3: 2.5, 0.5: 2.2, 0.8: 2.0}[sk] - (0.02 if t == 8 else 0.0)
    r = autotune.tune([Spec()], 2, 1, measure=lambda cf, t: times.get((cf, t), 9.0),
                      measure_skin=skin_time)
    assert r.best == {"cell_factor": 1.0, "scan_tile": 4, "verlet_skin": 0.8}
