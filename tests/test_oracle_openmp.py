"""The OpenMP build of the oracle (its per-particle loops on threads, used
only to time the all-cores CPU baseline) gives bit-identical results to the
single-threaded build: every particle's arithmetic and every reduction's
order are the same."""
import numpy as np
import pytest

import oracle
from paper_2003_01061_amd import workload as wk


@pytest.mark.parametrize("make,steps", [
    (lambda: wk.scaled_hole_2d(6001, seed=31, res=128), 25),
    (lambda: wk.scaled_ball_3d(6001, seed=32, res=32), 8),
    (lambda: wk.paper_square(eps_damp=0.1, max_phase1_steps=10, ramp_steps=20), 40),
])
def test_openmp_build_is_bit_identical(make, steps):
    wl = make()
    a = oracle.RefJob(wl)
    b = oracle.RefJob(wl, openmp=True)
    a.step(steps)
    b.step(steps)
    xa, va = a.state()
    xb, vb = b.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    for f in (oracle.F_AP, oracle.F_A, oracle.F_VT, oracle.F_GAMMA):
        assert np.array_equal(a.field(f), b.field(f))
    assert a.counters() == b.counters()
    for name, x in zip(("off", "ids", "rel"), zip(a.neighbors(), b.neighbors())):
        assert np.array_equal(*x), name
