"""The serving loop on the GPU: requests of both dimensions arrive while
others run, wait for slots and memory, share batches, and each result is
bit-identical to the same job run alone to convergence."""
import numpy as np
import pytest

from paper_2003_01061_amd import binding, serve
from paper_2003_01061_amd import workload as wk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(gpu):
    return gpu


def short_stream(n_jobs, seed):
    descs = wk.serving_stream(n_jobs, seed=seed, n_min=800, n_max=12_000,
                              max_phase1_steps=60, ramp_steps=20, phase2_steps=40)
    wls = [wk.build_job(d) for d in descs]
    t = wk.poisson_arrivals(n_jobs, rate=40.0, seed=seed)
    reqs = [serve.Request(d.idx, d.dim, d.n, float(t[q]), binding.JobSpec(w))
            for q, (d, w) in enumerate(zip(descs, wls))]
    return wls, reqs


@pytest.mark.parametrize("precision", [binding.SPH_FP32_MIXED, binding.SPH_FP64])
def test_served_results_equal_the_jobs_alone(precision):
    wls, reqs = short_stream(10, seed=11)
    srv = serve.Server(pool_bytes=192 << 20, slots=3, precision=precision, chunk=20,
                       keep_positions=True)
    res = srv.run(reqs)
    assert all(r.status == "ok" for r in res), [r.message for r in res]
    assert srv.stats.blocked_slots > 0            # requests waited for a slot
    assert {r.dim for r in res} == {2, 3}
    for r, wl in zip(res, wls):
        g = binding.SphMesh(wl, precision=precision, use_graph=1)
        g.step(r.steps)
        e = g.error()
        assert e["converged"] and e["step"] == r.steps
        assert np.array_equal(g.positions(), r.positions), r.idx
        assert g.counters()["interactions"] == r.interactions
        assert r.latency > 0 and r.admitted >= r.arrival
    s = serve.summarize(res, srv.stats)
    assert s["completed"] == 10 and s["latency_p99_s"] >= s["latency_p50_s"] > 0


def test_oversized_request_is_rejected_and_the_rest_served():
    wls, reqs = short_stream(4, seed=12)
    big = wk.scaled_hole_2d(400_000, seed=3, max_phase1_steps=60, ramp_steps=20,
                            phase2_steps=40)
    reqs.append(serve.Request(99, 2, big.n, 0.0, binding.JobSpec(big)))
    srv = serve.Server(pool_bytes=64 << 20, slots=4, chunk=20, max_job_steps=2000)
    assert srv.cap_particles[2] < big.n
    res = srv.run(reqs)
    by = {r.idx: r for r in res}
    assert by[99].status == "rejected"
    assert all(by[r.idx].status == "ok" for r in reqs if r.idx != 99)
