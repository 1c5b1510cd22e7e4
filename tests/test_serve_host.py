"""Host logic of the serving loop against a stand-in batch (no GPU): every
request finishes, admission never exceeds the slot cap or a batch's particle
and cell capacity, requests of one dimension are admitted in arrival order,
over-sized requests are rejected, and latencies are measured from arrival."""
import numpy as np
import pytest

from paper_2003_01061_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class Spec:
    def __init__(self, n, cells, steps_needed):
        self.n, self._cells, self.steps_needed = n, cells, steps_needed

    def cells(self):
        return self._cells


class FakeBatch:
    """Jobs converge after their own number of steps; a step costs time in
    proportion to the resident particles (the clock is shared)."""
    instances = []

    def __init__(self, dim, precision, max_particles, max_cells, max_jobs, max_neighbors,
                 scan_tile=0):
        self.dim, self.cap_p, self.cap_c, self.cap_j = dim, max_particles, max_cells, max_jobs
        self.jobs = {}
        self.log = []
        FakeBatch.instances.append(self)

    def add(self, spec):
        assert len(self.jobs) < self.cap_j
        assert sum(s.n for s, _ in self.jobs.values()) + spec.n <= self.cap_p
        assert sum(s.cells() for s, _ in self.jobs.values()) + spec.cells() <= self.cap_c
        slot = min(set(range(self.cap_j)) - set(self.jobs))
        self.jobs[slot] = [spec, 0]
        self.log.append(("add", spec, CLOCK.t))
        return slot

    def remove(self, j):
        del self.jobs[j]

    def step(self, k):
        CLOCK.t += k * 1e-6 * sum(s.n for s, _ in self.jobs.values())
        for v in self.jobs.values():
            v[1] = min(v[0].steps_needed, v[1] + k)

    def status(self):
        live = np.zeros(self.cap_j, bool)
        conv = np.zeros(self.cap_j, bool)
        steps = np.zeros(self.cap_j, np.int64)
        for j, (s, k) in self.jobs.items():
            live[j], conv[j], steps[j] = True, k >= s.steps_needed, k
        return live, conv, steps

    def positions(self, j):
        return np.full((self.jobs[j][0].n, 3), float(j))

    def error(self, j):
        return dict(e_sys=0.0, phase=4, converged=True, step=self.jobs[j][1])

    def counters(self, j):
        return dict(interactions=10 * self.jobs[j][0].n * self.jobs[j][1])


CLOCK = FakeClock()


def footprint(dim, precision, max_particles, max_cells, max_jobs, max_neighbors, scan_tile=0):
    return 1000 + 100 * max_particles + 8 * max_cells + 64 * max_jobs


def make_server(pool, slots, chunk=20):
    FakeBatch.instances.clear()
    CLOCK.t = 0.0
    return serve.Server(pool_bytes=pool, slots=slots, precision=1, chunk=chunk,
                        batch_factory=FakeBatch, footprint=footprint, clock=CLOCK,
                        sleep=CLOCK.sleep)


def stream(n_jobs, seed, rate):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_jobs))
    reqs = []
    for q in range(n_jobs):
        n = int(np.exp(rng.uniform(np.log(100), np.log(5000))))
        reqs.append(serve.Request(q, int(rng.choice([2, 3])), n, float(t[q]),
                                  Spec(n, n // 2, int(rng.integers(1, 12)) * 20)))
    return reqs


def test_every_request_finishes_within_the_caps():
    srv = make_server(pool=2_000_000, slots=5)
    reqs = stream(60, 1, rate=50.0)
    res = srv.run(reqs)
    assert all(r.status == "ok" for r in res)
    assert [r.idx for r in res] == list(range(60))
    for r, q in zip(res, reqs):
        assert r.admitted >= q.arrival and r.done > r.admitted
        assert r.steps == q.spec.steps_needed
    assert srv.stats.max_resident <= 5
    for d, ratio in ((2, 4.0), (3, 2.0)):   # the capacities the pool buys, and no more
        p = srv.cap_particles[d]
        assert footprint(d, 1, p, srv.cap_cells[d], 5, 0) <= 1_000_000
        assert footprint(d, 1, p + 1, int(ratio * (p + 1)), 5, 0) > 1_000_000
    s = serve.summarize(res, srv.stats)
    assert s["completed"] == 60 and s["latency_p50_s"] <= s["latency_p99_s"]


def test_admission_is_first_come_first_served_per_dimension():
    srv = make_server(pool=2_000_000, slots=3)
    reqs = stream(40, 2, rate=1e4)         # a burst: the queue builds up
    srv.run(reqs)
    for b in FakeBatch.instances:
        order = [s for (_, s, _) in b.log]
        want = sorted(order, key=lambda s: [q.arrival for q in reqs if q.spec is s][0])
        assert order == want
    assert srv.stats.blocked_slots > 0


def test_memory_bounds_admission_and_oversized_requests_are_rejected():
    srv = make_server(pool=1_200_000, slots=32)
    cap = srv.cap_particles[2]
    big = [serve.Request(q, 2, int(0.6 * cap), 0.0, Spec(int(0.6 * cap), 10, 40)) for q in range(3)]
    huge = serve.Request(3, 2, cap + 1, 0.0, Spec(cap + 1, 10, 40))
    res = srv.run(big + [huge])
    assert res[3].status == "rejected"
    done = sorted(r.done for r in res[:3])
    adm = sorted(r.admitted for r in res[:3])
    # two 60 % jobs never share the batch: each waits for the previous one
    assert adm[1] >= done[0] and adm[2] >= done[1]
    assert srv.stats.blocked_memory > 0


def test_a_job_that_never_converges_is_retired_at_the_step_limit():
    srv = make_server(pool=2_000_000, slots=4)
    srv.max_job_steps = 200
    reqs = [serve.Request(0, 2, 500, 0.0, Spec(500, 100, 10**9)),
            serve.Request(1, 2, 500, 0.0, Spec(500, 100, 60))]
    res = srv.run(reqs)
    assert res[0].status == "error" and "not converged" in res[0].message
    assert res[1].status == "ok" and res[1].steps == 60


def test_idle_server_waits_for_arrivals():
    srv = make_server(pool=2_000_000, slots=4)
    reqs = [serve.Request(0, 3, 500, 5.0, Spec(500, 100, 40))]
    res = srv.run(reqs)
    assert res[0].admitted >= 5.0 and res[0].latency > 0
