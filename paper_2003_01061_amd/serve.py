"""Serving: a request loop that admits meshing jobs of both dimensions into
device-resident batches and steps them with continuous batching.

* Admission.  The server owns a memory pool (bytes of device memory) and a
  number of job slots.  The pool is split between a 2D and a 3D batch, each
  allocated once with the particle and cell capacities its share buys (the
  library's own footprint formula).  A request is admitted, in arrival order
  per dimension, when a slot is free and its particles and cells fit beside
  the jobs already resident in its batch; otherwise it waits.  A request that
  could never fit is rejected at once.
* Continuous batching.  Every resident job advances in the one launch
  sequence of its batch; the two batches run on their own streams, so 2D and
  3D work overlaps on the device.  After every chunk of steps the server
  reads the per-job flags, retires converged jobs (positions copied to the
  host, latency stamped), which frees their slot and memory, and admits what
  is waiting.  A job's particles cross the host/device boundary only at admit
  and retire.
* Latency.  Time from a request's arrival to its converged positions on the
  host; the report gives p50 / p99 beside the throughput.

The device work is the library's (binding.SphBatch); this module is host
scheduling only, so it runs unchanged against a stand-in batch in CPU tests.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


@dataclass
class Request:
    idx: int
    dim: int
    n: int
    arrival: float          # seconds after the start of the run
    spec: object            # binding.JobSpec (or anything with .n and .cells())


@dataclass
class JobResult:
    idx: int
    dim: int
    n: int
    arrival: float
    admitted: float = float("nan")
    done: float = float("nan")
    steps: int = 0
    interactions: int = 0
    e_sys: float = float("nan")
    status: str = "ok"          # ok | rejected | error
    message: str = ""
    positions: Optional[np.ndarray] = None

    @property
    def latency(self):
        return self.done - self.arrival


@dataclass
class ServeStats:
    blocked_slots: int = 0      # admission rounds stopped by the slot cap
    blocked_memory: int = 0     # ... by the particle or cell capacity
    polls: int = 0
    chunks: int = 0
    max_resident: int = 0
    max_particles: dict = field(default_factory=dict)


class _Resident:
    def __init__(self, req, cells, admitted):
        self.req, self.cells, self.admitted = req, cells, admitted


class Server:
    """Continuous-batching server over one batch per dimension."""

    def __init__(self, pool_bytes=8 << 30, slots=32, precision=None, chunk=20,
                 max_neighbors=None, share=None, cells_per_particle=None,
                 batch_factory: Optional[Callable] = None,
                 footprint: Optional[Callable] = None,
                 clock=time.perf_counter, sleep=time.sleep, keep_positions=False,
                 max_job_steps=1 << 20, tuned=None):
        if precision is None or batch_factory is None or footprint is None:
            from . import binding
            precision = binding.SPH_FP32_MIXED if precision is None else precision
            batch_factory = batch_factory or binding.SphBatch
            footprint = footprint or binding.batch_footprint
        if int(slots) < 1 or int(chunk) < 1:
            raise ValueError("slots and chunk must be >= 1")
        self.precision = precision
        self.slots = int(slots)
        self.chunk = int(chunk)
        self.clock, self.sleep = clock, sleep
        self.keep_positions = keep_positions
        self.max_job_steps = int(max_job_steps)   # a job not converged by then is retired as an error
        # autotuned settings per dimension: {"cell_factor": .., "scan_tile": ..}
        self.tuned = {d: dict(c) for d, c in (tuned or {}).items()}
        self.max_neighbors = dict(max_neighbors or {2: 104, 3: 320})
        share = dict(share or {2: 0.5, 3: 0.5})
        ratio = dict(cells_per_particle or {2: 4.0, 3: 2.0})
        self.cap_particles, self.cap_cells, self.bytes = {}, {}, {}
        self.batches = {}
        for d in (2, 3):
            budget = int(pool_bytes * share[d])

            def fp(p, d=d):
                return footprint(dim=d, precision=precision, max_particles=int(p),
                                 max_cells=max(1, int(ratio[d] * p)), max_jobs=self.slots,
                                 max_neighbors=self.max_neighbors[d])
            base, per = fp(0), (fp(1 << 20) - fp(0)) / float(1 << 20)
            if base < 0 or per <= 0:
                raise ValueError("invalid batch capacities")
            p = max(0, int((budget - base) / per))
            while p > 0 and fp(p) > budget:      # the footprint is affine; guard rounding
                p -= 1
            self.cap_particles[d] = p
            self.cap_cells[d] = max(1, int(ratio[d] * p))
            self.bytes[d] = fp(p)
            self.batches[d] = batch_factory(d, precision, max_particles=p,
                                            max_cells=self.cap_cells[d], max_jobs=self.slots,
                                            max_neighbors=self.max_neighbors[d],
                                            scan_tile=self.tuned.get(d, {}).get("scan_tile", 0))
        self.stats = ServeStats()

    def footprint_bytes(self):
        return sum(self.bytes.values())

    def run(self, requests, progress=None):
        """Serve every request; returns one JobResult per request (in request
        order).  Arrival times are relative to the call."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.idx))
        results = {r.idx: JobResult(r.idx, r.dim, r.n, r.arrival) for r in reqs}
        queues = {2: deque(), 3: deque()}
        resident = {2: {}, 3: {}}
        used = {d: [0, 0] for d in (2, 3)}     # particles, cells
        finished = 0
        nxt = 0
        cells_of = {}
        spec_of = {}

        def spec(r):
            # the request's job with its dimension's tuned cell size
            if r.idx not in spec_of:
                cf = self.tuned.get(r.dim, {}).get("cell_factor")
                if cf is None:
                    spec_of[r.idx] = r.spec
                else:
                    from .autotune import with_cell_factor
                    spec_of[r.idx] = with_cell_factor(r.spec, cf)
            return spec_of[r.idx]
        t0 = self.clock()
        st = self.stats
        st.max_particles = {2: 0, 3: 0}

        def now():
            return self.clock() - t0

        while finished < len(reqs):
            t = now()
            while nxt < len(reqs) and reqs[nxt].arrival <= t:
                queues[reqs[nxt].dim].append(reqs[nxt])
                nxt += 1
            # admission, first come first served within each dimension
            for d in (2, 3):
                q = queues[d]
                while q:
                    r = q[0]
                    if r.idx not in cells_of:
                        cells_of[r.idx] = int(spec(r).cells())
                    cells = cells_of[r.idx]
                    if (cells < 0 or r.n > self.cap_particles[d] or cells > self.cap_cells[d]):
                        q.popleft()
                        res = results[r.idx]
                        res.status, res.done = "rejected", now()
                        res.message = "larger than the batch capacity" if cells >= 0 else "invalid job"
                        finished += 1
                        continue
                    if sum(len(x) for x in resident.values()) >= self.slots:
                        st.blocked_slots += 1
                        break
                    if (used[d][0] + r.n > self.cap_particles[d]
                            or used[d][1] + cells > self.cap_cells[d]):
                        st.blocked_memory += 1
                        break
                    q.popleft()
                    try:
                        job = self.batches[d].add(spec(r))
                    except Exception as e:       # refused by the library: report, go on
                        res = results[r.idx]
                        res.status, res.message, res.done = "error", str(e), now()
                        finished += 1
                        continue
                    resident[d][job] = _Resident(r, cells, now())
                    results[r.idx].admitted = resident[d][job].admitted
                    used[d][0] += r.n
                    used[d][1] += cells
                    st.max_particles[d] = max(st.max_particles[d], used[d][0])
            st.max_resident = max(st.max_resident, sum(len(x) for x in resident.values()))
            if not resident[2] and not resident[3]:
                if nxt < len(reqs):
                    self.sleep(max(0.0, reqs[nxt].arrival - now()))
                continue
            # one chunk on every busy batch (each on its own stream), then poll
            for d in (2, 3):
                if resident[d]:
                    self.batches[d].step(self.chunk)
                    st.chunks += 1
            for d in (2, 3):
                if not resident[d]:
                    continue
                b = self.batches[d]
                live, conv, steps = b.status()
                st.polls += 1
                for job in [j for j in resident[d] if conv[j] or steps[j] >= self.max_job_steps]:
                    rj = resident[d].pop(job)
                    res = results[rj.req.idx]
                    try:
                        if not conv[job]:
                            raise RuntimeError(f"not converged after {int(steps[job])} steps")
                        x = b.positions(job)
                        err = b.error(job)
                        cnt = b.counters(job)
                        res.done = now()
                        res.steps, res.e_sys = int(err["step"]), float(err["e_sys"])
                        res.interactions = int(cnt["interactions"])
                        if self.keep_positions:
                            res.positions = x
                    except Exception as e:
                        res.status, res.message, res.done = "error", str(e), now()
                    b.remove(job)
                    used[d][0] -= rj.req.n
                    used[d][1] -= rj.cells
                    finished += 1
                    if progress:
                        progress(res)
        return [results[r.idx] for r in sorted(reqs, key=lambda r: r.idx)]


def summarize(results, stats=None):
    """p50 / p99 latency, makespan and throughput of a finished run."""
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(0)
    t_first = min((r.arrival for r in results), default=0.0)
    t_last = max((r.done for r in ok), default=0.0)
    span = max(t_last - t_first, 1e-12)
    out = dict(jobs=len(results), completed=len(ok),
               rejected=sum(r.status == "rejected" for r in results),
               errors=sum(r.status == "error" for r in results),
               latency_p50_s=float(np.percentile(lat, 50)) if lat.size else None,
               latency_p99_s=float(np.percentile(lat, 99)) if lat.size else None,
               latency_max_s=float(lat.max()) if lat.size else None,
               makespan_s=span, jobs_per_s=len(ok) / span,
               interactions_per_s=sum(r.interactions for r in ok) / span,
               particle_steps_per_s=sum(r.n * r.steps for r in ok) / span)
    if stats is not None:
        out.update(blocked_slots=stats.blocked_slots, blocked_memory=stats.blocked_memory,
                   polls=stats.polls, max_resident=stats.max_resident)
    return out
