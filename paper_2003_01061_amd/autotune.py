"""Autotuner of the batched relaxation step.

The knobs are the ones that change speed but not the method:

* ``cell_factor`` -- cell side 2 h_min * cell_factor (per job).  Smaller cells
  follow the support disc (sphere) more tightly, so fewer candidates fail the
  predicate, but every particle visits more cell rows.  Changing it changes
  the canonical (cell, caller id) order of a neighbour list, hence the
  rounding of the force sums, never the list itself.
* ``scan_tile`` -- candidate records the neighbour scan loads and tests per
  pass (2, 4 or 8; per batch).  Results are bit-identical for every value.
* ``verlet_skin`` -- reach of the Verlet candidate lists beyond the cut-off
  radius, in units of h (0: a cell scan and a sort every step).  A wider skin
  means fewer rebuilds but more candidates to filter every step.  The lists
  are the cut-off lists whatever the skin; only the summation order changes.

The workgroup size is fixed at 256 (the kernels' occupancy is bounded by
their registers, and the per-wave accumulator stripes assume it) and the
list format is ELL, so neither is searched.

``tune`` times every (cell_factor, scan_tile) configuration of the grid on a
trial batch holding the given jobs (the graph-replayed step, after warm-up
steps), then every (skin, scan_tile) pair at the fastest cell factor, and
returns the fastest; ties keep the earlier (default-first) entry, and a
configuration replaces the default (or, at a skin, the best pair's tile) only
when it is faster by more than a noise margin.  The timing sources are injectable so
that the selection logic is testable without a GPU.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

DEFAULT = {"cell_factor": 1.0, "scan_tile": 4, "verlet_skin": 0.0}
CELL_FACTORS = (1.0, 0.75, 1.25)
SCAN_TILES = (4, 2, 8)
SKINS = (0.3, 0.5, 0.8)


@dataclass
class TuneResult:
    dim: int
    precision: int
    n_particles: int
    best: dict
    table: list = field(default_factory=list)   # one entry per configuration

    def speedup_over_default(self):
        base = next(r["ms_per_step"] for r in self.table
                    if r["cell_factor"] == DEFAULT["cell_factor"]
                    and r["scan_tile"] == DEFAULT["scan_tile"]
                    and r["verlet_skin"] == DEFAULT["verlet_skin"])
        return base / min(r["ms_per_step"] for r in self.table)


def with_cell_factor(spec, cf):
    """A copy of a binding.JobSpec whose parameters use cell side factor cf
    (the particle arrays are shared)."""
    from . import binding
    out = binding.JobSpec.__new__(binding.JobSpec)
    out.__dict__.update(spec.__dict__)
    out.params = binding.Params.from_buffer_copy(spec.params)
    out.params.cell_factor = float(cf)
    return out


def _time_config(specs, dim, precision, cf, tile, steps, warmup, max_neighbors, skin=0.0):
    from . import binding
    sp = [with_cell_factor(s, cf) for s in specs]
    b = binding.SphBatch(dim, precision, max_particles=sum(s.n for s in sp),
                         max_cells=sum(s.cells() for s in sp), max_jobs=len(sp),
                         max_neighbors=max_neighbors, use_graph=1, scan_tile=tile,
                         verlet_skin=skin)
    try:
        for s in sp:
            b.add(s)
        b.step(warmup)
        b.sync()
        t0 = time.perf_counter()
        b.step(steps)
        b.sync()
        return (time.perf_counter() - t0) / steps * 1e3
    finally:
        b.close()


def tune(specs: Sequence, dim: int, precision: int, cell_factors=CELL_FACTORS,
         scan_tiles=SCAN_TILES, steps=20, warmup=4, max_neighbors=0,
         measure: Optional[Callable] = None, min_gain=0.02, skins=SKINS,
         measure_skin: Optional[Callable] = None) -> TuneResult:
    """Time every (cell_factor, scan_tile) pair on a batch of ``specs``, then
    every (skin, scan_tile) pair at the fastest cell factor, and return the
    fastest; the default stays
    unless another configuration is faster by more than ``min_gain`` (timing
    noise must not flip the choice), and so does no skin.  ``measure(cf, tile)
    -> ms per step`` and ``measure_skin(cf, tile, skin)`` replace the GPU
    timing when given (an injected ``measure`` alone skips the skins)."""
    if not specs:
        raise ValueError("tune needs at least one job")
    if measure is None:
        def measure(cf, tile):
            return _time_config(specs, dim, precision, cf, tile, steps, warmup, max_neighbors)
        if measure_skin is None:
            def measure_skin(cf, tile, skin):
                return _time_config(specs, dim, precision, cf, tile, steps, warmup,
                                    max_neighbors, skin)
    grid = [(cf, t) for cf in cell_factors for t in scan_tiles]
    if (DEFAULT["cell_factor"], DEFAULT["scan_tile"]) not in grid:
        grid.insert(0, (DEFAULT["cell_factor"], DEFAULT["scan_tile"]))
    table = []
    for cf, t in grid:
        table.append({"cell_factor": cf, "scan_tile": t, "verlet_skin": 0.0,
                      "ms_per_step": float(measure(cf, t))})
    best = min(table, key=lambda r: r["ms_per_step"])   # first minimum wins ties
    default = table[grid.index((DEFAULT["cell_factor"], DEFAULT["scan_tile"]))]
    if best["ms_per_step"] * (1.0 + min_gain) > default["ms_per_step"]:
        best = default
    if measure_skin is not None:
        # the filter's batches differ from the scan's, so the tile is searched again
        for sk in skins:
            for t in scan_tiles:
                r = {"cell_factor": best["cell_factor"], "scan_tile": t, "verlet_skin": float(sk),
                     "ms_per_step": float(measure_skin(best["cell_factor"], t, sk))}
                table.append(r)
        # per skin, the tile of the best pair unless another tile beats it by
        # more than min_gain (so timing noise between near-equal tiles does
        # not decide); then the fastest skin
        per_skin = []
        for sk in skins:
            rows = [r for r in table[len(grid):] if r["verlet_skin"] == float(sk)]
            ref = next((r for r in rows if r["scan_tile"] == best["scan_tile"]), rows[0])
            fast = min(rows, key=lambda r: r["ms_per_step"])
            per_skin.append(fast if fast["ms_per_step"] * (1.0 + min_gain) <= ref["ms_per_step"] else ref)
        with_skin = min(per_skin, key=lambda r: r["ms_per_step"], default=None)
        if with_skin is not None and with_skin["ms_per_step"] * (1.0 + min_gain) <= best["ms_per_step"]:
            best = with_skin
    return TuneResult(dim, precision, int(sum(s.n for s in specs)),
                      {"cell_factor": best["cell_factor"], "scan_tile": best["scan_tile"],
                       "verlet_skin": best["verlet_skin"]},
                      table)
