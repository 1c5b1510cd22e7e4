"""Benchmark: particle-neighbour interactions/s of the feature-aware SPH
relaxation step on one MI355X.

Workload (default): the 2D unit square minus the disc r = 1/4, 250,000
particles, graded h = s h0 (1 + 4 d), h0 = 1/1024, seeded random init, 2,000
steps through both phases (Phase One capped at 1,200 steps), run once with
FP32 kernel sums + FP64 integration (the reported value) and once in plain
FP64.  A step is one pass of the whole hot path: hashing, sort, cell table,
neighbour list, both force sweeps, integration with projection and control.
The timed region starts with the particles resident in HBM and ends after
the last step; creation and the host copy of the result are outside it.

interactions = neighbour-list entries of every moving particle, once per step.

Prints one JSON line, with the roofline of the dominant kernel and the CPU
oracle baseline on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak in wave64 instructions/s: 256 CUs x 4 SIMDs, a wave64 VALU
# instruction occupies a 16-lane SIMD for 4 cycles, 2.4 GHz
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
# the same peak in lane operations (64 per wave64 instruction): 39.3e12/s
VALU_PEAK_LANE_OPS = VALU_PEAK_WAVE_INSTS * 64
COUNTERS_MD = os.path.join(ROOT, "profiles", "nbr_forces_square_hole_250k_counters.md")
COUNTERS_3D_MD = os.path.join(ROOT, "profiles", "cube_ball_2m_counters.md")
COUNTERS_ELL_MD = os.path.join(ROOT, "profiles", "ellipsoid_inclusions_20m_counters.md")
VERLET_SKIN_3D = 0.5   # the Verlet list skin the 3D leg also times (units of h)
KERNEL_SOURCES = ("paper_2003_01061_amd/csrc/sph_device.h", "paper_2003_01061_amd/csrc/sph_kernels.h")


def roofline(kernel, byts, avg_s, ctr, launches):
    """Roofline block of the dominant kernel.  Both fractions are computed:
    algorithmic HBM bytes per launch over the launch time against 8 TB/s, and
    (when counters of the current sources exist) VALU lane operations issued
    per launch over the launch time against the VALU issue peak.  The larger
    one names the bound."""
    hbm = byts / avg_s / 1e9
    blk = {"kernel": kernel, "avg_launch_us": avg_s * 1e6, "bytes_per_launch": byts,
           "launches": launches, "hbm_achieved_gbs": hbm, "hbm_frac": hbm / HBM_PEAK_GBS,
           "traffic": None, "traffic_frac": None, "valu_issue_frac": None}
    if ctr is not None:
        blk["traffic"] = ctr["traffic"]
        blk["traffic_frac"] = ctr["traffic"] / avg_s / 1e9 / HBM_PEAK_GBS
        blk["valu_issue_frac"] = ctr["valu"] / avg_s / VALU_PEAK_WAVE_INSTS
    if blk["valu_issue_frac"] is not None and blk["valu_issue_frac"] > blk["hbm_frac"]:
        ops = ctr["valu"] * 64 / avg_s / 1e12
        blk.update(bound="alu", achieved=ops, peak=VALU_PEAK_LANE_OPS / 1e12, unit="TOP/s",
                   frac=ops * 1e12 / VALU_PEAK_LANE_OPS)
    else:
        blk.update(bound="hbm", achieved=hbm, peak=HBM_PEAK_GBS, unit="GB/s",
                   frac=hbm / HBM_PEAK_GBS)
    return blk


def profiled_counters(cfg, path=COUNTERS_MD):
    """Counter figures of the dominant kernel from the committed rocprofv3
    summary, or None when the kernel sources changed since they were taken or
    the benchmark runs another configuration."""
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    want = "cell_factor={} scan_tile={}".format(float(cfg.get("cell_factor", 1.0)),
                                                int(cfg.get("scan_tile", 4)))
    if float(cfg.get("verlet_skin", 0.0)) > 0.0:   # the kernel that filters Verlet lists
        want += " verlet_skin={}".format(float(cfg["verlet_skin"]))
    # one fenced block of "key: value" lines per profiled configuration
    for block in re.findall(r"```\n(kernel: .*?)```", text, flags=re.S):
        kv = dict(re.findall(r"^(\w+): (.+)$", block, flags=re.M))
        if kv.get("kernel_source_sha256") == h.hexdigest() and kv.get("config") == want:
            return dict(traffic=float(kv["traffic_bytes_per_launch"]),
                        valu=float(kv["valu_insts_per_launch"]), waves=float(kv["waves_per_launch"]))
    return None


def kernel_bytes(name, wl, n_active, inter, real_bytes):
    """Algorithmic HBM bytes of one launch: every particle record or column
    read or written once, the neighbour list written or read once; gathers of
    neighbour records are cache traffic and not counted."""
    N = wl.n
    r4 = 4 * real_bytes                       # {ax, ay, az, 0} record
    if name == "nbr_forces":
        return N * 33 + n_active * (32 + 4 + r4) + inter * 4
    if name == "nbr_lists":
        return N * 33 + N * 4 + inter * 4
    if name == "sweep_b":
        return n_active * (32 + 32 + r4 + 1 + 4 + r4) + inter * 4
    if name == "integrate_hash":
        return N * (64 + 1 + 8) + n_active * (64 + r4)
    if name == "rank_gather":
        return N * 158
    if name == "scatter":
        return N * 24
    return None


def run_timed(wl, precision, steps, warmup, graph=True, cfg=None):
    from paper_2003_01061_amd import binding
    import torch
    cfg = cfg or {}
    torch.cuda.synchronize()
    tc = time.perf_counter()
    j = binding.SphMesh(wl, precision=precision, use_graph=int(graph), **cfg)
    j.sync()
    tw = time.perf_counter()
    # the warmup steps (untimed) also capture the step graphs
    j.step(warmup)
    j.sync()
    c0 = j.counters()["interactions"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    j.step(steps)
    j.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x = j.positions()
    t2 = time.perf_counter()
    c = j.counters()
    e = j.error()
    builds = j.list_builds()
    j.close()
    # seconds: the timed region (inputs resident in HBM); with_io adds the
    # creation (host -> device copy, initial hash) and the host copy of the result
    interactions = c["interactions"] - c0
    return dict(seconds=t1 - t0, seconds_with_io=(tw - tc) + (t2 - t0), interactions=interactions,
                escaped=c["escaped"], steps=c["steps"], e_sys=e["e_sys"], phase=e["phase"],
                converged=e["converged"], positions=x, builds=builds)


def phase_one_ends(j, wl, steps, seen):
    """Record, per moving feature, the step at which it left Phase One (read
    from its control state while it is in the transition or Phase Two)."""
    p = wl.params
    for f in range(len(wl.ftype)):
        if f in seen or wl.ftype[f] == 0 or not np.any(wl.feature == f):
            continue
        g = j.group_state(f)
        if g["phase"] == 2:
            seen[f] = steps - int(g["n_ph"])
        elif g["phase"] == 3:
            seen[f] = steps - p["ramp_steps"] - int(g["n_ph"])


def converge_run(wl, precision, cfg=None, max_steps=6000, chunk=100):
    """Run a job through both phases until every feature has converged (or
    max_steps): steps, wall time, and for every feature the step at which
    Phase One ended, and whether the error criterion (E_sys below the
    threshold) or the Phase One step cap ended it."""
    from paper_2003_01061_amd import binding
    import torch
    j = binding.SphMesh(wl, precision=precision, use_graph=1, **(cfg or {}))
    j.sync()
    # the first two steps capture the step graph (set-up, untimed)
    j.step(2)
    j.sync()
    torch.cuda.synchronize()
    c0 = j.counters()["interactions"]
    # the time of the steps alone: the control-state queries between chunks
    # (host round trips, one per feature) are left out
    sec, steps, ends = 0.0, 2, {}
    while steps < max_steps:
        t0 = time.perf_counter()
        j.step(chunk)
        j.sync()
        sec += time.perf_counter() - t0
        steps += chunk
        phase_one_ends(j, wl, steps, ends)
        if j.error()["converged"]:
            break
    c, e = j.counters(), j.error()
    x = j.positions()
    j.close()
    cap = wl.params["max_phase1_steps"]
    return dict(steps=int(c["steps"]), seconds=sec, converged=e["converged"], e_sys=e["e_sys"],
                escaped=c["escaped"], interactions_per_s=(c["interactions"] - c0) / sec,
                phase_one_end={str(f): {"step": s_, "by": "cap" if s_ >= cap else "criterion"}
                               for f, s_ in sorted(ends.items())},
                phase_one_cap=cap, positions=x)


def cube_ball_leg(args):
    """The 3D workload (unit cube minus a ball, 2,000,000 particles), FP32
    sums + FP64 integration: timed steps and the neighbour kernel's roofline.
    Its working set (~0.5 GB) is larger than the 256 MB Infinity Cache."""
    from paper_2003_01061_amd import binding
    from paper_2003_01061_amd import workload as wk
    wl = wk.cube_ball()
    prec = binding.SPH_FP32_MIXED
    r = run_timed(wl, prec, args.steps_3d, 3)
    others = {}
    for tag, p_ in (("fp64", binding.SPH_FP64), ("fp32_compensated", binding.SPH_FP32_COMPENSATED)):
        o = run_timed(wl, p_, args.steps_3d, 3)
        others[tag] = {"value": o["interactions"] / o["seconds"],
                       "ms_per_step": o["seconds"] / args.steps_3d * 1e3}
    stats, pc = profile_kernels(wl, prec, 5)
    per = {k: (ms / cnt if cnt else 0.0, cnt) for k, (ms, cnt) in stats.items()}
    n_active = int(np.sum(wl.ftype[wl.feature] != wk.SI))
    inter_step = pc["interactions"] / max(pc["steps"], 1)
    byts = kernel_bytes("nbr_forces", wl, n_active, inter_step, 4)
    ctr = profiled_counters({}, COUNTERS_3D_MD)
    # Verlet candidate lists (skin 0.5 h): the same steps, the particles
    # re-sorted and the lists rebuilt only when some particle has moved far
    # enough; the kernels' average over steps with and without a rebuild
    vcfg = {"verlet_skin": VERLET_SKIN_3D}
    rv = run_timed(wl, prec, args.steps_3d, 3, cfg=vcfg)
    vstats, vpc = profile_kernels(wl, prec, 10, vcfg)
    vper = {k: (ms / max(vpc["steps"], 1), cnt) for k, (ms, cnt) in vstats.items()}
    # the filter kernel's roofline: the same algorithmic bytes (its candidate
    # lists are extra traffic of the Verlet scheme, counted in "traffic")
    vms, vcnt = vstats["nbr_forces"]
    vinter = vpc["interactions"] / max(vpc["steps"], 1)
    verlet = {"verlet_skin": VERLET_SKIN_3D, "value": rv["interactions"] / rv["seconds"],
              "ms_per_step": rv["seconds"] / args.steps_3d * 1e3, "list_builds": rv["builds"],
              "kernel_us_per_step": {k: round(v[0] * 1e3, 2) for k, v in vper.items() if v[1]},
              "roofline": roofline("nbr_forces", kernel_bytes("nbr_forces", wl, n_active, vinter, 4),
                                   vms / max(vcnt, 1) * 1e-3, profiled_counters(vcfg, COUNTERS_3D_MD),
                                   vcnt)}
    return {"workload": "cube_ball_3d", "n_particles": wl.n, "steps": args.steps_3d,
            "value": r["interactions"] / r["seconds"], "unit": "interactions/s",
            "ms_per_step": r["seconds"] / args.steps_3d * 1e3,
            "interactions_per_step": r["interactions"] / args.steps_3d,
            "kernel_support": wl.params["kernel_support"],
            "boundary_scale": wl.params["boundary_scale"],
            "other_precisions": others,
            "verlet": verlet,
            "roofline": roofline("nbr_forces", byts, per["nbr_forces"][0] * 1e-3, ctr,
                                 per["nbr_forces"][1]),
            "kernel_avg_us": {k: round(v[0] * 1e3, 2) for k, v in per.items()}}


def profile_kernels(wl, precision, steps, cfg=None):
    """Per-kernel durations from HIP events recorded on the library's stream."""
    from paper_2003_01061_amd import binding
    j = binding.SphMesh(wl, precision=precision, use_graph=0, **(cfg or {}))
    j.profile(True)
    j.step(steps)
    stats = j.kernel_stats()
    c = j.counters()
    j.close()
    return stats, c


def quality(wl, x):
    """Converged mesh quality: the Delaunay mesh of the final positions with
    the paper's triangle measures, and nearest-neighbour distance / h_t."""
    from scipy.spatial import cKDTree
    from paper_2003_01061_amd import quality as mq
    from paper_2003_01061_amd.workload import _h_field
    pts = x[:, :wl.dim]
    d, _ = cKDTree(pts).query(pts, k=2)
    h = _h_field(x, wl.dim, wl.sizing, wl.holes)
    r = d[:, 1] / h
    return dict(mesh=mq.mesh_quality(x, wl.dim, wl.lo, wl.hi, wl.holes, domain=wl.domain, level=wl.level),
                nn_over_h_mean=float(r.mean()), nn_over_h_p1=float(np.percentile(r, 1)),
                nn_over_h_min=float(r.min()))


def _oracle_leg(wl, budget_s, openmp):
    import oracle
    j = oracle.RefJob(wl, openmp=openmp)
    t0 = time.perf_counter()
    steps = 0
    while True:
        j.step(1)
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    t = time.perf_counter() - t0
    return j.counters()["interactions"] / t, steps, t


def square_4352_leg():
    """The 4,352-particle unit square (h = 1/64, cut-off 2h) in plain FP64 for
    200 steps: a launch-bound job, timed like the headline."""
    from paper_2003_01061_amd import binding
    from paper_2003_01061_amd import workload as wk
    wl = wk.square_lattice()
    r = run_timed(wl, binding.SPH_FP64, 200, 5)
    return {"workload": "square_lattice_4352", "n_particles": wl.n, "precision": "fp64",
            "kernel_support": wl.params["kernel_support"], "steps": 200,
            "value": r["interactions"] / r["seconds"], "unit": "interactions/s",
            "ms_per_step": r["seconds"] / 200 * 1e3}


def cpu_baseline_square(threads):
    """The oracle on the whole 200-step run of the 4,352-particle square (the
    plain build, one thread)."""
    import oracle
    from paper_2003_01061_amd import workload as wk
    wl = wk.square_lattice()
    j = oracle.RefJob(wl)
    t0 = time.perf_counter()
    j.step(200)
    t = time.perf_counter() - t0
    return {"value": j.counters()["interactions"] / t, "unit": "interactions/s", "cores": 1,
            "kind": "oracle", "sample": f"all 200 steps of the 4,352-particle square, FP64 oracle, "
                                        f"single-threaded, {t:.1f} s"}


def cpu_baseline_3d(threads):
    """The OpenMP oracle on the first step of the 2M-particle cube minus a ball
    (its neighbour search from scratch included), one step being the bounded
    sample (~20 s on 16 threads)."""
    import oracle
    from paper_2003_01061_amd import workload as wk
    wl = wk.cube_ball()
    j = oracle.RefJob(wl, openmp=True)
    t0 = time.perf_counter()
    j.step(1)
    t = time.perf_counter() - t0
    return {"value": j.counters()["interactions"] / t, "unit": "interactions/s", "cores": threads,
            "kind": "oracle", "sample": f"first step of the 2M-particle 3D job, FP64 oracle, "
                                        f"OpenMP over particles on {threads} threads, {t:.1f} s"}


def cpu_baseline(wl, budget_s):
    """The FP64 oracle on this host: the plain single-threaded build and the
    OpenMP build (the same arithmetic, per-particle loops on every core the
    process may use), each on the first steps of the same workload."""
    nproc = os.cpu_count()
    avail = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS") or avail)
    v1, s1, t1 = _oracle_leg(wl, budget_s, False)
    vn, sn, tn = _oracle_leg(wl, budget_s, True)
    return dict(value=vn, unit="interactions/s", cores=threads, kind="oracle",
                sample=f"first {sn} steps of the same workload, FP64 oracle, OpenMP over "
                       f"particles on {threads} threads, {tn:.1f} s",
                nproc=nproc, cpus_available=avail,
                single_thread={"value": v1, "cores": 1,
                               "sample": f"first {s1} steps, single-threaded, {t1:.1f} s"},
                cube_ball_3d=cpu_baseline_3d(threads),
                square_4352=cpu_baseline_square(threads))


def ellipsoid_run(args):
    """The 16-ellipsoid workload (20,000,000 particles, h ratio 1:20) in
    FP32-mixed: autotuned cell factor and scan tile, then the full two-phase
    schedule (Phase One capped at 1,200 steps) until every feature has
    converged.  One JSON line: interactions/s over the run, time to the
    converged mesh, per-kernel times and the neighbour kernel's roofline."""
    import torch
    from paper_2003_01061_amd import autotune, binding
    from paper_2003_01061_amd import workload as wk
    t = time.perf_counter()
    wl = wk.ellipsoid_inclusions(max_phase1_steps=1200)
    print(f"[bench] ellipsoids n={wl.n} generated in {time.perf_counter() - t:.1f}s",
          file=sys.stderr, flush=True)
    prec = binding.SPH_FP32_MIXED
    cfg, tuned = {}, None
    if args.config is not None:
        cfg = json.loads(args.config)
    elif not args.no_tune:
        tr = autotune.tune([binding.JobSpec(wl)], 3, prec, steps=10, warmup=2)
        cfg, tuned = tr.best, dict(best=tr.best, speedup_over_default=tr.speedup_over_default(),
                                   table=tr.table)
        print(f"[bench] tuned {json.dumps(cfg)}", file=sys.stderr, flush=True)
    j = binding.SphMesh(wl, precision=prec, use_graph=1, **cfg)
    j.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    while steps < args.max_steps:
        j.step(100)
        steps += 100
        e = j.error()
        print(f"[bench] step {steps} e_sys {e['e_sys']:.3g} phase {e['phase']} "
              f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
        if e["converged"]:
            break
    j.sync()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    c, e = j.counters(), j.error()
    x = j.positions()
    j.close()
    stats, pc = profile_kernels(wl, prec, 5, cfg)
    per = {k: (ms / cnt if cnt else 0.0, cnt) for k, (ms, cnt) in stats.items()}
    n_active = int(np.sum(wl.ftype[wl.feature] != wk.SI))
    inter_step = pc["interactions"] / max(pc["steps"], 1)
    byts = kernel_bytes("nbr_forces", wl, n_active, inter_step, 4)
    avg_s = per["nbr_forces"][0] * 1e-3
    from scipy.spatial import cKDTree
    from paper_2003_01061_amd import quality as mq
    from paper_2003_01061_amd.workload import _h_field
    rng = np.random.default_rng(0)
    q = rng.choice(wl.n, 200_000, replace=False)
    d, _ = cKDTree(x).query(x[q], k=2)
    r = d[:, 1] / _h_field(x[q], 3, wl.sizing, wl.holes)
    region = ([0.45, 0.45, 0.45], [0.55, 0.55, 0.55])
    mesh = mq.mesh_quality(x, 3, wl.lo, wl.hi, wl.holes, region=region)
    out = {
        "metric": "particle-neighbour interactions/s per step, run to the converged mesh",
        "value": c["interactions"] / sec, "unit": "interactions/s", "n_gpus": 1,
        "steps": int(c["steps"]), "ms_per_step": sec / max(c["steps"], 1) * 1e3,
        "seconds_to_converged_mesh": sec, "converged": e["converged"],
        "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "ellipsoid_inclusions_3d", "n_particles": wl.n, "inclusions": 16,
                   "h_min": wl.sizing["h0"], "h_ratio": 20, "precision": "fp32 sums + fp64 integration",
                   "tuned": cfg},
        "autotune": tuned,
        "escaped": c["escaped"],
        "quality_sample": {"particles": int(len(q)), "nn_over_h_mean": float(r.mean()),
                           "nn_over_h_p1": float(np.percentile(r, 1)),
                           "mesh_region": region, "mesh": mesh},
        "roofline": roofline("nbr_forces", byts, avg_s, profiled_counters(cfg, COUNTERS_ELL_MD),
                             per["nbr_forces"][1]),
        "kernel_avg_us": {k: round(v[0] * 1e3, 2) for k, v in per.items()},
    }
    print(json.dumps(out))


# the paper's tables for its square and cube (sec. 4.1 Table "Square", sec. 4.5
# Table "Cube", rows of the proposed method; its own hardware and meshing)
PAPER_VALIDATION = {
    "paper_square": dict(G_avg=0.95, G_min=0.67, theta_max=94.85, theta_min=40.11,
                         theta_min_avg=56.23, n_theta_below_30=0, n_elements=4828,
                         runtime_s=5.07, n_iter=1600),
    "paper_cube": dict(theta_min=23.07, theta_max=146.74, gamma_min=0.27, gamma_avg=0.92,
                       theta_min_avg=56.88, slivers={"10": 0, "20": 0, "30": 28, "40": 1913},
                       n_elements=367839, runtime_s=1437.3, n_iter=7000),
    "paper_sphere01": dict(theta_min=22.33, theta_max=150.78, gamma_min=0.32, gamma_avg=0.91,
                           theta_min_avg=56.24, slivers={"10": 0, "20": 0, "30": 12, "40": 478},
                           n_elements=68757, runtime_s=448.35, n_iter=4600),
    "zalesak_disc": dict(G_avg=0.92, G_min=0.65, theta_max=97.73, theta_min=37.23,
                         theta_min_avg=53.50, n_theta_below_30=0, n_elements=4551,
                         runtime_s=15.00, n_iter=4200),
    "paper_sphere02": dict(theta_min=26.25, theta_max=143.78, gamma_min=0.32, gamma_avg=0.91,
                           slivers={"10": 0, "20": 0, "30": 18, "40": 1873},
                           n_elements=110706, runtime_s=236.42, n_iter=3800),
}


VALIDATION_PRESETS = {
    # the readings as printed: reach 2h, boundary term factor 1, no damping
    "printed": {},
    # the same with Phase One damping at the top of sec. 3.4.3's range
    # (eps = 0.2: every feature of the square leaves Phase One by the error
    # criterion on the oracle)
    "printed_damped": {"eps_damp": 0.2},
    # the mesh-quality calibration (reach 2.5h, boundary factor 2)
    "calibrated": {"kernel_support": 2.5, "boundary_scale": 2.0},
    # the same with Phase One damping (eps = 0.1, sec. 3.4.3's range) and a
    # time-step cap of 0.3 (the setting under which every feature of the
    # square leaves Phase One by the error criterion on the oracle)
    "calibrated_damped": {"kernel_support": 2.5, "boundary_scale": 2.0, "eps_damp": 0.1,
                          "dt_max": 0.3},
}


def validation_run(args):
    """The paper's square, cube, spheres and slotted disc run through both
    phases to convergence in FP32-mixed, under the printed readings and the
    calibrated presets: for every feature the step at which Phase One ended
    and whether the error criterion or the step cap ended it, the converged
    step, the wall time and the mesh quality, beside the paper's table values
    (context: other hardware, other meshing)."""
    from paper_2003_01061_amd import binding
    from paper_2003_01061_amd import quality as mq
    from paper_2003_01061_amd import workload as wk
    out = {}
    cap = args.validation_cap
    for name, make in (("paper_square", wk.paper_square), ("paper_cube", wk.paper_cube),
                       ("paper_sphere01", wk.paper_sphere01),
                       ("paper_sphere02", wk.paper_sphere02), ("zalesak_disc", wk.zalesak_disc)):
        out[name] = {"paper": PAPER_VALIDATION[name]}
        for preset, over in VALIDATION_PRESETS.items():
            wl = make(max_phase1_steps=cap, **over)
            # Sphere02's sizing changes h by half per support radius: its lists
            # reach ~330 entries during the relaxation, above the 3D default
            cfg = {"max_neighbors": 512} if wl.dim == 3 else {}
            r = converge_run(wl, binding.SPH_FP32_MIXED, cfg, max_steps=cap + 1000)
            x = r.pop("positions")
            r.update(particles=wl.n, h_scale=wl.scale, params=over,
                     mesh=mq.mesh_quality(x, wl.dim, wl.lo, wl.hi, wl.holes, domain=wl.domain,
                                          level=wl.level))
            out[name][preset] = r
            print(f"[bench] {name} {preset}: {json.dumps(r)}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "steps and time to the converged mesh, mesh quality",
                      "data": "synthetic", "precision": "fp32 sums + fp64 integration",
                      "phase_one_cap": cap, "cases": out}))


def _build_job(desc):
    from paper_2003_01061_amd import workload as wk
    return wk.build_job(desc)


def serving(args):
    """The serving stream: n_jobs requests of both dimensions, N log-uniform in
    [1e3, 5e5], FP32 sums + FP64 integration, full two-phase schedule.  First
    all requests at t = 0 (closed loop): its completion rate is the saturation
    rate.  Then Poisson arrivals at the given fractions of that rate."""
    import multiprocessing as mp
    from paper_2003_01061_amd import binding, serve
    from paper_2003_01061_amd import workload as wk
    descs = wk.serving_stream(args.serve_jobs, seed=4)
    t0 = time.perf_counter()
    order = sorted(descs, key=lambda d: -d.n)
    with mp.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        built = pool.map(_build_job, order, chunksize=1)
    wl_of = {d.idx: w for d, w in zip(order, built)}
    specs = {d.idx: binding.JobSpec(wl_of[d.idx]) for d in descs}
    print(f"[bench] serving stream: {len(descs)} jobs, "
          f"{sum(d.n for d in descs)} particles, built in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    # autotune per dimension on the median-size request of that dimension
    from paper_2003_01061_amd import autotune
    tuned, tuning = {}, {}
    if not args.no_tune:
        for d in (2, 3):
            ds = sorted((x for x in descs if x.dim == d), key=lambda x: x.n)
            if not ds:
                continue
            med = ds[len(ds) // 2]
            # serving batches keep the cell scan (no Verlet lists): no skins
            r = autotune.tune([specs[med.idx]], d, binding.SPH_FP32_MIXED, steps=10, warmup=2,
                              max_neighbors=320 if d == 3 else 104, skins=())
            tuned[d] = r.best
            tuning[str(d)] = dict(job_particles=med.n, best=r.best,
                                  speedup_over_default=r.speedup_over_default())
        print(f"[bench] serving tuned: {json.dumps(tuning)}", file=sys.stderr, flush=True)
    srv = serve.Server(pool_bytes=int(args.serve_pool_gib * (1 << 30)), slots=args.serve_slots,
                       precision=binding.SPH_FP32_MIXED, chunk=args.serve_chunk, tuned=tuned)

    def one(rate):
        t = wk.poisson_arrivals(len(descs), rate, seed=4)
        reqs = [serve.Request(d.idx, d.dim, d.n, float(t[q]), specs[d.idx])
                for q, d in enumerate(descs)]
        srv.stats = serve.ServeStats()
        done = [0]

        def progress(r):
            done[0] += 1
            if done[0] % 32 == 0:
                print(f"[bench] serving: {done[0]} jobs done", file=sys.stderr, flush=True)

        res = srv.run(reqs, progress=progress)
        out = serve.summarize(res, srv.stats)
        out["arrival_rate_per_s"] = None if not np.isfinite(rate) else rate
        print(f"[bench] serving rate={rate:.3g}/s: " + json.dumps(out), file=sys.stderr, flush=True)
        return out

    closed = one(float("inf"))
    sat = closed["jobs_per_s"]
    runs = {"closed_loop": closed}
    for f in args.serve_rates:
        runs[f"poisson_{f:g}x"] = one(f * sat)
    return dict(jobs=len(descs), particles=int(sum(d.n for d in descs)),
                jobs_2d=sum(d.dim == 2 for d in descs), pool_bytes=srv.footprint_bytes(),
                slots=args.serve_slots, chunk_steps=args.serve_chunk,
                capacity_particles={str(k): v for k, v in srv.cap_particles.items()},
                saturation_jobs_per_s=sat, autotune=tuning, runs=runs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--n", type=int, default=250_000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--config", type=str, default=None,
                    help="JSON tuning of the headline job (cell_factor, scan_tile, verlet_skin) "
                         "used instead of the autotuner's choice, e.g. for profiling runs")
    ap.add_argument("--pmc-cell-factor", type=float, default=1.0,
                    help="cell factor of the 'step' counter pass")
    ap.add_argument("--pmc-scan-tile", type=int, default=4, choices=[2, 4, 8],
                    help="scan tile of the 'step' counter pass")
    ap.add_argument("--pmc-skin", type=float, default=0.0,
                    help="Verlet list skin of the counter passes (units of h; 0 = cell scan)")
    ap.add_argument("--pmc-precision", choices=["mixed", "compensated", "fp64"], default="mixed",
                    help="precision of the 'step' and 'step3d' counter passes")
    ap.add_argument("--no-converge", action="store_true",
                    help="skip the runs to the converged mesh (profiling runs)")
    ap.add_argument("--pmc-pass", choices=["step", "step3d", "stepell", "copy"], default=None,
                    help="counter-collection pass for rocprofv3 --pmc: 'step' runs --steps "
                         "eagerly launched FP32-mixed steps of the workload (default tuning), "
                         "'step3d' the same on the 2M-particle cube minus a ball, 'stepell' on "
                         "the 20M-particle ellipsoid job (tuning from --config), "
                         "'copy' one 256 MiB device copy (counter calibration); prints no JSON")
    ap.add_argument("--workload", choices=["square_hole", "ellipsoids", "validation"],
                    default="square_hole",
                    help="ellipsoids: the 20M-particle inclusion workload run to convergence; "
                         "validation: the paper's square and cube run to convergence "
                         "(each its own JSON line; not the headline)")
    ap.add_argument("--max-steps", type=int, default=6000,
                    help="step cap of the runs to the converged mesh")
    ap.add_argument("--steps-3d", type=int, default=40,
                    help="timed steps of the 2M-particle 3D leg")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--validation-cap", type=int, default=4000,
                    help="Phase One step cap of the validation runs")
    ap.add_argument("--serve-jobs", type=int, default=256)
    ap.add_argument("--serve-rates", type=float, nargs="*", default=[0.9])
    ap.add_argument("--serve-pool-gib", type=float, default=8.0)
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-chunk", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(a multi-GPU decomposition is designed but not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_2003_01061_amd import binding
    from paper_2003_01061_amd import workload as wk

    if args.pmc_pass == "copy":
        a = torch.ones(1 << 25, dtype=torch.float64, device="cuda")   # 256 MiB
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] copy pass: {a.numel() * 8} bytes read, {b.numel() * 8} written",
              file=sys.stderr, flush=True)
        return
    if args.workload == "ellipsoids":
        ellipsoid_run(args)
        return
    if args.workload == "validation":
        validation_run(args)
        return
    pmc_prec = {"mixed": binding.SPH_FP32_MIXED, "compensated": binding.SPH_FP32_COMPENSATED,
                "fp64": binding.SPH_FP64}[args.pmc_precision]
    if args.pmc_pass == "stepell":
        wle = wk.ellipsoid_inclusions(max_phase1_steps=1200)
        cfg = json.loads(args.config) if args.config else {}
        j = binding.SphMesh(wle, precision=pmc_prec, use_graph=0, **cfg)
        j.step(args.steps)
        j.sync()
        print(f"[bench] stepell pass: {args.steps} steps {json.dumps(cfg)}", file=sys.stderr, flush=True)
        return
    if args.pmc_pass == "step3d":
        wl3 = wk.cube_ball()
        j = binding.SphMesh(wl3, precision=pmc_prec, use_graph=0, verlet_skin=args.pmc_skin)
        j.step(args.steps)
        j.sync()
        print(f"[bench] step3d pass: {args.steps} steps", file=sys.stderr, flush=True)
        return
    wl = wk.square_hole(n_total=args.n)
    if args.pmc_pass == "step":
        j = binding.SphMesh(wl, precision=pmc_prec, use_graph=0,
                            cell_factor=args.pmc_cell_factor, scan_tile=args.pmc_scan_tile,
                            verlet_skin=args.pmc_skin)
        j.step(args.steps)
        j.sync()
        c = j.counters()
        print(f"[bench] step pass: {args.steps} steps, {c['interactions']} interactions",
              file=sys.stderr, flush=True)
        return
    print(f"[bench] workload square_hole n={wl.n} scale={wl.scale:.4f}", file=sys.stderr, flush=True)
    cfg, tuned = {}, None
    if args.config is not None:
        cfg = json.loads(args.config)
    elif not args.no_tune:
        from paper_2003_01061_amd import autotune
        t = autotune.tune([binding.JobSpec(wl)], 2, binding.SPH_FP32_MIXED, steps=20, warmup=4)
        cfg = t.best
        tuned = dict(best=t.best, speedup_over_default=t.speedup_over_default(), table=t.table)
        print(f"[bench] tuned {json.dumps(t.best)} ({t.speedup_over_default():.3f}x over default)",
              file=sys.stderr, flush=True)
    r32 = run_timed(wl, binding.SPH_FP32_MIXED, args.steps, args.warmup, cfg=cfg)
    print(f"[bench] fp32-mixed {r32['seconds']:.3f}s", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64 = run_timed(wl, binding.SPH_FP64, args.steps, args.warmup, cfg=cfg)
        print(f"[bench] fp64 {r64['seconds']:.3f}s", file=sys.stderr, flush=True)
    r32c = run_timed(wl, binding.SPH_FP32_COMPENSATED, args.steps, args.warmup, cfg=cfg)
    print(f"[bench] fp32-compensated {r32c['seconds']:.3f}s", file=sys.stderr, flush=True)
    value = r32["interactions"] / r32["seconds"]

    stats, pc = profile_kernels(wl, binding.SPH_FP32_MIXED, args.profile_steps, cfg)
    per = {k: (ms / cnt if cnt else 0.0, cnt) for k, (ms, cnt) in stats.items()}
    dom = max((k for k in stats if kernel_bytes(k, wl, 1, 1, 4) is not None),
              key=lambda k: stats[k][0])
    n_active = int(np.sum(wl.ftype[wl.feature] != wk.SI))
    inter_step = pc["interactions"] / max(pc["steps"], 1)
    byts = kernel_bytes(dom, wl, n_active, inter_step, 4)
    avg_s = per[dom][0] * 1e-3
    ctr = profiled_counters(cfg) if dom == "nbr_forces" else None
    print(f"[bench] profile: " + ", ".join(f"{k}={v[0]*1e3:.1f}us" for k, v in per.items()),
          file=sys.stderr, flush=True)

    # the same workload run to the converged mesh in both precisions, whatever
    # --steps is: FP32-mixed against FP64 at equal converged quality
    conv = {}
    for tag, prec in (("fp32", binding.SPH_FP32_MIXED), ("fp64", binding.SPH_FP64)):
        if (tag == "fp64" and args.no_fp64) or args.no_converge:
            continue
        c_ = converge_run(wl, prec, cfg, max_steps=args.max_steps)
        c_["quality"] = quality(wl, c_.pop("positions"))
        conv[tag] = c_
        print(f"[bench] converged {tag}: {c_['steps']} steps {c_['seconds']:.2f}s "
              f"{c_['interactions_per_s']:.3g}/s", file=sys.stderr, flush=True)

    leg3d = None if args.no_3d else cube_ball_leg(args)
    leg_c1 = square_4352_leg()
    print(f"[bench] square 4352 FP64: {leg_c1['value']:.3g}/s, {leg_c1['ms_per_step']:.4f} ms/step",
          file=sys.stderr, flush=True)
    if leg3d is not None:
        print(f"[bench] cube_ball 3D: {leg3d['value']:.3g}/s, nbr_forces "
              f"{leg3d['roofline']['avg_launch_us']:.0f}us", file=sys.stderr, flush=True)

    srv = None if args.no_serve else serving(args)
    lat = None
    if srv is not None:
        key = next((k for k in srv["runs"] if k.startswith("poisson")), "closed_loop")
        lat = [srv["runs"][key]["latency_p50_s"], srv["runs"][key]["latency_p99_s"]]

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args.cpu_seconds)

    out = {
        "metric": "particle-neighbour interactions/s per step (FP32 vs FP64) + p50/p99 job latency",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "square_hole_2d", "n_particles": wl.n, "h0": 1.0 / 1024,
                   "h_scale": round(wl.scale, 6), "grad": 4.0, "hole_radius": 0.25,
                   "kernel_support": wl.params["kernel_support"],
                   "boundary_scale": wl.params["boundary_scale"],
                   "max_phase1_steps": wl.params["max_phase1_steps"],
                   "steps": args.steps, "precision": "fp32 sums + fp64 integration",
                   "parallelism": "single GPU", "tuned": cfg},
        "autotune": tuned,
        "pcie_inclusive": {"value": r32["interactions"] / r32["seconds_with_io"],
                           "seconds": r32["seconds_with_io"],
                           "note": "create (host->device copy, first hash) + steps + positions "
                                   "(device->host); not the reported value"},
        "fp64": None if r64 is None else {
            "value": r64["interactions"] / r64["seconds"],
            "ms_per_step": r64["seconds"] / args.steps * 1e3,
            "e_sys": r64["e_sys"], "phase": r64["phase"],
            "max_abs_position_diff_vs_fp32": float(np.abs(r64["positions"] - r32["positions"]).max()),
        },
        "timed_region_state": {"e_sys": r32["e_sys"], "phase": r32["phase"],
                               "converged": r32["converged"], "escaped": r32["escaped"]},
        "fp32_compensated": {
            "value": r32c["interactions"] / r32c["seconds"],
            "ms_per_step": r32c["seconds"] / args.steps * 1e3,
            "note": "FP32 pair terms summed in FP32 with Neumaier compensation (the reported "
                    "value sums FP32 terms in FP64)",
            "max_abs_position_diff_vs_fp32": float(np.abs(r32c["positions"] - r32["positions"]).max()),
            "max_abs_position_diff_vs_fp64": None if r64 is None else
            float(np.abs(r32c["positions"] - r64["positions"]).max())},
        "converged": conv,
        "fp32_vs_fp64_at_convergence": None if "fp64" not in conv or "fp32" not in conv else {
            "interactions_per_s_ratio": conv["fp32"]["interactions_per_s"] / conv["fp64"]["interactions_per_s"],
            "G_avg": [conv["fp32"]["quality"]["mesh"].get("G_avg"), conv["fp64"]["quality"]["mesh"].get("G_avg")],
            "theta_min_avg": [conv["fp32"]["quality"]["mesh"].get("theta_min_avg"),
                              conv["fp64"]["quality"]["mesh"].get("theta_min_avg")]},
        "cube_ball_3d": leg3d,
        "square_4352_fp64": leg_c1,
        "latency_p50_p99_s": lat,
        "serving": srv,
        "roofline": roofline(dom, byts, avg_s, ctr, per[dom][1]),
        "kernel_avg_us": {k: round(v[0] * 1e3, 2) for k, v in per.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
