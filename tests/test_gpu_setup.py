"""sph_mesh_create from the problem statement (the library places the
particles: sec. 3.2 split, sec. 3.6 sampling) and device memory from the
caller's allocator, through the C ABI on the GPU."""
import copy

import numpy as np
import pytest

import oracle
from paper_2003_01061_amd import binding
from paper_2003_01061_amd import workload as wk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(gpu):
    return gpu


def _unscaled(wl):
    sz = dict(wl.sizing)
    sz["h0"] = sz["h0"] / wl.scale
    if sz["kind"] in (wk.H_LINEAR_FROM_POINT, wk.H_SHELL):
        sz["grad"] = sz["grad"] / wl.scale
    return sz


@pytest.mark.parametrize("make,res", [(lambda: wk.square_hole(n_total=20000, res=256), 256),
                                      (lambda: wk.cube_ball(n_total=30011, res=48), 48),
                                      (lambda: wk.paper_sphere01(res=48), 48)])
def test_create_from_the_problem_statement(make, res):
    """The job holds exactly the host set-up's particles (the generator's
    split), and its steps follow the oracle fed those particles."""
    wl = make()
    p = dict(wl.params, n_particles=wl.n, seed=5, mass_res=res)
    g = binding.SphMesh.from_problem(wl.dim, wl.lo, wl.hi, wl.holes, _unscaled(wl), p,
                                     domain=wl.domain)
    info = g.setup_info()
    assert info["counts"] == [int(np.sum(wl.feature == f)) for f in range(len(wl.ftype))]
    assert abs(info["h_scale"] - wl.scale) <= 1e-9 * wl.scale
    host = binding.job_setup(wl.dim, wl.lo, wl.hi, wl.holes, _unscaled(wl), p, domain=wl.domain)
    x0, f0 = g.positions(with_feature=True)
    assert np.array_equal(x0, host["xyz"]) and np.array_equal(f0, host["feature"])
    ref_wl = copy.copy(wl)
    ref_wl.xyz, ref_wl.feature = host["xyz"], host["feature"]
    ref_wl.sizing = dict(_unscaled(wl), h0=host["h0"], grad=host["grad"])
    ref = oracle.RefJob(ref_wl)
    K = 20 if wl.dim == 2 else 6
    ref.step(K)
    g.step(K)
    ext = float(np.max(wl.hi[:wl.dim] - wl.lo[:wl.dim]))
    assert np.abs(g.positions() - ref.state()[0]).max() <= 1e-12 * ext
    assert g.counters()["interactions"] == ref.counters()["interactions"]


def test_device_memory_from_the_callers_allocator():
    """A job whose device memory comes from PyTorch's caching allocator runs
    bit-identically to one on hipMalloc, holds that memory while it lives,
    and gives it back when destroyed."""
    import torch
    torch.cuda.set_device(0)
    wl = wk.scaled_hole_2d(20011, seed=21, res=512)
    plain = binding.SphMesh(wl, use_graph=1)
    plain.step(15)
    before = torch.cuda.memory_allocated()
    alloc = binding.torch_allocator()
    g = binding.SphMesh(wl, use_graph=1, allocator=alloc)
    held = torch.cuda.memory_allocated() - before
    assert held >= g.device_bytes() > 0
    g.step(15)
    assert np.array_equal(g.positions(), plain.positions())
    g.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    # a batch with the allocator too
    spec = binding.JobSpec(wl)
    b = binding.SphBatch(2, max_particles=wl.n, max_cells=spec.cells(), max_jobs=1, allocator=alloc)
    j = b.add(spec)
    b.step(15)
    assert np.array_equal(b.positions(j), plain.positions())
    b.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
