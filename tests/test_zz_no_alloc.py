"""The entry point that allocates nothing (sph_mesh_control_replay_noalloc)
against the allocating one it mirrors (sph_mesh_control_replay), through the
C ABI, on two calls in a row, the second with a shorter series: identical
phases, resets and E_sys.  Its scratch is a fixed device array shared by the
calls, so the second call also shows that each call starts from a fresh
control state."""
import numpy as np
import pytest
import torch

from paper_2003_01061_amd import binding
from paper_2003_01061_amd import workload as wk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu(gpu):
    return gpu


def _series(n, seed):
    rng = np.random.default_rng(seed)
    vbar = 1.0 + 1e-7 * rng.standard_normal(n)
    vbar[: n // 3] += np.linspace(1e-3, 0.0, n // 3)         # settles after a third
    dt = rng.uniform(1e-3, 1e-2, n)
    dt[n // 5] = 1e-5                                         # a time-step drop
    return vbar, dt


def _noalloc(params, vbar, dt):
    dev = torch.device("cuda", 0)
    n = vbar.size
    v = torch.tensor(vbar, dtype=torch.float64, device=dev)
    d = torch.tensor(dt, dtype=torch.float64, device=dev)
    ph = torch.full((n,), -1, dtype=torch.int32, device=dev)
    rs = torch.full((n,), -1, dtype=torch.int32, device=dev)
    es = torch.full((n,), -1.0, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    binding.control_replay_noalloc(params, n, v.data_ptr(), d.data_ptr(), ph.data_ptr(),
                                   rs.data_ptr(), es.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    return ph.cpu().numpy(), rs.cpu().numpy(), es.cpu().numpy()


def test_noalloc_replay_equals_the_allocating_entry_point():
    torch.cuda.set_device(0)
    p = wk.default_params(max_phase1_steps=900, ramp_steps=60, ramp_halving=10, phase2_steps=100)
    for n, seed in ((3000, 1), (1100, 2)):        # the second call is shorter
        vbar, dt = _series(n, seed)
        want = binding.control_replay(p, vbar, dt)
        got = _noalloc(p, vbar, dt)
        for w, g in zip(want, got):
            assert np.array_equal(w, g)
        phases = set(want[0].tolist())
        assert {1, 2, 3} <= phases, phases


def test_noalloc_replay_rejects_a_series_over_the_maximum():
    p = wk.default_params()
    with pytest.raises(binding.SphError) as e:
        binding.control_replay_noalloc(p, 1000001, 0, 0, 0, 0, 0, None)
    assert e.value.status == 1 and "maximum" in str(e.value)
