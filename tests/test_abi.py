"""CPU checks of the C ABI: the library builds, loads, and exports every
entry point that include/sph_mesh.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sph_mesh.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_mesh_\w+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for core in ("sph_mesh_create", "sph_mesh_step", "sph_mesh_positions", "sph_mesh_error"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2003_01061_amd import binding
    lib = binding.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(binding.exported_symbols()) == set(declared_functions())


def test_kernel_names_need_no_gpu():
    from paper_2003_01061_amd import binding
    L = binding.lib()
    names = [L.sph_mesh_kernel_name(k).decode() for k in range(L.sph_mesh_kernel_count())]
    assert "nbr_forces" in names and "sweep_b" in names


def test_invalid_arguments_fail_before_touching_the_gpu():
    from paper_2003_01061_amd import binding
    from paper_2003_01061_amd import workload as wk
    wl = wk.square_lattice(n_side=4)
    bad = dict(wl.params)
    bad["window_samples"] = 0
    with pytest.raises(binding.SphError) as e:
        binding.SphMesh(wl, params=bad)
    assert e.value.status == 1
    wl.feature = wl.feature.copy()
    wl.feature[0] = 99
    with pytest.raises(binding.SphError):
        binding.SphMesh(wl)


def test_struct_layout_matches_header():
    """ctypes mirrors of the header structs have the C sizes."""
    from paper_2003_01061_amd import binding
    assert ctypes.sizeof(binding.Geometry) == 4 + 4 + 48 + 8 + 8   # padded
    assert ctypes.sizeof(binding.Sizing) == 8 + 24 + 24
