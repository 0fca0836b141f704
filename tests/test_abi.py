"""CPU-side checks of the C-ABI library: it loads, and exports every function
the public header declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gsim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsim_[a-z_]+)\s*\(", src)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for need in ("gsim_mesh_upload", "gsim_particles_set", "gsim_geodesic_pairs", "gsim_compute_forces",
                 "gsim_displace_on_surface", "gsim_step"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2404_19751_amd import gsim
    if not os.path.exists(gsim.LIB_PATH):
        pytest.fail("HIP library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(gsim.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(gsim.EXPORTS) == declared_functions()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2404_19751_amd import gsim
    saved = gsim._lib
    gsim._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            gsim.load(str(tmp_path / "missing.so"))
    finally:
        gsim._lib = saved
