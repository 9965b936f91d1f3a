"""The C-ABI library loads on the CPU and exports every entry point that
include/discomatch.h declares (no compute calls here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "discomatch.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dm_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_declared_symbols():
    so = os.path.join(ROOT, "paper_2310_08230_amd", "libdiscomatch.so")
    assert os.path.exists(so), "build the library first (paper_2310_08230_amd/build.py)"
    lib = ctypes.CDLL(so)
    names = _declared()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    lib.dm_version.restype = ctypes.c_char_p
    assert lib.dm_version().startswith(b"discomatch")


def test_binding_exposes_abi_names():
    import paper_2310_08230_amd as m
    for n in ("build_product_space", "build_costs", "dual_solve", "round_primal", "lower_bound",
              "SmoothedBound", "Context"):
        assert hasattr(m, n)


def test_binding_sets_argtypes_for_every_entry_point():
    """Every declared entry point has its argument types set, so ctypes
    converts the Python integers and pointers exactly as the header says."""
    import paper_2310_08230_amd as m
    L = m.lib()
    missing = [n for n in _declared() if getattr(L, n).argtypes is None]
    assert not missing, missing
