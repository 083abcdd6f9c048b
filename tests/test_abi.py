"""Host-side checks of the C ABI: the library loads and exports every symbol
that include/dda.h declares (no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_0908_0863_amd", "libdda.so")


def _declared():
    src = open(os.path.join(ROOT, "include", "dda.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?(dda_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["dda_open", "dda_target_create", "dda_set_occupancy", "dda_set_permittivity",
              "dda_build_spectrum", "dda_matvec", "dda_solve", "dda_cross_sections", "dda_grad_cabs_eps"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdda.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_lists_every_declared_symbol():
    import importlib.util
    spec = importlib.util.spec_from_file_location("dda_binding_src", os.path.join(ROOT, "paper_0908_0863_amd", "dda.py"))
    src = open(spec.origin).read()
    for n in _declared():
        assert f'"{n}"' in src, n
