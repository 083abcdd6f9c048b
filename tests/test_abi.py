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


def _header():
    return open(os.path.join(ROOT, "include", "dda.h")).read()


def test_binding_constants_match_header():
    """Every DDA_* enumerator the binding defines has the header's value."""
    from paper_0908_0863_amd import dda
    vals = {k: int(v) for k, v in re.findall(r"\b(DDA_[A-Z0-9_]+)\s*=\s*(-?\d+)", _header())}
    seen = 0
    for k, v in vals.items():
        if hasattr(dda, k):
            assert getattr(dda, k) == v, k
            seen += 1
    assert seen >= 20
    # every solver value is reachable by name
    solvers = [v for k, v in vals.items() if k in ("DDA_BICGSTAB", "DDA_QMR_SYM", "DDA_BICG_SYM", "DDA_CGS",
                                                    "DDA_TFQMR", "DDA_BICG", "DDA_QMR", "DDA_RBICGSTAB",
                                                    "DDA_MLBICGSTAB")]
    assert sorted(set(dda._SOLVER.values())) == sorted(solvers)


@pytest.mark.parametrize("struct", ["dda_solve_opts", "dda_solve_info", "dda_batch_item"])
def test_binding_struct_fields_follow_header(struct):
    """The ctypes structures list the header's fields in the header's order."""
    from paper_0908_0863_amd import dda
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + struct + ";", _header()).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(\w+)\s*;", body)
    assert [f for f, _ in getattr(dda, struct)._fields_] == fields


def test_solve_options_marshalling():
    """Solver names of the paper's Table 3 map to the header's values and the
    options structure carries every field in order (no GPU needed)."""
    from paper_0908_0863_amd import dda
    o = dda.Target.make_opts(solver="rbicgstab", precision="mixed", tol=1e-7, inner_tol=2e-4, max_iter=50,
                             max_outer=3, jacobi=False, check_every=6, use_graph=True, solver_param=3)
    assert (o.solver, o.precision, o.max_iter, o.max_outer) == (dda.DDA_RBICGSTAB, dda.DDA_SOLVE_MIXED, 50, 3)
    assert (o.tol, o.inner_tol, o.jacobi, o.check_every, o.use_graph, o.solver_param) == (1e-7, 2e-4, 0, 6, 1, 3)
    names = {"bicg": dda.DDA_BICG, "bicg_sym": dda.DDA_BICG_SYM, "cocg": dda.DDA_BICG_SYM,
             "bicgstab": dda.DDA_BICGSTAB, "cgs": dda.DDA_CGS, "mlbicgstab": dda.DDA_MLBICGSTAB,
             "qmr": dda.DDA_QMR, "qmr_sym": dda.DDA_QMR_SYM, "rbicgstab": dda.DDA_RBICGSTAB, "tfqmr": dda.DDA_TFQMR}
    for n, v in names.items():
        assert dda.Target.make_opts(solver=n).solver == v
    with pytest.raises(KeyError):
        dda.Target.make_opts(solver="gmres")
