"""Error behaviour of the C ABI as the header states it: invalid arguments
(DDA_EINVAL), calls out of order (DDA_ESTATE) and missed tolerances
(DDA_ENOTCONV, with the last iterate and its info returned).  Every case is
rejected on the host before any kernel sees the bad input, or is a normal
solve stopped by its iteration limit."""
import numpy as np
import pytest

from paper_0908_0863_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dda():
    from paper_0908_0863_amd import dda as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return m


@pytest.fixture(scope="module")
def lib(dda):
    return dda.Library(0)


def _code(exc_info):
    return exc_info.value.code


@pytest.mark.parametrize("K,J,P,kd", [(0, 4, 4, 0.3), (4, -1, 4, 0.3), (4, 4, 4, 0.0), (4, 4, 4, float("nan"))])
def test_target_create_rejects_bad_lattice(dda, lib, K, J, P, kd):
    with pytest.raises(dda.DDAError) as e:
        dda.Target(lib, K, J, P, kd)
    assert _code(e) == dda.DDA_EINVAL


def test_out_of_order_and_bad_material(dda, lib):
    t = dda.Target(lib, 4, 3, 2, 0.4)
    with pytest.raises(dda.DDAError) as e:
        t.set_permittivity(2.0, "ldr")                   # before the occupancy
    assert _code(e) == dda.DDA_ESTATE
    with pytest.raises(dda.DDAError) as e:
        t.set_occupancy(np.zeros((2, 3, 4), np.uint8))   # no occupied site
    assert _code(e) == dda.DDA_EINVAL
    nd = t.set_occupancy(np.ones((2, 3, 4), np.uint8))
    assert nd == 24
    x = torch.zeros((1, 3, nd), dtype=torch.complex128, device="cuda")
    with pytest.raises(dda.DDAError) as e:
        t.matvec(x)                                      # no polarisability yet
    assert _code(e) == dda.DDA_ESTATE
    with pytest.raises(dda.DDAError) as e:
        t.set_permittivity(1.0, "ldr")                   # eps = 1: alpha = 0
    assert _code(e) == dda.DDA_EINVAL
    with pytest.raises(dda.DDAError) as e:
        t.set_permittivity(-2.0, "cm")                   # the Clausius-Mossotti pole
    assert _code(e) == dda.DDA_EINVAL
    t.set_permittivity(2.0 + 0.1j, "ldr")
    with pytest.raises(dda.DDAError) as e:
        t.matvec(x)                                      # spectrum not built
    assert _code(e) == dda.DDA_ESTATE
    t.build_spectrum()
    y = t.matvec(x)
    assert torch.count_nonzero(y).item() == 0
    with pytest.raises(dda.DDAError) as e:
        t.set_option(dda.DDA_OPT_SCHEDULE, 3)            # no such schedule
    assert _code(e) == dda.DDA_EINVAL
    with pytest.raises(dda.DDAError) as e:
        t.solve(khat=[[0, 0, 1]], ehat=[[1, 0, 0]], tol=2.0)
    assert _code(e) == dda.DDA_EINVAL
    with pytest.raises(dda.DDAError) as e:
        t.solve(khat=[[0, 0, 1]], ehat=[[1, 0, 0]], solver="rbicgstab", solver_param=5)   # l above 4
    assert _code(e) == dda.DDA_EINVAL
    with pytest.raises(dda.DDAError) as e:
        t.far_field(t.solve(khat=[[0, 0, 1]], ehat=[[1, 0, 0]])[0], [[1.0, 1.0, 0.0]])  # not a unit vector
    assert _code(e) == dda.DDA_EINVAL


@pytest.mark.parametrize("solver,param", [("bicgstab", 0), ("qmr_sym", 0), ("bicg_sym", 0), ("cgs", 0), ("tfqmr", 0),
                                          ("bicg", 0), ("qmr", 0), ("rbicgstab", 2), ("mlbicgstab", 3)])
def test_iteration_limit_reports_not_converged(dda, lib, solver, param):
    w = inputs.workload("sphere16")
    t = dda.Target(lib, 16, 16, 16, w["kd"])
    nd = t.set_occupancy(w["occ"])
    t.set_permittivity(np.full(nd, w["m"] ** 2), "ldr")
    t.build_spectrum()
    kw = dict(khat=w["khat"][:1], ehat=w["ehat"][:1], solver=solver, solver_param=param, precision="fp64", tol=1e-12,
              max_iter=3, max_outer=1)
    with pytest.raises(dda.NotConverged):
        t.solve(**kw)
    P, info = t.solve(raise_on_fail=False, **kw)
    assert info[0]["converged"] == 0 and info[0]["iterations"] <= 4
    assert 1e-12 < info[0]["rel_residual"] < 1.0        # a partial solution, not garbage
    assert torch.isfinite(torch.view_as_real(P)).all()


def _sphere16(dda, lib):
    w = inputs.workload("sphere16")
    t = dda.Target(lib, 16, 16, 16, w["kd"])
    nd = t.set_occupancy(w["occ"])
    t.set_permittivity(np.full(nd, w["m"] ** 2), "ldr")
    t.build_spectrum()
    return t, w


def test_non_finite_right_hand_side_rejected(dda, lib):
    t, w = _sphere16(dda, lib)
    E = t.incident_field(w["khat"][:1], w["ehat"][:1])
    E[0, 1, 5] = complex(float("nan"), 0.0)
    with pytest.raises(dda.DDAError) as e:
        t.solve(einc=E, S=[0.0], solver="bicgstab", precision="fp64", tol=1e-8)
    assert _code(e) == dda.DDA_EINVAL
    with pytest.raises(dda.DDAError) as e:
        t.set_option(dda.DDA_OPT_INJECT_BREAKDOWN, -1)
    assert _code(e) == dda.DDA_EINVAL


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_injected_breakdown_restarts_from_true_residual(dda, lib, precision):
    """Two BiCGSTAB inner solves that start from a zero shadow vector break
    down in their first step (rhat^H v = 0); the refinement loop restarts each
    time from the FP64 true residual and the solve still reaches the answer of
    the undisturbed one."""
    t, w = _sphere16(dda, lib)
    kw = dict(khat=w["khat"][:1], ehat=w["ehat"][:1], solver="bicgstab", precision=precision, tol=1e-10,
              inner_tol=1e-4)
    P0, i0 = t.solve(**kw)
    t.set_option(dda.DDA_OPT_INJECT_BREAKDOWN, 2)
    P1, i1 = t.solve(**kw)
    assert i0[0]["converged"] and i1[0]["converged"]
    # two wasted refinement steps, then at least one that solves (in mixed
    # precision the first breakdown also switches the inner solves to FP64)
    assert i1[0]["outer_iterations"] >= 3
    if precision == "fp64":
        assert i0[0]["outer_iterations"] == 1
    assert (torch.linalg.norm(P1 - P0) / torch.linalg.norm(P0)).item() < 1e-8
    P2, i2 = t.solve(**kw)  # the injections are used up
    assert i2[0]["outer_iterations"] == i0[0]["outer_iterations"]


@pytest.mark.parametrize("solver", ["qmr_sym", "tfqmr"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_step_that_worsens_the_residual_is_taken_back(dda, lib, solver, precision):
    """A refinement step applied with the wrong sign (fault injection from the
    host) leaves the true residual larger than before: the loop restores P and
    the residual of that step's start, and the solve still ends at the answer
    of the undisturbed one (in mixed precision on FP64 inner solves).  Two
    right-hand sides, both disturbed."""
    t, w = _sphere16(dda, lib)
    kw = dict(khat=w["khat"], ehat=w["ehat"], solver=solver, precision=precision, tol=1e-10, inner_tol=1e-4)
    P0, i0 = t.solve(**kw)
    with pytest.raises(dda.DDAError) as e:
        t.set_option(dda.DDA_OPT_INJECT_BAD_STEP, -1)
    assert _code(e) == dda.DDA_EINVAL
    t.set_option(dda.DDA_OPT_INJECT_BAD_STEP, 1)
    P1, i1 = t.solve(**kw)
    for r in range(len(i0)):
        assert i0[r]["converged"] and i1[r]["converged"]
        # the taken-back step counts; in mixed precision the FP64 inner solves
        # that follow it can need fewer steps than the undisturbed solve
        assert i1[r]["outer_iterations"] >= 2
        if precision == "fp64":
            assert i1[r]["outer_iterations"] == i0[r]["outer_iterations"] + 1
        assert torch.isfinite(torch.view_as_real(P1[r])).all()
        assert (torch.linalg.norm(P1[r] - P0[r]) / torch.linalg.norm(P0[r])).item() < 1e-8
