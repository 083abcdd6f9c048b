"""The seeded input generators (CPU): the workloads have the shapes, dipole
counts and optics of the configurations they stand for, the aggregate
ensemble has the stated size and parameter ranges, and the incidence
directions are unit vectors with orthonormal polarisations.  The generators
hold none of the method's arithmetic."""
import math

import numpy as np
import pytest

from paper_0908_0863_amd import inputs


@pytest.mark.parametrize("name,lattice,nd,m", [
    ("sphere16", (16, 16, 16), 2176, 1.33 + 0.01j),
    ("cube64", (64, 64, 64), 262144, 1.5 + 0.02j),
    ("ellipsoid96", (96, 96, 96), 206192, 1.7 + 0.1j),
    ("sphere128", (128, 128, 128), 1099136, 1.6 + 0.05j),
    ("sphere10", (10, 10, 10), 552, 1.6 + 0.05j),
    ("sphere200", (200, 200, 200), 4188896, 1.63631 + 0.372j),
    ("cube100", (100, 100, 100), 1000000, 1.63631 + 0.372j),
])
def test_workload_shapes_counts_and_optics(name, lattice, nd, m):
    w = inputs.workload(name)
    assert (w["K"], w["J"], w["P"]) == lattice
    assert w["occ"].shape == lattice[::-1] and w["occ"].dtype == np.uint8
    assert int(w["occ"].sum()) == nd
    assert w["m"] == pytest.approx(m)
    assert w["kd"] > 0


@pytest.mark.parametrize("name,x", [("sphere16", 1.0), ("cube64", 10.0), ("ellipsoid96", 15.0), ("sphere128", 20.0)])
def test_workload_size_parameters(name, x):
    """x = k a_eff with a_eff = (3 N_d / 4 pi)^(1/3) (d = 1)."""
    w = inputs.workload(name)
    nd = int(w["occ"].sum())
    assert w["kd"] * (3 * nd / (4 * math.pi)) ** (1 / 3) == pytest.approx(x, rel=1e-12)


def test_ellipsoid_orientations_are_orthonormal():
    w = inputs.workload("ellipsoid96")
    kh, eh = np.asarray(w["khat"]), np.asarray(w["ehat"])
    assert kh.shape == (128, 3) and eh.shape == (128, 3)
    assert np.allclose(np.linalg.norm(kh, axis=1), 1.0, atol=1e-14)
    assert np.allclose(np.linalg.norm(eh, axis=1), 1.0, atol=1e-14)
    assert np.abs(np.sum(kh * eh, axis=1)).max() < 1e-14
    # the two polarisations of one direction are orthogonal
    assert np.abs(np.sum(eh[0::2] * eh[1::2], axis=1)).max() < 1e-14


def test_aggregate_ensemble_ranges_and_reproducibility():
    a1 = inputs.aggregates(4, 40)
    a2 = inputs.aggregates(4, 40)
    assert len(a1) == 40
    for p, q in zip(a1, a2):
        assert p["L"] == q["L"] and np.array_equal(p["occ"], q["occ"]) and p["m"] == q["m"]
        assert 32 <= p["L"] <= 128 and p["occ"].shape == (p["L"],) * 3
        assert 1.3 <= p["m"].real <= 1.8 and 0.001 <= p["m"].imag <= 0.3
        assert int(p["occ"].sum()) > 0


def test_complex_gaussian_is_seeded():
    a = inputs.complex_gaussian(5, (2, 3, 7))
    assert a.dtype == np.complex128 and a.shape == (2, 3, 7)
    assert np.array_equal(a, inputs.complex_gaussian(5, (2, 3, 7)))
    assert not np.array_equal(a, inputs.complex_gaussian(6, (2, 3, 7)))
