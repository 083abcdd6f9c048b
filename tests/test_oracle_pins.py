"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a closed form, a
conservation law, a printed value or an independent library routine, chosen so
that a dropped term, a sign or an index mistake in the oracle fails at least one.
"""
import math

import numpy as np
import pytest

import oracle as ora
from paper_0908_0863_amd import inputs
from tests.conftest import read_golden

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# --- P1: the sphere rule reproduces every N_d the paper prints --------------

def test_sphere_counts_match_paper():
    for K, nd, *_ in read_golden("sphere_counts.txt"):
        assert inputs.sphere_count(int(K)) == int(nd), K


def test_sphere_array_matches_count_and_sites_order():
    occ = inputs.sphere(18)
    assert int(occ.sum()) == 3112
    s = ora.sites_of(occ)
    lin = s[:, 2] * 18 * 18 + s[:, 1] * 18 + s[:, 0]
    assert np.all(np.diff(lin) > 0)


# --- the interaction tensor -------------------------------------------------

def _dipole_field(k, r, p):
    """Field at r of an oscillating dipole p at the origin (Jackson, Classical
    Electrodynamics, Eq. 9.18, Gaussian units, time factor e^{-i w t}):
    E = e^{ikr} { k^2 (n x p) x n / r + [3 n (n.p) - p] (1/r^3 - i k / r^2) }."""
    rr = np.linalg.norm(r)
    n = r / rr
    return np.exp(1j * k * rr) * (k * k * np.cross(np.cross(n, p), n) / rr
                                  + (3 * n * np.dot(n, p) - p) * (1 / rr ** 3 - 1j * k / rr ** 2))


@pytest.mark.parametrize("r", [(1, 0, 0), (0, 2, 0), (1, -2, 3), (-3, 1, -1), (5, 4, -2)])
def test_neg_green_is_minus_dipole_field(r):
    k = 0.37
    t = ora.neg_green(k, r)
    T = np.array([[t[0], t[1], t[2]], [t[1], t[3], t[4]], [t[2], t[4], t[5]]])
    for p in np.eye(3):
        np.testing.assert_allclose(-T @ p, _dipole_field(k, np.array(r, float), p), rtol=1e-13, atol=1e-15)


def test_neg_green_parities_match_table1():
    """Odd/even behaviour of each component under a reflection of one axis is
    what Table 1 of the paper lists."""
    signs = {row[0]: [int(v) for v in row[1:]] for row in read_golden("table1_signs.txt")}
    k = 0.8
    r = np.array([2.0, 3.0, 5.0])
    t0 = ora.neg_green(k, r)
    for ax, name in enumerate("xyz"):
        rm = r.copy()
        rm[ax] = -rm[ax]
        t1 = ora.neg_green(k, rm)
        np.testing.assert_allclose(t1, np.array(signs[name]) * t0, rtol=1e-14)


# --- P2: single dipole, two dipoles -----------------------------------------

def test_single_dipole_closed_form():
    k = 0.3
    sites = np.zeros((1, 3), np.int32)
    eps = 2.5 + 0.4j
    ainv = ora.alpha_inv(eps, k, "ldr", 0.0)
    alpha = 1.0 / ainv
    E = ora.einc(sites, k, [0, 0, 1], [1, 0, 0])
    P = ora.solve_dense(sites, k, ainv, E)
    np.testing.assert_allclose(P[:, 0], [alpha, 0, 0], rtol=1e-15)
    cext = ora.c_ext(k, E, P)
    csca = ora.c_sca_quadrature(sites, k, P, 24, 48)
    cabs = ora.c_abs(k, ainv, P)
    assert cext == pytest.approx(4 * math.pi * k * alpha.imag, rel=1e-14)
    assert csca == pytest.approx(8 * math.pi / 3 * k ** 4 * abs(alpha) ** 2, rel=1e-13)
    assert cabs == pytest.approx(cext - csca, rel=1e-12, abs=1e-18)
    assert ora.c_sca_double_sum(sites, k, P) == pytest.approx(csca, rel=1e-13)


@pytest.mark.parametrize("pol", ["parallel", "perpendicular"])
def test_two_dipoles_closed_form(pol):
    """Two identical dipoles a distance d apart along x, plane wave along z.
    Both see the same incident field; by symmetry P1 = P2 = P with
    (alpha^{-1} - G_aa(d)) P = E0, where from the dipole field
    G_xx(d x) = 2 e^{ikd}(1 - ikd)/d^3 (field along the axis) and
    G_yy(d x) = e^{ikd}(k^2 d^2 - 1 + ikd)/d^3 (field across the axis)."""
    k, d = 0.45, 3
    sites = np.array([[0, 0, 0], [d, 0, 0]], np.int32)
    eps = 3.0 + 0.1j
    ainv = ora.alpha_inv(eps, k, "rr")
    if pol == "parallel":
        e, G = np.array([1.0, 0, 0]), 2 * np.exp(1j * k * d) * (1 - 1j * k * d) / d ** 3
    else:
        e, G = np.array([0, 1.0, 0]), np.exp(1j * k * d) * (k * k * d * d - 1 + 1j * k * d) / d ** 3
    E = ora.einc(sites, k, [0, 0, 1], e)
    P = ora.solve_dense(sites, k, ainv, E)
    expect = 1.0 / (ainv - G)
    a = 0 if pol == "parallel" else 1
    np.testing.assert_allclose(P[a], [expect, expect], rtol=1e-14)
    np.testing.assert_allclose(np.delete(P, a, axis=0), 0, atol=1e-16)


# --- P3c: symmetry, LU --------------------------------------------------------

def _cluster(n, seed=1, box=6):
    rng = np.random.default_rng(seed)
    pts = set()
    while len(pts) < n:
        pts.add(tuple(rng.integers(0, box, 3)))
    lin = sorted(pts, key=lambda p: (p[2], p[1], p[0]))
    return np.array(lin, np.int32)


def test_matrix_is_complex_symmetric_bitwise():
    sites = _cluster(25)
    ainv = ora.alpha_inv(np.full(25, 2.0 + 0.3j), 0.5, "ldr", 0.2)
    A = ora.dense_matrix(sites, 0.5, ainv)
    assert np.array_equal(A, A.T)


def test_dense_matvec_equals_matrix_product():
    sites = _cluster(40, seed=3)
    k = 0.6
    ainv = ora.alpha_inv(np.full(40, 1.7 + 0.2j), k, "ldr")
    x = inputs.complex_gaussian(0, (3, 40))
    A = ora.dense_matrix(sites, k, ainv)
    y = ora.dense_matvec(sites, k, ainv, x)
    np.testing.assert_allclose(y.ravel(), A @ x.ravel(), rtol=1e-13)
    rows = np.array([5, 0, 39])
    yr = ora.dense_matvec(sites, k, ainv, x, rows=rows)
    np.testing.assert_allclose(yr, y[:, rows], rtol=1e-15)


def test_lu_matches_lapack():
    sites = _cluster(30, seed=4)
    k = 0.9
    ainv = ora.alpha_inv(np.full(30, 2.2 + 0.5j), k, "ldr")
    A = ora.dense_matrix(sites, k, ainv)
    b = inputs.complex_gaussian(1, (90, 2))
    np.testing.assert_allclose(ora.lu_solve(A, b), np.linalg.solve(A, b), rtol=1e-11)


def test_bicgstab_reaches_lu_solution():
    sites = _cluster(30, seed=5)
    k = 0.5
    ainv = ora.alpha_inv(np.full(30, 1.5 + 0.05j), k, "ldr")
    E = ora.einc(sites, k, [0, 0, 1], [1, 0, 0])
    x, it = ora.bicgstab(lambda v: ora.dense_matvec(sites, k, ainv, v.reshape(3, 30)).ravel(),
                         E.ravel(), tol=1e-12)
    P = ora.solve_dense(sites, k, ainv, E)
    assert it < 200
    np.testing.assert_allclose(x.reshape(3, 30), P, rtol=1e-9, atol=1e-12 * np.abs(P).max())


# --- P3: optical theorem and energy conservation ------------------------------

@pytest.mark.parametrize("presc", ["rr", "ldr"])
def test_optical_theorem_cluster(presc):
    """C_ext = C_abs + C_sca holds exactly for any solution of the DDA system;
    C_sca here is the independent far-field quadrature."""
    sites = _cluster(30, seed=7)
    k = 0.7
    eps = 2.4 + 0.6j
    S = ora.ldr_S([0, 0, 1], [1, 0, 0])
    ainv = ora.alpha_inv(np.full(30, eps), k, presc, S)
    E = ora.einc(sites, k, [0, 0, 1], [1, 0, 0])
    P = ora.solve_dense(sites, k, ainv, E)
    cext, cabs = ora.c_ext(k, E, P), ora.c_abs(k, ainv, P)
    csca = ora.c_sca_quadrature(sites, k, P)
    assert cext == pytest.approx(cabs + csca, rel=1e-11)
    assert ora.c_sca_double_sum(sites, k, P) == pytest.approx(csca, rel=1e-11)


def test_real_permittivity_does_not_absorb():
    """For real eps the radiative term -(2/3) i k^3 in alpha^{-1} makes the dipoles
    lossless: C_abs = 0 and C_ext = C_sca (quadrature)."""
    sites = _cluster(20, seed=8)
    k = 0.6
    ainv = ora.alpha_inv(np.full(20, 2.25 + 0j), k, "ldr", 0.0)
    E = ora.einc(sites, k, [1, 0, 0], [0, 0, 1])
    P = ora.solve_dense(sites, k, ainv, E)
    assert abs(ora.c_abs(k, ainv, P)) < 1e-13 * ora.c_ext(k, E, P)
    assert ora.c_ext(k, E, P) == pytest.approx(ora.c_sca_quadrature(sites, k, P), rel=1e-11)


# --- P3b: Rayleigh limit ------------------------------------------------------

@pytest.mark.parametrize("K,tol", [(10, 0.02), (16, 0.01)])
def test_rayleigh_small_sphere(K, tol):
    """Q_abs -> 4 x Im L, Q_sca -> (8/3) x^4 |L|^2, L = (eps-1)/(eps+2), as x -> 0;
    the lattice discretisation error shrinks with N_d."""
    occ = inputs.sphere(K)
    sites = ora.sites_of(occ)
    nd = sites.shape[0]
    x = 0.05
    k = x / ora.a_eff(nd)
    eps = (1.33 + 0.01j) ** 2
    ainv = ora.alpha_inv(np.full(nd, eps), k, "ldr", 0.0)
    E = ora.einc(sites, k, [0, 0, 1], [1, 0, 0])
    P = ora.solve_dense(sites, k, ainv, E)
    area = math.pi * ora.a_eff(nd) ** 2
    L = (eps - 1) / (eps + 2)
    qabs = ora.c_abs(k, ainv, P) / area
    qsca = ora.c_sca_quadrature(sites, k, P, 8, 16) / area
    assert qabs == pytest.approx(4 * x * L.imag, rel=tol)
    assert qsca == pytest.approx(8 / 3 * x ** 4 * abs(L) ** 2, rel=tol)


# --- circulant embedding (Sec. 3, Appendix A) ---------------------------------

@pytest.mark.parametrize("dims,pads", [((4, 3, 5), (7, 5, 9)), ((4, 3, 5), (8, 6, 10)),
                                       ((3, 4, 2), (9, 8, 4)), ((1, 1, 1), (1, 1, 1)),
                                       ((2, 1, 1), (3, 1, 1)), ((5, 2, 3), (12, 3, 5))])
def test_circulant_spectrum_gives_dense_convolution(dims, pads):
    """ifftn(Y . fftn(x zero-padded))[first octant] + alpha^{-1} x = dense A x for
    any padded size >= 2n - 1 (the convolution theorem of Eq. circdiagl1
    extended to three levels, Appendix A)."""
    K, J, P = dims
    Kpp, Jpp, Ppp = pads
    rng = np.random.default_rng(11)
    occ = (rng.random((P, J, K)) < 0.7).astype(np.uint8)
    occ.flat[0] = 1
    sites = ora.sites_of(occ)
    nd = sites.shape[0]
    k = 0.55
    ainv = ora.alpha_inv(np.full(nd, 2.0 + 0.3j), k, "ldr")
    x = inputs.complex_gaussian(2, (3, nd))
    Y = ora.circulant_spectrum(K, J, P, Kpp, Jpp, Ppp, k, half=False)
    Xg = np.zeros((3, Ppp, Jpp, Kpp), np.complex128)
    Xg[:, sites[:, 2], sites[:, 1], sites[:, 0]] = x
    Xf = np.fft.fftn(Xg, axes=(1, 2, 3))
    comp = [[0, 1, 2], [1, 3, 4], [2, 4, 5]]
    Q = np.stack([sum(Y[comp[a][b]] * Xf[b] for b in range(3)) for a in range(3)])
    yg = np.fft.ifftn(Q, axes=(1, 2, 3))
    y = yg[:, sites[:, 2], sites[:, 1], sites[:, 0]] + ainv[None, :] * x
    yd = ora.dense_matvec(sites, k, ainv, x)
    np.testing.assert_allclose(y, yd, rtol=0, atol=1e-13 * np.abs(yd).max())


def test_spectrum_mirror_parities_match_table1():
    """The DFT keeps the mirror parity of each tensor component: Y(n''-f) = s Y(f)
    along every axis with the Table 1 sign s, so the octant [0, n''/2] holds
    the whole spectrum (the access rule of Sec. 3, with signs)."""
    signs = {row[0]: [int(v) for v in row[1:]] for row in read_golden("table1_signs.txt")}
    K, J, P = 4, 5, 3
    Kpp, Jpp, Ppp = 8, 10, 6
    Y = ora.circulant_spectrum(K, J, P, Kpp, Jpp, Ppp, 0.4, half=False)
    for c in range(6):
        Yc = Y[c]
        for ax, name, n in ((2, "x", Kpp), (1, "y", Jpp), (0, "z", Ppp)):
            f = np.arange(n)
            mirrored = np.take(Yc, (-f) % n, axis=ax)
            np.testing.assert_allclose(mirrored, signs[name][c] * Yc, atol=1e-12)


# --- gradient -----------------------------------------------------------------

def test_gradient_adjoint_matches_exact_finite_differences():
    sites = _cluster(18, seed=12)
    nd = 18
    k = 0.5
    rng = np.random.default_rng(13)
    eps = 2.0 + rng.uniform(0, 1, nd) + 1j * rng.uniform(0.05, 0.4, nd)
    S = 0.3
    E = ora.einc(sites, k, [0, 0, 1], [1, 0, 0])
    g, _ = ora.grad_cabs_adjoint_dense(sites, k, eps, "ldr", S, E)
    sel = [0, 5, 17]
    fd = ora.grad_cabs_woodbury_fd(sites, k, eps, "ldr", S, E, sel, h=1e-5)
    np.testing.assert_allclose(fd, g[sel], rtol=1e-7, atol=1e-9 * np.abs(g).max())
    # brute force: re-solve the whole system at eps_n +- h
    n = 5
    h = 1e-5 * abs(eps[n])
    vals = []
    for d in (h, -h, 1j * h, -1j * h):
        e2 = eps.copy()
        e2[n] += d
        ai = ora.alpha_inv(e2, k, "ldr", S)
        P = ora.solve_dense(sites, k, ai, E)
        vals.append(ora.c_abs(k, ai, P))
    brute = (vals[0] - vals[1]) / (2 * h) + 1j * (vals[2] - vals[3]) / (2 * h)
    assert brute.real == pytest.approx(g[n].real, rel=1e-6, abs=1e-9)
    assert brute.imag == pytest.approx(g[n].imag, rel=1e-6, abs=1e-9)


# --- far field, amplitude and Mueller matrices (next step after the solve) --

def test_far_field_is_the_limit_of_the_dipole_field():
    """R e^{-ikR} E(R n) of a dipole p at r0 (Jackson's exact field) tends to the
    oracle's F(n) as R grows; the O(1/R) remainder shrinks tenfold per decade."""
    k = 0.6
    r0 = np.array([2.0, -1.0, 3.0])
    p = np.array([0.3 + 0.2j, -0.1 + 0.5j, 0.4 - 0.3j])
    n = np.array([0.48, -0.6, 0.64])
    n = n / np.linalg.norm(n)
    F = ora.far_field(np.array([r0], np.int32), k, p.reshape(3, 1), n.reshape(1, 3))[0]
    errs = []
    for R in (1e4, 1e5):
        E = _dipole_field(k, R * n - r0, p)
        errs.append(np.linalg.norm(R * np.exp(-1j * k * R) * E - F) / np.linalg.norm(F))
    assert errs[1] < 2e-3 and errs[1] < 0.2 * errs[0]


def test_optical_theorem_from_forward_amplitude():
    """C_ext = (4 pi / k) Im(e^* . F(k-hat)) = (4 pi / k^2) Re S2(0) for a solved
    cluster, against the extinction sum C_ext = 4 pi k sum Im(E^* . P)."""
    sites = _cluster(20, seed=3)
    k = 0.8
    ainv = ora.alpha_inv(np.full(20, 2.2 + 0.4j), k, "rr")
    Ex = ora.einc(sites, k, [0, 0, 1], [1, 0, 0])
    Ey = ora.einc(sites, k, [0, 0, 1], [0, 1, 0])
    Px = ora.solve_dense(sites, k, ainv, Ex)
    Py = ora.solve_dense(sites, k, ainv, Ey)
    fwd = np.array([[0.0, 0.0, 1.0]])
    Fx = ora.far_field(sites, k, Px, fwd)[0]
    assert 4 * math.pi / k * np.imag(Fx[0]) == pytest.approx(ora.c_ext(k, Ex, Px), rel=1e-12)
    S = ora.amplitude_matrix_z(ora.far_field(sites, k, Px, fwd), ora.far_field(sites, k, Py, fwd), [0.0], [0.0], k)
    assert 4 * math.pi / k ** 2 * np.real(S[0, 1]) == pytest.approx(ora.c_ext(k, Ex, Px), rel=1e-12)


def test_rayleigh_dipole_amplitude_and_mueller():
    """A single isotropic dipole (P = alpha E0): S1 = -i k^3 alpha, S2 = S1 cos(theta),
    S3 = S4 = 0 (Bohren & Huffman Sec. 5.2), so M11 = |S1|^2 (1 + cos^2)/2,
    M12 = -|S1|^2 sin^2 / 2, M33 = M44 = |S1|^2 cos, all others 0."""
    k, alpha = 0.7, 0.3 + 0.1j
    th = np.array([0.2, 0.9, 1.6, 2.5])
    ph = np.array([0.3, 2.0, 4.1, 5.5])
    dirs = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    origin = np.zeros((1, 3), np.int32)
    Fx = ora.far_field(origin, k, np.array([[alpha], [0], [0]]), dirs)
    Fy = ora.far_field(origin, k, np.array([[0], [alpha], [0]]), dirs)
    S = ora.amplitude_matrix_z(Fx, Fy, th, ph, k)
    s1 = -1j * k ** 3 * alpha
    np.testing.assert_allclose(S[:, 0], s1, rtol=1e-14)
    np.testing.assert_allclose(S[:, 1], s1 * np.cos(th), rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(S[:, 2:], 0, atol=1e-16)
    M = ora.mueller_from_amplitude(S)
    a2 = abs(s1) ** 2
    ref = np.zeros((4, 4, 4))
    ref[:, 0, 0] = ref[:, 1, 1] = a2 * (1 + np.cos(th) ** 2) / 2
    ref[:, 0, 1] = ref[:, 1, 0] = -a2 * np.sin(th) ** 2 / 2
    ref[:, 2, 2] = ref[:, 3, 3] = a2 * np.cos(th)
    np.testing.assert_allclose(M, ref, atol=1e-14 * a2)


def test_mueller_of_a_pure_amplitude_matrix():
    """A Mueller matrix from one amplitude matrix is non-depolarising:
    sum_ij M_ij^2 = 4 M11^2; the identity Jones matrix gives the identity."""
    rng = np.random.default_rng(2)
    S = rng.normal(size=(6, 4)) + 1j * rng.normal(size=(6, 4))
    M = ora.mueller_from_amplitude(S)
    np.testing.assert_allclose(np.sum(M ** 2, axis=(1, 2)), 4 * M[:, 0, 0] ** 2, rtol=1e-12)
    np.testing.assert_allclose(ora.mueller_from_amplitude([[1, 1, 0, 0]])[0], np.eye(4), atol=1e-15)


# --- anisotropic, multi-material composition (Sec. 2: a material per direction)

def test_single_anisotropic_dipole_closed_form():
    """alpha = diag(ax, ay, az): an x-polarised wave along z excites P = ax x,
    a y-polarised one P = ay y; C_ext = 4 pi k Im(a_c), C_sca = (8 pi/3) k^4 |a_c|^2."""
    k = 0.4
    a = np.array([0.8 + 0.3j, 0.2 + 0.05j, 1.1 + 0.7j])
    ainv = (1.0 / a).reshape(3, 1)
    site = np.zeros((1, 3), np.int32)
    for c, e in ((0, [1, 0, 0]), (1, [0, 1, 0])):
        E = ora.einc(site, k, [0, 0, 1], e)
        P = ora.solve_dense(site, k, ainv, E)
        assert P[c, 0] == pytest.approx(a[c], rel=1e-14)
        assert ora.c_ext(k, E, P) == pytest.approx(4 * math.pi * k * a[c].imag, rel=1e-13)
        csca = ora.c_sca_quadrature(site, k, P)
        assert csca == pytest.approx(8 * math.pi / 3 * k ** 4 * abs(a[c]) ** 2, rel=1e-12)


def test_composition_reduces_to_isotropic_and_keeps_the_optical_theorem():
    sites = _cluster(24, seed=4)
    k, S = 0.6, 0.0
    mats = [2.3 + 0.4j, 1.7 + 0.05j]
    iso = ora.alpha_inv_composition(mats, np.zeros((3, 24), int), k, "ldr", S)
    np.testing.assert_array_equal(iso, np.broadcast_to(ora.alpha_inv(mats[0], k, "ldr", S), (3, 24)))
    flags = np.random.default_rng(3).integers(0, 2, (3, 24))
    ainv = ora.alpha_inv_composition(mats, flags, k, "ldr", S)
    A = ora.dense_matrix(sites, k, ainv)
    assert np.array_equal(A, A.T)
    E = ora.einc(sites, k, [0, 0, 1], [1, 0, 0])
    P = ora.solve_dense(sites, k, ainv, E)
    cext, cabs = ora.c_ext(k, E, P), ora.c_abs(k, ainv, P)
    assert cext == pytest.approx(cabs + ora.c_sca_quadrature(sites, k, P), rel=1e-11)


# --- the LDR orientation factor S = sum_a (khat_a ehat_a)^2 (Sec. 1 names LDR) --
# Pinned by geometry, not by re-typing the formula: an axis-aligned wave has no
# product k_a e_a; on a body diagonal every k_a^2 is 1/3 and sum_a e_a^2 = 1;
# for an orthonormal triad (e1, e2, khat) every axis obeys
# e1_a^2 + e2_a^2 + k_a^2 = 1, so S(e1) + S(e2) = sum_a k_a^2 (1 - k_a^2).  A
# dropped square, (khat . ehat)^2 (identically 0) or a swapped operand fails.

def _transverse_pair(khat, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(3)
    e1 = v - np.dot(v, khat) * khat
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(khat, e1)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_ldr_S_vanishes_along_lattice_axes(axis):
    khat = np.eye(3)[axis]
    for seed in range(4):
        e1, e2 = _transverse_pair(khat, seed)
        assert ora.ldr_S(khat, e1) == 0.0
        assert ora.ldr_S(-khat, e2) == 0.0


def test_ldr_S_is_one_third_on_the_body_diagonal():
    for signs in ([1, 1, 1], [1, -1, 1], [-1, -1, 1]):
        khat = np.array(signs, float) / math.sqrt(3.0)
        for seed in range(5):
            e1, e2 = _transverse_pair(khat, seed)
            assert ora.ldr_S(khat, e1) == pytest.approx(1.0 / 3.0, abs=1e-15)
            assert ora.ldr_S(khat, e2) == pytest.approx(1.0 / 3.0, abs=1e-15)


def test_ldr_S_transverse_sum_rule():
    rng = np.random.default_rng(11)
    for _ in range(20):
        khat = rng.standard_normal(3)
        khat /= np.linalg.norm(khat)
        e1, e2 = _transverse_pair(khat, int(rng.integers(1 << 30)))
        want = float(np.sum(khat ** 2 * (1.0 - khat ** 2)))
        assert ora.ldr_S(khat, e1) + ora.ldr_S(khat, e2) == pytest.approx(want, abs=1e-15)
        assert 0.0 <= ora.ldr_S(khat, e1) <= 0.5 + 1e-15  # k_a^2 e_a^2 <= (k_a^2 + e_a^2) / 4 as k_a^2 + e_a^2 <= 1


def test_ldr_S_enters_alpha_inv_through_b3_only():
    """Only the b3 S eps kd^2 term depends on S: the difference of two S values
    is b3 (S1 - S2) eps kd^2, and S = 0 leaves the CM + b1 + b2 eps form."""
    eps, kd = 2.3 + 0.4j, 0.3
    a1 = ora.alpha_inv(eps, kd, "ldr", 1.0 / 3.0)
    a0 = ora.alpha_inv(eps, kd, "ldr", 0.0)
    assert a1 - a0 == pytest.approx(ora.LDR_B3 * eps * kd ** 2 / 3.0, rel=1e-12)
    rr = ora.alpha_inv(eps, kd, "rr")
    assert a0 - rr == pytest.approx((ora.LDR_B1 + ora.LDR_B2 * eps) * kd ** 2, rel=1e-12)
