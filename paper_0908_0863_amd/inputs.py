"""Seeded synthetic inputs: target geometries, incident directions and random
vectors.

This module holds none of the DDA arithmetic (no interaction tensor, no
polarisability, no transform); it only produces lattices, occupancies and
numbers.  Both the HIP library's tests and the CPU oracle consume it.

Occupancy arrays are uint8 [P][J][K] (z, y, x; x fastest), matching the linear
site index n = k*J*K + j*K + i of the paper's Appendix A.
"""
from __future__ import annotations

import math

import numpy as np


def sphere(K: int) -> np.ndarray:
    """Sphere on a K^3 lattice: site (i, j, k) occupied iff
    |r - c|^2 <= (K/2)^2 with c = ((K-1)/2, (K-1)/2, (K-1)/2).  Evaluated in
    exact integers as sum (2x - (K-1))^2 <= K^2.  This rule reproduces every
    occupied-site count the paper prints (18^3 -> 3,112 in Sec. 4; 200^3 ...
    600^3 in Sec. 6 and its system-size table)."""
    a = (2 * np.arange(K, dtype=np.int64) - (K - 1)) ** 2
    d = a[:, None, None] + a[None, :, None] + a[None, None, :]
    return (d <= K * K).astype(np.uint8)


def sphere_count(K: int) -> int:
    """Occupied count of ``sphere(K)``, computed plane by plane (no K^3 array)."""
    a = (2 * np.arange(K, dtype=np.int64) - (K - 1)) ** 2
    s2 = a[:, None] + a[None, :]
    tot = 0
    for z in range(K):
        tot += int(np.count_nonzero(s2 + a[z] <= K * K))
    return tot


def cube(K: int, J: int | None = None, P: int | None = None) -> np.ndarray:
    """Completely filled rectangular lattice."""
    J = K if J is None else J
    P = K if P is None else P
    return np.ones((P, J, K), dtype=np.uint8)


def ellipsoid(K: int, J: int, P: int, a: float, b: float, c: float) -> np.ndarray:
    """Ellipsoid with semi-axes (a, b, c) along (x, y, z), centred on the
    lattice centre, exact integer test
    (2x-(K-1))^2 b^2 c^2 + (2y-(J-1))^2 a^2 c^2 + (2z-(P-1))^2 a^2 b^2 <= 4 a^2 b^2 c^2
    for integer semi-axes."""
    a2, b2, c2 = int(a * a), int(b * b), int(c * c)
    x = (2 * np.arange(K, dtype=np.int64) - (K - 1)) ** 2
    y = (2 * np.arange(J, dtype=np.int64) - (J - 1)) ** 2
    z = (2 * np.arange(P, dtype=np.int64) - (P - 1)) ** 2
    lhs = z[:, None, None] * a2 * b2 + y[None, :, None] * a2 * c2 + x[None, None, :] * b2 * c2
    return (lhs <= 4 * a2 * b2 * c2).astype(np.uint8)


def aggregate(rng: np.random.Generator, n_monomers: int, radius: float = 4.0,
              min_lattice: int = 32, max_lattice: int = 128):
    """Random cluster of touching spheres by sequential attachment: each new
    centre sits at distance 2*radius from a randomly chosen existing centre, in
    a uniformly random direction, and is rejected if it comes closer than
    2*radius to any other centre.  Voxelised on a cubic lattice of the bounding
    box extent (at least ``min_lattice``): a site is occupied iff it lies within
    ``radius`` of some centre.  Returns (occ, L) or None if L > max_lattice."""
    centres = [np.zeros(3)]
    tries = 0
    while len(centres) < n_monomers:
        tries += 1
        if tries > 200 * n_monomers:
            break
        base = centres[rng.integers(len(centres))]
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        c = base + 2.0 * radius * u
        C = np.array(centres)
        if np.min(np.linalg.norm(C - c, axis=1)) < 2.0 * radius - 1e-9:
            continue
        centres.append(c)
    C = np.array(centres)
    lo = C.min(0) - radius
    hi = C.max(0) + radius
    L = int(math.ceil(float((hi - lo).max()))) + 1
    L = max(L, min_lattice)
    if L > max_lattice:
        return None
    mid = (lo + hi) / 2.0
    off = mid - (L - 1) / 2.0
    g = np.arange(L, dtype=np.float64)
    occ = np.zeros((L, L, L), dtype=np.uint8)
    for c in C - off:
        zs = slice(max(0, int(c[2] - radius) - 1), min(L, int(c[2] + radius) + 2))
        ys = slice(max(0, int(c[1] - radius) - 1), min(L, int(c[1] + radius) + 2))
        xs = slice(max(0, int(c[0] - radius) - 1), min(L, int(c[0] + radius) + 2))
        d2 = ((g[zs, None, None] - c[2]) ** 2 + (g[None, ys, None] - c[1]) ** 2
              + (g[None, None, xs] - c[0]) ** 2)
        occ[zs, ys, xs] |= (d2 <= radius * radius).astype(np.uint8)
    return occ, L


def aggregates(seed: int, count: int = 40):
    """``count`` aggregate targets of 20..200 monomers with refractive index
    m ~ U(1.3, 1.8) + i U(0.001, 0.3); regenerates any that overflow 128^3."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = int(rng.integers(20, 201))
        r = aggregate(rng, n)
        if r is None:
            continue
        occ, L = r
        m = complex(rng.uniform(1.3, 1.8), rng.uniform(0.001, 0.3))
        out.append(dict(occ=occ, L=L, m=m, monomers=n))
    return out


def directions(seed: int, n: int):
    """n propagation directions uniform on the sphere (cos theta ~ U[-1,1],
    phi ~ U[0, 2 pi)) with the two polarisations theta-hat and phi-hat.
    Returns khat [n][3], e1 [n][3], e2 [n][3] (real)."""
    rng = np.random.default_rng(seed)
    ct = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    khat = np.stack([st * np.cos(ph), st * np.sin(ph), ct], 1)
    e1 = np.stack([ct * np.cos(ph), ct * np.sin(ph), -st], 1)
    e2 = np.stack([-np.sin(ph), np.cos(ph), np.zeros(n)], 1)
    return khat, e1, e2


def complex_gaussian(seed: int, shape, dtype=np.complex128) -> np.ndarray:
    """Seeded standard complex Gaussian array."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return (z / math.sqrt(2.0)).astype(dtype)


def kd_from_size_parameter(x: float, nd: int) -> float:
    """kd from the size parameter x = k a_eff with a_eff = (3 N_d / 4 pi)^(1/3) d."""
    return x / ((3.0 * nd / (4.0 * math.pi)) ** (1.0 / 3.0))


# --- the workloads used by the tests and the benchmark ----------------------

def workload(name: str) -> dict:
    """Named synthetic workloads.  Returns occupancy, lattice, refractive index,
    kd and the incident directions/polarisations."""
    zhat = np.array([0.0, 0.0, 1.0])
    xh = np.array([1.0, 0.0, 0.0])
    yh = np.array([0.0, 1.0, 0.0])
    if name == "sphere16":     # sphere, m = 1.33 + 0.01i, x = 1, 2 polarisations along +z
        occ = sphere(16)
        nd = int(occ.sum())
        return dict(name=name, occ=occ, K=16, J=16, P=16, m=1.33 + 0.01j,
                    kd=kd_from_size_parameter(1.0, nd), khat=[zhat, zhat], ehat=[xh, yh])
    if name == "cube64":       # filled cube, m = 1.5 + 0.02i, x = 10, one polarisation
        occ = cube(64)
        nd = int(occ.size)
        return dict(name=name, occ=occ, K=64, J=64, P=64, m=1.5 + 0.02j,
                    kd=kd_from_size_parameter(10.0, nd), khat=[zhat], ehat=[xh])
    if name == "ellipsoid96":  # semi-axes 48, 32, 32; m = 1.7 + 0.1i, x = 15; 64 dirs x 2 pols
        occ = ellipsoid(96, 96, 96, 48, 32, 32)
        nd = int(occ.sum())
        kh, e1, e2 = directions(3, 64)
        khat = [k for k in kh for _ in range(2)]
        ehat = [e for pair in zip(e1, e2) for e in pair]
        return dict(name=name, occ=occ, K=96, J=96, P=96, m=1.7 + 0.1j,
                    kd=kd_from_size_parameter(15.0, nd), khat=khat, ehat=ehat)
    if name == "sphere128":    # m = 1.6 + 0.05i, x = 20
        occ = sphere(128)
        nd = int(occ.sum())
        return dict(name=name, occ=occ, K=128, J=128, P=128, m=1.6 + 0.05j,
                    kd=kd_from_size_parameter(20.0, nd), khat=[zhat], ehat=[xh])
    if name == "sphere10":     # 10^3 version of sphere128: same m and kd
        occ = sphere(10)
        big = sphere_count(128)
        return dict(name=name, occ=occ, K=10, J=10, P=10, m=1.6 + 0.05j,
                    kd=kd_from_size_parameter(20.0, big), khat=[zhat], ehat=[xh])
    if name == "sphere200":    # the paper's benchmark sphere (Sec. 6, Table 3): same optics as cube100
        occ = sphere(200)
        nd = int(occ.sum())
        lam, a = 3.175, 0.5
        x = 2.0 * math.pi * a / lam
        return dict(name=name, occ=occ, K=200, J=200, P=200, m=1.63631 + 0.372j,
                    kd=kd_from_size_parameter(x, nd), khat=[zhat], ehat=[xh])
    if name == "cube100":      # the paper's validation cube (Sec. 6): x = 0.989478
        occ = cube(100)
        lam, a = 3.175, 0.5
        x = 2.0 * math.pi * a / lam
        return dict(name=name, occ=occ, K=100, J=100, P=100, m=1.63631 + 0.372j,
                    kd=kd_from_size_parameter(x, 100 ** 3), khat=[zhat], ehat=[xh])
    raise KeyError(name)
