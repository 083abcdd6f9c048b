"""The plain-C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, gcc) runs its matrix-vector product (all rows and a row
subset), dense matrix, LU solve and far-field quadrature on a small seeded
target without a report, and agrees with the regular build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as ora
from paper_0908_0863_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", os.path.join(ROOT, "oracle", "dda_oracle.c"),
           os.path.join(ROOT, "tests", "oracle_sanitized_main.c"), "-o", exe, "-lm"]
    try:
        subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    except subprocess.CalledProcessError as e:
        if b"asan" in e.stderr.lower() and b"cannot find" in e.stderr.lower():
            pytest.skip("sanitizer runtime not installed")
        raise
    rng = np.random.default_rng(31)
    occ = (rng.random((4, 5, 6)) < 0.6).astype(np.uint8)
    occ.flat[0] = 1
    sites = np.ascontiguousarray(ora.sites_of(occ), dtype=np.int32)
    nd = sites.shape[0]
    kd = 0.37
    ainv = np.ascontiguousarray(ora.alpha_inv(np.full(nd, 2.1 + 0.3j), kd, "ldr", 0.2), np.complex128)
    ainv3 = np.ascontiguousarray(np.tile(ainv, 3))
    x = np.ascontiguousarray(inputs.complex_gaussian(5, (3, nd)), np.complex128)
    rows = np.ascontiguousarray(np.sort(rng.choice(nd, 7, replace=False)).astype(np.int64))
    ncos, nphi = ora.quadrature_sizes(sites, kd)
    cosn, wcos = np.polynomial.legendre.leggauss(ncos)
    inp = tmp_path / "in.bin"
    with open(inp, "wb") as f:
        np.array([nd, rows.size, ncos, nphi], np.int64).tofile(f)
        np.array([kd], np.float64).tofile(f)
        sites.tofile(f)
        ainv3.tofile(f)
        x.tofile(f)
        rows.tofile(f)
        np.ascontiguousarray(cosn).tofile(f)
        np.ascontiguousarray(wcos).tofile(f)
    out = tmp_path / "out.bin"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe, str(inp), str(out)], capture_output=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr.decode()[-3000:]
    assert b"runtime error" not in r.stderr and b"AddressSanitizer" not in r.stderr, r.stderr.decode()[-3000:]
    raw = np.fromfile(out, dtype=np.uint8)
    n3 = 3 * nd
    off = 0

    def take(count, dt):
        nonlocal off
        b = np.dtype(dt).itemsize * count
        v = raw[off:off + b].view(dt)
        off += b
        return v

    y = take(n3, np.complex128).reshape(3, nd)
    yr = take(3 * rows.size, np.complex128).reshape(3, rows.size)
    z = take(n3, np.complex128).reshape(3, nd)
    csca = take(1, np.float64)[0]
    info = take(1, np.int32)[0]
    assert off == raw.size and info == 0
    yo = ora.dense_matvec(sites, kd, ainv, x)
    assert np.linalg.norm(y - yo) <= 1e-13 * np.linalg.norm(yo)
    assert np.linalg.norm(yr - yo[:, rows]) <= 1e-13 * np.linalg.norm(yo[:, rows])
    zo = ora.solve_dense(sites, kd, ainv, x)
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)
    assert csca == pytest.approx(ora.c_sca_quadrature(sites, kd, zo), rel=1e-12)
