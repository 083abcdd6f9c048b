"""The allocation-free product dda_matvec_noalloc (for callers that cannot
allocate device memory) against dda_matvec, through the C ABI: two calls in a
row, the second with a smaller input, bit for bit with the schedule fixed and
within the oracle bars with the tuned one; no device memory is taken; inputs
beyond the scratch limit are rejected."""
import numpy as np
import pytest

import oracle as ora
from paper_0908_0863_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    from paper_0908_0863_amd import dda
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return dda.Library(0)


def _target(lib, occ, kd, eps):
    from paper_0908_0863_amd import dda
    P, J, K = occ.shape
    t = dda.Target(lib, K, J, P, kd)
    nd = t.set_occupancy(occ)
    t.set_permittivity(np.full(nd, eps), "ldr")
    t.build_spectrum()
    return t, nd


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("sched", [0, 6])
def test_noalloc_matches_matvec_two_calls_second_smaller(lib, sched):
    from paper_0908_0863_amd import dda
    big, nd_big = _target(lib, inputs.sphere(16), 0.3, 2.2 + 0.1j)
    rng = np.random.default_rng(71)
    occ_small = (rng.random((8, 7, 8)) < 0.6).astype(np.uint8)  # K'' = P'' = 16: every schedule exists
    occ_small.flat[0] = 1
    small, nd_small = _target(lib, occ_small, 0.45, 1.9 + 0.05j)
    cases = [(big, nd_big, 3, inputs.sphere(16), 0.3, 2.2 + 0.1j), (small, nd_small, 1, occ_small, 0.45, 1.9 + 0.05j)]
    for t, nd, nrhs, occ, kd, eps in cases:
        try:
            t.set_option(dda.DDA_OPT_SCHEDULE, sched)
        except dda.DDAError:
            pytest.skip(f"no schedule {sched}")
    outs = []
    for t, nd, nrhs, occ, kd, eps in cases:  # the second call is the smaller one
        S = [0.05 * r for r in range(nrhs)]
        x = inputs.complex_gaussian(72 + nrhs, (nrhs, 3, nd))
        for dt in (torch.complex128, torch.complex64):
            xd = torch.from_numpy(x).to("cuda", dt)
            outs.append((t, nd, nrhs, occ, kd, eps, S, x, xd, torch.empty_like(xd)))
    # a first round of calls (the runtime loads code and sets up its own state
    # on the first launches of a process), then a second round during which
    # the device's free memory must not move
    for t, nd, nrhs, occ, kd, eps, S, x, xd, y_na in outs:
        t.matvec_noalloc(xd, y_na, S=S, jacobi=True)
    first = [o[-1].clone() for o in outs]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for t, nd, nrhs, occ, kd, eps, S, x, xd, y_na in outs:
        t.matvec_noalloc(xd, y_na, S=S, jacobi=True)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0  # no device memory was taken
    for o, y1 in zip(outs, first):
        assert torch.equal(o[-1], y1)  # the shared scratch keeps no state between calls
    for t, nd, nrhs, occ, kd, eps, S, x, xd, y_na in outs:
        y_ref = t.matvec(xd, S=S, jacobi=True)  # the allocating entry point, same schedule
        assert torch.equal(y_na, y_ref), (nd, nrhs, xd.dtype)
        sites = ora.sites_of(occ)
        for r in range(nrhs):
            ainv = ora.alpha_inv(np.full(nd, eps), kd, "ldr", S[r])
            s = 1.0 / np.sqrt(ainv)
            yo = s * ora.dense_matvec(sites, kd, ainv, s * x[r])
            tol = 1e-12 if xd.dtype == torch.complex128 else 2e-6
            yr = y_na[r].cpu().numpy()
            assert _rel(yr, yo) < tol
            assert np.abs(yr - yo).max() <= tol * np.abs(yo).max()


def test_noalloc_rejects_inputs_beyond_the_scratch(lib):
    from paper_0908_0863_amd import dda
    t, nd = _target(lib, np.ones((64, 64, 64), np.uint8), 0.25, 2.25 + 0.06j)
    x = torch.zeros((1, 3, nd), dtype=torch.complex128, device="cuda")  # FP64 64^3: 75 MB of workspace
    y = torch.empty_like(x)
    with pytest.raises(dda.DDAError) as e:
        t.matvec_noalloc(x, y)
    assert e.value.code == dda.DDA_EINVAL and "scratch" in str(e.value)
    x32 = torch.from_numpy(inputs.complex_gaussian(3, (1, 3, nd)).astype(np.complex64)).cuda()
    y32 = torch.empty_like(x32)
    t.matvec_noalloc(x32, y32)  # FP32, one right-hand side: fits
    assert torch.equal(y32, t.matvec(x32)) or _rel(y32.cpu().numpy(), t.matvec(x32).cpu().numpy()) < 2e-6
