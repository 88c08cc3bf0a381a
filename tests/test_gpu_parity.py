"""GPU parity: the HIP split-FFT matvec (through the C ABI) against the FP64 CPU
oracle on the same seeded inputs.

Tolerances (relative L2 over all entries): complex128 <= 1e-12, complex64
<= 1e-5, both against the FP64 oracle.
"""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}
NP = {"c128": np.complex128, "c64": np.complex64}


@pytest.fixture(scope="module")
def sf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_17981_amd as sf
    return sf


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _run(sf, coeffs, x, dtype, method="split", schedule="auto"):
    n = oracle.grid_of(coeffs)
    b = coeffs.shape[0]
    _say(f"n={n} b={b} dtype={dtype} method={method} sched={schedule} nrhs={x.shape[0]}")
    plan = sf.Plan(n, b, torch.from_numpy(coeffs).cuda(), dtype=dtype, method=method,
                   max_nrhs=x.shape[0], schedule=schedule)
    xd = torch.from_numpy(x.astype(NP[dtype])).cuda()
    ws = plan.alloc_workspace(x.shape[0])
    y = plan.apply(xd, workspace=ws)
    torch.cuda.synchronize()
    out = y.cpu().numpy().astype(np.complex128)
    plan.close()
    return out


SMALL = [
    # (grid, b) -- several tiles per pass and ragged last tiles
    ((24,), 1), ((40,), 3), ((10, 12), 1), ((16, 40), 3), ((6, 10, 12), 1), ((5, 12, 40), 3),
    ((8, 6, 10), 3), ((4, 3, 2, 5), 1), ((2, 3, 4, 2, 2), 1), ((16, 16, 16), 3),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid,b", SMALL)
def test_split_matches_dense_small(sf, grid, b, dtype):
    coeffs = wl.iid_coeffs(7, grid, b)
    x = wl.vectors(8, grid, b, 2)
    want = oracle.dense_matvec(coeffs, x) if math.prod(grid) * b <= 4096 else \
        oracle.embed_matvec(coeffs, x)
    for sched in ("breadth", "depth"):
        got = _run(sf, coeffs, x, dtype, "split", sched)
        err = wl.relative_l2(got, want)
        assert err <= TOL[dtype], (sched, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid,b", [((24,), 1), ((10, 12), 3), ((6, 10, 12), 1), ((4, 3, 2, 5), 3)])
def test_embed_baseline_matches_dense(sf, grid, b, dtype):
    coeffs = wl.iid_coeffs(9, grid, b)
    x = wl.vectors(10, grid, b, 2)
    want = oracle.dense_matvec(coeffs, x)
    got = _run(sf, coeffs, x, dtype, "embed")
    assert wl.relative_l2(got, want) <= TOL[dtype]


def test_plain_16_c128_against_dense(sf):
    """16^3 scalar, i.i.d. coefficients on the 31^3 offset grid, FP64, one vector."""
    coeffs, x = wl.plain_16()
    want = oracle.dense_matvec(coeffs, x)
    for sched in ("breadth", "depth"):
        got = _run(sf, coeffs, x, "c128", "split", sched)
        assert wl.relative_l2(got, want) <= 1e-12
    got = _run(sf, coeffs, x, "c128", "embed")
    assert wl.relative_l2(got, want) <= 1e-12


@pytest.mark.parametrize("grid,b", [((8, 6, 10), 3), ((40, 48), 1)])
def test_delta_and_shift_kernels(sf, grid, b):
    x = wl.vectors(11, grid, b, 1)
    got = _run(sf, wl.delta_coeffs(grid, b), x, "c128")
    assert wl.relative_l2(got, x) <= 1e-13
    r0 = tuple((v // 3) * (-1) ** l for l, v in enumerate(grid))
    coeffs = wl.shifted_delta_coeffs(grid, b, r0, b - 1, 0)
    got = _run(sf, coeffs, x, "c128")
    assert wl.relative_l2(got, oracle.dense_matvec(coeffs, x)) <= 1e-12


@pytest.fixture(scope="module")
def green64():
    coeffs, x = wl.green_64()
    want = oracle.embed_matvec(coeffs, x)
    rng = np.random.default_rng(2024)
    pts = np.stack([rng.integers(0, 64, 64) for _ in range(3)], axis=1)
    rows = oracle.sampled_rows(coeffs, x, pts)
    return coeffs, x, want, pts, rows


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("method", ["split", "embed"])
def test_green_64_full_size(sf, green64, dtype, method):
    """64^3 grid, 3x3 Green blocks (k=0.7): full-size parity against the FP64
    embedding oracle, which is itself checked on sampled direct-sum rows."""
    coeffs, x, want, pts, rows = green64
    ref_rows = np.stack([want[(slice(None), slice(None)) + tuple(p)] for p in pts], axis=-1)
    assert wl.relative_l2(ref_rows, rows) <= 1e-13
    got = _run(sf, coeffs, x, dtype, method)
    err = wl.relative_l2(got, want)
    _say(f"green64 {dtype} {method} rel_l2={err:.3e}")
    assert err <= TOL[dtype]


def test_multi_rhs_and_depth_schedule(sf):
    grid, b = (12, 10, 16), 3
    coeffs = wl.iid_coeffs(12, grid, b)
    x = wl.vectors(13, grid, b, 5)
    want = oracle.embed_matvec(coeffs, x)
    for dtype in ("c128", "c64"):
        for sched in ("breadth", "depth"):
            got = _run(sf, coeffs, x, dtype, "split", sched)
            assert wl.relative_l2(got, want) <= TOL[dtype]


def test_apply_rejects_bad_arguments(sf):
    grid, b = (8, 8), 1
    plan = sf.Plan(grid, b, torch.from_numpy(wl.iid_coeffs(1, grid, b)).cuda(), dtype="c64")
    x = torch.zeros((1, 1, 8, 8), dtype=torch.complex64, device="cuda")
    with pytest.raises(sf.SfftError):
        plan.apply(x, y=x)  # y aliases x
    ws = torch.empty(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(sf.SfftError):
        plan.apply(x, workspace=ws)  # too small
    with pytest.raises(ValueError):
        plan.apply(x.to(torch.complex128))
    plan.close()
