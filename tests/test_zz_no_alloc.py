"""GPU: sfft_apply_noalloc (workspace from the library's static device scratch)
against sfft_apply with a caller workspace, through the C ABI: the same kernels
and schedule, so the products must agree bit for bit (and with the FP64
oracle), on two calls in a row with the second smaller, and an oversized
request is refused before anything runs."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_17981_amd as sf
    return sf


def _noalloc(N, plan, x, y):
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return N.lib.sfft_apply_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                    x.shape[0], st)


@pytest.mark.parametrize("dtype,tdt,tol", [("c64", torch.complex64, 1e-5), ("c128", torch.complex128, 1e-12)])
def test_noalloc_matches_apply(sf, dtype, tdt, tol):
    from paper_2406_17981_amd import _native as N
    cases = [((24, 20, 32), 3, 4, "depth"), ((12, 10, 16), 3, 2, "breadth")]  # second call smaller
    for grid, b, nrhs, sched in cases:
        print(f"[case] noalloc n={grid} b={b} nrhs={nrhs} {dtype} {sched}", flush=True)
        coeffs = wl.green_coeffs(grid, 0.8)
        x = wl.vectors(105, grid, b, nrhs)
        plan = sf.Plan(grid, b, torch.from_numpy(coeffs).cuda(), dtype=dtype, max_nrhs=nrhs, schedule=sched)
        xd = torch.from_numpy(x).to(tdt).cuda()
        y_ref = plan.apply(xd, workspace=plan.alloc_workspace(nrhs))
        y = torch.full_like(xd, complex(float("nan"), float("nan")))
        assert _noalloc(N, plan, xd, y) == N.OK, N.lib.sfft_last_error()
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        got = y.cpu().numpy().astype(np.complex128)
        assert wl.relative_l2(got, oracle.embed_matvec(coeffs, x)) <= tol
        plan.close()


def test_noalloc_refuses_oversized_and_empty_is_a_no_op(sf):
    from paper_2406_17981_amd import _native as N
    grid, b = (128, 128, 128), 3
    plan = sf.Plan(grid, b, torch.zeros((b, b, 255, 255, 255), dtype=torch.complex128, device="cuda"),
                   dtype="c64", max_nrhs=2, schedule="depth")
    assert plan.workspace_size(2) > (128 << 20)
    x = torch.zeros((2, b) + grid, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    assert _noalloc(N, plan, x, y) == N.INVALID_ARG
    assert b"static scratch" in N.lib.sfft_last_error()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert N.lib.sfft_apply_noalloc(plan.handle, None, None, 0, st) == N.OK
    plan.close()
