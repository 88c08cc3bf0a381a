"""GPU: one batched Arnoldi step (sfft_arnoldi_step_multi) against FP64 NumPy.

Classical Gram-Schmidt with a second pass only where the first removed more
than half of ||w||^2: a generic w takes one pass, a w that lies almost in the
basis span takes two, and both come out orthogonal to the basis to working
precision; each job's results are bitwise the same alone and in a shared call."""

import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def native():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_17981_amd import _native
    return _native


def _basis(rng, n, m):
    a = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    q, _ = np.linalg.qr(a)
    return q.T.copy()                            # (m, n), orthonormal rows


def _step(N, jobs, dtype):
    """jobs: list of (V (m, n) or None, w (n,)) host arrays; returns
    [(hcol, vout)] from one call."""
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    keep = []
    arr = (N.ArnoldiJob * len(jobs))()
    for a, (V, w) in zip(arr, jobs):
        n = w.size
        m = 0 if V is None else V.shape[0]
        Vd = torch.from_numpy(V).to(tdt).cuda() if m else torch.empty((1, n), dtype=tdt, device="cuda")
        wd = torch.from_numpy(w).to(tdt).cuda()
        vo = torch.empty(n, dtype=tdt, device="cuda")
        hc = torch.zeros(m + 1, dtype=torch.complex128, device="cuda")
        keep.append((Vd, wd, vo, hc))
        a.V, a.ldv, a.m = Vd.data_ptr(), n, m
        a.w, a.vout, a.n, a.hcol = wd.data_ptr(), vo.data_ptr(), n, hc.data_ptr()
    need = C.c_size_t()
    N.check(N.lib.sfft_arnoldi_scratch_size(len(jobs), arr, C.byref(need)), "sfft_arnoldi_scratch_size")
    scratch = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device="cuda")
    code = N.C64 if dtype == "c64" else N.C128
    st = torch.cuda.current_stream().cuda_stream
    N.check(N.lib.sfft_arnoldi_step_multi(len(jobs), arr, code, C.c_void_p(scratch.data_ptr()),
                                          scratch.numel(), C.c_void_p(st)), "sfft_arnoldi_step_multi")
    torch.cuda.synchronize()
    return [(hc.cpu().numpy(), vo.cpu().numpy().astype(np.complex128)) for _, _, vo, hc in keep]


@pytest.mark.parametrize("dtype,tol,orth", [("c128", 1e-12, 1e-13), ("c64", 2e-5, 2e-6)])
def test_arnoldi_step_matches_fp64_gram_schmidt(native, dtype, tol, orth):
    rng = np.random.default_rng(7)
    n, m = 5000, 7                               # 5 chunks of 1024 entries, the last ragged
    V = _basis(rng, n, m)
    if dtype == "c64":                           # the basis as the device stores it
        V = V.astype(np.complex64).astype(np.complex128)
    generic = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    near = V.T @ (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    near = near + 1e-6 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    start = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    jobs = [(V, generic), (V, near), (None, start)]
    out = _step(native, jobs, dtype)
    for (Vj, w), (hcol, vout) in zip(jobs, out):
        if Vj is None:
            assert abs(hcol[0].real - np.linalg.norm(w)) <= tol * np.linalg.norm(w)
            assert np.linalg.norm(vout - w / np.linalg.norm(w)) <= 10 * tol
            continue
        if dtype == "c64":
            w = w.astype(np.complex64).astype(np.complex128)
        h = Vj.conj() @ w                        # exact projections of an orthonormal basis
        r = w - Vj.T @ h
        # projections and residual norm, relative to ||w||
        assert np.abs(hcol[:m] - h).max() <= 10 * tol * np.linalg.norm(w)
        assert abs(hcol[m].real - np.linalg.norm(r)) <= 10 * tol * np.linalg.norm(w)
        # the new basis vector: unit norm and orthogonal to the basis
        assert abs(np.linalg.norm(vout) - 1.0) <= 10 * tol
        assert np.abs(Vj.conj() @ vout).max() <= orth
        # Arnoldi relation for this column: w = V h + hcol[m] vout
        assert np.linalg.norm(w - Vj.T @ hcol[:m] - hcol[m].real * vout) <= 10 * tol * np.linalg.norm(w)
    # bitwise independent of the other jobs in the call
    for job, (hcol, vout) in zip(jobs, out):
        alone = _step(native, [job], dtype)[0]
        assert np.array_equal(alone[0], hcol) and np.array_equal(alone[1], vout)
