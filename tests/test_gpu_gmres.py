"""GPU: restarted GMRES(m) with FP64 iterative refinement on the scattering
operator A = I - diag(chi) T (sfft_gmres_solve), checked with the FP64 oracle's
product: the returned residual is the true one and meets the tolerance."""

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


def _ball_chi(n, b, radius, amp):
    """Susceptibility amp on a ball of the given radius around the grid centre, 0 elsewhere."""
    idx = np.indices(n)
    r2 = sum((idx[l] - n[l] / 2) ** 2 for l in range(len(n)))
    chi = np.zeros((b,) + tuple(n), dtype=np.complex128)
    chi[:, r2 <= radius * radius] = amp
    return chi


def _oracle_residual(coeffs, chi, rhs, x):
    ax = x - chi * oracle.embed_matvec(coeffs, x[None])[0]
    return np.linalg.norm((rhs - ax).ravel()) / np.linalg.norm(rhs.ravel())


@pytest.mark.parametrize("lo_dtype,m,tol", [("c64", 20, 1e-6), ("c64", 20, 1e-10), ("c128", 30, 1e-11)])
def test_gmres_green_32(sf, lo_dtype, m, tol):
    """32^3 grid, 3x3 Green blocks (k = 0.7), chi = 0.05 (1 + 0.5i) on a ball of
    radius 5 (515 grid points): restarts happen (m = 20 < the ~30 steps the
    problem needs), complex64 Krylov steps reach 1e-10 through the FP64
    refinement, and the oracle's A x confirms the reported residual."""
    n, b = (32, 32, 32), 3
    coeffs = wl.green_coeffs(n, 0.7)
    chi = _ball_chi(n, b, 5, 0.05 * (1 + 0.5j))
    rhs = wl.vectors(503, n, b, 1)[0]
    cd = torch.from_numpy(coeffs).cuda()
    hi = sf.Plan(n, b, cd, dtype="c128")
    lo = hi if lo_dtype == "c128" else sf.Plan(n, b, cd, dtype="c64", parity=wl.green_parity(3))
    print(f"[case] gmres n={n} lo={lo_dtype} m={m} tol={tol}", flush=True)
    x, info = sf.gmres_solve(lo, hi, torch.from_numpy(chi).cuda(), torch.from_numpy(rhs).cuda(), m=m,
                             max_cycles=40, tol=tol)
    torch.cuda.synchronize()
    print(f"[case] gmres info {info}", flush=True)
    assert info["converged"] and info["rel_residual"] <= tol
    if m < 30:
        assert info["cycles"] >= 2  # restarted
    res = _oracle_residual(coeffs, chi, rhs, x.cpu().numpy())
    assert res <= 1.05 * tol + 1e-14, res
    assert abs(res - info["rel_residual"]) <= 1e-3 * res + 1e-14
    hi.close()
    if lo is not hi:
        lo.close()


def test_gmres_trivial_cases(sf):
    """chi = 0 (A = I) gives x = b with at most two complex64 products (one
    step leaves the complex64 rounding of b / ||b||, which one more step, in
    the same cycle or after an FP64 restart, removes); b = 0 gives x = 0 with
    nothing to do; a wrong plan pairing or workspace is refused."""
    n, b = (8, 6, 10), 3
    coeffs = wl.green_coeffs(n, 0.9)
    cd = torch.from_numpy(coeffs).cuda()
    hi = sf.Plan(n, b, cd, dtype="c128")
    lo = sf.Plan(n, b, cd, dtype="c64")
    rhs = torch.from_numpy(wl.vectors(504, n, b, 1)[0]).cuda()
    zero = torch.zeros_like(rhs)
    x, info = sf.gmres_solve(lo, hi, zero, rhs, m=5, tol=1e-12)
    assert info["converged"] and info["cycles"] <= 2 and info["matvecs"] <= 2, info
    assert torch.allclose(x, rhs, rtol=0, atol=1e-11 * rhs.abs().max().item())
    x, info = sf.gmres_solve(lo, hi, zero, zero, m=5, tol=1e-12)
    assert info["converged"] and info["matvecs"] == 0 and torch.count_nonzero(x) == 0
    other = sf.Plan((8, 6, 12), b, torch.from_numpy(wl.green_coeffs((8, 6, 12), 0.9)).cuda(), dtype="c128")
    with pytest.raises(sf.SfftError, match="INVALID_ARG"):
        sf.gmres_solve(lo, other, zero, rhs)
    with pytest.raises(sf.SfftError, match="INVALID_ARG"):
        sf.gmres_solve(hi, lo, zero, rhs)  # the residual plan must be complex128
    with pytest.raises(sf.SfftError, match="workspace too small"):
        sf.gmres_solve(lo, hi, zero, rhs, workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    for p in (hi, lo, other):
        p.close()


def test_gmres_on_a_long_level(sf):
    """A one-level 4096-point problem (carried as two plan levels in both
    plans) with a decaying scalar kernel and chi = 0.1 on a window: the
    complex64 / complex128 plan pair is accepted and the oracle's A x confirms
    the residual."""
    n, b = (4096,), 1
    r = np.arange(-(n[0] - 1), n[0])
    coeffs = (np.exp(0.9j * np.abs(r)) / (1.0 + np.abs(r)))[None, None].astype(np.complex128)
    chi = np.zeros((b,) + n, dtype=np.complex128)
    chi[:, 1000:3000] = 0.1
    rhs = wl.vectors(505, n, b, 1)[0]
    cd = torch.from_numpy(coeffs).cuda()
    hi = sf.Plan(n, b, cd, dtype="c128")
    lo = sf.Plan(n, b, cd, dtype="c64")
    print(f"[case] gmres long level n={n}", flush=True)
    x, info = sf.gmres_solve(lo, hi, torch.from_numpy(chi).cuda(), torch.from_numpy(rhs).cuda(), m=30,
                             max_cycles=40, tol=1e-9)
    torch.cuda.synchronize()
    print(f"[case] gmres info {info}", flush=True)
    assert info["converged"] and info["rel_residual"] <= 1e-9
    res = _oracle_residual(coeffs, chi, rhs, x.cpu().numpy())
    assert res <= 1.05e-9 + 1e-14, res
    hi.close()
    lo.close()
