"""GPU: the out-of-core product (vectors in host memory, the device holding
the plan and slabs only) against the in-core depth-first product (bit for bit:
the same kernels do the same per-pencil work) and the FP64 oracle, with
budgets that force many slabs, uneven last slabs and tile-aligned row slabs."""

import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}
TDT = {"c128": torch.complex128, "c64": torch.complex64}


@pytest.fixture(scope="module")
def sf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_17981_amd as sf
    return sf


CASES = [((24, 20, 32), 3, "green", 2), ((40, 48), 1, "iid", 3), ((10, 12, 6, 8), 2, "iid", 1),
         ((12, 10, 16), 3, "mirrored", 2), ((14, 9, 10), 1, "iid", 2), ((64, 64, 64), 3, "green", 1)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid,b,kind,nrhs", CASES)
def test_out_of_core_matches_in_core(sf, grid, b, kind, nrhs, dtype):
    d = len(grid)
    par = None
    if kind in ("green", "mirrored"):
        coeffs = wl.green_coeffs(grid, 0.9)
        par = wl.green_parity(d) if kind == "mirrored" else None
    else:
        coeffs = wl.iid_coeffs(110, grid, b)
    x = wl.vectors(111, grid, b, nrhs)
    print(f"[case] ooc n={grid} b={b} {kind} nrhs={nrhs} {dtype}", flush=True)
    plan = sf.Plan(grid, b, torch.from_numpy(coeffs).cuda(), dtype=dtype, parity=par, max_nrhs=nrhs,
                   schedule="depth")
    xd = torch.from_numpy(x).to(TDT[dtype]).cuda()
    y_in = plan.apply(xd, workspace=plan.alloc_workspace(nrhs)).cpu()
    xh = torch.from_numpy(x).to(TDT[dtype]).pin_memory()
    vb = xd.numel() * xd.element_size()
    rows8 = 8 * (d - 1) * vb // grid[0] + 7  # row slabs of 8 level-1 indices: many slabs, uneven last one
    ran = 0
    for budget in (rows8, 2 * rows8 + 12345, 4 * vb):
        try:
            _, used = plan.ooc_sizes(nrhs, budget)
        except sf.SfftError as e:  # row slabs start on leaf-tile boundaries: a few grids need more rows
            assert "budget too small" in str(e) and budget < 4 * vb
            continue
        assert used <= budget
        ran += 1
        y = plan.apply_ooc(xh, device_budget=budget)
        torch.cuda.synchronize()
        assert torch.equal(y, y_in), budget
    assert ran >= 2
    want = oracle.embed_matvec(coeffs, x)
    assert wl.relative_l2(y.numpy().astype(np.complex128), want) <= TOL[dtype]
    plan.close()


def test_out_of_core_refusals(sf):
    grid = (16, 12)
    coeffs = torch.from_numpy(wl.iid_coeffs(112, grid, 1)).cuda()
    plan = sf.Plan(grid, 1, coeffs, dtype="c64")
    with pytest.raises(sf.SfftError, match="budget too small"):
        plan.ooc_sizes(1, 64)
    emb = sf.Plan(grid, 1, coeffs, dtype="c64", method="embed")
    with pytest.raises(sf.SfftError, match="UNSUPPORTED"):
        emb.ooc_sizes(1, 1 << 20)
    one = sf.Plan((32,), 1, torch.from_numpy(wl.iid_coeffs(113, (32,), 1)).cuda(), dtype="c64")
    with pytest.raises(sf.SfftError, match="UNSUPPORTED"):
        one.ooc_sizes(1, 1 << 20)
    for p in (plan, emb, one):
        p.close()


@pytest.mark.parametrize("grid,b", [((4096,), 1), ((3072, 6), 2)])
def test_out_of_core_with_a_long_level(sf, grid, b):
    """A level above 2048 is carried as two plan levels, so even a one-level
    grid has the level-1 split the out-of-core product works on."""
    coeffs = wl.iid_coeffs(114, grid, b)
    x = wl.vectors(115, grid, b, 2)
    print(f"[case] ooc long level n={grid} b={b}", flush=True)
    plan = sf.Plan(grid, b, torch.from_numpy(coeffs).cuda(), dtype="c128", max_nrhs=2, schedule="depth")
    xd = torch.from_numpy(x).cuda()
    y_in = plan.apply(xd, workspace=plan.alloc_workspace(2)).cpu()
    xh = torch.from_numpy(x).pin_memory()
    vb = xd.numel() * xd.element_size()
    ran = 0
    for budget in (vb // 2, vb, 4 * vb):
        try:
            _, used = plan.ooc_sizes(2, budget)
        except sf.SfftError as e:
            assert "budget too small" in str(e) and budget < 4 * vb
            continue
        assert used <= budget
        ran += 1
        y = plan.apply_ooc(xh, device_budget=budget)
        torch.cuda.synchronize()
        assert torch.equal(y, y_in), budget
    assert ran >= 1
    assert wl.relative_l2(y_in.numpy(), oracle.embed_matvec(coeffs, x)) <= TOL["c128"]
    plan.close()
