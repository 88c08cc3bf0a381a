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


def _run(sf, coeffs, x, dtype, method="split", schedule="auto", parity=None, info=None):
    n = oracle.grid_of(coeffs)
    b = coeffs.shape[0]
    _say(f"n={n} b={b} dtype={dtype} method={method} sched={schedule} nrhs={x.shape[0]} "
         f"mirrored={parity is not None}")
    plan = sf.Plan(n, b, torch.from_numpy(coeffs).cuda(), dtype=dtype, method=method,
                   max_nrhs=x.shape[0], schedule=schedule, parity=parity)
    if info is not None:
        info.update(plan.info())
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
    ((2, 3, 2, 2, 4, 2), 1), ((2, 2, 3, 2, 2, 5), 3),  # d = 6, the most levels a plan takes
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid,b", SMALL)
def test_split_matches_dense_small(sf, grid, b, dtype, monkeypatch):
    # slab schedule with the smallest slabs (a few level-1 indices each, the
    # last one ragged): many slab walks per product
    monkeypatch.setenv("SFFT_SLAB_MB", "0.000001")
    coeffs = wl.iid_coeffs(7, grid, b)
    x = wl.vectors(8, grid, b, 2)
    want = oracle.dense_matvec(coeffs, x) if math.prod(grid) * b <= 4096 else \
        oracle.embed_matvec(coeffs, x)
    for sched in ("breadth", "depth", "slab"):
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


def test_multi_rhs_and_depth_schedule(sf, monkeypatch):
    monkeypatch.setenv("SFFT_SLAB_MB", "0.02")  # slabs of a few level-1 indices at 5 RHS
    grid, b = (12, 10, 16), 3
    coeffs = wl.iid_coeffs(12, grid, b)
    x = wl.vectors(13, grid, b, 5)
    want = oracle.embed_matvec(coeffs, x)
    for dtype in ("c128", "c64"):
        for sched in ("breadth", "depth", "slab"):
            got = _run(sf, coeffs, x, dtype, "split", sched)
            assert wl.relative_l2(got, want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid,b", [((256, 128, 4), 1), ((6, 4, 128), 3), ((8, 256), 3), ((128, 6, 10), 3),
                                    ((6, 1024), 3), ((1024, 10), 1), ((512, 40), 3), ((1024, 40), 1)])
def test_long_levels_match_oracle(sf, grid, b, dtype):
    """Levels of length 128 and more in every position: strided passes of those
    lengths form their split phases from one per-lane value, leaves of those
    lengths use the multiply-add butterflies, block product and merge, and
    leaves of length 1024 transform their pencils one after another through
    one LDS row, and strided passes of length 512 and 1024, whose tiles are
    narrower than a 128-byte line, run in XCD-contiguous order (512 x 40 and
    1024 x 40: 45 and 20 tiles, grids rounded up to a multiple of 8); every
    output against the FP64 oracle, both schedules."""
    coeffs = wl.green_coeffs(grid, 0.8) if b == 3 and len(grid) == 3 else wl.iid_coeffs(61, grid, b)
    x = wl.vectors(62, grid, b, 2)
    want = oracle.embed_matvec(coeffs, x)
    for sched in ("breadth", "depth"):
        got = _run(sf, coeffs, x, dtype, "split", sched)
        err = wl.relative_l2(got, want)
        _say(f"long levels {grid} b={b} {dtype} {sched} rel_l2={err:.3e}")
        assert err <= TOL[dtype], (sched, err)


MIXED_RADIX = [((6, 80), 3), ((96, 10), 1), ((10, 96), 3), ((80, 12), 1), ((384, 6), 3), ((6, 384), 1),
               ((4, 80, 96), 3), ((96, 6, 80), 1), ((384, 4, 6), 3)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid,b", MIXED_RADIX)
def test_mixed_radix_levels_match_oracle(sf, grid, b, dtype):
    """Levels of length 80 ([2,8,5] passes, [5,4,4] leaf), 96 ([4,8,3] / [2,4,4,3])
    and 384 ([4,8,4,3] / [2,4,4,4,3]) in the strided and the leaf position, whose
    FP64 symbols come from 160-, 192- and 768-point transforms; these are the
    lengths of the uneven-grid batch (96 x 80 x 64, 512 x 384) and of the 96^3
    serving grid. Every output against the FP64 oracle, both schedules."""
    coeffs = wl.iid_coeffs(71, grid, b)
    x = wl.vectors(72, grid, b, 2)
    want = oracle.embed_matvec(coeffs, x)
    for sched in ("breadth", "depth"):
        got = _run(sf, coeffs, x, dtype, "split", sched)
        err = wl.relative_l2(got, want)
        _say(f"mixed radix {grid} b={b} {dtype} {sched} rel_l2={err:.3e}")
        assert err <= TOL[dtype], (sched, err)
    got = _run(sf, coeffs, x, dtype, "embed")
    assert wl.relative_l2(got, want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid", [(6, 80), (96, 10), (384, 6), (6, 384), (4, 80, 96), (96, 6, 80)])
def test_mixed_radix_levels_mirrored(sf, grid, dtype):
    """Green blocks stored mirrored (Section II.C) on levels of length 80, 96 and
    384: the leaf's mirror reads (bin M > n read as 2n - M) on odd lengths of the
    even-bin and odd-bin halves, both schedules."""
    coeffs = wl.green_coeffs(grid, 0.6)
    x = wl.vectors(73, grid, 3, 2)
    want = oracle.embed_matvec(coeffs, x)
    for sched in ("breadth", "depth"):
        info = {}
        got = _run(sf, coeffs, x, dtype, "split", sched, parity=wl.green_parity(len(grid)), info=info)
        assert info["compressed"] == 1
        err = wl.relative_l2(got, want)
        _say(f"mixed radix mirrored {grid} {dtype} {sched} rel_l2={err:.3e}")
        assert err <= TOL[dtype], (sched, err)


@pytest.mark.parametrize("grid,nrhs", [((64, 64, 64), 16), ((64, 24, 10), 401)])
def test_large_launch_matches_single_rhs_applies(sf, grid, nrhs):
    """b=3, complex64, breadth-first, many right-hand sides: 64^3 with 16 of them
    runs level-2 passes of 12288 workgroups, 64 x 24 x 10 with 401 passes of 9023
    and 24060 (not multiples of 8: the grids are rounded up and 1 and 4 work items
    are past the end); all use the XCD-contiguous block order, and the leaf takes several
    right-hand sides per symbol fetch; the single-RHS applies' passes are small
    launches of 128-lane workgroups (16-pencil tiles at length 64) where the
    many-RHS passes take 256 lanes (32 pencils). None of this changes any entry's
    arithmetic, so
    every right-hand side must equal its own single-RHS apply (dispatch order, one
    right-hand side per leaf lane group) bit for bit: a tile skipped or done twice
    would not. The first right-hand side is also checked against the FP64 oracle."""
    coeffs = wl.green_coeffs(grid, 0.7) if grid == (64, 64, 64) else wl.iid_coeffs(41, grid, 3)
    x = wl.vectors(42, grid, 3, nrhs)
    _say(f"block order n={grid} nrhs={nrhs}")
    plan = sf.Plan(grid, 3, torch.from_numpy(coeffs).cuda(), dtype="c64", max_nrhs=nrhs, schedule="breadth")
    xd = torch.from_numpy(x.astype(np.complex64)).cuda()
    ws = plan.alloc_workspace(nrhs)
    y = plan.apply(xd, workspace=ws)
    for r in range(nrhs):
        y1 = plan.apply(xd[r:r + 1].contiguous(), workspace=ws)
        assert torch.equal(y[r:r + 1], y1), r
    torch.cuda.synchronize()
    got = y[:1].cpu().numpy().astype(np.complex128)
    plan.close()
    want = oracle.embed_matvec(coeffs, x[:1])
    assert wl.relative_l2(got, want) <= TOL["c64"]


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


def _odd_scalar_coeffs(n, seed):
    """Scalar generator odd along every level: prod_l sgn(r_l) * g(|r|)."""
    rng = np.random.default_rng(seed)
    r = wl.offsets(n)
    dist = np.sqrt(sum(np.asarray(v, dtype=float) ** 2 for v in r))
    g = np.cos(1.1 * dist) + 1j * np.sin(0.4 * dist + rng.standard_normal())
    sgn = np.ones(dist.shape)
    for v in r:
        sgn = sgn * np.sign(v)
    return (sgn * g)[None, None].astype(np.complex128)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid", [(6, 10, 12), (5, 12, 40), (16, 16, 16), (10, 12)])
def test_mirrored_symbols_green(sf, grid, dtype, monkeypatch):
    """Green blocks with symbols stored mirrored (Section II.C): same product,
    every schedule (the slab one with slabs of a few level-1 indices: the
    leaf reads the mirrored rows from a slab's pencil offset)."""
    monkeypatch.setenv("SFFT_SLAB_MB", "0.000001")
    coeffs = wl.green_coeffs(grid, 0.7)
    x = wl.vectors(21, grid, 3, 2)
    want = oracle.embed_matvec(coeffs, x)
    par = wl.green_parity(len(grid))
    for sched in ("breadth", "depth", "slab"):
        info = {}
        got = _run(sf, coeffs, x, dtype, "split", sched, parity=par, info=info)
        assert info["compressed"] == 1
        esz = 8 if dtype == "c64" else 16
        # Green blocks are symmetric: 6 stored components of 9
        assert info["block_symmetry"] == 1
        row = info["mirror_row"]  # n + 1, or n + E/2 with lane pairs
        assert grid[-1] + 1 <= row <= grid[-1] + max(1, grid[-1] // 2)
        assert info["symbol_bytes"] == 6 * math.prod(v + 1 for v in grid[:-1]) * row * esz
        assert wl.relative_l2(got, want) <= TOL[dtype], sched


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid", [(6, 10, 12), (8, 5, 16)])
def test_mirrored_symbols_skew(sf, grid, dtype):
    coeffs = wl.skew_coeffs(grid, 1.3)
    x = wl.vectors(22, grid, 3, 1)
    want = oracle.embed_matvec(coeffs, x)
    got = _run(sf, coeffs, x, dtype, "split", parity=wl.skew_parity(3))
    assert wl.relative_l2(got, want) <= TOL[dtype]


@pytest.mark.parametrize("grid", [(5, 6), (12, 10, 3), (40,)])
def test_mirrored_symbols_odd_scalar(sf, grid):
    coeffs = _odd_scalar_coeffs(grid, 5)
    x = wl.vectors(23, grid, 1, 2)
    want = oracle.dense_matvec(coeffs, x)
    par = np.full((1, 1, len(grid)), wl.ODD, dtype=np.int32)
    got = _run(sf, coeffs, x, "c128", "split", parity=par)
    assert wl.relative_l2(got, want) <= 1e-12
    # a declared symmetry that the coefficients do not have is refused at
    # plan creation (checked exactly on the device), naming the level
    bad = np.full((1, 1, len(grid)), wl.EVEN, dtype=np.int32)
    with pytest.raises(sf.SfftError, match="INVALID_ARG.*level 1"):
        sf.Plan(grid, 1, torch.from_numpy(coeffs).cuda(), dtype="c128", parity=bad)
    # one level wrong, the others right: still refused
    bad = par.copy()
    bad[0, 0, -1] = wl.EVEN
    with pytest.raises(sf.SfftError, match=f"level {len(grid)}"):
        sf.Plan(grid, 1, torch.from_numpy(coeffs).cuda(), dtype="c128", parity=bad)


def test_declared_parity_checked_exactly(sf):
    """The parity check is exact: a single coefficient changed by one ulp
    breaks it, at creation and at update (where the plan keeps its symbols)."""
    grid = (6, 10, 12)
    green = wl.green_coeffs(grid, 0.9)
    par = wl.green_parity(3)
    near = green.copy()
    near[0, 1, 2, 3, 4] = np.nextafter(near[0, 1, 2, 3, 4].real, np.inf) + 1j * near[0, 1, 2, 3, 4].imag
    with pytest.raises(sf.SfftError, match="component \\(0, 1\\)"):
        sf.Plan(grid, 3, torch.from_numpy(near).cuda(), dtype="c64", parity=par)
    x = torch.from_numpy(wl.vectors(24, grid, 3, 1).astype(np.complex64)).cuda()
    plan = sf.Plan(grid, 3, torch.from_numpy(green).cuda(), dtype="c64", parity=par)
    y0 = plan.apply(x)
    # block-symmetric but with one (0,1)/(1,0) pair perturbed alike: same
    # block symmetry, broken parity
    near[1, 0, 2, 3, 4] = near[0, 1, 2, 3, 4]
    with pytest.raises(sf.SfftError, match="INVALID_ARG"):
        plan.update(torch.from_numpy(near).cuda())
    assert torch.equal(plan.apply(x), y0)
    plan.close()


def _blocks_with_symmetry(seed, grid, b, kind):
    c = wl.iid_coeffs(seed, grid, b)
    if kind == "sym":
        c = c + np.swapaxes(c, 0, 1)
    elif kind == "anti":
        c = c - np.swapaxes(c, 0, 1)
    return c


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("b", [2, 4])
@pytest.mark.parametrize("grid", [(24,), (10, 12), (6, 10, 12), (16, 8, 64), (4, 3, 2, 5)])
def test_block_sizes_two_and_four(sf, grid, b, dtype):
    """b = 2 and b = 4 blocks (Algorithm 1's block data T[bId] for any block
    size): general blocks and exactly (anti)symmetric ones, whose b(b+1)/2
    stored components the plan detects, against the FP64 oracle, both
    schedules and the embedding baseline."""
    x = wl.vectors(81, grid, b, 2)
    for kind, bs in (("iid", 0), ("sym", 1), ("anti", 2)):
        coeffs = _blocks_with_symmetry(80, grid, b, kind)
        want = oracle.dense_matvec(coeffs, x) if math.prod(grid) * b <= 4096 else oracle.embed_matvec(coeffs, x)
        for sched in ("breadth", "depth"):
            info = {}
            got = _run(sf, coeffs, x, dtype, "split", sched, info=info)
            assert info["block_symmetry"] == bs, kind
            err = wl.relative_l2(got, want)
            _say(f"b={b} {grid} {kind} {dtype} {sched} rel_l2={err:.3e}")
            assert err <= TOL[dtype], (kind, sched, err)
        got = _run(sf, coeffs, x, dtype, "embed")
        assert wl.relative_l2(got, want) <= TOL[dtype], (kind, "embed")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("b", [1, 2, 4])
@pytest.mark.parametrize("grid", [(10, 12), (6, 10, 12), (5, 8, 16)])
def test_mirrored_storage_any_block_size(sf, grid, b, dtype):
    """Mirrored symbols (Section II.C) for blocks of 1, 2 and 4 with a random
    even/odd pattern per (component, level), coefficients exactly of that
    parity."""
    d = len(grid)
    par = np.random.default_rng(82 + b).integers(1, 3, (b, b, d)).astype(np.int32)
    coeffs = wl.parity_coeffs(83, grid, b, par)
    x = wl.vectors(84, grid, b, 2)
    want = oracle.embed_matvec(coeffs, x)
    for sched in ("breadth", "depth"):
        info = {}
        got = _run(sf, coeffs, x, dtype, "split", sched, parity=par, info=info)
        assert info["compressed"] == 1
        err = wl.relative_l2(got, want)
        _say(f"mirrored b={b} {grid} {dtype} {sched} rel_l2={err:.3e}")
        assert err <= TOL[dtype], (sched, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_green_64_mirrored_full_size(sf, green64, dtype):
    """The symmetric-kernel variant of the 64^3 Green workload."""
    coeffs, x, want, _, _ = green64
    info = {}
    got = _run(sf, coeffs, x, dtype, "split", parity=wl.green_parity(3), info=info)
    err = wl.relative_l2(got, want)
    _say(f"green64 mirrored {dtype} rel_l2={err:.3e} symbol_bytes={info['symbol_bytes']}")
    # lane pairs: 64 + E/2 entries per last-level row (E = 8 entries per lane
    # in the complex64 leaf, 4 in the complex128 one) instead of 65
    row = 68 if dtype == "c64" else 66
    assert info["mirror_row"] == row
    assert info["symbol_bytes"] == 6 * 65 ** 2 * row * (8 if dtype == "c64" else 16)
    assert err <= TOL[dtype]


@pytest.fixture(scope="module")
def large_golden():
    """FP64 oracle values of the 256 x 256 x 128 products at 128 grid points
    (tests/golden/make_large_rows.py: corners, both ends of every axis, first
    and last pencils of leaf tiles, random interior points)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_256_rows.npz")
    g = np.load(path)
    cfg = wl.LARGE_256
    assert tuple(g["n"]) == tuple(cfg["n"]) and float(g["k"]) == cfg["k"] and int(g["seed_x"]) == cfg["seed_x"]
    return {k: g[k] for k in g.files}


def _large_case(sf, coeffs, x, pts, dtype, parity, schedule):
    n = wl.LARGE_256["n"]
    _say(f"large n={n} dtype={dtype} mirrored={parity is not None} sched={schedule} nrhs={x.shape[0]}")
    plan = sf.Plan(n, 3, torch.from_numpy(coeffs).cuda(), dtype=dtype, parity=parity,
                   max_nrhs=x.shape[0], schedule=schedule)
    info = plan.info()
    xd = torch.from_numpy(x.astype(NP[dtype])).cuda()
    y = plan.apply(xd, workspace=plan.alloc_workspace(x.shape[0]))
    torch.cuda.synchronize()
    idx = torch.from_numpy(np.ravel_multi_index(pts.T, n)).cuda()
    got = y.reshape(x.shape[0], 3, -1)[:, :, idx].cpu().numpy().astype(np.complex128)
    plan.close()
    del xd, y
    torch.cuda.empty_cache()
    return got, info


def test_large_green_and_skew_full_size(sf, large_golden):
    """256 x 256 x 128 grid, 3x3 blocks, 8 right-hand sides, complex64 (FP64 symbols):
    Green k=1.3 and the skew-symmetric kernel, general and mirrored symbols, both
    schedules, each against the stored FP64 oracle values at 128 grid points of
    every right-hand side (per-point relative error too, so one wrong pencil or
    tile cannot hide in the norm)."""
    cfg = wl.LARGE_256
    n, nrhs = cfg["n"], cfg["nrhs"]
    pts = large_golden["points"]
    x = wl.vectors(cfg["seed_x"], n, 3, nrhs)
    for name, make, par in (("green", lambda: wl.green_coeffs(n, cfg["k"]), wl.green_parity(3)),
                            ("skew", lambda: wl.skew_coeffs(n, cfg["k"]), wl.skew_parity(3))):
        coeffs = make()
        want = large_golden[name]
        cases = [(None, "depth"), (par, "depth")] if name == "skew" else \
            [(None, "depth"), (None, "breadth"), (par, "depth"), (par, "breadth")]
        for parity, sched in cases:
            got, info = _large_case(sf, coeffs, x, pts, "c64", parity, sched)
            err = wl.relative_l2(got, want)
            scale = np.linalg.norm(want, axis=(0, 1)).max()
            worst = float(np.abs(got - want).max() / scale)
            _say(f"large {name} mirrored={parity is not None} {sched} rel_l2={err:.3e} worst={worst:.3e} "
                 f"symbol_bytes={info['symbol_bytes']} workspace={info['workspace_bytes']}")
            assert err <= 1e-5
            assert worst <= 1e-5
        del coeffs


def test_serving_grid_96(sf):
    """The 96^3 grid of the serving stream (every level of length 96: [4,8,3]
    passes, [2,4,4,3] leaf, 192-point FP64 symbol transforms), 3x3 Green blocks,
    complex64, depth-first as the server runs it, general and mirrored symbols,
    against direct sums at sampled points and the grid's corners."""
    n = (96, 96, 96)
    coeffs = wl.green_coeffs(n, 1.1)
    x = wl.vectors(63, n, 3, 1)
    rng = np.random.default_rng(64)
    corners = np.array([[0, 0, 0], [95, 95, 95], [0, 0, 95], [95, 0, 0], [0, 95, 0], [48, 47, 95]])
    pts = np.concatenate([np.stack([rng.integers(0, 96, 26) for _ in range(3)], axis=1), corners])
    want = oracle.sampled_rows(coeffs, x, pts)
    idx = torch.from_numpy(np.ravel_multi_index(pts.T, n)).cuda()
    for parity in (None, wl.green_parity(3)):
        _say(f"serving grid n={n} mirrored={parity is not None}")
        plan = sf.Plan(n, 3, torch.from_numpy(coeffs).cuda(), dtype="c64", parity=parity, max_nrhs=1,
                       schedule="depth")
        y = plan.apply(torch.from_numpy(x.astype(np.complex64)).cuda())
        got = y.reshape(1, 3, -1)[:, :, idx].cpu().numpy().astype(np.complex128)
        plan.close()
        err = wl.relative_l2(got, want)
        _say(f"serving grid 96^3 mirrored={parity is not None} rel_l2={err:.3e}")
        assert err <= TOL["c64"]


@pytest.mark.parametrize("mirrored", [False, True])
@pytest.mark.parametrize("n", [(1024, 1024), (128, 128, 128)])
def test_largest_serving_grids(sf, n, mirrored):
    """The largest grids of the serving stream, 1024 x 1024 and 128^3, 3x3 Green
    blocks, complex64, depth-first as the server runs them. At 1024^2 the
    length-1024 passes have 4-pencil tiles (XCD-contiguous order), the
    length-1024 leaf runs its pencils one after another through one LDS row,
    and the symbols come from 2048-point FP64 transforms; at 128^3 every level
    has length 128. Checked against direct sums at sampled output points and
    the grid's corners."""
    d = len(n)
    coeffs = wl.green_coeffs(n, 0.9)
    x = wl.vectors(61, n, 3, 1)
    rng = np.random.default_rng(62)
    corners = np.array([[0] * d, [v - 1 for v in n], [0] * (d - 1) + [n[-1] - 1], [n[0] // 2] + [0] * (d - 1)])
    pts = np.concatenate([np.stack([rng.integers(0, v, 12) for v in n], axis=1), corners])
    want = oracle.sampled_rows(coeffs, x, pts)
    _say(f"serving grid n={n} mirrored={mirrored}")
    plan = sf.Plan(n, 3, torch.from_numpy(coeffs).cuda(), dtype="c64",
                   parity=wl.green_parity(d) if mirrored else None, max_nrhs=1, schedule="depth")
    y = plan.apply(torch.from_numpy(x.astype(np.complex64)).cuda())
    idx = torch.from_numpy(np.ravel_multi_index(pts.T, n)).cuda()
    got = y.reshape(1, 3, -1)[:, :, idx].cpu().numpy().astype(np.complex128)
    plan.close()
    del y
    torch.cuda.empty_cache()
    assert wl.relative_l2(got, want) <= TOL["c64"]


# ---------------------------------------------------------------------------
# Degenerate and empty inputs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid,b", [((1, 12, 10), 3), ((6, 1, 8), 1), ((16, 1), 3), ((1, 1, 24), 1)])
def test_levels_of_size_one(sf, grid, b, dtype):
    """A level of size 1 only has offset 0; the product still equals the
    dense definition (the plan drops such levels internally)."""
    coeffs = wl.iid_coeffs(31, grid, b)
    x = wl.vectors(32, grid, b, 2)
    want = oracle.dense_matvec(coeffs, x)
    got = _run(sf, coeffs, x, dtype, "split")
    assert wl.relative_l2(got, want) <= TOL[dtype]
    plan = sf.Plan(grid, b, torch.from_numpy(coeffs).cuda(), dtype=dtype)
    assert plan.info()["n"] == tuple(grid) and plan.info()["d"] == len(grid)
    plan.close()


def test_single_point_grid_is_rejected(sf):
    grid = (1, 1)
    with pytest.raises(sf.SfftError, match="UNSUPPORTED"):
        sf.Plan(grid, 1, torch.from_numpy(wl.iid_coeffs(1, grid, 1)).cuda(), dtype="c64")


def test_empty_batch_is_a_no_op(sf):
    import ctypes as C
    from paper_2406_17981_amd import _native as N
    grid, b = (8, 6, 10), 3
    coeffs = wl.iid_coeffs(41, grid, b)
    plan = sf.Plan(grid, b, torch.from_numpy(coeffs).cuda(), dtype="c64")
    assert plan.workspace_size(0) == 0
    # through the C ABI with NULL buffers
    assert N.lib.sfft_apply(plan.handle, None, None, 0, None, 0, None) == 0
    # through the binding with (0, b, *n) tensors
    x0 = torch.empty((0, b) + grid, dtype=torch.complex64, device="cuda")
    y0 = plan.apply(x0)
    assert tuple(y0.shape) == (0, b) + grid
    # an empty problem inside a batch leaves the others intact
    x = wl.vectors(42, grid, b, 2)
    xd = torch.from_numpy(x.astype(np.complex64)).cuda()
    y = torch.empty_like(xd)
    y_empty = torch.empty_like(x0)
    sf.apply_multi([plan, plan], [x0, xd], [y_empty, y])
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.complex128)
    assert wl.relative_l2(got, oracle.embed_matvec(coeffs, x)) <= TOL["c64"]
    assert N.lib.sfft_apply(plan.handle, None, None, -1, None, 0, None) != 0
    plan.close()


# ---------------------------------------------------------------------------
# Block symmetry of the coefficients (detected exactly at plan creation)
# ---------------------------------------------------------------------------
def _plan_info_and_product(sf, coeffs, x, dtype, parity=None):
    info = {}
    got = _run(sf, coeffs, x, dtype, "split", parity=parity, info=info)
    return info, got


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_block_symmetry_detection_and_products(sf, dtype, monkeypatch):
    grid = (6, 10, 12)
    x = wl.vectors(51, grid, 3, 2)
    green = wl.green_coeffs(grid, 0.8)
    skew = wl.skew_coeffs(grid, 1.1)
    iid = wl.iid_coeffs(52, grid, 3)
    # symmetric except one offset of one pair: not symmetric
    near = green.copy()
    near[0, 1, 3, 4, 5] += 1e-9
    # pair (0, 1) symmetric, pairs with 2 antisymmetric: neither pattern
    mixed = iid.copy()
    mixed[1, 0] = mixed[0, 1]
    mixed[2, 0] = -mixed[0, 2]
    mixed[2, 1] = -mixed[1, 2]
    cases = [("iid", iid, 0, 9), ("green", green, 1, 6), ("skew", skew, 2, 6), ("near", near, 0, 9),
             ("mixed", mixed, 0, 9)]
    general = None  # symbol bytes with all 9 components stored (tiles padded as the leaf needs)
    for name, coeffs, bs, ns in cases:
        info, got = _plan_info_and_product(sf, coeffs, x, dtype)
        general = general or info["symbol_bytes"]
        assert info["block_symmetry"] == bs, name
        assert info["symbol_bytes"] * 9 == general * ns, name
        assert wl.relative_l2(got, oracle.embed_matvec(coeffs, x)) <= TOL[dtype], name
    # the embedding baseline stores the same components
    info_g, info_s = {}, {}
    _run(sf, iid, x, dtype, "embed", info=info_g)
    got = _run(sf, green, x, dtype, "embed", info=info_s)
    assert info_s["block_symmetry"] == 1 and info_s["symbol_bytes"] * 9 == info_g["symbol_bytes"] * 6
    assert wl.relative_l2(got, oracle.embed_matvec(green, x)) <= TOL[dtype]
    # switching the detection off stores all 9 and gives the same product
    monkeypatch.setenv("SFFT_NO_BLOCK_SYMMETRY", "1")
    info, got_off = _plan_info_and_product(sf, green, x, dtype)
    assert info["block_symmetry"] == 0 and info["symbol_bytes"] == general
    monkeypatch.delenv("SFFT_NO_BLOCK_SYMMETRY")
    _, got_on = _plan_info_and_product(sf, green, x, dtype)
    assert wl.relative_l2(got_on, got_off) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_block_symmetry_with_mirrored_storage(sf, dtype):
    grid = (8, 6, 10)
    x = wl.vectors(53, grid, 3, 1)
    for coeffs, par, bs in ((wl.green_coeffs(grid, 0.9), wl.green_parity(3), 1),
                            (wl.skew_coeffs(grid, 1.2), wl.skew_parity(3), 2)):
        info, got = _plan_info_and_product(sf, coeffs, x, dtype, parity=par)
        assert info["compressed"] == 1 and info["block_symmetry"] == bs
        assert wl.relative_l2(got, oracle.embed_matvec(coeffs, x)) <= TOL[dtype]


# ---------------------------------------------------------------------------
# Plan update (new coefficients of the same shape and block symmetry)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("kind,mirrored,method", [("green", False, "split"), ("green", True, "split"),
                                                  ("green", False, "embed"), ("skew", False, "split"),
                                                  ("skew", True, "split")])
def test_plan_update_equals_a_fresh_plan(sf, dtype, kind, mirrored, method):
    """A plan made for the Green (block-symmetric) or skew (block
    antisymmetric) kernel at k=0.7 and updated to k=1.1 gives bit for bit what
    a plan made at k=1.1 gives (the same symbol generation into the same
    layout), and matches the FP64 oracle. Coefficients without the plan's block
    symmetry (i.i.d. blocks) are refused, and the plan keeps its symbols."""
    grid = (16, 12, 10)
    make = wl.green_coeffs if kind == "green" else wl.skew_coeffs
    ca, cb = make(grid, 0.7), make(grid, 1.1)
    par = (wl.green_parity(3) if kind == "green" else wl.skew_parity(3)) if mirrored else None
    x = wl.vectors(55, grid, 3, 2)
    xd = torch.from_numpy(x.astype(NP[dtype])).cuda()
    _say(f"plan update n={grid} dtype={dtype} kind={kind} mirrored={mirrored} method={method}")
    plan = sf.Plan(grid, 3, torch.from_numpy(ca).cuda(), dtype=dtype, parity=par, max_nrhs=2, method=method)
    fresh = sf.Plan(grid, 3, torch.from_numpy(cb).cuda(), dtype=dtype, parity=par, max_nrhs=2, method=method)
    ya = plan.apply(xd)
    plan.update(torch.from_numpy(cb).cuda())
    yb = plan.apply(xd)
    assert torch.equal(yb, fresh.apply(xd))
    assert not torch.equal(ya, yb)
    want = oracle.embed_matvec(cb, x)
    assert wl.relative_l2(yb.cpu().numpy().astype(np.complex128), want) <= TOL[dtype]
    with pytest.raises(sf.SfftError):
        plan.update(torch.from_numpy(wl.iid_coeffs(3, grid, 3)).cuda())
    assert torch.equal(plan.apply(xd), yb)
    assert plan.info()["block_symmetry"] == (1 if kind == "green" else 2)
    torch.cuda.synchronize()
    plan.close()
    fresh.close()


# ---------------------------------------------------------------------------
# Level sizes without length-specialised kernels (runtime-length kernels)
# ---------------------------------------------------------------------------
RUNTIME_LENGTHS = [((7,), 1), ((14, 9), 3), ((21, 10), 2), ((35, 6, 4), 1), ((49, 5), 4), ((9, 15, 25), 3),
                   ((36, 100), 1), ((6, 7, 8), 3), ((12, 343), 1), ((1000,), 2), ((2, 1960), 1), ((28, 3, 14), 4)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid,b", RUNTIME_LENGTHS)
def test_runtime_length_levels_match_oracle(sf, grid, b, dtype):
    """Level sizes with prime factors in {2, 3, 5, 7} but no length-specialised
    kernels (7, 9, 14, 15, 21, 25, 35, 36, 49, 100, 343, 1000, 1960 and the
    FP64 symbol lengths 2 n_l, e.g. 686, 2000, 3920) run on the runtime-length
    kernels (radix 8, 4, 2, 3, 5, 7 stages in LDS), alone and next to
    length-specialised levels; every output against the FP64 oracle, both
    schedules and the embedding baseline."""
    from paper_2406_17981_amd import _native as N
    assert any(N.lib.sfft_length_supported(v) == 2 for v in grid)
    coeffs = wl.iid_coeffs(91, grid, b)
    x = wl.vectors(92, grid, b, 2)
    want = oracle.dense_matvec(coeffs, x) if math.prod(grid) * b <= 4096 else oracle.embed_matvec(coeffs, x)
    for sched in ("breadth", "depth"):
        got = _run(sf, coeffs, x, dtype, "split", sched)
        err = wl.relative_l2(got, want)
        _say(f"runtime length {grid} b={b} {dtype} {sched} rel_l2={err:.3e}")
        assert err <= TOL[dtype], (sched, err)
    got = _run(sf, coeffs, x, dtype, "embed")
    assert wl.relative_l2(got, want) <= TOL[dtype], "embed"


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid", [(14, 9), (7, 21, 5), (25, 6, 49), (15,)])
def test_runtime_length_levels_mirrored(sf, grid, dtype):
    """Mirrored symbols (Section II.C) on runtime-length levels, odd and even
    sizes, b = 3 with a random even/odd pattern and block symmetry."""
    d = len(grid)
    par = np.random.default_rng(93).integers(1, 3, (3, 3, d)).astype(np.int32)
    par = np.maximum(par, np.swapaxes(par, 0, 1))  # symmetric pattern, so symmetric blocks can carry it
    coeffs = wl.parity_coeffs(94, grid, 3, par)
    coeffs = (coeffs + np.swapaxes(coeffs, 0, 1)) / 2
    x = wl.vectors(95, grid, 3, 2)
    want = oracle.embed_matvec(coeffs, x)
    for sched in ("breadth", "depth"):
        info = {}
        got = _run(sf, coeffs, x, dtype, "split", sched, parity=par, info=info)
        assert info["compressed"] == 1 and info["block_symmetry"] == 1
        err = wl.relative_l2(got, want)
        _say(f"runtime length mirrored {grid} {dtype} {sched} rel_l2={err:.3e}")
        assert err <= TOL[dtype], (sched, err)


def test_unsupported_level_sizes(sf):
    """Prime factors outside {2, 3, 5, 7} are refused before any device work,
    naming the size (levels above 2048 are carried as several plan levels:
    tests/test_gpu_long_levels.py)."""
    for grid in ((11,), (8, 22), (4099,)):
        coeffs = torch.zeros((1, 1) + tuple(2 * v - 1 for v in grid), dtype=torch.complex128, device="cuda")
        with pytest.raises(sf.SfftError, match="UNSUPPORTED"):
            sf.Plan(grid, 1, coeffs, dtype="c64")


# ---------------------------------------------------------------------------
# Adjoint: y = T^H x from the plan's symbols conjugated and transposed
# ---------------------------------------------------------------------------
ADJ_CASES = [((10, 12), 1, "iid", None), ((6, 10, 12), 3, "iid", None), ((6, 10, 12), 3, "green", "mirrored"),
             ((8, 6, 10), 3, "skew", "mirrored"), ((8, 6, 10), 3, "skew", None), ((5, 8, 16), 2, "parity", "mirrored"),
             ((4, 3, 2, 5), 4, "iid", None), ((14, 9), 4, "sym", None), ((7, 10), 2, "anti", None)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid,b,kind,storage", ADJ_CASES)
def test_adjoint_matches_oracle(sf, grid, b, kind, storage, dtype):
    """sfft_apply_adjoint against the FP64 oracle's product with the generator
    t^H(r) = t(-r)^H (general, block-symmetric, block-antisymmetric and mirrored
    storage, b = 1..4, a runtime-length level), both schedules and the
    embedding baseline; plus <u, T v> = <T^H u, v> on the device results."""
    d = len(grid)
    par = None
    if kind == "green":
        coeffs, par = wl.green_coeffs(grid, 0.8), wl.green_parity(d)
    elif kind == "skew":
        coeffs, par = wl.skew_coeffs(grid, 1.2), wl.skew_parity(d)
    elif kind == "parity":
        par = np.random.default_rng(96).integers(1, 3, (b, b, d)).astype(np.int32)
        coeffs = wl.parity_coeffs(97, grid, b, par)
    else:
        coeffs = _blocks_with_symmetry(98, grid, b, kind)
    if storage != "mirrored":
        par = None
    x = wl.vectors(99, grid, b, 2)
    want = oracle.embed_matvec(oracle.adjoint_coeffs(coeffs), x)
    want_fwd = oracle.embed_matvec(coeffs, x)
    cd = torch.from_numpy(coeffs).cuda()
    xd = torch.from_numpy(x.astype(NP[dtype])).cuda()
    runs = [("split", "breadth"), ("split", "depth")] + ([("embed", "auto")] if par is None else [])
    for method, sched in runs:
        _say(f"adjoint {grid} b={b} {kind} {storage} {dtype} {method} {sched}")
        plan = sf.Plan(grid, b, cd, dtype=dtype, method=method, parity=par, max_nrhs=2, schedule=sched)
        ws = plan.alloc_workspace(2)
        with pytest.raises(sf.SfftError, match="INVALID_ARG"):
            plan.apply(xd, workspace=ws, adjoint=True)  # not enabled yet
        plan.enable_adjoint()
        assert plan.info()["adjoint_symbol_bytes"] == plan.info()["symbol_bytes"]
        yh = plan.apply(xd, workspace=ws, adjoint=True)
        yf = plan.apply(xd, workspace=ws)
        torch.cuda.synchronize()
        gh = yh.cpu().numpy().astype(np.complex128)
        gf = yf.cpu().numpy().astype(np.complex128)
        plan.close()
        err = wl.relative_l2(gh, want)
        _say(f"adjoint rel_l2={err:.3e}")
        assert err <= TOL[dtype], (method, sched, err)
        assert wl.relative_l2(gf, want_fwd) <= TOL[dtype]
        # <x_1, T x_0> = <T^H x_1, x_0> with the device products
        lhs = np.vdot(x[1], gf[0])
        rhs = np.vdot(gh[1], x[0])
        assert abs(lhs - rhs) <= 10 * TOL[dtype] * np.linalg.norm(x[1]) * np.linalg.norm(gf[0])


def test_adjoint_follows_plan_update(sf):
    """After sfft_plan_update the adjoint symbols are those of the new operator."""
    grid = (16, 12, 10)
    ca, cb = wl.green_coeffs(grid, 0.7), wl.green_coeffs(grid, 1.1)
    ca[0, 0] *= 1 + 0.5j  # no longer Hermitian-like: T^H differs from T
    cb[0, 0] *= 1 - 0.3j
    x = wl.vectors(100, grid, 3, 1)
    plan = sf.Plan(grid, 3, torch.from_numpy(ca).cuda(), dtype="c128", parity=wl.green_parity(3))
    plan.enable_adjoint()
    plan.update(torch.from_numpy(cb).cuda())
    y = plan.apply(torch.from_numpy(x).cuda(), adjoint=True)
    torch.cuda.synchronize()
    want = oracle.embed_matvec(oracle.adjoint_coeffs(cb), x)
    assert wl.relative_l2(y.cpu().numpy(), want) <= 1e-12
    plan.close()


def test_one_plan_on_two_streams_with_distinct_workspaces(sf):
    """A plan is immutable after creation, so applies of one plan on two streams
    at once, each with its own workspace, must give the same bits as
    applies one after another (both schedules)."""
    grid, b = (24, 20, 32), 3
    coeffs = wl.green_coeffs(grid, 0.8)
    xa = torch.from_numpy(wl.vectors(120, grid, b, 2).astype(np.complex64)).cuda()
    xb = torch.from_numpy(wl.vectors(121, grid, b, 2).astype(np.complex64)).cuda()
    for sched in ("depth", "breadth"):
        plan = sf.Plan(grid, b, torch.from_numpy(coeffs).cuda(), dtype="c64", max_nrhs=2, schedule=sched)
        ya_ref = plan.apply(xa, workspace=plan.alloc_workspace(2))
        yb_ref = plan.apply(xb, workspace=plan.alloc_workspace(2))
        torch.cuda.synchronize()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        w1, w2 = plan.alloc_workspace(2), plan.alloc_workspace(2)
        ya, yb = torch.empty_like(xa), torch.empty_like(xb)
        torch.cuda.synchronize()
        for _ in range(20):  # interleaved launches on both streams
            plan.apply(xa, ya, w1, stream=s1)
            plan.apply(xb, yb, w2, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(ya, ya_ref) and torch.equal(yb, yb_ref), sched
        plan.close()
