"""GPU: a seeded sweep of mixed configurations against the FP64 oracle.

Each case draws the number of levels (1..4), level sizes from the
length-specialised and runtime-length kernels (odd and even, with prime
factors 2, 3, 5, 7), the block size (1..4), general or mirrored symbol
storage (a random even/odd pattern per component and level), the dtype, the
number of right-hand sides and the schedule; it compares the product with
the oracle's embedding (complex128 <= 1e-12, complex64 <= 1e-5 relative L2),
checks that the 2^k per-device shares for a random k sum to it and the
adjoint against the oracle's product with t^H(r) = t(-r)^H. Random sets of
these problems then run as batches in every graph form."""

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
SIZES = [2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 14, 15, 16, 20, 21, 24, 25, 28, 32, 35, 36, 40, 48, 49, 64, 80, 96,
         100, 128, 160, 192, 256, 384]
SCHEDULES = ["auto", "breadth", "depth", "slab"]
NCASE = 120


def _draw(i):
    rng = np.random.default_rng(7000 + i)
    d = int(rng.integers(1, 5))
    cap = {1: 4096, 2: 6000, 3: 6000, 4: 3000}[d]  # grid points, so the oracle stays fast
    while True:
        grid = tuple(int(rng.choice(SIZES)) for _ in range(d))
        if math.prod(grid) <= cap and math.prod(grid) > 1:
            break
    b = int(rng.integers(1, 5))
    mirrored = bool(rng.integers(0, 2))
    dtype = ["c128", "c64"][int(rng.integers(0, 2))]
    nrhs = int(rng.integers(1, 4))
    sched = SCHEDULES[int(rng.integers(0, len(SCHEDULES)))]
    k = int(rng.integers(1, d)) if d > 1 else 0
    return dict(grid=grid, b=b, mirrored=mirrored, dtype=dtype, nrhs=nrhs, sched=sched, k=k, seed=7100 + i)


@pytest.fixture(scope="module")
def sf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_17981_amd as sf
    return sf


@pytest.mark.parametrize("i", range(NCASE))
def test_sweep_case(sf, i, monkeypatch):
    c = _draw(i)
    grid, b, d = c["grid"], c["b"], len(c["grid"])
    print(f"[case] sweep {i}: {c}", flush=True)
    sys.stdout.flush()
    monkeypatch.setenv("SFFT_SLAB_MB", "0.001")  # several slabs even on these small grids
    par = None
    if c["mirrored"]:
        par = np.random.default_rng(c["seed"]).integers(1, 3, (b, b, d)).astype(np.int32)
        coeffs = wl.parity_coeffs(c["seed"], grid, b, par)
    else:
        coeffs = wl.iid_coeffs(c["seed"], grid, b)
    x = wl.vectors(c["seed"] + 1, grid, b, c["nrhs"])
    want = oracle.embed_matvec(coeffs, x)
    plan = sf.Plan(grid, b, torch.from_numpy(coeffs).cuda(), dtype=c["dtype"], max_nrhs=c["nrhs"],
                   schedule=c["sched"], parity=par)
    assert plan.info()["compressed"] == int(c["mirrored"])
    xd = torch.from_numpy(x.astype(NP[c["dtype"]])).cuda()
    y = plan.apply(xd, workspace=plan.alloc_workspace(c["nrhs"]))
    torch.cuda.synchronize()
    err = wl.relative_l2(y.cpu().numpy().astype(np.complex128), want)
    assert err <= TOL[c["dtype"]], ("apply", err)
    # the per-device shares of a 2^k-way split by branch (k below the plan's
    # levels; levels of size 1 are not drawn)
    k = min(c["k"], sum(v > 1 for v in grid) - 1)
    total = None
    for prefix in range(1 << k):
        sh = plan.apply_subtree(k, prefix, xd)
        total = sh.clone() if total is None else total + sh
    torch.cuda.synchronize()
    err = wl.relative_l2(total.cpu().numpy().astype(np.complex128), want)
    assert err <= TOL[c["dtype"]], ("shares", k, err)
    # the adjoint from the same symbols: generator t^H(r) = t(-r)^H
    plan.enable_adjoint()
    yh = plan.apply(xd, workspace=plan.alloc_workspace(c["nrhs"]), adjoint=True)
    torch.cuda.synchronize()
    err = wl.relative_l2(yh.cpu().numpy().astype(np.complex128),
                         oracle.embed_matvec(oracle.adjoint_coeffs(coeffs), x))
    assert err <= TOL[c["dtype"]], ("adjoint", err)
    plan.close()


NBATCH = 12


@pytest.mark.parametrize("j", range(NBATCH))
def test_sweep_batch(sf, j, monkeypatch):
    """A random set of 2 to 6 of the sweep's problems in one sfft_apply_multi
    call, in each graph form (the library's timed choice, per-problem chains,
    grouped lanes), replayed three times: every output equals the problem's
    own apply bit for bit."""
    rng = np.random.default_rng(9000 + j)
    picks = [int(v) for v in rng.choice(NCASE, size=int(rng.integers(2, 7)), replace=False)]
    print(f"[case] batch sweep {j}: cases {picks}", flush=True)
    monkeypatch.setenv("SFFT_SLAB_MB", "0.001")
    plans, xs, singles = [], [], []
    for i in picks:
        c = _draw(i)
        grid, b, d = c["grid"], c["b"], len(c["grid"])
        par = None
        if c["mirrored"]:
            par = np.random.default_rng(c["seed"]).integers(1, 3, (b, b, d)).astype(np.int32)
            coeffs = wl.parity_coeffs(c["seed"], grid, b, par)
        else:
            coeffs = wl.iid_coeffs(c["seed"], grid, b)
        plan = sf.Plan(grid, b, torch.from_numpy(coeffs).cuda(), dtype=c["dtype"], max_nrhs=c["nrhs"],
                       schedule=c["sched"], parity=par)
        x = torch.from_numpy(wl.vectors(c["seed"] + 1, grid, b, c["nrhs"]).astype(NP[c["dtype"]])).cuda()
        plans.append(plan)
        xs.append(x)
        singles.append(plan.apply(x, workspace=plan.alloc_workspace(c["nrhs"])))
    torch.cuda.synchronize()
    ws = torch.empty(max(sf.workspace_size_multi(plans, [x.shape[0] for x in xs]), 1), dtype=torch.uint8,
                     device="cuda")
    for form in ("auto", "chains", "grouped"):
        if form == "auto":
            monkeypatch.delenv("SFFT_BATCH_MODE", raising=False)
        else:
            monkeypatch.setenv("SFFT_BATCH_MODE", form)
        ys = [torch.zeros_like(x) for x in xs]
        for rep in range(3):
            for y in ys:
                y.zero_()
            torch.cuda.synchronize()
            sf.apply_multi(plans, xs, ys, workspace=ws)
            torch.cuda.synchronize()
            for i, (y, ysingle) in enumerate(zip(ys, singles)):
                assert torch.equal(y, ysingle), (form, rep, picks[i])
    for p in plans:
        p.close()
