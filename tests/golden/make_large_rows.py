"""Writes tests/golden/large_256_rows.npz: FP64 oracle values of the
256 x 256 x 128, 3x3-block, 8-right-hand-side products at sampled grid points.

    python tests/golden/make_large_rows.py [--workers N]

Only ``oracle`` (the circulant-embedding product, computed one right-hand side
at a time to bound host memory at about 30 GB) and the seeded generators in
``workloads`` are used; nothing from the HIP path. The points are chosen so a
wrong tile, pencil or boundary shows: the eight grid corners, both ends of
every axis with the other coordinates drawn at random, pencils of both
parities along the second axis (a leaf tile of the length-128 innermost level
holds two neighbouring pencils), and random interior points.
"""

from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import oracle.toeplitz as OT  # noqa: E402
import workloads as wl  # noqa: E402

OUT = os.path.join(HERE, "large_256_rows.npz")


def sample_points(n, seed=5021):
    rng = np.random.default_rng(seed)
    pts = []
    for c in range(8):  # corners
        pts.append([(n[l] - 1) if (c >> l) & 1 else 0 for l in range(3)])
    for l in range(3):  # both ends of every axis
        for end in (0, n[l] - 1):
            for _ in range(4):
                p = [int(rng.integers(0, v)) for v in n]
                p[l] = end
                pts.append(p)
    for par in (0, 1):  # first and last pencil of leaf tiles (second axis even / odd)
        for _ in range(24):
            p = [int(rng.integers(0, v)) for v in n]
            p[1] = 2 * int(rng.integers(0, n[1] // 2)) + par
            pts.append(p)
    while len(pts) < 128:
        pts.append([int(rng.integers(0, v)) for v in n])
    return np.asarray(pts, dtype=np.int64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=min(16, len(os.sched_getaffinity(0))))
    a = ap.parse_args()
    OT.set_workers(a.workers)
    cfg = wl.LARGE_256
    n, nrhs = cfg["n"], cfg["nrhs"]
    pts = sample_points(n)
    x = wl.vectors(cfg["seed_x"], n, 3, nrhs)
    out = dict(points=pts, n=np.asarray(n), k=np.float64(cfg["k"]), seed_x=np.int64(cfg["seed_x"]))
    idx = tuple(pts[:, l] for l in range(3))
    for name, make in (("green", wl.green_coeffs), ("skew", wl.skew_coeffs)):
        coeffs = make(n, cfg["k"])
        vals = np.empty((nrhs, 3, len(pts)), dtype=np.complex128)
        for r in range(nrhs):
            t0 = time.time()
            y = oracle.embed_matvec(coeffs, x[r:r + 1])
            vals[r] = y[0][(slice(None),) + idx]
            del y
            print(f"{name} rhs {r}: {time.time() - t0:.1f} s", flush=True)
        out[name] = vals
        del coeffs
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
