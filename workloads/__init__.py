"""Seeded synthetic inputs for multilevel block-Toeplitz matrix-vector products.

This module is shared by the CPU oracle's tests, the GPU parity tests and the
benchmark. It holds random draws and the closed-form coupling kernels t(r) that
define test matrices, and nothing of the split-FFT method itself: no Fourier
transform, no embedding, no phase split, no merge.

Conventions (used everywhere in this repository):

* ``n`` is the grid, a tuple ``(n_1, ..., n_d)``; level ``l`` of the Toeplitz
  structure is C-order axis ``l`` (axis 1 outermost).
* Coefficients are an array of shape ``(b, b, 2n_1-1, ..., 2n_d-1)``; the
  offset ``r_l`` sits at index ``r_l + n_l - 1``. The matrix is
  ``T[(a, i), (c, j)] = t(i - j)[a, c]``.
* Vectors are ``(nrhs, b, n_1, ..., n_d)`` (a single vector may drop ``nrhs``).
* Random complex entries have independent real and imaginary parts drawn from
  N(0, 1): zero mean, unit variance (the paper's Results section uses complex
  entries with zero-mean random parts of adjustable variance).
* Draw order inside one seed: coefficients first, then vectors in RHS order.
"""

from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np

EVEN = 1
ODD = 2
NONE = 0


def _grid(n: Sequence[int]) -> Tuple[int, ...]:
    n = tuple(int(v) for v in n)
    if not n or any(v < 1 for v in n):
        raise ValueError(f"bad grid {n}")
    return n


def complex_normal(rng: np.random.Generator, shape, scale: float = 1.0) -> np.ndarray:
    """Complex array, real and imaginary parts i.i.d. N(0, scale^2)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * scale


def offsets(n: Sequence[int]):
    """Open meshgrid of the integer offsets r_l in [-(n_l-1), n_l-1] per axis."""
    n = _grid(n)
    return np.meshgrid(*[np.arange(-(v - 1), v) for v in n], indexing="ij", sparse=True)


def coeff_shape(n: Sequence[int], b: int) -> Tuple[int, ...]:
    n = _grid(n)
    return (b, b) + tuple(2 * v - 1 for v in n)


def iid_coeffs(seed: int, n: Sequence[int], b: int = 1) -> np.ndarray:
    """I.i.d. complex-normal coefficients on the full offset grid."""
    rng = np.random.default_rng(seed)
    return complex_normal(rng, coeff_shape(n, b))


def vectors(seed: int, n: Sequence[int], b: int = 1, nrhs: int = 1) -> np.ndarray:
    """I.i.d. complex-normal input vectors, shape (nrhs, b, *n)."""
    rng = np.random.default_rng(seed)
    return complex_normal(rng, (nrhs, b) + _grid(n))


def iid_problem(seed_coeffs: int, seed_x: int, n, b=1, nrhs=1):
    return iid_coeffs(seed_coeffs, n, b), vectors(seed_x, n, b, nrhs)


def _unit_offsets3(n: Sequence[int]):
    """Offsets as 3-vectors: d=3 uses (r1, r2, r3); d=2 uses (r1, r2, 0); d=1 uses (r1, 0, 0)."""
    n = _grid(n)
    if len(n) > 3:
        raise ValueError("3-vector kernels need d <= 3")
    r = [a.astype(np.float64) for a in offsets(n)]
    shape = tuple(2 * v - 1 for v in n)
    comps = [np.broadcast_to(a, shape) for a in r]
    while len(comps) < 3:
        comps.append(np.zeros(shape))
    rx, ry, rz = comps
    dist = np.sqrt(rx * rx + ry * ry + rz * rz)
    return (rx, ry, rz), dist


def green_coeffs(n: Sequence[int], k: float = 0.7, self_term: float = 2.0) -> np.ndarray:
    """Dyadic Green-function-like 3x3 kernel.

    t(r) = exp(i k |r|) / |r| * (I - rhat rhat^T) for r != 0 and t(0) = self_term * I.
    Block symmetric; component (a, c) is even along every axis when a == c and
    odd along axes a and c (even elsewhere) when a != c.
    """
    (rx, ry, rz), dist = _unit_offsets3(n)
    comps = (rx, ry, rz)
    safe = np.where(dist > 0, dist, 1.0)
    g = np.exp(1j * k * safe) / safe
    out = np.zeros((3, 3) + dist.shape, dtype=np.complex128)
    zero = dist == 0
    for a in range(3):
        for c in range(3):
            rr = comps[a] * comps[c] / (safe * safe)
            val = g * ((1.0 if a == c else 0.0) - rr)
            val = np.where(zero, self_term if a == c else 0.0, val)
            out[a, c] = val
    return out


def green_coeffs_device(n: Sequence[int], k: float = 0.7, self_term: float = 2.0, device="cuda"):
    """green_coeffs evaluated with torch on a device (complex128), for callers
    that need many large coefficient arrays quickly (the serving workload)."""
    import torch
    n = _grid(n)
    if len(n) > 3:
        raise ValueError("3-vector kernels need d <= 3")
    axes = [torch.arange(-(v - 1), v, dtype=torch.float64, device=device) for v in n]
    grids = torch.meshgrid(*axes, indexing="ij")
    shape = grids[0].shape
    comps = list(grids) + [torch.zeros(shape, dtype=torch.float64, device=device)] * (3 - len(n))
    dist = torch.sqrt(comps[0] ** 2 + comps[1] ** 2 + comps[2] ** 2)
    zero = dist == 0
    safe = torch.where(zero, torch.ones_like(dist), dist)
    g = torch.polar(1.0 / safe, k * safe)
    out = torch.empty((3, 3) + tuple(shape), dtype=torch.complex128, device=device)
    for a in range(3):
        for c in range(a, 3):
            rr = comps[a] * comps[c] / (safe * safe)
            val = g * ((1.0 if a == c else 0.0) - rr)
            val = torch.where(zero, torch.full_like(val, self_term if a == c else 0.0), val)
            out[a, c] = val
            if c != a:
                out[c, a] = val
    return out


def skew_coeffs(n: Sequence[int], k: float = 1.3) -> np.ndarray:
    """Skew-symmetric 3x3 kernel t(r) = exp(i k |r|)/|r| * [rhat]_x with t(0) = 0.

    [a]_x is the cross-product matrix ([a]_x v = a x v). The block is skew
    symmetric (t(r)^T = -t(r)) and the kernel is odd under r -> -r; component
    (a, c) with a != c is odd along the third axis g (g != a, c) and even along
    the other two; the diagonal is zero.
    """
    (rx, ry, rz), dist = _unit_offsets3(n)
    safe = np.where(dist > 0, dist, 1.0)
    g = np.where(dist > 0, np.exp(1j * k * safe) / safe, 0.0)
    ux, uy, uz = rx / safe, ry / safe, rz / safe
    out = np.zeros((3, 3) + dist.shape, dtype=np.complex128)
    out[0, 1] = -uz * g
    out[0, 2] = uy * g
    out[1, 0] = uz * g
    out[1, 2] = -ux * g
    out[2, 0] = -uy * g
    out[2, 1] = ux * g
    return out


def green_parity(d: int) -> np.ndarray:
    """Per-(component, level) parity of green_coeffs on a d-level grid (b=3).

    Returns an int array (3, 3, d) with EVEN / ODD entries. Axis l of the grid
    carries the 3-vector component l (components beyond d are identically 0
    along the offsets, so they are even).
    """
    m = np.full((3, 3, d), EVEN, dtype=np.int32)
    for a in range(3):
        for c in range(3):
            if a != c:
                for ax in (a, c):
                    if ax < d:
                        m[a, c, ax] = ODD
    return m


def skew_parity(d: int) -> np.ndarray:
    """Per-(component, level) parity of skew_coeffs (b=3, d<=3)."""
    m = np.full((3, 3, d), EVEN, dtype=np.int32)
    for a in range(3):
        for c in range(3):
            if a != c:
                g = 3 - a - c
                if g < d:
                    m[a, c, g] = ODD
    return m


def parity_coeffs(seed: int, n: Sequence[int], b: int, parity: np.ndarray) -> np.ndarray:
    """I.i.d. complex-normal coefficients made exactly even or odd per
    (component, level): parity is an int array (b, b, d) of EVEN / ODD / NONE;
    along a level marked EVEN the array is replaced by (c + c mirrored)/2,
    along one marked ODD by (c - c mirrored)/2 (its r_l = 0 plane becomes 0).
    Mirroring an axis of offsets maps r_l to -r_l; the two halves are formed by
    the same IEEE operations, so the symmetry holds bit for bit."""
    n = _grid(n)
    c = iid_coeffs(seed, n, b)
    parity = np.asarray(parity).reshape(b, b, len(n))
    for a in range(b):
        for cc in range(b):
            comp = c[a, cc]
            for l in range(len(n)):
                f = np.flip(comp, axis=l)
                if parity[a, cc, l] == EVEN:
                    comp = (comp + f) / 2
                elif parity[a, cc, l] == ODD:
                    comp = (comp - f) / 2
            c[a, cc] = comp
    return c


def delta_coeffs(n: Sequence[int], b: int = 1) -> np.ndarray:
    """t(0) = I, t(r != 0) = 0: the identity matrix."""
    n = _grid(n)
    out = np.zeros(coeff_shape(n, b), dtype=np.complex128)
    centre = tuple(v - 1 for v in n)
    for a in range(b):
        out[(a, a) + centre] = 1.0
    return out


def shifted_delta_coeffs(n: Sequence[int], b: int, r0: Sequence[int], a: int, c: int,
                         value: complex = 1.0) -> np.ndarray:
    """Single nonzero coefficient t(r0)[a, c] = value."""
    n = _grid(n)
    out = np.zeros(coeff_shape(n, b), dtype=np.complex128)
    idx = tuple(int(r) + v - 1 for r, v in zip(r0, n))
    out[(a, c) + idx] = value
    return out


def constant_coeffs(n: Sequence[int], value: complex = 1.0) -> np.ndarray:
    """t(r) = value for every offset (scalar)."""
    n = _grid(n)
    return np.full(coeff_shape(n, 1), value, dtype=np.complex128)


def separable_factors(seed: int, n: Sequence[int]):
    """Per-axis random 1-D Toeplitz generators a_l(r_l), r_l in [-(n_l-1), n_l-1]."""
    n = _grid(n)
    rng = np.random.default_rng(seed)
    return [complex_normal(rng, (2 * v - 1,)) for v in n]


def separable_coeffs(factors) -> np.ndarray:
    """t(r) = prod_l a_l(r_l) (scalar), built from separable_factors."""
    out = np.ones((), dtype=np.complex128)
    for f in factors:
        out = np.multiply.outer(out, f)
    return out.reshape((1, 1) + out.shape)


# ---------------------------------------------------------------------------
# The synthetic workloads of the benchmark and parity suites.
# ---------------------------------------------------------------------------

PLAIN_16 = dict(name="plain-16^3-b1-c128", n=(16, 16, 16), b=1, seed_coeffs=101, seed_x=102)
GREEN_64 = dict(name="green-64^3-b3", n=(64, 64, 64), b=3, k=0.7, seed_x=202)
LARGE_256 = dict(name="green-256x256x128-b3-8rhs", n=(256, 256, 128), b=3, k=1.3, nrhs=8,
                 seed_x=502)
BATCH_GRIDS = [(48, 40, 32), (64, 64, 32), (96, 80, 64), (512, 384)]


def plain_16():
    """Scalar d=3 16^3 problem: i.i.d. coefficients on the 31^3 offset grid and one vector."""
    c = PLAIN_16
    return iid_problem(c["seed_coeffs"], c["seed_x"], c["n"], 1, 1)


def green_64(nrhs: int = 1):
    """d=3 64^3 grid with 3x3 Green blocks (k=0.7, self term 2I) and one vector."""
    c = GREEN_64
    return green_coeffs(c["n"], c["k"]), vectors(c["seed_x"], c["n"], 3, nrhs)


def batch_problems():
    """Uneven-grid batch: every grid of BATCH_GRIDS with b=1 (i.i.d.) and b=3 (Green k=0.7),
    8 right-hand sides each: 8 problems, 64 right-hand sides in all."""
    probs = []
    for q, n in enumerate(BATCH_GRIDS):
        for bi, b in enumerate((1, 3)):
            idx = 2 * q + bi
            if b == 1:
                coeffs = iid_coeffs(300 + idx, n, 1)
            else:
                coeffs = green_coeffs(n, 0.7)
            x = vectors(310 + idx, n, b, 8)
            probs.append(dict(n=n, b=b, coeffs=coeffs, x=x))
    return probs


def poisson_arrivals(seed: int, rate: float, count: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream with the given mean rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def relative_l2(got: np.ndarray, ref: np.ndarray) -> float:
    """||got - ref||_2 / ||ref||_2 over all entries."""
    ref = np.asarray(ref)
    den = float(np.linalg.norm(ref.ravel()))
    num = float(np.linalg.norm((np.asarray(got) - ref).ravel()))
    return num / den if den > 0 else num


__all__ = [n for n in dir() if not n.startswith("_")]
del math
