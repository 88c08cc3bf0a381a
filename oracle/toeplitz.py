"""FP64 CPU oracle: multilevel block-Toeplitz matvec, plain and slow.

TEST INFRASTRUCTURE ONLY (see the package docstring). No function here is used
by the HIP library or its Python binding.

Conventions (shared with the seeded generators in ``workloads``):

* grid ``n = (n_1, ..., n_d)``; level l of the Toeplitz structure is C-order
  axis l of the grid (level 1 outermost);
* coefficients ``t`` of shape ``(b, b, 2n_1-1, ..., 2n_d-1)``, offset r_l at
  index r_l + n_l - 1; the matrix is ``T[(a, i), (c, j)] = t(i - j)[a, c]``;
* vectors ``(nrhs, b, n_1, ..., n_d)``;
* branch bit-vector ``p = (p_1, ..., p_d)``, p_l = 1 when the branch took the
  odd (phase-shifted) child at level l; flat branch index
  ``q = sum_l p_l * 2**(d - l)`` (C order over p);
* forward DFT unnormalised with kernel exp(-2 pi i j k / n), inverse DFT
  carries 1/n (NumPy's convention).

Readings taken where the paper is ambiguous or garbled (all fixed by the
mathematics and pinned in the tests):

1. phase operator P along level l: Phi_l[k] = exp(-i pi k / n_l), k = 0..n_l-1
   (the sign that makes the odd coefficients of the 2n-point transform come
   out of the proof in Section II.A);
2. the relation between F(v~) and F(v), F(Pv) is an interleave: even bins of
   the 2n-point transform are F(v), odd bins are F(Pv);
3. merge (Section II.A, after the inverse along that level):
   v = (v_even + conj(Phi) * v_odd) / 2;
4. the embedding pad s_0 (introduction) is 0;
5. T[bId] is the parity sub-lattice C^[p_1::2, ..., p_d::2] of the
   unnormalised d-dimensional transform of the embedded generator.
"""

from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple

import numpy as np
import scipy.fft

__all__ = [
    "grid_of", "dense_operator", "dense_matvec", "embedded_generator", "embed_symbol",
    "embed_matvec", "embed_matvec_with_symbol", "adjoint_coeffs", "branch_symbols", "phase",
    "split_branch_sum", "split_branch_sum_with_symbol", "lazy_order", "lazy_costs",
    "sampled_rows", "compress_symbol", "expand_symbol", "c_embed", "c_split",
    "c_split_closed", "ratio_c", "ratio_c_asymptotic", "ratio_m", "ratio_m_sym",
    "mem_embed", "mem_split", "branch_index",
]

_WORKERS = None  # scipy.fft default (1 thread) unless set by the caller


def set_workers(w):
    """Thread count handed to scipy.fft (None = library default)."""
    global _WORKERS
    _WORKERS = w


def grid_of(coeffs: np.ndarray) -> Tuple[int, ...]:
    """Grid n from a coefficient array of shape (b, b, 2n_1-1, ..., 2n_d-1)."""
    if coeffs.ndim < 3 or coeffs.shape[0] != coeffs.shape[1]:
        raise ValueError(f"coefficient shape {coeffs.shape} is not (b, b, 2n-1, ...)")
    for m in coeffs.shape[2:]:
        if m % 2 != 1:
            raise ValueError(f"offset axis of even length {m}")
    return tuple((m + 1) // 2 for m in coeffs.shape[2:])


def _as_vectors(x: np.ndarray, b: int, n: Sequence[int]) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    if x.shape == (b,) + tuple(n):
        x = x[None]
    if x.shape[1:] != (b,) + tuple(n):
        raise ValueError(f"vector shape {x.shape} does not match b={b}, n={n}")
    return x


# ---------------------------------------------------------------------------
# O1: the matrix itself
# ---------------------------------------------------------------------------

def dense_operator(coeffs: np.ndarray) -> np.ndarray:
    """The multilevel block-Toeplitz matrix, written out.

    T[(a, i), (c, j)] = t(i - j)[a, c] for grid points i, j (translation
    invariance gives this structure; Algorithm 1 promises y = T v). Rows and
    columns run over (a, i_1, ..., i_d) in C order.
    """
    n = grid_of(coeffs)
    b = coeffs.shape[0]
    s = math.prod(n)
    pts = np.indices(n).reshape(len(n), s)
    off = tuple((pts[l][:, None] - pts[l][None, :] + n[l] - 1).astype(np.int32)
                for l in range(len(n)))
    T = np.empty((b, s, b, s), dtype=np.complex128)
    for a in range(b):
        for c in range(b):
            T[a, :, c, :] = coeffs[(a, c) + off]
    return T.reshape(b * s, b * s)


def dense_matvec(coeffs: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = T x by the dense O((b s)^2) product (tiny grids only)."""
    n = grid_of(coeffs)
    b = coeffs.shape[0]
    x = _as_vectors(x, b, n)
    T = dense_operator(coeffs)
    flat = x.reshape(x.shape[0], -1)
    return (flat @ T.T).reshape(x.shape)


# ---------------------------------------------------------------------------
# O2: the standard multilevel circulant embedding (introduction)
# ---------------------------------------------------------------------------

def embedded_generator(coeffs: np.ndarray) -> np.ndarray:
    """Circulant embedding of every level: n -> 2n ("extending the diagonal bands").

    Along each level the coefficient of offset r moves to position r mod 2n;
    position n (the pad entry s_0 of the introduction's 2x2 example) is 0.
    Result shape (b, b, 2n_1, ..., 2n_d).
    """
    n = grid_of(coeffs)
    b = coeffs.shape[0]
    out = np.zeros((b, b) + tuple(2 * v for v in n), dtype=np.complex128)
    targets = [np.mod(np.arange(-(v - 1), v), 2 * v) for v in n]
    out[(slice(None), slice(None)) + np.ix_(*targets)] = coeffs
    return out


def embed_symbol(coeffs: np.ndarray) -> np.ndarray:
    """Unnormalised d-dimensional DFT of the embedded generator, (b, b, 2n_1, ..., 2n_d)."""
    c = embedded_generator(coeffs)
    axes = tuple(range(2, c.ndim))
    return scipy.fft.fftn(c, axes=axes, workers=_WORKERS)


def embed_matvec(coeffs: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = T x through the standard circulant embedding (introduction).

    Pad every level of x with zeros to 2n, transform, multiply point by point by
    the b x b blocks of the embedded symbol, inverse transform, keep the first
    n entries along every level (the projection).
    """
    return embed_matvec_with_symbol(embed_symbol(coeffs), x)


def embed_matvec_with_symbol(C: np.ndarray, x: np.ndarray) -> np.ndarray:
    """embed_matvec for an embedded symbol C = embed_symbol(coeffs) computed
    beforehand (shape (b, b, 2n_1, ..., 2n_d)), so repeated products with one
    operator transform the generator once."""
    b = C.shape[0]
    n = tuple(v // 2 for v in C.shape[2:])
    x = _as_vectors(x, b, n)
    d = len(n)
    xp = np.zeros(x.shape[:2] + tuple(2 * v for v in n), dtype=np.complex128)
    xp[(slice(None), slice(None)) + tuple(slice(0, v) for v in n)] = x
    axes = tuple(range(2, 2 + d))
    X = scipy.fft.fftn(xp, axes=axes, workers=_WORKERS)
    Y = np.einsum("ac...,rc...->ra...", C, X)
    y = scipy.fft.ifftn(Y, axes=axes, workers=_WORKERS)
    return y[(slice(None), slice(None)) + tuple(slice(0, v) for v in n)].copy()


def adjoint_coeffs(coeffs: np.ndarray) -> np.ndarray:
    """Generator of the conjugate transpose: T^H[(a, i), (c, j)] = conj(T[(c, j), (a, i)])
    = conj(t(j - i)[c, a]), so t^H(r)[a, c] = conj(t(-r)[c, a]). Reversing
    every offset axis maps index r_l + n_l - 1 to -r_l + n_l - 1."""
    d = coeffs.ndim - 2
    flipped = coeffs[(slice(None), slice(None)) + (slice(None, None, -1),) * d]
    return np.conj(np.swapaxes(flipped, 0, 1)).copy()


# ---------------------------------------------------------------------------
# Branch data T[bId] and Algorithm 1
# ---------------------------------------------------------------------------

def branch_index(p: Sequence[int]) -> int:
    """Flat branch index q of the parity bit-vector p (p_1 most significant)."""
    q = 0
    for bit in p:
        q = 2 * q + int(bit)
    return q


def branch_symbols(coeffs: np.ndarray) -> np.ndarray:
    """T[bId] for every branch: the 2^d parity sub-lattices of the embedded symbol.

    Section II.C splits the fully embedded, transformed generator into 2^d parts
    of s coefficients each; part p holds C^[2j + p] (j over the n-grid).
    Returns shape (2^d, b, b, n_1, ..., n_d), branch index as in branch_index.
    """
    n = grid_of(coeffs)
    d = len(n)
    C = embed_symbol(coeffs)
    b = coeffs.shape[0]
    out = np.empty((2 ** d, b, b) + n, dtype=np.complex128)
    for q in range(2 ** d):
        p = [(q >> (d - 1 - l)) & 1 for l in range(d)]
        out[q] = C[(slice(None), slice(None)) + tuple(slice(pl, None, 2) for pl in p)]
    return out


def phase(nl: int) -> np.ndarray:
    """Diagonal of the phase operator P along a level of size n_l (Section II.A)."""
    return np.exp(-1j * np.pi * np.arange(nl) / nl)


def _along(arr: np.ndarray, vec: np.ndarray, axis: int) -> np.ndarray:
    shape = [1] * arr.ndim
    shape[axis] = vec.shape[0]
    return arr * vec.reshape(shape)


def split_branch_sum(coeffs: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = T x as the sum over the 2^d parity branches, without recursion.

    Section II.A applied to every level at once: the bins 2j + p of the
    2n-point transform of the zero-padded vector are the n-point transform of
    Phi^p x (Phi^p = prod over levels of Phi_l^(p_l)), and the first n entries
    of the 2n-point inverse transform are half the sum over the two parities of
    conj(Phi)^p times the n-point inverse transform of those bins. With the
    parity sub-lattices T_p = T[bId] of the embedded symbol (Section II.C):

        y = 2^-d  sum_p  conj(Phi^p) . iFFT_n( T_p . FFT_n( Phi^p . x ) )

    where FFT_n is the unpadded d-dimensional transform and T_p . acts as the
    b x b block product at every frequency. Every branch is evaluated on its
    own; nothing is shared between branches.
    """
    return split_branch_sum_with_symbol(embed_symbol(coeffs), x)


def split_branch_sum_with_symbol(C: np.ndarray, x: np.ndarray) -> np.ndarray:
    """split_branch_sum for an embedded symbol C = embed_symbol(coeffs) computed
    beforehand; branch q reads its parity sub-lattice T[bId] of C."""
    b = C.shape[0]
    n = tuple(v // 2 for v in C.shape[2:])
    d = len(n)
    x = _as_vectors(x, b, n)
    axes = tuple(range(2, 2 + d))
    y = np.zeros_like(x)
    for q in range(2 ** d):
        p = [(q >> (d - 1 - l)) & 1 for l in range(d)]
        Tq = C[(slice(None), slice(None)) + tuple(slice(pl, None, 2) for pl in p)]
        v = x
        for l in range(d):
            if p[l]:
                v = _along(v, phase(n[l]), 2 + l)
        V = scipy.fft.fftn(v, axes=axes, workers=_WORKERS)
        W = np.einsum("ac...,rc...->ra...", Tq, V)
        w = scipy.fft.ifftn(W, axes=axes, workers=_WORKERS)
        for l in range(d):
            if p[l]:
                w = _along(w, np.conj(phase(n[l])), 2 + l)
        y += w
    return y / 2 ** d


def lazy_order(d: int):
    """Events of the lazy (depth-first) evaluation of the d-level branch tree.

    Section II: a node at depth k holds one vector; splitting it along level
    k + 1 creates the phase-shifted odd child, the even subtree is finished
    before the odd one is started, and the two results are merged along level
    k + 1 before the node is left. Entering a node at depth l >= 1 transforms
    its vector along level l and leaving it transforms back. The events are
    built here from the leaves' binary branch indices in increasing order
    (p_1 most significant, even before odd): between leaf q - 1 and leaf q the
    trailing odd levels of q - 1 are closed (inverse transform, merge) and the
    deepest even level of q - 1 is left and re-entered as its odd sibling.

    Returns a list of tuples: ("split", l), ("fft", l), ("leaf", q),
    ("ifft", l), ("merge", l) with levels l = 1..d.
    """
    ev = []
    for l in range(1, d + 1):
        ev += [("split", l), ("fft", l)]
    for q in range(2 ** d):
        if q > 0:
            prev = q - 1
            k = 0
            while (prev >> k) & 1:
                k += 1          # trailing odd levels d, d-1, ..., d-k+1 of leaf q-1
            for l in range(d, d - k, -1):
                ev += [("ifft", l), ("merge", l)]
            top = d - k          # deepest even level of leaf q-1: becomes odd
            ev += [("ifft", top), ("fft", top)]
            for l in range(top + 1, d + 1):
                ev += [("split", l), ("fft", l)]
        ev.append(("leaf", q))
    for l in range(d, 0, -1):
        ev += [("ifft", l), ("merge", l)]
    return ev


def lazy_costs(n: Sequence[int], b: int = 1, nrhs: int = 1) -> Dict[str, object]:
    """Work units and live vectors of the lazy evaluation (Section II.C units).

    Walks lazy_order: an FFT or inverse FFT along level l costs
    (entries of one vector) * log2(n_l), a split or merge costs one phase
    multiply per entry, a leaf costs b^2 scalar products per grid point and
    right-hand side. The input is one live vector, a split adds one, a merge
    frees one. Returns fft, phase, mult, total, fft_calls / ifft_calls per
    level, the leaves in visiting order, and the peak number of live vectors.
    """
    n = tuple(n)
    d = len(n)
    s = math.prod(n)
    units = s * b * nrhs
    out = dict(fft=0.0, phase=0, mult=0, fft_calls={}, ifft_calls={}, leaves=[], peak=1)
    live = 1
    for kind, arg in lazy_order(d):
        if kind in ("fft", "ifft"):
            out["fft"] += units * math.log2(n[arg - 1])
            key = "fft_calls" if kind == "fft" else "ifft_calls"
            out[key][arg] = out[key].get(arg, 0) + 1
        elif kind == "split":
            out["phase"] += units
            live += 1
            out["peak"] = max(out["peak"], live)
        elif kind == "merge":
            out["phase"] += units
            live -= 1
        else:
            out["mult"] += nrhs * b * b * s
            out["leaves"].append(arg)
    out["live_at_end"] = live
    out["total"] = out["fft"] + out["phase"] + out["mult"]
    return out


# ---------------------------------------------------------------------------
# O4: direct sums at sampled output points
# ---------------------------------------------------------------------------

def sampled_rows(coeffs: np.ndarray, x: np.ndarray, points: np.ndarray) -> np.ndarray:
    """y[:, :, i] = sum_j sum_c t(i - j)[:, c] x[:, c, j] at the given grid points.

    points: int array (K, d). Returns (nrhs, b, K). Cost O(K b^2 s).
    """
    n = grid_of(coeffs)
    b = coeffs.shape[0]
    x = _as_vectors(x, b, n)
    points = np.asarray(points, dtype=np.int64).reshape(-1, len(n))
    out = np.empty((x.shape[0], b, points.shape[0]), dtype=np.complex128)
    xf = x.reshape(x.shape[0], b, -1)
    for kk, i in enumerate(points):
        # t(i - j) for all j: offsets i_l - j_l, i.e. a reversed window of each offset axis
        sl = tuple(slice(int(i[l]) + n[l] - 1, (int(i[l]) - 1 if i[l] > 0 else None), -1)
                   for l in range(len(n)))
        for a in range(b):
            acc = np.zeros(x.shape[0], dtype=np.complex128)
            for c in range(b):
                slab = np.ascontiguousarray(coeffs[(a, c) + sl]).reshape(-1)
                acc += xf[:, c, :] @ slab
            out[:, a, kk] = acc
    return out


# ---------------------------------------------------------------------------
# Symmetric / skew-symmetric symbol storage (Section II.C)
# ---------------------------------------------------------------------------

def compress_symbol(C: np.ndarray, parity: np.ndarray) -> Dict[Tuple[int, int], np.ndarray]:
    """Keep, per block component, only bins m_l in [0, n_l] along mirrored levels.

    C: embedded symbol (b, b, 2n_1, ..., 2n_d). parity: (b, b, d) with 1 (even
    generator along that level: C^[2n - m] = C^[m]), 2 (odd generator:
    C^[2n - m] = 2 C^[0] - C^[m]) or 0 (no symmetry: keep all 2n bins).
    Returns {(a, c): array}. With every level mirrored this stores prod(n_l + 1)
    values per component instead of prod(2 n_l).
    """
    b = C.shape[0]
    n = tuple(v // 2 for v in C.shape[2:])
    out = {}
    for a in range(b):
        for c in range(b):
            sl = tuple(slice(0, n[l] + 1) if parity[a, c, l] else slice(None)
                       for l in range(len(n)))
            out[(a, c)] = C[(a, c) + sl].copy()
    return out


def expand_symbol(comp: Dict[Tuple[int, int], np.ndarray], parity: np.ndarray,
                  n: Sequence[int]) -> np.ndarray:
    """Inverse of compress_symbol: rebuild all 2n_l bins level by level."""
    n = tuple(n)
    d = len(n)
    b = parity.shape[0]
    out = np.empty((b, b) + tuple(2 * v for v in n), dtype=np.complex128)
    for (a, c), half in comp.items():
        arr = half
        for l in range(d):
            if parity[a, c, l] == 0:
                continue
            ax = l
            nl = n[l]
            mirrored = np.flip(np.take(arr, np.arange(1, nl), axis=ax), axis=ax)  # bins n-1..1
            if parity[a, c, l] == 1:
                tail = mirrored
            else:
                zero = np.take(arr, [0], axis=ax)
                tail = 2.0 * zero - mirrored
            arr = np.concatenate([arr, tail], axis=ax)  # bins 0..n, then n+1..2n-1
        out[a, c] = arr
    return out


# ---------------------------------------------------------------------------
# Section II.C: operation counts and memory ratios
# ---------------------------------------------------------------------------

def c_embed(n: Sequence[int]) -> float:
    """C_embed: FFTs of the 2^d s embedded vector (forward and inverse) + 2^d s multiplies."""
    n = tuple(n)
    d = len(n)
    s = math.prod(n)
    return 2 ** (d + 1) * s * math.log2(2 ** d * s) + 2 ** d * s


def c_split(n: Sequence[int]) -> float:
    """C_split as a sum over levels: 2^l forward and 2^l inverse FFTs at level l,
    the 2^d leaf multiplies, and a split plus a merge at every inner node."""
    n = tuple(n)
    d = len(n)
    s = math.prod(n)
    fft = 2 * sum(2 ** l * s * math.log2(n[l - 1]) for l in range(1, d + 1))
    mult = 2 ** d * s
    ph = 2 * sum(2 ** l * s for l in range(0, d))
    return fft + mult + ph


def c_split_closed(nl: int, d: int) -> float:
    """Closed form of C_split for equal level sizes: 2(2^d-1) s (2 log2 n + 1) + 2^d s."""
    s = nl ** d
    return 2 * (2 ** d - 1) * s * (2 * math.log2(nl) + 1) + 2 ** d * s


def ratio_c(nl: int, d: int) -> float:
    """R_c = C_embed / C_split at finite n (Eq. CompRatio, first form)."""
    return c_embed((nl,) * d) / c_split((nl,) * d)


def ratio_c_asymptotic(d: int) -> float:
    """Limit of R_c as n -> infinity: d / (2 - 2^(1-d))."""
    return d / (2.0 - 2.0 ** (1 - d))


def ratio_m(d: int) -> float:
    """R_m = (2^d s + 2^d s) / ((d+1) s + 2^d s) (Eq. MemRatio)."""
    return 2.0 / ((d + 1) * 2.0 ** (-d) + 1.0)


def ratio_m_sym(d: int) -> float:
    """R_m,sym = (2^d s + s) / ((d+1) s + s) (Eq. MemRatioSym, symbol stored in s)."""
    return (2.0 ** d + 1.0) / (d + 2.0)


def mem_embed(n: Sequence[int], b: int = 1, nrhs: int = 1) -> Dict[str, int]:
    """Entries held by the standard embedding: padded vectors and the full symbol."""
    d = len(n)
    s = math.prod(n)
    return dict(vectors=2 ** d * s * b * nrhs, symbol=2 ** d * s * b * b)


def mem_split(n: Sequence[int], b: int = 1, nrhs: int = 1, unique_components: int | None = None
              ) -> Dict[str, int]:
    """Entries held by Algorithm 1 under lazy evaluation: (d+1) vectors and the branch
    data (2^d s per component, or prod(n_l + 1) per unique component when stored
    mirrored)."""
    d = len(n)
    s = math.prod(n)
    sym = 2 ** d * s * b * b if unique_components is None else \
        unique_components * math.prod(v + 1 for v in n)
    return dict(vectors=(d + 1) * s * b * nrhs, symbol=sym)
