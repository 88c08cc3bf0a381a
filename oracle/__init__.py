"""CPU FP64 oracle for multilevel block-Toeplitz matrix-vector products.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or link
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it. It shares no code with the HIP library
and imports nothing from the product package; its inputs come from the seeded
generators in ``workloads``.

Everything here is plain NumPy/SciPy in float64/complex128, written for a reader
to check against the paper (Siron & Molesky, "A Split Fast Fourier Transform
Algorithm for Block Toeplitz Matrix-Vector Multiplication") by eye:

* ``dense_operator`` / ``dense_matvec``: the matrix written out, y = T v.
* ``embedded_generator`` / ``embed_matvec``: the standard multilevel circulant
  embedding of the introduction (pad every level to 2n, FFT, diagonal
  multiply, inverse FFT, keep the first n along every level).
* ``split_branch_sum``: the split identity of Section II.A on every level as a
  non-recursive sum over the 2^d parity branches with their symbols T[bId].
* ``lazy_order`` / ``lazy_costs``: the lazy (depth-first) evaluation order of
  the branch tree, built from the branch indices, with its work units and
  live vectors (Section II.C counts, the (d+1) peak).
* ``embed_matvec_with_symbol``: the embedding product for a symbol transformed
  beforehand; ``adjoint_coeffs``: the generator of T^H.
* ``sampled_rows``: direct sums for a few output indices (large grids).
* ``branch_symbols`` / ``compress_symbols`` / ``expand_symbols``: the per-branch
  Toeplitz data T[bId] and its symmetric storage (Section II.C).
* ``c_embed``, ``c_split``, ``ratio_*``: Eqs. (CompRatio), (MemRatio),
  (MemRatioSym) and Table I.

Parity status: every function here is pinned by ``tests/test_oracle.py``
against closed forms, brute force or the paper's printed values; none is
"parity unpinned".
"""

from .toeplitz import *  # noqa: F401,F403
from .toeplitz import __all__  # noqa: F401
