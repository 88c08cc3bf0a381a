"""Split-FFT multilevel block-Toeplitz matrix-vector products on AMD MI355X.

A from-scratch HIP implementation (gfx950) of the lazy-embedding /
eager-projection algorithm of Siron & Molesky (Algorithm 1), with the
standard multilevel circulant embedding as an in-library baseline. The
native library is ``libsfft.so`` (C ABI in ``include/sfft.h``); this package
only marshals torch device tensors into it.
"""

from . import _native
from ._native import SfftError
from .plan import Plan, apply_multi, batch_last_form, gmres_solve, gmres_workspace_size, workspace_size_multi

supported_length = lambda L: bool(_native.lib.sfft_length_supported(int(L)))  # noqa: E731

__all__ = ["Plan", "apply_multi", "batch_last_form", "workspace_size_multi", "gmres_solve", "gmres_workspace_size", "SfftError",
           "supported_length"]
