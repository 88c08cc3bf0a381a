"""Python face of the C ABI: a Plan over torch device tensors.

PyTorch provides device memory and streams only; every step of the product
runs in libsfft.so's HIP kernels.
"""

from __future__ import annotations

import ctypes as C
import math
from typing import Optional, Sequence

import torch

from . import _native as N

_DTYPES = {"c64": (N.C64, torch.complex64), "c128": (N.C128, torch.complex128)}
_METHODS = {"split": N.SPLIT, "embed": N.EMBED}
_SCHEDS = {"auto": N.SCHED_AUTO, "breadth": N.SCHED_BREADTH, "depth": N.SCHED_DEPTH, "slab": N.SCHED_SLAB}


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _require_device(t: torch.Tensor, name: str, dtype: torch.dtype):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """y = T x for a d-level block-Toeplitz T (Algorithm 1 or the embedding baseline).

    n: level sizes (n_1 outermost); b: block size; coeffs: complex128 device
    tensor (b, b, 2n_1-1, ..., 2n_d-1) (host arrays are copied to the device);
    dtype "c64" | "c128"; method "split" | "embed"; parity: optional
    (b, b, d) int array of 0 / 1 (even) / 2 (odd) for mirrored symbol storage;
    schedule "auto" | "breadth" | "depth" | "slab".
    """

    def __init__(self, n: Sequence[int], b: int, coeffs, dtype: str = "c64", method: str = "split",
                 parity=None, max_nrhs: int = 1, schedule: str = "auto", stream=None):
        self.n = tuple(int(v) for v in n)
        self.d = len(self.n)
        self.b = int(b)
        self.dtype_code, self.torch_dtype = _DTYPES[dtype]
        self.dtype = dtype
        self.method = method
        if not isinstance(coeffs, torch.Tensor) or not coeffs.is_cuda:
            coeffs = torch.as_tensor(coeffs, dtype=torch.complex128).to("cuda")
        _require_device(coeffs, "coeffs", torch.complex128)
        want = (self.b, self.b) + tuple(2 * v - 1 for v in self.n)
        if tuple(coeffs.shape) != want:
            raise ValueError(f"coeffs shape {tuple(coeffs.shape)} != {want}")
        n_arr = (C.c_int64 * self.d)(*self.n)
        par_ptr = None
        if parity is not None:
            import numpy as np
            par = np.ascontiguousarray(np.asarray(parity, dtype=np.int32).reshape(-1))
            if par.size != self.b * self.b * self.d:
                raise ValueError("parity must have b*b*d entries")
            self._par = (C.c_int32 * par.size)(*par.tolist())
            par_ptr = self._par
        h = C.c_void_p()
        st = N.lib.sfft_plan_create(C.byref(h), self.d, n_arr, self.b, C.c_void_p(coeffs.data_ptr()),
                                    self.dtype_code, _METHODS[method], par_ptr, int(max_nrhs),
                                    _SCHEDS[schedule], C.c_void_p(_stream_handle(stream)))
        N.check(st, "sfft_plan_create")
        self._h = h
        self.max_nrhs = int(max_nrhs)

    # -- queries ---------------------------------------------------------
    @property
    def handle(self) -> C.c_void_p:
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def info(self) -> dict:
        inf = N.SfftInfo()
        N.check(N.lib.sfft_plan_info(self.handle, C.byref(inf)), "sfft_plan_info")
        return dict(d=inf.d, n=tuple(inf.n[:inf.d]), b=inf.b, dtype=inf.dtype, method=inf.method,
                    schedule=inf.schedule, compressed=inf.compressed, max_nrhs=inf.max_nrhs,
                    symbol_bytes=inf.symbol_bytes, table_bytes=inf.table_bytes,
                    workspace_bytes=inf.workspace_bytes, vector_elems=inf.vector_elems,
                    block_symmetry=inf.block_symmetry, adjoint_symbol_bytes=inf.adjoint_symbol_bytes,
                    tile_mode=tuple(inf.tile_mode[:inf.d]), mirror_row=inf.mirror_row,
                    plan_n=tuple(inf.plan_n[:inf.plan_d]), pencil_len=tuple(inf.pencil_len[:inf.plan_d]),
                    radix=tuple(tuple(r for r in inf.radix[l] if r) for l in range(inf.plan_d)),
                    leaf_radix=tuple(r for r in inf.leaf_radix if r), peak_bytes=inf.peak_bytes)

    def workspace_size(self, nrhs: int) -> int:
        out = C.c_size_t()
        N.check(N.lib.sfft_workspace_size(self.handle, int(nrhs), C.byref(out)), "sfft_workspace_size")
        return int(out.value)

    def vector_shape(self, nrhs: int):
        return (int(nrhs), self.b) + self.n

    def alloc_workspace(self, nrhs: int) -> Optional[torch.Tensor]:
        nb = self.workspace_size(nrhs)
        if nb == 0:
            return None
        return torch.empty(nb, dtype=torch.uint8, device="cuda")

    # -- apply -----------------------------------------------------------
    def apply(self, x: torch.Tensor, y: Optional[torch.Tensor] = None,
              workspace: Optional[torch.Tensor] = None, stream=None, adjoint: bool = False) -> torch.Tensor:
        """y = T x (or y = T^H x with adjoint=True, after enable_adjoint()); x is
        (nrhs, b, *n) (or (b, *n)) of the plan dtype, on the device."""
        _require_device(x, "x", self.torch_dtype)
        squeeze = x.dim() == self.d + 1
        xs = x.unsqueeze(0) if squeeze else x
        if tuple(xs.shape[1:]) != (self.b,) + self.n:
            raise ValueError(f"x shape {tuple(x.shape)} does not match b={self.b}, n={self.n}")
        nrhs = xs.shape[0]
        if y is None:
            y = torch.empty_like(xs)
        else:
            _require_device(y, "y", self.torch_dtype)
            if y.numel() != xs.numel():
                raise ValueError("y has the wrong size")
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous device tensor")
            ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
        fn = N.lib.sfft_apply_adjoint if adjoint else N.lib.sfft_apply
        st = fn(self.handle, C.c_void_p(xs.data_ptr()), C.c_void_p(y.data_ptr()), nrhs,
                C.c_void_p(ws_ptr) if ws_ptr else None, ws_bytes, C.c_void_p(_stream_handle(stream)))
        N.check(st, "sfft_apply_adjoint" if adjoint else "sfft_apply")
        return y.view(x.shape) if squeeze else y

    __call__ = apply

    def workspace_size_subtree(self, k: int, nrhs: int) -> int:
        out = C.c_size_t()
        N.check(N.lib.sfft_workspace_size_subtree(self.handle, int(k), int(nrhs), C.byref(out)),
                "sfft_workspace_size_subtree")
        return int(out.value)

    def apply_subtree(self, k: int, prefix: int, x: torch.Tensor, y: Optional[torch.Tensor] = None,
                      workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """One device's share of T x split over 2^k devices by branch: the
        contribution of the branches whose parities along levels 1..k are the
        bits of prefix (bit l-1 for level l; levels of size 1 do not count).
        The 2^k shares sum to T x. workspace: workspace_size_subtree(k, nrhs)
        bytes (allocated here when omitted)."""
        _require_device(x, "x", self.torch_dtype)
        squeeze = x.dim() == self.d + 1
        xs = x.unsqueeze(0) if squeeze else x
        if tuple(xs.shape[1:]) != (self.b,) + self.n:
            raise ValueError(f"x shape {tuple(x.shape)} does not match b={self.b}, n={self.n}")
        nrhs = xs.shape[0]
        if y is None:
            y = torch.empty_like(xs)
        else:
            _require_device(y, "y", self.torch_dtype)
            if y.numel() != xs.numel():
                raise ValueError("y has the wrong size")
        if workspace is None:
            nb = self.workspace_size_subtree(k, nrhs)
            workspace = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous device tensor")
            ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
        st = N.lib.sfft_apply_subtree(self.handle, int(k), int(prefix), C.c_void_p(xs.data_ptr()),
                                      C.c_void_p(y.data_ptr()), nrhs, C.c_void_p(ws_ptr) if ws_ptr else None,
                                      ws_bytes, C.c_void_p(_stream_handle(stream)))
        N.check(st, "sfft_apply_subtree")
        return y.view(x.shape) if squeeze else y

    def ooc_sizes(self, nrhs: int, device_budget: int):
        """(host workspace bytes, device workspace bytes) of apply_ooc for a
        device budget (sfft_ooc_sizes)."""
        h, d = C.c_size_t(), C.c_size_t()
        N.check(N.lib.sfft_ooc_sizes(self.handle, int(nrhs), int(device_budget), C.byref(h), C.byref(d)),
                "sfft_ooc_sizes")
        return int(h.value), int(d.value)

    def apply_ooc(self, x: torch.Tensor, y: Optional[torch.Tensor] = None, device_budget: int = 1 << 30,
                  host_ws: Optional[torch.Tensor] = None, device_ws: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
        """y = T x with x and y in host memory (sfft_apply_ooc): the device
        holds the plan and slabs of at most device_budget bytes. x: CPU tensor
        (nrhs, b, *n) of the plan dtype, preferably pinned."""
        if x.is_cuda or x.dtype != self.torch_dtype or not x.is_contiguous():
            raise ValueError(f"x must be a contiguous host tensor of {self.torch_dtype}")
        xs = x.unsqueeze(0) if x.dim() == self.d + 1 else x
        if tuple(xs.shape[1:]) != (self.b,) + self.n:
            raise ValueError(f"x shape {tuple(x.shape)} does not match b={self.b}, n={self.n}")
        nrhs = xs.shape[0]
        hb, db = self.ooc_sizes(nrhs, device_budget)
        if y is None:
            y = torch.empty(xs.shape, dtype=self.torch_dtype, pin_memory=True)
        if y.is_cuda or y.dtype != self.torch_dtype or y.numel() != xs.numel() or not y.is_contiguous():
            raise ValueError("y must be a contiguous host tensor of x's size and dtype")
        if host_ws is None:
            host_ws = torch.empty(hb, dtype=torch.uint8, pin_memory=True)
        if device_ws is None:
            device_ws = torch.empty(db, dtype=torch.uint8, device="cuda")
        N.check(N.lib.sfft_apply_ooc(self.handle, C.c_void_p(xs.data_ptr()), C.c_void_p(y.data_ptr()), nrhs,
                                     C.c_void_p(host_ws.data_ptr()), host_ws.numel(),
                                     C.c_void_p(device_ws.data_ptr()), device_ws.numel(),
                                     C.c_void_p(_stream_handle(stream))), "sfft_apply_ooc")
        return y.view(x.shape)

    def enable_adjoint(self, stream=None) -> None:
        """Build the symbols of T^H (sfft_plan_enable_adjoint) so that
        apply(..., adjoint=True) computes y = T^H x."""
        N.check(N.lib.sfft_plan_enable_adjoint(self.handle, C.c_void_p(_stream_handle(stream))),
                "sfft_plan_enable_adjoint")

    def autotune(self, nrhs: int = 1, use_cache: bool = True, stream=None) -> float:
        """Pick the fastest schedule / leaf grouping for nrhs right-hand sides on
        the device (microseconds per apply, -1 when taken from the cache)."""
        best = C.c_double()
        N.check(N.lib.sfft_plan_autotune(self.handle, int(nrhs), int(use_cache),
                                         C.c_void_p(_stream_handle(stream)), C.byref(best)),
                "sfft_plan_autotune")
        return float(best.value)

    # -- profiling hooks -------------------------------------------------
    def profile(self, kinds=("leaf",)):
        """Bracket later launches of the given kernel kinds with HIP events."""
        names = {"forward": N.KIND_FORWARD, "leaf": N.KIND_LEAF, "inverse": N.KIND_INVERSE,
                 "copy": N.KIND_COPY}
        mask = 0
        for k in kinds:
            mask |= 1 << names[k]
        N.check(N.lib.sfft_profile_enable(self.handle, mask), "sfft_profile_enable")

    def profile_read(self, kind="leaf", reset=True):
        """(total milliseconds, launches) of the recorded launches of one kind."""
        names = {"forward": N.KIND_FORWARD, "leaf": N.KIND_LEAF, "inverse": N.KIND_INVERSE,
                 "copy": N.KIND_COPY}
        ms = C.c_double()
        cnt = C.c_int64()
        N.check(N.lib.sfft_profile_read(self.handle, names[kind], C.byref(ms), C.byref(cnt), int(reset)),
                "sfft_profile_read")
        return float(ms.value), int(cnt.value)

    def update(self, coeffs, stream=None) -> None:
        """New coefficients of the same shape and block symmetry: the symbols
        are regenerated in place (sfft_plan_update). Earlier applies of the
        plan must be ordered before `stream`."""
        if not isinstance(coeffs, torch.Tensor) or not coeffs.is_cuda:
            coeffs = torch.as_tensor(coeffs, dtype=torch.complex128).to("cuda")
        _require_device(coeffs, "coeffs", torch.complex128)
        want = (self.b, self.b) + tuple(2 * v - 1 for v in self.n)
        if tuple(coeffs.shape) != want:
            raise ValueError(f"coeffs shape {tuple(coeffs.shape)} != {want}")
        N.check(N.lib.sfft_plan_update(self.handle, C.c_void_p(coeffs.data_ptr()),
                                       C.c_void_p(_stream_handle(stream))), "sfft_plan_update")

    def close(self):
        if getattr(self, "_h", None) is not None:
            N.lib.sfft_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_size_multi(plans: Sequence[Plan], nrhs: Sequence[int]) -> int:
    k = len(plans)
    arr = (C.c_void_p * k)(*[p.handle.value for p in plans])
    nr = (C.c_int64 * k)(*[int(v) for v in nrhs])
    out = C.c_size_t()
    N.check(N.lib.sfft_workspace_size_multi(k, arr, nr, C.byref(out)), "sfft_workspace_size_multi")
    return int(out.value)


def apply_multi(plans: Sequence[Plan], xs: Sequence[torch.Tensor], ys: Sequence[torch.Tensor],
                workspace: Optional[torch.Tensor] = None, stream=None):
    """Problem i: ys[i] = T_i xs[i], all in one call of the C ABI."""
    k = len(plans)
    if not (len(xs) == len(ys) == k):
        raise ValueError("plans, xs and ys must have the same length")
    nr = []
    for p, x, y in zip(plans, xs, ys):
        _require_device(x, "x", p.torch_dtype)
        _require_device(y, "y", p.torch_dtype)
        if x.numel() % (p.b * math.prod(p.n)) or y.numel() != x.numel():
            raise ValueError("bad vector size")
        nr.append(x.numel() // (p.b * math.prod(p.n)))
    arr = (C.c_void_p * k)(*[p.handle.value for p in plans])
    xa = (C.c_void_p * k)(*[x.data_ptr() for x in xs])
    ya = (C.c_void_p * k)(*[y.data_ptr() for y in ys])
    na = (C.c_int64 * k)(*nr)
    if workspace is None:
        nb = workspace_size_multi(plans, nr)
        workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    st = N.lib.sfft_apply_multi(k, arr, xa, ya, na, C.c_void_p(workspace.data_ptr()),
                                workspace.numel(), C.c_void_p(_stream_handle(stream)))
    N.check(st, "sfft_apply_multi")
    return ys


def batch_last_form() -> Optional[str]:
    """Graph form the last apply_multi replayed: "chains", "grouped" or None."""
    return {0: "chains", 1: "grouped"}.get(int(N.lib.sfft_batch_last_form()))


def gmres_workspace_size(lo: Plan, hi: Plan, m: int) -> int:
    out = C.c_size_t()
    N.check(N.lib.sfft_gmres_workspace_size(lo.handle, hi.handle, int(m), C.byref(out)),
            "sfft_gmres_workspace_size")
    return int(out.value)


def gmres_solve(lo: Plan, hi: Plan, chi: torch.Tensor, rhs: torch.Tensor, x: Optional[torch.Tensor] = None,
                m: int = 30, max_cycles: int = 50, tol: float = 1e-6,
                workspace: Optional[torch.Tensor] = None, stream=None):
    """Solve (I - diag(chi) T) x = rhs by restarted GMRES(m) (sfft_gmres_solve):
    Krylov steps with lo's products, the true residual in FP64 with hi (a
    complex128 plan of the same T). chi, rhs, x: complex128 device tensors of
    shape (b, *n); x holds the initial guess (zero when None) and receives the
    solution. Returns (x, info dict)."""
    shape = (lo.b,) + lo.n
    for name, t in (("chi", chi), ("rhs", rhs)):
        _require_device(t, name, torch.complex128)
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}")
    if x is None:
        x = torch.zeros(shape, dtype=torch.complex128, device=rhs.device)
    _require_device(x, "x", torch.complex128)
    if tuple(x.shape) != shape:
        raise ValueError(f"x must have shape {shape}")
    if workspace is None:
        workspace = torch.empty(gmres_workspace_size(lo, hi, m), dtype=torch.uint8, device=rhs.device)
    inf = N.GmresInfo()
    N.check(N.lib.sfft_gmres_solve(lo.handle, hi.handle, C.c_void_p(chi.data_ptr()), C.c_void_p(rhs.data_ptr()),
                                   C.c_void_p(x.data_ptr()), int(m), int(max_cycles), float(tol),
                                   C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                   C.c_void_p(_stream_handle(stream)), C.byref(inf)), "sfft_gmres_solve")
    return x, dict(cycles=inf.cycles, matvecs=inf.matvecs, fp64_matvecs=inf.fp64_matvecs,
                   rel_residual=inf.rel_residual, rel_residual_estimate=inf.rel_residual_estimate,
                   converged=bool(inf.converged))
