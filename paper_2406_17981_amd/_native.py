"""ctypes declarations of libsfft.so (include/sfft.h). Argument marshalling only.

The library must be built in-tree (``python -m paper_2406_17981_amd.build``);
importing this module without it raises ImportError: there is no fallback.
torch is imported first so that the library binds to the same HIP runtime
instance torch already loaded (both carry the soname libamdhip64.so.7).
"""

from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (load torch's HIP runtime before the library)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsfft.so")

OK, INVALID_ARG, UNSUPPORTED, OUT_OF_MEMORY, HIP_ERROR = range(5)
C64, C128 = 0, 1
SPLIT, EMBED = 0, 1
SCHED_AUTO, SCHED_BREADTH, SCHED_DEPTH, SCHED_SLAB = 0, 1, 2, 3
PARITY_NONE, PARITY_EVEN, PARITY_ODD = 0, 1, 2

# every function include/sfft.h declares
EXPORTS = [
    "sfft_plan_create", "sfft_workspace_size", "sfft_apply", "sfft_workspace_size_multi",
    "sfft_apply_multi", "sfft_plan_info", "sfft_plan_destroy", "sfft_status_string",
    "sfft_last_error", "sfft_length_supported", "sfft_profile_enable", "sfft_profile_read",
    "sfft_plan_autotune", "sfft_arnoldi_scratch_size", "sfft_arnoldi_step_multi", "sfft_plan_update",
    "sfft_plan_enable_adjoint", "sfft_apply_adjoint", "sfft_gmres_workspace_size", "sfft_gmres_solve",
    "sfft_apply_noalloc", "sfft_apply_each", "sfft_ooc_sizes", "sfft_apply_ooc", "sfft_batch_last_form",
    "sfft_workspace_size_subtree", "sfft_apply_subtree",
]
KIND_FORWARD, KIND_LEAF, KIND_INVERSE, KIND_COPY = range(4)


class SfftInfo(C.Structure):
    _fields_ = [
        ("d", C.c_int), ("n", C.c_int64 * 8), ("b", C.c_int), ("dtype", C.c_int),
        ("method", C.c_int), ("schedule", C.c_int), ("compressed", C.c_int),
        ("max_nrhs", C.c_int64), ("symbol_bytes", C.c_size_t), ("table_bytes", C.c_size_t),
        ("workspace_bytes", C.c_size_t), ("vector_elems", C.c_int64), ("block_symmetry", C.c_int),
        ("adjoint_symbol_bytes", C.c_size_t), ("tile_mode", C.c_int * 8), ("mirror_row", C.c_int64),
        ("plan_d", C.c_int), ("plan_n", C.c_int64 * 8), ("pencil_len", C.c_int64 * 8),
        ("radix", (C.c_int * 8) * 8), ("leaf_radix", C.c_int * 8), ("peak_bytes", C.c_size_t),
    ]


class ArnoldiJob(C.Structure):
    _fields_ = [
        ("V", C.c_void_p), ("ldv", C.c_int64), ("m", C.c_int64), ("w", C.c_void_p),
        ("vout", C.c_void_p), ("n", C.c_int64), ("hcol", C.c_void_p),
    ]


class GmresInfo(C.Structure):
    _fields_ = [
        ("cycles", C.c_int64), ("matvecs", C.c_int64), ("fp64_matvecs", C.c_int64),
        ("rel_residual", C.c_double), ("rel_residual_estimate", C.c_double), ("converged", C.c_int),
    ]


class SfftError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        super().__init__(f"{where}: {_status_name(status)}: {msg}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2406_17981_amd/build.py`")
    lib = C.CDLL(LIB_PATH)
    vp, i64, sz = C.c_void_p, C.c_int64, C.c_size_t
    P64 = C.POINTER(C.c_int64)
    lib.sfft_plan_create.argtypes = [C.POINTER(vp), C.c_int, P64, C.c_int, vp, C.c_int, C.c_int,
                                     C.POINTER(C.c_int32), i64, C.c_int, vp]
    lib.sfft_workspace_size.argtypes = [vp, i64, C.POINTER(sz)]
    lib.sfft_apply.argtypes = [vp, vp, vp, i64, vp, sz, vp]
    lib.sfft_workspace_size_multi.argtypes = [C.c_int, C.POINTER(vp), P64, C.POINTER(sz)]
    lib.sfft_apply_multi.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), P64, vp, sz,
                                     vp]
    lib.sfft_plan_info.argtypes = [vp, C.POINTER(SfftInfo)]
    lib.sfft_plan_destroy.argtypes = [vp]
    lib.sfft_plan_update.argtypes = [vp, vp, vp]
    lib.sfft_plan_enable_adjoint.argtypes = [vp, vp]
    lib.sfft_apply_adjoint.argtypes = [vp, vp, vp, i64, vp, sz, vp]
    lib.sfft_apply_noalloc.argtypes = [vp, vp, vp, i64, vp]
    lib.sfft_workspace_size_subtree.argtypes = [vp, C.c_int, i64, C.POINTER(sz)]
    lib.sfft_apply_subtree.argtypes = [vp, C.c_int, C.c_uint32, vp, vp, i64, vp, sz, vp]
    lib.sfft_ooc_sizes.argtypes = [vp, i64, sz, C.POINTER(sz), C.POINTER(sz)]
    lib.sfft_apply_ooc.argtypes = [vp, vp, vp, i64, vp, sz, vp, sz, vp]
    lib.sfft_apply_each.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), P64, C.POINTER(vp),
                                    C.POINTER(sz), vp, C.POINTER(C.c_int)]
    lib.sfft_gmres_workspace_size.argtypes = [vp, vp, C.c_int, C.POINTER(sz)]
    lib.sfft_gmres_solve.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_double, vp, sz, vp,
                                     C.POINTER(GmresInfo)]
    lib.sfft_status_string.argtypes = [C.c_int]
    lib.sfft_status_string.restype = C.c_char_p
    lib.sfft_last_error.argtypes = []
    lib.sfft_last_error.restype = C.c_char_p
    lib.sfft_batch_last_form.argtypes = []
    lib.sfft_length_supported.argtypes = [i64]
    lib.sfft_profile_enable.argtypes = [vp, C.c_uint]
    lib.sfft_profile_read.argtypes = [vp, C.c_int, C.POINTER(C.c_double), P64, C.c_int]
    lib.sfft_plan_autotune.argtypes = [vp, i64, C.c_int, vp, C.POINTER(C.c_double)]
    lib.sfft_arnoldi_scratch_size.argtypes = [C.c_int, C.POINTER(ArnoldiJob), C.POINTER(sz)]
    lib.sfft_arnoldi_step_multi.argtypes = [C.c_int, C.POINTER(ArnoldiJob), C.c_int, vp, sz, vp]
    for name in EXPORTS:
        fn = getattr(lib, name)
        if fn.restype is C.c_int or fn.restype is None:
            fn.restype = C.c_int
    _check_single_hip_runtime()
    return lib


def _check_single_hip_runtime():
    """Fail loudly if two different libamdhip64 copies ended up in the process."""
    try:
        paths = set()
        with open("/proc/self/maps") as f:
            for ln in f:
                if "libamdhip64" in ln:
                    paths.add(os.path.realpath(ln.split()[-1]))
        if len(paths) > 1:
            raise ImportError(f"two HIP runtimes loaded: {sorted(paths)}")
    except OSError:
        pass


lib = _load()


def _status_name(s: int) -> str:
    try:
        return lib.sfft_status_string(s).decode()
    except Exception:  # pragma: no cover
        return str(s)


def check(status: int, where: str):
    if status != OK:
        raise SfftError(status, where, lib.sfft_last_error().decode())
