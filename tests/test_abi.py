"""The C-ABI library loads on the host and exports every function include/sfft.h
declares. No compute call is made here (no GPU in this environment)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfft.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sfft_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("sfft_plan_create", "sfft_apply", "sfft_apply_multi", "sfft_workspace_size",
                 "sfft_plan_info", "sfft_plan_destroy", "sfft_status_string"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2406_17981_amd import _native
    lib = ctypes.CDLL(_native.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_native.EXPORTS) == _declared()


def test_host_only_calls():
    from paper_2406_17981_amd import _native as N
    assert N.lib.sfft_status_string(N.INVALID_ARG) == b"SFFT_INVALID_ARG"
    assert N.lib.sfft_length_supported(64) == 1
    for L in (7, 9, 14, 15, 21, 25, 35, 36, 49, 100, 343, 1000, 2187, 4096):  # runtime-length kernels
        assert N.lib.sfft_length_supported(L) == 2, L
    for L in (0, 1, 11, 22, 26, 4097, 5000, 8192):
        assert N.lib.sfft_length_supported(L) == 0, L
    for L in (16, 40, 48, 64, 80, 96, 128, 160, 192, 256, 384, 512, 768, 1024, 2048):
        assert N.lib.sfft_length_supported(L) == 1, L
    assert N.lib.sfft_batch_last_form() == -1  # no batch graph replayed in this process


def test_argument_validation_without_a_device():
    """Validation happens before any HIP call, so it is testable on the host."""
    from paper_2406_17981_amd import _native as N
    h = ctypes.c_void_p()
    n = (ctypes.c_int64 * 3)(16, 16, 16)
    fake = ctypes.c_void_p(0x1000)
    assert N.lib.sfft_plan_create(None, 3, n, 1, fake, 0, 0, None, 1, 0, None) == N.INVALID_ARG
    assert N.lib.sfft_plan_create(ctypes.byref(h), 0, n, 1, fake, 0, 0, None, 1, 0, None) == N.INVALID_ARG
    assert N.lib.sfft_plan_create(ctypes.byref(h), 7, n, 1, fake, 0, 0, None, 1, 0, None) == N.UNSUPPORTED
    assert N.lib.sfft_plan_create(ctypes.byref(h), 3, n, 5, fake, 0, 0, None, 1, 0, None) == N.INVALID_ARG
    assert b"block size" in N.lib.sfft_last_error()
    assert N.lib.sfft_plan_create(ctypes.byref(h), 3, n, 1, None, 0, 0, None, 1, 0, None) == N.INVALID_ARG
    assert N.lib.sfft_plan_create(ctypes.byref(h), 3, n, 1, fake, 5, 0, None, 1, 0, None) == N.INVALID_ARG
    n11 = (ctypes.c_int64 * 3)(16, 11, 16)  # prime factor 11: outside {2, 3, 5, 7}
    assert N.lib.sfft_plan_create(ctypes.byref(h), 3, n11, 1, fake, 0, 0, None, 1, 0, None) == N.UNSUPPORTED
    assert b"11" in N.lib.sfft_last_error() or b"22" in N.lib.sfft_last_error()
    assert N.lib.sfft_apply(None, fake, fake, 1, None, 0, None) == N.INVALID_ARG
    assert N.lib.sfft_plan_update(None, fake, None) == N.INVALID_ARG
    assert b"null" in N.lib.sfft_last_error()


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle (it is test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_2406_17981_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", txt, re.M), f
                assert "oracle/" not in txt, f


def test_arnoldi_scratch_and_validation_without_a_device():
    """Scratch sizes and argument checks of the batched Arnoldi step are host
    logic: per job, one FP64 complex partial per 1024-entry chunk and basis
    vector plus one for the norms, and m + 2 more, rounded up to 256 bytes."""
    from paper_2406_17981_amd import _native as N
    b = ctypes.c_size_t(123)
    assert N.lib.sfft_arnoldi_scratch_size(0, None, ctypes.byref(b)) == N.OK and b.value == 0
    jobs = (N.ArnoldiJob * 2)()
    for j, (n, m) in zip(jobs, ((5000, 7), (3000, 0))):
        j.V, j.ldv, j.m, j.n = 0x1000, n, m, n
        j.w, j.vout, j.hcol = 0x2000, 0x3000, 0x4000
    assert N.lib.sfft_arnoldi_scratch_size(2, jobs, ctypes.byref(b)) == N.OK

    def per_job(n, m):
        raw = (-(-n // 1024) * (m + 1) + m + 2) * 16
        return -(-raw // 256) * 256
    assert b.value == per_job(5000, 7) + per_job(3000, 0)
    need = b.value
    fake = ctypes.c_void_p(0x5000)
    assert N.lib.sfft_arnoldi_step_multi(2, jobs, 9, fake, need, None) == N.INVALID_ARG       # dtype
    assert N.lib.sfft_arnoldi_step_multi(2, jobs, N.C64, fake, need - 1, None) == N.INVALID_ARG
    assert b"scratch" in N.lib.sfft_last_error()
    jobs[0].m = 65                                                                              # > 64
    assert N.lib.sfft_arnoldi_scratch_size(2, jobs, ctypes.byref(b)) == N.OK
    assert N.lib.sfft_arnoldi_step_multi(2, jobs, N.C64, fake, b.value, None) == N.INVALID_ARG
    jobs[0].m, jobs[0].ldv = 7, 4999                                                            # ldv < n
    assert N.lib.sfft_arnoldi_step_multi(2, jobs, N.C64, fake, need, None) == N.INVALID_ARG
    assert b"Arnoldi job" in N.lib.sfft_last_error()
    assert N.lib.sfft_arnoldi_step_multi(0, None, N.C64, None, 0, None) == N.OK               # empty step


def test_info_struct_layout_matches_the_header(tmp_path):
    """The ctypes mirror of sfft_info has the C struct's size and field offsets
    (compiled from include/sfft.h with the host C compiler)."""
    import shutil
    import subprocess
    from paper_2406_17981_amd import _native as N
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    fields = [f for f, _ in N.SfftInfo._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"sfft.h\"\nint main(void) {\n"
                   + "  printf(\"%zu\\n\", sizeof(sfft_info));\n"
                   + "".join(f"  printf(\"%zu\\n\", offsetof(sfft_info, {f}));\n" for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got[0] == ctypes.sizeof(N.SfftInfo)
    assert got[1:] == [getattr(N.SfftInfo, f).offset for f in fields]
