"""The runtime's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

paper_2406_17981_amd/build.py links tests/native/sfft_host_check.cpp with the
runtime units whose host code is instrumented (-Xarch_host -fsanitize=...;
device code as in the regular build). Host mode runs the calls that need no
GPU; GPU mode drives every entry point of include/sfft.h on small problems and
checks that schedules and entry points agree bit for bit. A sanitizer report
ends the program with a nonzero status."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "paper_2406_17981_amd", "sfft_host_check")
ENV = dict(os.environ,
           ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:protect_shadow_gap=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(mode, timeout):
    if not os.path.exists(BIN):
        pytest.skip("sanitizer host check not built (python paper_2406_17981_amd/build.py)")
    print(f"[case] sanitizer host check, mode {mode}", flush=True)
    p = subprocess.run([BIN, mode], env=ENV, capture_output=True, text=True, timeout=timeout)
    out = p.stdout + p.stderr
    print(out[-4000:], flush=True)
    return p.returncode, out


def test_host_paths_under_sanitizers():
    rc, out = _run("host", 120)
    assert rc == 0 and f"host check ok (host)" in out


@pytest.mark.gpu
def test_every_entry_point_under_sanitizers():
    rc, out = _run("gpu", 300)
    assert rc == 0 and "host check ok (gpu)" in out
