"""Build libsfft.so (HIP kernels, runtime and C ABI) for gfx950, in-tree.

    python paper_2406_17981_amd/build.py [-j N]

(run as a script: importing the package would load the library it builds)

Every call recompiles every source: one object per pencil length listed in
csrc/lengths.def (kernels_len.hip with -DSFFT_LEN=<L>), the runtime, and a
shared-library link. Objects go to _build/ at the repository root; the
library is written next to this file.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsfft.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled on purpose; hipcc's host pass warns
# that it does not know the feature, which is harmless.
# Contraction is off: every fused multiply-add in the kernels is explicit, so
# results do not depend on which instantiation of a kernel ran.
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         f"-I{os.path.join(ROOT, 'include')}"]


def lengths():
    txt = open(os.path.join(CSRC, "lengths.def")).read()
    return [int(v) for v in re.findall(r"SFFT_X\((\d+)\)", txt)]


def _run(cmd):
    t0 = time.time()
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(ln for ln in p.stdout.splitlines() if "packed-fp32-ops" not in ln)
    return p.returncode, out, time.time() - t0


def _stale(src: str, obj: str) -> bool:
    """True when obj is missing or older than its source, a header, or this script."""
    if not os.path.exists(obj):
        return True
    deps = [src, __file__] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".def"))]
    deps += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every unit (incremental=True: only those older than their
    sources or any header) and link libsfft.so."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    units = []
    for L in lengths():
        units.append((os.path.join(CSRC, "kernels_len.hip"), os.path.join(BUILD, f"kernels_L{L}.o"),
                      [f"-DSFFT_LEN={L}"]))
    units.append((os.path.join(CSRC, "runtime.hip"), os.path.join(BUILD, "runtime.o"), []))
    units.append((os.path.join(CSRC, "batch.hip"), os.path.join(BUILD, "batch.o"), []))
    units.append((os.path.join(CSRC, "krylov.hip"), os.path.join(BUILD, "krylov.o"), []))
    units.append((os.path.join(CSRC, "generic_kernels.hip"), os.path.join(BUILD, "generic_kernels.o"), []))
    units.append((os.path.join(CSRC, "gmres.hip"), os.path.join(BUILD, "gmres.o"), []))
    # biggest lengths first so the slowest compiles start early
    units.sort(key=lambda u: -int(re.search(r"(\d+)", os.path.basename(u[1])).group(1))
               if "kernels_L" in u[1] else 0)
    cmds = [[HIPCC] + FLAGS + extra + ["-c", src, "-o", obj] for src, obj, extra in units
            if not incremental or _stale(src, obj)]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    failed = [(c, r) for c, r in zip(cmds, results) if r[0] != 0]
    if failed:
        for c, (rc, out, _) in failed:
            sys.stderr.write(" ".join(c) + "\n" + out + "\n")
        raise RuntimeError(f"{len(failed)} HIP compile step(s) failed")
    if verbose:
        for c, (_, out, dt) in zip(cmds, results):
            print(f"{dt:6.1f}s {os.path.basename(c[-1])}")
    tmp = LIB + ".tmp"
    rc, out, _ = _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp]
                      + [u[1] for u in units])
    if rc != 0:
        raise RuntimeError("link failed:\n" + out)
    os.replace(tmp, LIB)
    build_host_check(units, jobs, incremental)
    return LIB


# Host code of the runtime units instrumented by AddressSanitizer and
# UndefinedBehaviorSanitizer (-Xarch_host: the device code stays the regular
# build's), linked with the length kernels into tests/native/sfft_host_check.
HOST_CHECK = os.path.join(PKG, "sfft_host_check")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build_host_check(units, jobs, incremental=False):
    asan = os.path.join(BUILD, "asan")
    os.makedirs(asan, exist_ok=True)
    driver = os.path.join(ROOT, "tests", "native", "sfft_host_check.cpp")
    san_units = [(src, os.path.join(asan, os.path.basename(obj))) for src, obj, extra in units
                 if "kernels_L" not in obj]
    san_units.append((driver, os.path.join(asan, "sfft_host_check.o")))
    cmds = [[HIPCC] + FLAGS + SAN + ["-c", src, "-o", obj] for src, obj in san_units
            if not incremental or _stale(src, obj)]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    failed = [(c, r) for c, r in zip(cmds, results) if r[0] != 0]
    if failed:
        for c, (rc, out, _) in failed:
            sys.stderr.write(" ".join(c) + "\n" + out + "\n")
        raise RuntimeError(f"{len(failed)} sanitizer compile step(s) failed")
    objs = [obj for _, obj in san_units] + [obj for _, obj, _ in units if "kernels_L" in obj]
    rc, out, _ = _run([HIPCC, f"--offload-arch={ARCH}"] + SAN + ["-o", HOST_CHECK] + objs)
    if rc != 0:
        raise RuntimeError("host check link failed:\n" + out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--incremental", action="store_true", help="recompile only out-of-date units")
    a = ap.parse_args()
    t0 = time.time()
    path = build(a.j, a.v, a.incremental)
    print(f"built {path} in {time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
