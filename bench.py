#!/usr/bin/env python3
"""Benchmark of the split-FFT multilevel block-Toeplitz matvec on one MI355X.

Headline workload (the default): d = 3 levels, 256 x 256 x 128 grid, 3 x 3
Green-function blocks t(r) = exp(i k |r|)/|r| (I - rhat rhat^T), k = 1.3,
self term 2 I; 8 seeded complex-normal right-hand sides per apply, complex64
data path with FP64-generated symbols and twiddles. A step is one apply of the
whole hot path to the 8 right-hand sides (forward split passes, fused leaf,
inverse merge passes) in Algorithm 1's depth-first order, inputs resident in
HBM; value = matvecs/s = 8 / step time.

Prints ONE JSON line: the split path's throughput, its apply latency
percentiles (warm and after a 1 GiB cache scrub), the dominant kernel's
roofline, breadth-first / mirrored-symbol / skew-kernel variants and the full
circulant embedding on the same GPU with measured device memory, and the FP64
CPU oracle timed on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
    python bench.py --workload green64|batch|serve|gmres   (the other configurations)
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "block-Toeplitz matvecs/s & HBM roofline %, split-FFT vs full embed; p99 latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2406_17981_amd/csrc/fft_engine.hpp",
                  "paper_2406_17981_amd/csrc/axis_kernels.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic_large(kernel: str):
    """HBM bytes per launch of a 256x256x128 kernel from the committed rocprofv3
    PMC summary, or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "large_pmc_traffic.json")
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("kernels", {}).get(kernel, {}).get("measured_bytes")


def measured_traffic(kernel: str):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, or None when
    absent or taken on kernel sources that have changed since."""
    path = os.path.join(ROOT, "profiles", "leaf_pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("kernel") != kernel:
        return None
    return rec.get("bytes_per_launch")


def stream_copy_gbs(nbytes=1 << 30, reps=20):
    """Device-to-device copy bandwidth (read + write bytes per second) of a
    streaming copy of nbytes: the practical HBM ceiling on this machine. The copy
    is torch's elementwise kernel (b = a + 0), one short contiguous run per
    thread over the whole grid, which moves about a quarter more than
    Tensor.copy_'s blit kernel (hipMemcpy)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.add(a, 0.0, out=b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.add(a, 0.0, out=b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / dt / 1e9


COPY_PROBE_BYTES = 1 << 30


def pmc_probe(workload="green64"):
    """Run under rocprofv3 --pmc: a plain device copy of COPY_PROBE_BYTES (read
    and written once each) next to twelve headline matvecs (or three depth-first
    applies of the 256x256x128 workload), so the counters of the kernels can be
    scaled by those of a copy of known size."""
    import torch
    import workloads as wl
    import paper_2406_17981_amd as sf
    # the counters describe the kernels built from these sources
    log(f"[pmc-probe] kernel_source_hash {kernel_source_hash()}")
    a = torch.empty(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    if workload == "large":
        import numpy as np
        cfg = wl.LARGE_256
        n, nrhs = cfg["n"], cfg["nrhs"]
        cd = wl.green_coeffs_device(n, cfg["k"])
        x = torch.from_numpy(wl.vectors(cfg["seed_x"], n, 3, nrhs).astype(np.complex64)).cuda()
        y = torch.empty_like(x)
        for parity in (None, wl.green_parity(3)):  # general, then mirrored symbols
            plan = sf.Plan(n, 3, cd, dtype="c64", max_nrhs=nrhs, schedule="depth", parity=parity)
            ws = plan.alloc_workspace(nrhs)
            for _ in range(3):
                plan.apply(x, y, ws)
            torch.cuda.synchronize()
            plan.close()
            del ws
            torch.cuda.empty_cache()
            log(f"pmc probe: {'mirrored' if parity is not None else 'general'} symbols done")
        return
    coeffs, x_host = wl.green_64(1)
    plan = sf.Plan(wl.GREEN_64["n"], 3, torch.from_numpy(coeffs).cuda(), dtype="c64", method="split",
                   schedule="breadth")  # the 64^3 workload's schedule
    x = torch.from_numpy(x_host).to(torch.complex64).cuda()
    y = torch.empty_like(x)
    ws = plan.alloc_workspace(1)
    for _ in range(12):
        plan.apply(x, y, ws)
    torch.cuda.synchronize()
    log("pmc probe done")


def pmc_summarize(fetch_dir, write_dir, out_path, probe_log):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the leaf kernel, scaled by the
    copy probe's counters, written as JSON for the roofline's traffic field."""
    import csv
    import glob

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if r.get("Counter_Name") == counter]
        return rows

    def per_kernel(rows):
        agg = {}
        for r in rows:
            agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return agg

    out = {}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        agg = per_kernel(load(d, counter))
        copy = [v for k, v in agg.items() if "copyBuffer" in k or "copy" in k.lower() and "sfft" not in k]
        copy_kib = max(copy[0]) if copy else None
        leaf = [v for k, v in agg.items() if k.startswith("void sfft::k_leaf<float, 64, 3, 2, false, 1>")]
        leaf_kib = sorted(leaf[0])[len(leaf[0]) // 2] if leaf else None
        scale = COPY_PROBE_BYTES / (copy_kib * 1024.0) if copy_kib else None
        out[key] = dict(copy_kib=copy_kib, leaf_kib_median=leaf_kib, scale=scale,
                        leaf_bytes=leaf_kib * 1024.0 * scale if (leaf_kib and scale) else None)
    total = None
    if out["fetch"]["leaf_bytes"] is not None and out["write"]["leaf_bytes"] is not None:
        total = out["fetch"]["leaf_bytes"] + out["write"]["leaf_bytes"]
    rec = dict(kernel="sfft::k_leaf<float, 64, 3, 2, false, 1>", kernel_source_hash=probe_source_hash(probe_log),
               bytes_per_launch=total, detail=out,
               command="rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -- python3 bench.py --pmc-probe")
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


PROF_ROWS = 40  # kernel rows in a statistics table (the rest summed in one row)
VGPR_NOTE = ("VGPRs as rocprofv3 reports them, in units of two registers: the code objects' own counts "
             "(`.amdhsa_next_free_vgpr`, rounded up to a multiple of 8) are twice these, e.g. 136 for "
             "`k_leaf<float, 128, 3, 2, false, 1>`.")


def prof_summarize(db_path, out_path, title, command):
    """Kernel statistics from a rocprofv3 results database (--kernel-trace):
    launches, mean / min / max duration per kernel and workgroup count, with
    the registers and LDS of each kernel, as a Markdown table."""
    import sqlite3
    con = sqlite3.connect(db_path)
    rows = con.execute(
        "select name, grid_x / workgroup_x, count(*), avg(duration), min(duration), max(duration), "
        "sum(duration), max(vgpr_count), max(lds_size) from kernels group by name, grid_x, workgroup_x "
        "order by sum(duration) desc").fetchall()
    total = sum(r[6] for r in rows)
    lines = [f"# {title}", "", "Command (repository root, one MI355X):", "```", command, "```", "",
             VGPR_NOTE, "",
             "| kernel | workgroups | launches | mean (us) | min (us) | max (us) | share of kernel time | VGPRs | LDS (B) |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for name, wg, cnt, avg, mn, mx, tot, vgpr, lds in rows[:PROF_ROWS]:
        short = name.replace("(sfft::PassArgs)", "").replace("void ", "")
        if len(short) > 90:
            short = short[:87] + "..."
        lines.append(f"| `{short}` | {wg} | {cnt} | {avg / 1e3:.1f} | {mn / 1e3:.1f} | {mx / 1e3:.1f} | "
                     f"{100.0 * tot / total:.1f}% | {vgpr} | {lds} |")
    if len(rows) > PROF_ROWS:
        rest = rows[PROF_ROWS:]
        lines.append(f"| {len(rest)} further kernels | | {sum(r[2] for r in rest)} | | | | "
                     f"{100.0 * sum(r[6] for r in rest) / total:.1f}% | | |")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {out_path}")


# kernels of one depth-first 256x256x128 apply (8 right-hand sides) and their
# algorithmic bytes per launch: a leaf reads and writes one branch vector
# (1.61 GB each) and reads the quarter of the 3.22 GB of symbols its branch
# needs; a pass moves three branch vectors
LARGE_PMC_KERNELS = {
    "sfft::k_leaf<float, 128, 3, 2, false, 1>": 2 * 1610612736 + 805306368,
    # mirrored symbols: a branch's parities select a quarter of the stored
    # 6 x 257 x 257 x 130 entries along the outer two levels (rows of 128 + 2
    # entries: lane pairs of the 32-lane, 4-entry leaf)
    "sfft::k_leaf<float, 128, 3, 2, true, 1>": 2 * 1610612736 + 6 * 129 * 129 * 130 * 8,
    "sfft::k_strided<float, 256, 0, 256>": 3 * 1610612736,
    "sfft::k_strided<float, 256, 1, 256>": 3 * 1610612736,
}


def probe_source_hash(probe_log):
    """Kernel source hash that a --pmc-probe run printed (its stderr log)."""
    for ln in open(probe_log):
        if ln.startswith("[pmc-probe] kernel_source_hash "):
            return ln.split()[-1]
    raise SystemExit(f"{probe_log}: no kernel_source_hash line from --pmc-probe")


def pmc_summarize_large(fetch_dir, write_dir, out_path, probe_log):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE of the 256x256x128 kernels, scaled by
    the copy probe's counters, against their algorithmic bytes; stamped with the
    kernel source hash the probe reported."""
    import csv
    import glob

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if r.get("Counter_Name") == counter]
        return rows

    res = {}
    scales = {}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = load(d, counter)
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        scales[key] = COPY_PROBE_BYTES / (max(copy) * 1024.0) if copy else None
        for name in LARGE_PMC_KERNELS:
            vals = sorted(float(r["Counter_Value"]) for r in rows if r["Kernel_Name"].startswith("void " + name))
            if vals and scales[key]:
                res.setdefault(name, {})[key] = vals[len(vals) // 2] * 1024.0 * scales[key]
                res[name]["launches"] = len(vals)
    out = {}
    for name, alg in LARGE_PMC_KERNELS.items():
        r = res.get(name, {})
        if "fetch" in r and "write" in r:
            out[name] = dict(fetch_bytes=r["fetch"], write_bytes=r["write"], measured_bytes=r["fetch"] + r["write"],
                             algorithmic_bytes=alg, ratio=(r["fetch"] + r["write"]) / alg, launches=r["launches"])
    rec = dict(workload="256x256x128, b=3, 8 right-hand sides, c64, split depth-first", scales=scales,
               kernel_source_hash=probe_source_hash(probe_log), kernels=out,
               command="rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -- python3 bench.py --workload large --pmc-probe")
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


LARGE_LEAF = "sfft::k_leaf<float, 128, 3, 2, false, 1>"


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_large(coeffs, x_host, budget_s):
    """The FP64 oracle (circulant embedding, symbol transformed once before the
    timed loop) on one right-hand side of the 256x256x128 workload, with
    scipy.fft using all host cores and then one core; then the oracle's split
    product (the sum over parity branches) once with all cores."""
    import numpy as np
    import oracle
    import oracle.toeplitz as OT
    cores = len(os.sched_getaffinity(0))
    OT.set_workers(cores)
    t0 = time.perf_counter()
    C = oracle.embed_symbol(coeffs)
    t_sym = time.perf_counter() - t0
    log(f"[cpu] embedded symbol in {t_sym:.1f} s ({cores} workers)")
    runs, ref = {}, None
    for workers, budget in ((cores, budget_s), (1, 0.0)):
        OT.set_workers(workers)
        reps, t0 = 0, time.perf_counter()
        while True:
            y = oracle.embed_matvec_with_symbol(C, x_host[:1])
            reps += 1
            if ref is None:
                ref = y
            if time.perf_counter() - t0 >= budget:
                break
        wall = time.perf_counter() - t0
        runs[workers] = dict(matvecs_per_s=round(reps / wall, 5), reps=reps, wall_s=round(wall, 2))
        log(f"[cpu] workers={workers}: {reps} matvecs in {wall:.1f} s")
    # the oracle's split product (sum over the 2^d parity branches) on the same
    # right-hand side and symbol, all cores: the CPU side of split vs embed
    OT.set_workers(cores)
    t0 = time.perf_counter()
    ys = oracle.split_branch_sum_with_symbol(C, x_host[:1])
    t_split = time.perf_counter() - t0
    split = dict(matvecs_per_s=round(1.0 / t_split, 5), reps=1, wall_s=round(t_split, 2),
                 rel_l2_vs_embed=float(f"{float(np.linalg.norm(ys - ref) / np.linalg.norm(ref)):.3e}"))
    log(f"[cpu] split branch sum, workers={cores}: 1 matvec in {t_split:.1f} s")
    OT.set_workers(None)
    del C, ys
    best = runs[cores]
    return ref, dict(value=best["matvecs_per_s"], unit="matvecs/s", cores=cores, kind="oracle",
                     sample=f"{best['reps']} FP64 matvecs (1 right-hand side each) of the same 256x256x128 "
                            f"b=3 Green workload through oracle.embed_matvec_with_symbol, symbol transformed "
                            f"once beforehand ({t_sym:.1f} s, not timed); scipy.fft workers={cores}",
                     cpu_model=cpu_model(), per_workers={str(k): v for k, v in runs.items()},
                     split_branch_sum=split)


def pmc_counters_table(pmc_dir, out_path, title, command):
    """Median per-dispatch value of every counter of a rocprofv3 --pmc run
    (CSV output) for the 256x256x128 leaf kernels, as a Markdown table."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    vals = {}
    for r in rows:
        name = r["Kernel_Name"]
        for k in LARGE_PMC_KERNELS:
            if name.startswith("void " + k):
                vals.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    counters = sorted({c for v in vals.values() for c in v})
    lines = [f"# {title}", "", "Command (repository root, one MI355X):", "```", command, "```", "",
             "Median per dispatch over the probe's launches of each kernel.", "",
             "| kernel | " + " | ".join(counters) + " |", "|---|" + "---:|" * len(counters)]
    for k, cv in vals.items():
        cells = []
        for c in counters:
            v = sorted(cv.get(c, []))
            cells.append(f"{v[len(v) // 2]:.4g}" if v else "")
        lines.append(f"| `{k}` | " + " | ".join(cells) + " |")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {out_path}")


def bench_large(args):
    """Headline: 256 x 256 x 128 grid, 3x3 Green blocks (k=1.3, self term 2I),
    8 right-hand sides per apply, complex64 data path with FP64-generated
    symbols and twiddles, split product in Algorithm 1's depth-first order.
    Beside it: breadth-first, mirrored symbols, the skew-symmetric kernel and
    the full circulant embedding on the same GPU, apply latency percentiles,
    the dominant kernel's roofline and the FP64 CPU oracle."""
    import numpy as np
    import torch
    import workloads as wl
    import paper_2406_17981_amd as sf

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    dev = torch.cuda.get_device_properties(0)
    log(f"device: {dev.name}, {dev.multi_processor_count} CUs")
    cfg = wl.LARGE_256
    n, nrhs, b = cfg["n"], cfg["nrhs"], 3
    d = len(n)
    log("generating coefficients and vectors on the host")
    coeffs = wl.green_coeffs(n, cfg["k"])
    x_host = wl.vectors(cfg["seed_x"], n, b, nrhs)
    x = torch.from_numpy(x_host.astype(np.complex64)).cuda()
    y = torch.empty_like(x)
    vb = x.numel() * 8  # V: bytes of one set of 8 right-hand sides
    golden = np.load(os.path.join(ROOT, "tests", "golden", "large_256_rows.npz"))
    pts = golden["points"]
    pidx = torch.from_numpy(np.ravel_multi_index(pts.T, n)).cuda()

    def sampled_err(kname):
        got = y.reshape(nrhs, b, -1)[:, :, pidx].cpu().numpy().astype(np.complex128)
        return wl.relative_l2(got, golden[kname])

    results, rel = {}, {}
    headline = {}
    for kname in ("green", "skew"):
        if kname == "skew":
            del coeffs_d
            torch.cuda.empty_cache()
            ck = wl.skew_coeffs(n, cfg["k"])
        else:
            ck = coeffs
        coeffs_d = torch.from_numpy(ck).cuda()
        if kname == "skew":
            del ck
        par = wl.green_parity(3) if kname == "green" else wl.skew_parity(3)
        cases = [("split_depth", "split", "depth", None), ("split_breadth", "split", "breadth", None),
                 ("split_depth_mirrored", "split", "depth", par), ("embed", "embed", "auto", None)]
        if kname == "skew":
            cases = [cases[0], cases[2], cases[3]]
        for label, method, sched, parity in cases:
            key = f"{kname}_{label}"
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            plan = sf.Plan(n, b, coeffs_d, dtype="c64", method=method, parity=parity, max_nrhs=nrhs,
                           schedule=sched)
            ws = plan.alloc_workspace(nrhs)
            torch.cuda.synchronize()
            held = free0 - torch.cuda.mem_get_info()[0]
            info = plan.info()
            head = key == "green_split_depth"
            log(f"[{key}] timing {args.steps} applies after {args.warmup}")
            ms, leaf = time_plan(plan, x, y, ws, args.steps, args.warmup, profile_leaf=head)
            rel[key] = float(f"{sampled_err(kname):.3e}")
            r = dict(ms_per_apply=round(ms, 4), matvecs_per_s=round(nrhs * 1e3 / ms, 2),
                     schedule=["auto", "breadth", "depth", "slab"][info["schedule"]],
                     symbol_bytes=info["symbol_bytes"], workspace_bytes=info["workspace_bytes"],
                     model_device_bytes=info["symbol_bytes"] + info["table_bytes"] + info["workspace_bytes"] + 2 * vb,
                     measured_device_bytes=int(held) + 2 * vb)
            if head or key in ("green_embed", "green_split_depth_mirrored"):
                warm = apply_latencies(plan, x, y, ws, max(100, args.steps), pct=(50, 99))
                cold = apply_latencies(plan, x, y, ws, 30, scrub_bytes=1 << 30, pct=(50, 99))
                r["latency_ms"] = {"warm": {"p50": warm[0] / 1e3, "p99": warm[1] / 1e3},
                                   "cold": {"p50": cold[0] / 1e3, "p99": cold[1] / 1e3}}
            if head:
                headline = dict(ms=ms, leaf=leaf, info=info)
                y_c64 = y.clone()
                r["device_shares"] = time_shares(plan, x, y, nrhs, max(10, args.steps // 2))
            results[key] = r
            log(f"[{key}] {ms:.3f} ms per apply ({r['matvecs_per_s']:.0f} matvecs/s), "
                f"sampled rel L2 {rel[key]:.2e}, device bytes {r['measured_device_bytes'] / 1e9:.2f} GB")
            plan.close()
            del ws
            torch.cuda.empty_cache()
        if kname == "green":
            # FP64 residual of the complex64 product: the same product through a
            # complex128 plan, compared on the device in FP64
            plan = sf.Plan(n, b, coeffs_d, dtype="c128", method="split", max_nrhs=nrhs, schedule="depth")
            x128 = x.to(torch.complex128)
            y128 = plan.apply(x128, workspace=plan.alloc_workspace(nrhs))
            fp64_rel = (torch.linalg.vector_norm(y_c64.to(torch.complex128) - y128)
                        / torch.linalg.vector_norm(y128)).item()
            log(f"[green] rel L2 of the c64 product against the c128 product: {fp64_rel:.3e}")
            plan.close()
            del x128, y128
            torch.cuda.empty_cache()
    del coeffs_d, x
    torch.cuda.empty_cache()

    ms = headline["ms"]
    info = headline["info"]
    leaf_ms, leaf_cnt = headline["leaf"]
    sampled_applies = len(range(0, args.steps, PROFILE_EVERY))
    per_apply = leaf_cnt / max(sampled_applies, 1)
    leaf_avg_s = leaf_ms / max(leaf_cnt, 1) * 1e-3
    S = info["symbol_bytes"]
    b_alg = 2 * vb + S  # compulsory bytes of one apply: x read, y written, stored symbols read once
    achieved = b_alg / (leaf_avg_s * per_apply) / 1e9
    kernel_bytes = (2 * vb + S / per_apply)  # one leaf launch: its branch in and out, its quarter of the symbols
    model_bytes = (2 ** (d + 2) - 6) * vb + S  # every level's pass moves its branch vectors once
    copy_gbs = stream_copy_gbs()
    roofline = dict(
        bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
        frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic_large(LARGE_LEAF),
        kernel=LARGE_LEAF, avg_launch_us=round(leaf_avg_s * 1e6, 1), launches_per_apply=per_apply,
        algorithmic_bytes_per_apply=int(b_alg),
        algorithmic_bytes_per_launch=int(b_alg / per_apply),
        note="achieved = (2V + S) / (leaf launches per apply x mean leaf launch time); V = one set of 8 "
             "right-hand sides, S = stored symbol bytes",
        kernel_own=dict(bytes_per_launch=int(kernel_bytes), achieved=round(kernel_bytes / leaf_avg_s / 1e9, 1),
                        frac=round(kernel_bytes / leaf_avg_s / 1e9 / HBM_PEAK_GBS, 4)),
        whole_apply=dict(algorithmic_bytes=int(b_alg), achieved=round(b_alg / (ms * 1e-3) / 1e9, 1),
                         frac=round(b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         model_bytes=int(model_bytes), model_achieved=round(model_bytes / (ms * 1e-3) / 1e9, 1),
                         model_frac=round(model_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)),
        stream_copy_gbs=round(copy_gbs, 1))

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline (~{args.cpu_seconds:.0f} s with all cores, then one rep on one core, then one split rep)")
        ref, cpu = cpu_baseline_large(coeffs, x_host, args.cpu_seconds)
        rel["green_split_depth_full_rhs0_vs_cpu_oracle"] = float(
            f"{wl.relative_l2(y_c64[:1].cpu().numpy().astype(np.complex128), ref):.3e}")
        del ref
    g = results
    line = {
        "metric": METRIC,
        "value": g["green_split_depth"]["matvecs_per_s"],
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": g["green_split_depth"]["ms_per_apply"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "green-256x256x128-b3-k1.3-8rhs", "grid": list(n), "b": b, "nrhs": nrhs,
                   "method": "split", "schedule": "depth",
                   "kernel": "3x3 Green blocks exp(ik|r|)/|r| (I - rr^T), k=1.3, self 2I",
                   "step": "one apply of 8 right-hand sides (8 matvecs)"},
        "roofline": roofline,
        "latency_ms": g["green_split_depth"].get("latency_ms"),
        "cpu_baseline": cpu,
        "variants": g,
        "split_vs_embed": {
            "speedup": round(g["green_embed"]["ms_per_apply"] / g["green_split_depth"]["ms_per_apply"], 3),
            "device_bytes_ratio_embed_over_split": round(
                g["green_embed"]["model_device_bytes"] / g["green_split_depth"]["model_device_bytes"], 3),
            "device_bytes_ratio_embed_over_split_mirrored": round(
                g["green_embed"]["model_device_bytes"] / g["green_split_depth_mirrored"]["model_device_bytes"], 3),
            "measured_device_bytes_ratio_embed_over_split": round(
                g["green_embed"]["measured_device_bytes"] / g["green_split_depth"]["measured_device_bytes"], 3),
            "device_bytes_note": "model: symbols + tables + workspace + x + y as the plans report them; measured: "
                                 "hipMemGetInfo before plan creation and after the workspace allocation, plus x and "
                                 "y (it can include plan-creation scratch the stream-ordered pool keeps cached)",
            "skew_speedup_mirrored": round(g["skew_embed"]["ms_per_apply"]
                                           / g["skew_split_depth_mirrored"]["ms_per_apply"], 3)},
        "fp64_residual_c64_vs_c128": float(f"{fp64_rel:.3e}"),
        "rel_l2_vs_fp64_oracle": rel,
        "rel_l2_note": "sampled: all 8 right-hand sides at 128 grid points against stored FP64 oracle values "
                       "(tests/golden/large_256_rows.npz)",
    }
    print(json.dumps(line), flush=True)


def bench_batch(args):
    """Uneven-grid batch: 48x40x32, 64x64x32, 96x80x64 and 512x384, each with
    scalar (i.i.d.) and 3x3 Green blocks, 8 right-hand sides each (64 in all),
    complex64. One step = the whole batch, issued as one apply per problem, or
    as one sfft_apply_multi graph launch in each graph form (per-problem
    chains, grouped lanes) and as the library's timed choice between them."""
    import numpy as np
    import torch
    import workloads as wl
    import paper_2406_17981_amd as sf
    probs = wl.batch_problems()
    plans, xs, ys, tuned = [], [], [], []
    for pr in probs:
        plan = sf.Plan(pr["n"], pr["b"], torch.from_numpy(pr["coeffs"]).cuda(), dtype="c64",
                       max_nrhs=pr["x"].shape[0])
        tuned.append(plan.autotune(pr["x"].shape[0], use_cache=False))
        plans.append(plan)
        xs.append(torch.from_numpy(pr["x"]).to(torch.complex64).cuda())
        ys.append(torch.empty_like(xs[-1]))
    nrhs_total = sum(x.shape[0] for x in xs)
    wss = [p.alloc_workspace(x.shape[0]) for p, x in zip(plans, xs)]

    def seq():
        for p, x, y, w in zip(plans, xs, ys, wss):
            p.apply(x, y, w)

    wsm = torch.empty(max(sf.workspace_size_multi(plans, [x.shape[0] for x in xs]), 1), dtype=torch.uint8,
                      device="cuda")

    def multi():
        sf.apply_multi(plans, xs, ys, workspace=wsm)

    res = {}
    forms = {}
    saved = os.environ.get("SFFT_BATCH_MODE")
    for name, fn, form in (("sequential_applies", seq, None), ("graph_chains", multi, "chains"),
                           ("graph_grouped", multi, "grouped"), ("apply_multi_graph", multi, "auto")):
        if form == "auto":
            os.environ.pop("SFFT_BATCH_MODE", None)
        elif form is not None:
            os.environ["SFFT_BATCH_MODE"] = form
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        if form is not None:
            forms[name] = sf.batch_last_form()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        res[name] = dict(ms_per_batch=round(ms, 4), matvecs_per_s=round(nrhs_total * 1e3 / ms, 1))
        if name in forms:
            res[name]["form"] = forms[name]
        log(f"[batch {name}] {ms:.3f} ms per batch of {nrhs_total} RHS")
    if saved is None:
        os.environ.pop("SFFT_BATCH_MODE", None)
    else:
        os.environ["SFFT_BATCH_MODE"] = saved
    line = {"workload": "batch-8-problems-64rhs-c64",
            "problems": [dict(grid=list(pr["n"]), b=pr["b"], nrhs=int(pr["x"].shape[0]),
                              schedule=["auto", "breadth", "depth", "slab"][p.info()["schedule"]], tuned_us=round(t, 1))
                         for pr, p, t in zip(probs, plans, tuned)],
            "steps": args.steps, "warmup": args.warmup, "results": res,
            "graph_speedup": round(res["sequential_applies"]["ms_per_batch"] / res["apply_multi_graph"]["ms_per_batch"], 3)}
    print(json.dumps(line), flush=True)


def bench_gmres(args):
    """Krylov solve: (I - diag(chi) T) x = b by restarted GMRES(40) to a
    relative residual of 1e-8, on a 96^3 grid with 3x3 Green blocks (k = 0.7),
    chi = 0.05 (1 + 0.5i) on a ball of radius 12 cells (about 7,200 points);
    Krylov steps with complex64 products (mirrored symbols, autotuned schedule), true residuals and
    the refinement in FP64 with a complex128 plan. Time to solution (plans
    built beforehand), products per second, and the FP64 oracle's residual of
    the returned x on the host."""
    import numpy as np
    import torch
    import oracle
    import workloads as wl
    import paper_2406_17981_amd as sf
    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    n, b, tol, m = (96, 96, 96), 3, 1e-8, 40
    coeffs = wl.green_coeffs(n, 0.7)
    idx = np.indices(n)
    r2 = sum((idx[l] - n[l] / 2) ** 2 for l in range(3))
    chi = np.zeros((b,) + n, dtype=np.complex128)
    chi[:, r2 <= 12 * 12] = 0.05 * (1 + 0.5j)
    rhs = wl.vectors(506, n, b, 1)[0]
    cd = torch.from_numpy(coeffs).cuda()
    hi = sf.Plan(n, b, cd, dtype="c128", schedule="depth")
    lo = sf.Plan(n, b, cd, dtype="c64", parity=wl.green_parity(3))
    lo.autotune(nrhs=1, use_cache=False)  # schedule and pass widths of the Krylov product, by timing
    chi_d, rhs_d = torch.from_numpy(chi).cuda(), torch.from_numpy(rhs).cuda()
    ws = torch.empty(sf.gmres_workspace_size(lo, hi, m), dtype=torch.uint8, device="cuda")
    sf.gmres_solve(lo, hi, chi_d, rhs_d, m=m, max_cycles=1, tol=1e-1, workspace=ws)  # warm-up
    torch.cuda.synchronize()
    runs = []
    for _ in range(max(1, min(args.steps, 5))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = sf.gmres_solve(lo, hi, chi_d, rhs_d, m=m, max_cycles=60, tol=tol, workspace=ws)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t0, info))
        log(f"[gmres] {runs[-1][0] * 1e3:.1f} ms, {info}")
    wall, info = min(runs, key=lambda r: r[0])
    xh = x.cpu().numpy()
    ax = xh - chi * oracle.embed_matvec(coeffs, xh[None])[0]
    res = float(np.linalg.norm((rhs - ax).ravel()) / np.linalg.norm(rhs.ravel()))
    log(f"[gmres] oracle residual {res:.3e}")
    prods = info["matvecs"] + info["fp64_matvecs"]
    line = {"workload": "gmres-green-96^3-b3-k0.7-chi-ball12", "m": m, "tol": tol,
            "ms_to_solution": round(wall * 1e3, 3), "runs_ms": [round(r[0] * 1e3, 3) for r in runs],
            "cycles": info["cycles"], "c64_matvecs": info["matvecs"], "fp64_matvecs": info["fp64_matvecs"],
            "matvecs_per_s": round(prods / wall, 1), "converged": info["converged"],
            "rel_residual": info["rel_residual"], "oracle_rel_residual": float(f"{res:.3e}"),
            "chi_points": int((chi[0] != 0).sum()),
            "c64_schedule": ["auto", "breadth", "depth", "slab"][lo.info()["schedule"]]}
    lo.close()
    hi.close()
    print(json.dumps(line), flush=True)


def bench_serve(args):
    """Serving: Poisson arrivals (mean 200 req/s, seed 401), half d=2 grids
    {128..1024}^2 and half d=3 {32..128}^3, 3x3 Green kernels with k ~ U[0.5,1.5],
    each request a 30-step Arnoldi chain of matvecs. Continuous batching in
    complex64 with mirrored symbols under an HBM budget, against the plain
    FP64 path (one request at a time, full symbols) on the same stream."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2406_17981_amd import serve
    reqs = serve.poisson_requests(401, 200.0, args.requests)
    coeff_fn = lambda n, k: wl.green_coeffs_device(n, k, device="cuda")  # noqa: E731
    for n in ((8, 8), (4, 4, 4)):  # first-use warm-up of the coefficient generator's device ops
        coeff_fn(n, 1.0)
    torch.cuda.synchronize()
    out = {}
    for name, mk, max_active, nreq in (
            ("batched_c64", lambda: serve.GpuExecutor(coeff_fn, wl.green_parity, dtype="c64", mirrored=True,
                                                       **({} if args.schedule == "auto" else
                                                          {"schedule": args.schedule})), 256,
             len(reqs)),
            ("single_fp64", lambda: serve.SingleRequestExecutor(coeff_fn, None, dtype="c128", mirrored=False), 1,
             len(reqs) if args.single_requests is None else min(len(reqs), args.single_requests))):
        rs = serve.poisson_requests(401, 200.0, nreq)
        ex = mk()
        srv = serve.Server(ex, budget_bytes=int(args.budget_gb * (1 << 30)), max_active=max_active)
        log(f"[serve {name}] {nreq} requests")
        t0 = time.perf_counter()
        done = srv.run(rs)
        torch.cuda.synchronize()
        summ = serve.latency_summary(done)
        gm = [r.result["gmres_residual"] for r in done if r.result]
        summ["gmres_residual_median"] = float(f"{float(np.median(gm)):.3e}") if gm else None
        summ.update(wall_s=round(time.perf_counter() - t0, 3), server_steps=srv.steps_run,
                    host_s_admit=round(srv.time_in["admit"], 3), host_s_step=round(srv.time_in["step"], 3),
                    host_s_step_waiting_for_device=round(ex.wait_s, 3),
                    host_s_finish=round(srv.time_in["finish"], 3),
                    mean_batch=round(sum(srv.batch_sizes) / max(len(srv.batch_sizes), 1), 2),
                    peak_reserved_gb=round(srv.peak_reserved / 2 ** 30, 2))
        out[name] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in summ.items()}
        log(f"[serve {name}] p50 {summ['p50_s']:.3f} s p99 {summ['p99_s']:.3f} s, "
            f"{summ['matvecs_per_s']:.0f} matvecs/s")
        ex.close()
        del ex, srv
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "serve-poisson200-green-b3-arnoldi30", "results": out,
                      "budget_gb": args.budget_gb}), flush=True)


PROFILE_EVERY = 10  # leaf launches bracketed by HIP events: every 10th apply of the timed region


def time_plan(plan, x, y, ws, steps, warmup, profile_leaf=False):
    """Mean wall time per apply (ms) over `steps` applies after `warmup`; with
    profile_leaf, the leaf launches of every PROFILE_EVERY-th timed apply are
    bracketed by HIP events on the apply stream (an event pair delays the
    launches around it, so bracketing them all would slow the region it
    measures), returning (total leaf ms, launches) as well."""
    import torch
    for _ in range(warmup):
        plan.apply(x, y, ws)
    torch.cuda.synchronize()
    if profile_leaf:
        plan.profile_read("leaf", reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        sample = profile_leaf and i % PROFILE_EVERY == 0
        if sample:
            plan.profile(("leaf",))
        plan.apply(x, y, ws)
        if sample:
            plan.profile(())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    leaf = plan.profile_read("leaf", reset=True) if profile_leaf else None
    return (t1 - t0) * 1e3 / steps, leaf


def time_shares(plan, x, y, nrhs, reps):
    """One device's share of the product when it is split over 2^k devices by
    branch (Plan.apply_subtree, k = 1 and 2; the shares sum to T x): mean time
    per share (ms, wall clock over reps calls after two warm-up calls) for the
    first and the last branch prefix, and the share's workspace. The
    cross-device sum of the shares is not part of it."""
    import torch
    out = {"note": "ms per share of all right-hand sides (apply_subtree); k levels split across 2^k devices; "
                   "the sum-reduce across devices is not included"}
    for k in (1, 2):
        nb = plan.workspace_size_subtree(k, nrhs)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda") if nb else None
        times = []
        for prefix in (0, (1 << k) - 1):
            for _ in range(2):
                plan.apply_subtree(k, prefix, x, y, workspace=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                plan.apply_subtree(k, prefix, x, y, workspace=ws)
            torch.cuda.synchronize()
            times.append(round((time.perf_counter() - t0) * 1e3 / reps, 4))
        out[f"k{k}"] = {"ms_per_share": {"prefix_0": times[0], f"prefix_{(1 << k) - 1}": times[1]},
                        "workspace_bytes": nb}
        log(f"[shares] k={k}: {times[0]:.3f} / {times[1]:.3f} ms per share (first / last prefix)")
        del ws
    return out


def apply_latencies(plan, x, y, ws, reps, scrub_bytes=0, pct=(10, 50, 90)):
    """Per-apply device time (HIP events around each apply on the current
    stream), optionally after a fill of scrub_bytes that evicts the
    memory-side cache; returns the percentiles pct in microseconds."""
    import numpy as np
    import torch
    scrub = torch.empty(max(scrub_bytes // 4, 1), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    plan.apply(x, y, ws)
    torch.cuda.synchronize()
    for i in range(reps):
        if scrub_bytes:
            scrub.fill_(float(i))
        ev[i][0].record(st)
        plan.apply(x, y, ws)
        ev[i][1].record(st)
    torch.cuda.synchronize()
    us = np.array([a.elapsed_time(b) * 1e3 for a, b in ev])
    del scrub
    torch.cuda.empty_cache()
    return tuple(round(float(v), 2) for v in np.percentile(us, list(pct)))


def time_plan_cold(plan, x, y, ws, reps, scrub_bytes=1 << 30):
    """Cold-cache timing: before every apply, a 1 GiB fill evicts the 256 MB
    memory-side cache, so symbols and vectors stream from HBM. Returns the
    mean apply time (ms, events around the apply only) and the leaf record."""
    import torch
    scrub = torch.empty(scrub_bytes // 4, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    plan.apply(x, y, ws)
    torch.cuda.synchronize()
    plan.profile(("leaf",))
    plan.profile_read("leaf", reset=True)
    for i in range(reps):
        scrub.fill_(float(i))
        ev[i][0].record(st)
        plan.apply(x, y, ws)
        ev[i][1].record(st)
    torch.cuda.synchronize()
    leaf = plan.profile_read("leaf", reset=True)
    plan.profile(())
    ms = sum(a.elapsed_time(b) for a, b in ev) / reps
    del scrub
    torch.cuda.empty_cache()
    return ms, leaf


def cpu_baseline(coeffs, x, budget_s):
    """The FP64 oracle's circulant-embedding matvec timed on the host cores."""
    import oracle
    reps, t0 = 0, time.perf_counter()
    c0 = os.times()
    ref = None
    while True:
        ref = oracle.embed_matvec(coeffs, x)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    wall = time.perf_counter() - t0
    c1 = os.times()
    cpu = (c1.user - c0.user) + (c1.system - c0.system)
    cores = max(1, int(round(cpu / wall)))
    return ref, dict(value=reps / wall, unit="matvecs/s", cores=cores, kind="oracle",
                     sample=f"{reps} full FP64 matvecs of the same 64^3 b=3 Green workload through "
                            f"oracle.embed_matvec (symbol transform included each call), "
                            f"{wall:.1f} s wall")


def bench_green64(args):
    """64^3 grid, 3x3 Green blocks (k=0.7), one right-hand side per apply: the split
    path in complex64 and complex128, mirrored symbols, all 9 components, and the
    full embedding, with the leaf's roofline and the FP64 CPU oracle."""
    import numpy as np
    import torch
    import workloads as wl
    import paper_2406_17981_amd as sf

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    dev = torch.cuda.get_device_properties(0)
    log(f"device: {dev.name}, {dev.multi_processor_count} CUs")

    cfg = wl.GREEN_64
    n, b, nrhs = cfg["n"], cfg["b"], 1
    coeffs, x_host = wl.green_64(nrhs)
    coeffs_d = torch.from_numpy(coeffs).cuda()
    s = math.prod(n)
    d = len(n)

    # breadth-first by default here: at 64^3 with one right-hand side it is the
    # autotuner's choice (fewer, larger launches), and the counters in
    # profiles/leaf_pmc_traffic.* are taken on it
    sched64 = "breadth" if args.schedule == "auto" else args.schedule
    results = {}
    outputs = {}
    variants = [("split", "c64"), ("split", "c128"), ("embed", "c64"), ("embed", "c128"),
                ("split_mirrored", "c64"), ("split_mirrored", "c128"), ("split_all9", "c64")]
    if args.variants == "headline":
        variants = variants[:1]
    headline_leaf = None
    cold = lat_warm = lat_cold = None
    for vmethod, dtype in variants:
        method = "split" if vmethod.startswith("split") else "embed"
        parity = wl.green_parity(3) if vmethod == "split_mirrored" else None
        tdt = torch.complex64 if dtype == "c64" else torch.complex128
        esz = 8 if dtype == "c64" else 16
        # split_all9: the symbols of all 9 block components, as for a kernel
        # without block symmetry (the Green blocks are symmetric: 6 are stored)
        if vmethod == "split_all9":
            os.environ["SFFT_NO_BLOCK_SYMMETRY"] = "1"
        plan = sf.Plan(n, b, coeffs_d, dtype=dtype, method=method, max_nrhs=nrhs,
                       schedule=sched64, parity=parity)
        os.environ.pop("SFFT_NO_BLOCK_SYMMETRY", None)
        info = plan.info()
        x = torch.from_numpy(x_host).to(tdt).cuda()
        y = torch.empty_like(x)
        ws = plan.alloc_workspace(nrhs)
        head = (vmethod, dtype) == variants[0]
        log(f"[{vmethod} {dtype}] timing {args.steps} steps after {args.warmup} warmup")
        ms, leaf = time_plan(plan, x, y, ws, args.steps, args.warmup, profile_leaf=head)
        if head:
            cold = time_plan_cold(plan, x, y, ws, max(10, min(args.steps, 50)))
            lat_warm = apply_latencies(plan, x, y, ws, 100)
            lat_cold = apply_latencies(plan, x, y, ws, 50, scrub_bytes=1 << 30)
        vbytes = nrhs * b * s * esz
        dev_bytes = info["symbol_bytes"] + info["table_bytes"] + info["workspace_bytes"] + 2 * vbytes
        results[f"{vmethod}_{dtype}"] = dict(
            matvecs_per_s=nrhs * 1e3 / ms, ms_per_matvec=ms, schedule=["auto", "breadth", "depth", "slab"][info["schedule"]],
            device_bytes=dev_bytes, symbol_bytes=info["symbol_bytes"],
            workspace_bytes=info["workspace_bytes"], vector_bytes=vbytes,
            block_symmetry=info["block_symmetry"])
        outputs[f"{vmethod}_{dtype}"] = y.cpu().numpy().astype(np.complex128)
        if head:
            headline_leaf = (leaf, info, vbytes, ms)
        plan.close()
        del x, y, ws
        torch.cuda.empty_cache()

    if args.variants == "all":
        # context: the same operator on 8 right-hand sides per apply (the leaf
        # fetches each symbol block once for the right-hand sides of a workgroup)
        x8 = torch.from_numpy(wl.vectors(203, n, b, 8).astype(np.complex64)).cuda()
        plan = sf.Plan(n, b, coeffs_d, dtype="c64", method="split", max_nrhs=8, schedule=sched64)
        y8 = torch.empty_like(x8)
        ws8 = plan.alloc_workspace(8)
        ms8, _ = time_plan(plan, x8, y8, ws8, max(args.steps // 4, 10), args.warmup)
        results["split_c64_8rhs"] = dict(matvecs_per_s=8e3 / ms8, ms_per_apply=ms8,
                                         schedule=["auto", "breadth", "depth", "slab"][plan.info()["schedule"]])
        plan.close()
        del x8, y8, ws8
        torch.cuda.empty_cache()

    (leaf_ms, leaf_cnt), info, vbytes, ms = headline_leaf
    leaf_avg_s = leaf_ms / max(leaf_cnt, 1) * 1e-3
    # a breadth-first leaf launch takes every branch prefix of levels 1..d-1,
    # a depth-first one a single branch (and the symbols of that branch)
    nbr = 2 ** (d - 1) if info["schedule"] == 1 else 1
    leaf_alg_bytes = 2 * nbr * vbytes + info["symbol_bytes"] * nbr // 2 ** (d - 1)
    achieved = leaf_alg_bytes / leaf_avg_s / 1e9
    leaf_kernel = f"sfft::k_leaf<float, 64, 3, 2, false, {info['block_symmetry']}>"
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic(leaf_kernel),
                    kernel=leaf_kernel, avg_launch_us=round(leaf_avg_s * 1e6, 2),
                    launches=leaf_cnt, algorithmic_bytes_per_launch=int(leaf_alg_bytes))

    cold_ms, (cold_leaf_ms, cold_cnt) = cold
    cold_leaf_s = cold_leaf_ms / max(cold_cnt, 1) * 1e-3
    roofline["cold"] = dict(avg_launch_us=round(cold_leaf_s * 1e6, 2),
                            achieved=round(leaf_alg_bytes / cold_leaf_s / 1e9, 1),
                            frac=round(leaf_alg_bytes / cold_leaf_s / 1e9 / HBM_PEAK_GBS, 4),
                            ms_per_matvec=round(cold_ms / nrhs, 5), launches=cold_cnt,
                            note="1 GiB fill before each apply evicts the memory-side cache")

    copy_gbs = stream_copy_gbs()
    roofline["stream_copy_gbs"] = round(copy_gbs, 1)
    roofline["frac_of_stream_copy"] = round(achieved / copy_gbs, 4)
    # the whole product: every level's pass moves its branch vectors once,
    # (2^(d+2) - 6) V over the d-1 forward passes, the leaf and the d-1
    # inverse passes, plus the stored symbols once
    path_bytes = (2 ** (d + 2) - 6) * vbytes + info["symbol_bytes"]
    path_gbs = path_bytes / (ms * 1e-3) / 1e9
    roofline["whole_matvec"] = dict(bytes_per_matvec=int(path_bytes), achieved=round(path_gbs, 1),
                                    frac=round(path_gbs / HBM_PEAK_GBS, 4),
                                    frac_of_stream_copy=round(path_gbs / copy_gbs, 4))

    cpu = None
    rel = {}
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline, ~{args.cpu_seconds:.0f} s")
        ref, cpu = cpu_baseline(coeffs, x_host, args.cpu_seconds)
        for k, v in outputs.items():
            rel[k] = wl.relative_l2(v, ref)

    head = results["split_c64"]
    emb = results.get("embed_c64")
    line = {
        "metric": METRIC,
        "value": round(head["matvecs_per_s"], 2),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_matvec"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "green-64^3-b3-k0.7", "grid": list(n), "b": b, "nrhs": nrhs,
                   "method": "split", "schedule": head["schedule"],
                   "kernel": "3x3 Green blocks exp(ik|r|)/|r| (I - rr^T), k=0.7, self 2I"},
        "roofline": roofline,
        "latency_us": {"warm": dict(zip(("p10", "p50", "p90"), lat_warm)),
                       "cold": dict(zip(("p10", "p50", "p90"), lat_cold)),
                       "note": "device time per apply (events around each apply); cold: after a 1 GiB fill"},
        "cpu_baseline": cpu,
        "variants": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                     for k, v in results.items()},
        "speedup_vs_embed": {dt: round(results[f"split_{dt}"]["matvecs_per_s"] /
                                       results[f"embed_{dt}"]["matvecs_per_s"], 3)
                             for dt in ("c64", "c128") if f"embed_{dt}" in results},
        "device_bytes_ratio_embed_over_split": {
            dt: round(results[f"embed_{dt}"]["device_bytes"] / results[f"split_{dt}"]["device_bytes"], 4)
            for dt in ("c64", "c128") if f"embed_{dt}" in results},
        "rel_l2_vs_fp64_oracle": {k: float(f"{v:.3e}") for k, v in rel.items()},
    }
    if emb is None:
        line.pop("speedup_vs_embed")
    print(json.dumps(line), flush=True)



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed applies (default 20 large, 1000 green64, 50 batch)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed applies first (default 5 large; 2000 green64, whose applies are "
                         "short and would otherwise run before the GPU clocks ramp up; 5 batch)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "breadth", "depth", "slab"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default="all", choices=["all", "headline"])
    ap.add_argument("--pmc-probe", action="store_true", help="workload for rocprofv3 --pmc runs")
    ap.add_argument("--requests", type=int, default=400, help="serve: requests in the stream")
    ap.add_argument("--single-requests", type=int, default=None,
                    help="serve: requests for the FP64 path (default: the same stream)")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve: HBM budget")
    ap.add_argument("--workload", default="large", choices=["large", "green64", "batch", "serve", "gmres"],
                    help="large (default, the headline): 256x256x128, b=3, 8 RHS, split vs embed; "
                         "green64: the 64^3 one-RHS configuration; "
                         "batch: 8 uneven-grid problems, 64 RHS, one graph; serve: the Poisson stream; "
                         "gmres: restarted GMRES on I - chi T, 96^3 Green blocks")
    ap.add_argument("--pmc-summarize", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON", "PROBE_LOG"),
                    help="PROBE_LOG: stderr of one of the --pmc-probe runs (names the kernel sources measured)")
    ap.add_argument("--prof-summarize", nargs=4, metavar=("RESULTS_DB", "OUT_MD", "TITLE", "COMMAND"),
                    help="write a kernel-statistics table from a rocprofv3 --kernel-trace results database")
    ap.add_argument("--pmc-table", nargs=4, metavar=("PMC_DIR", "OUT_MD", "TITLE", "COMMAND"),
                    help="write the leaf kernels' counters of a rocprofv3 --pmc run (CSV) as a table")
    args = ap.parse_args()
    steps_default, warmup_default = {"large": (20, 5), "batch": (50, 5), "green64": (1000, 2000), "gmres": (3, 1)}.get(
        args.workload, (1, 0))
    if args.steps is None:
        args.steps = steps_default
    if args.warmup is None:
        args.warmup = warmup_default

    if args.prof_summarize:
        prof_summarize(*args.prof_summarize)
        return
    if args.pmc_table:
        pmc_counters_table(*args.pmc_table)
        return
    if args.pmc_summarize:
        (pmc_summarize_large if args.workload == "large" else pmc_summarize)(*args.pmc_summarize)
        return
    if args.pmc_probe:
        pmc_probe(args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "one device's share of a branch-split product is timed on one GPU instead (device_shares).",
              file=sys.stderr)
        sys.exit(2)

    {"large": bench_large, "green64": bench_green64, "batch": bench_batch, "serve": bench_serve,
     "gmres": bench_gmres}[args.workload](args)


if __name__ == "__main__":
    main()
