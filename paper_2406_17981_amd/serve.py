"""Continuous-batching server for Krylov chains of block-Toeplitz matvecs.

Each request is a GMRES-style Arnoldi chain on its own operator T (a 3x3
Green-function block-Toeplitz matrix on a d = 2 or 3 grid): v_0 = b/||b||,
then `steps` times w = T v_j, orthogonalise w against v_0..v_j, normalise.
The server

* admits arrived requests first-come first-served while their device memory
  (plan symbols and tables, workspace, the Krylov basis, and the transient
  coefficient / FP64 symbol scratch of plan creation) fits an HBM budget;
  requests that do not fit wait in the queue;
* advances every active request by one Arnoldi step per server step: the
  matvecs of all active requests are issued over several streams so their
  kernels overlap on the device, then one sfft_arnoldi_step_multi call
  orthogonalises all of them;
* admits new requests between steps as slots and memory free up (continuous
  batching), and records arrival, admission and completion times;
* finishes a request with the GMRES solve of T x = b on its chain: the small
  least-squares problem min ||beta e_1 - H y|| on the host and x = V y on the
  device. The host does not wait for the device between steps: a finished
  chain's Hessenberg matrix is copied back asynchronously and the request
  completes once that copy has landed, while later steps are already queued;
* keeps the plans of finished requests for reuse: a new request on the same
  grid takes one over and only regenerates its symbols (sfft_plan_update),
  so admission allocates and frees no device memory; idle plans count
  against the budget and are closed when an admission needs the room;
* isolates failures: a request larger than the whole budget, one whose
  admission raises (say an allocation failure) and one whose step or
  completion fails end alone with an error result, their memory returned;
  the others carry on. Requests can be cancelled (queued, waiting or
  active) and may carry a deadline after which they are cancelled.

Every kernel is deterministic and works on one request's buffers only, so a
request's results are bitwise the same alone and in any mix.

The device work is behind an executor interface so the scheduler can be
tested on the host with a mock executor.
"""

from __future__ import annotations

import concurrent.futures as cf
import ctypes as C
import math
import queue as queue_mod
import threading
import time
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the stream starts
    n: tuple                       # grid
    k: float                       # Green-function wavenumber
    steps: int = 30                # matvecs in the chain
    seed: int = 0                  # seeds the start vector
    deadline: Optional[float] = None  # seconds after arrival; cancelled when exceeded
    # filled by the server
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Optional[dict] = None
    status: str = "pending"        # "ok", "error" or "cancelled" once it has left the server

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


def poisson_requests(seed: int, rate: float, count: int, steps: int = 30,
                     d2_sizes=(128, 256, 512, 1024), d3_sizes=(32, 64, 96, 128),
                     k_range=(0.5, 1.5)) -> List[Request]:
    """Poisson arrivals (exponential gaps, mean 1/rate); half d = 2 grids, half
    d = 3, sizes uniform over the given sets, k uniform over k_range."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for i in range(count):
        if rng.random() < 0.5:
            nn = int(rng.choice(d2_sizes))
            n = (nn, nn)
        else:
            nn = int(rng.choice(d3_sizes))
            n = (nn, nn, nn)
        out.append(Request(rid=i, arrival=float(t[i]), n=n, k=float(rng.uniform(*k_range)), steps=steps,
                           seed=4000 + i))
    return out


class Executor:
    """Device side of the server (one implementation per backend)."""

    def bytes_needed(self, req: Request) -> tuple:
        """(resident bytes, extra transient bytes during admission)."""
        raise NotImplementedError

    def admit(self, req: Request) -> object:
        raise NotImplementedError

    def admit_start(self, req: Request) -> cf.Future:
        """Starts admitting req; the future's result is the slot handle (or
        the admission's exception). The default admits synchronously."""
        fut = cf.Future()
        try:
            fut.set_result(self.admit(req))
        except Exception as e:  # noqa: BLE001
            fut.set_exception(e)
        return fut

    def step(self, slots: Sequence[object]) -> Optional[List[tuple]]:
        """One Arnoldi step for each slot. Returns (index into slots, message)
        for every slot whose step failed (None or [] when all succeeded); a
        failed slot takes no further steps."""
        raise NotImplementedError

    def finish_start(self, slot: object) -> None:
        """Starts fetching a finished chain's results without waiting."""

    def finish_ready(self, slot: object) -> bool:
        """True once finish(slot) would not wait for the device."""
        return True

    def finish_wait(self, slot: object) -> None:
        """Blocks until finish_ready(slot)."""

    def finish(self, slot: object) -> dict:
        raise NotImplementedError

    def release(self, slot: object) -> None:
        raise NotImplementedError

    def idle_bytes(self, req: Optional[Request] = None) -> int:
        """Device bytes kept for reuse outside any request, less what admitting
        `req` would take over (counted in its own bytes_needed)."""
        return 0

    def trim(self, req: Optional[Request] = None) -> None:
        """Frees the memory idle_bytes(req) counts."""


@dataclass
class _Slot:
    req: Request
    handle: object
    reserved: int
    done_steps: int = 0


ADMITTED, WAIT, REJECTED = "admitted", "wait", "rejected"


class Server:
    """Admission by HBM budget, continuous batching, completion bookkeeping,
    per-request failure isolation and cancellation."""

    def __init__(self, executor: Executor, budget_bytes: int, max_active: int = 256,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = max_active
        self.clock = clock
        self.sleep = sleep
        self.reserved = 0
        self.peak_reserved = 0
        self.steps_run = 0
        self.batch_sizes: List[int] = []
        self.time_in = dict(admit=0.0, step=0.0, finish=0.0)  # host seconds per phase
        self.failed = 0
        self.cancelled = 0
        self._cancel = set()
        self._admitting = []  # (request, future of its slot, resident, transient bytes)

    def cancel(self, rid: int) -> None:
        """Cancels request rid wherever it is (not yet arrived, queued, active);
        takes effect at the next server step boundary. Thread-safe."""
        self._cancel.add(rid)

    def _end(self, req: Request, status: str, result: Optional[dict], t0: float, finished: List[Request]) -> None:
        req.status = status
        req.result = result
        req.done = self.clock() - t0
        if status == "error":
            self.failed += 1
        elif status == "cancelled":
            self.cancelled += 1
        finished.append(req)

    def _try_admit(self, req: Request, now: float, active: List[_Slot], draining: int = 0) -> str:
        resident, transient = self.ex.bytes_needed(req)
        if resident + transient > self.budget:
            req.result = dict(error=f"needs {resident + transient} bytes, more than the budget of {self.budget}")
            return REJECTED
        if len(active) + draining + len(self._admitting) >= self.max_active:
            return WAIT
        if self.reserved + resident + transient + self.ex.idle_bytes(req) > self.budget and self.ex.idle_bytes(req):
            self.ex.trim(req)
        if self.reserved + resident + transient + self.ex.idle_bytes(req) > self.budget:
            return WAIT
        self.reserved += resident + transient
        self.peak_reserved = max(self.peak_reserved, self.reserved)
        t = self.clock()
        fut = self.ex.admit_start(req)
        self.time_in["admit"] += self.clock() - t
        req.admitted = now
        self._admitting.append((req, fut, resident, transient))
        return ADMITTED

    def _collect_admissions(self, active: List[_Slot], t0: float, finished: List[Request], wait: bool) -> None:
        """Moves finished admissions to the active set (in admission order);
        with wait, blocks for the oldest one first."""
        if wait and self._admitting:
            t = self.clock()
            cf.wait([self._admitting[0][1]])
            self.time_in["admit"] += self.clock() - t
        keep = []
        for req, fut, resident, transient in self._admitting:
            if not fut.done():
                keep.append((req, fut, resident, transient))
                continue
            exc = fut.exception()
            if exc is not None:  # one request's failure must not end the others
                self.reserved -= resident + transient
                self._end(req, "error", dict(error=f"admission failed: {type(exc).__name__}: {exc}"), t0, finished)
            else:
                self.reserved -= transient
                active.append(_Slot(req, fut.result(), resident))
        self._admitting = keep

    def _retire(self, s: _Slot, status: str, result: dict, t0: float, finished: List[Request]) -> None:
        """Ends an active or draining slot that did not complete normally."""
        try:
            self.ex.release(s.handle)
        except Exception as e:  # noqa: BLE001
            result = dict(result, release_error=f"{type(e).__name__}: {e}")
        self.reserved -= s.reserved
        self._end(s.req, status, result, t0, finished)

    def _complete(self, s: _Slot, t0: float, finished: List[Request]) -> None:
        t = self.clock()
        try:
            result = self.ex.finish(s.handle)
        except Exception as e:  # noqa: BLE001
            self._retire(s, "error", dict(error=f"completion failed: {type(e).__name__}: {e}"), t0, finished)
            self.time_in["finish"] += self.clock() - t
            return
        self.ex.release(s.handle)
        self.time_in["finish"] += self.clock() - t
        self.reserved -= s.reserved
        self._end(s.req, "ok", result, t0, finished)

    def _expired(self, req: Request, now: float) -> bool:
        return req.rid in self._cancel or (req.deadline is not None and now - req.arrival > req.deadline)

    def run(self, requests: Sequence[Request]) -> List[Request]:
        pending = sorted(requests, key=lambda r: r.arrival)
        queue: List[Request] = []
        active: List[_Slot] = []
        draining: List[_Slot] = []   # chains done, results on their way back
        finished: List[Request] = []
        t0 = self.clock()
        i = 0
        while i < len(pending) or queue or active or draining or self._admitting:
            still = []
            for s in draining:
                if self.ex.finish_ready(s.handle):
                    self._complete(s, t0, finished)
                else:
                    still.append(s)
            draining = still
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival <= now:
                queue.append(pending[i])
                i += 1
            # cancellations and deadlines (queued and active requests)
            keep = []
            for r in queue:
                if self._expired(r, now):
                    self._end(r, "cancelled", dict(cancelled=True), t0, finished)
                else:
                    keep.append(r)
            queue = keep
            keep = []
            for s in active:
                if self._expired(s.req, now):
                    self._retire(s, "cancelled", dict(cancelled=True, steps_done=s.done_steps), t0, finished)
                else:
                    keep.append(s)
            active = keep
            while queue:
                outcome = self._try_admit(queue[0], self.clock() - t0, active, len(draining))
                if outcome == WAIT:
                    break
                r = queue.pop(0)
                if outcome == REJECTED:
                    self._end(r, "error", r.result, t0, finished)
            self._collect_admissions(active, t0, finished, wait=not active and not draining)
            if not active:
                if draining:
                    self.ex.finish_wait(draining[0].handle)
                elif i < len(pending) and not self._admitting:
                    self.sleep(max(0.0, pending[i].arrival - (self.clock() - t0)))
                continue
            t = self.clock()
            failures = self.ex.step([s.handle for s in active]) or []
            self.time_in["step"] += self.clock() - t
            self.steps_run += 1
            self.batch_sizes.append(len(active))
            bad = dict(failures)
            still = []
            for k, s in enumerate(active):
                if k in bad:
                    self._retire(s, "error", dict(error=f"step failed: {bad[k]}", steps_done=s.done_steps), t0,
                                 finished)
                    continue
                s.done_steps += 1
                if s.done_steps >= s.req.steps:
                    self.ex.finish_start(s.handle)
                    draining.append(s)
                else:
                    still.append(s)
            active = still
        return finished


def latency_summary(reqs: Sequence[Request]) -> dict:
    """Latency percentiles and throughput over the requests that completed
    (failed and cancelled ones are counted apart)."""
    ok = [r for r in reqs if r.latency is not None and r.status in ("ok", "pending")]
    lat = np.array([r.latency for r in ok])
    if lat.size == 0:
        return {}
    span = max(r.done for r in ok) - min(r.arrival for r in ok)
    mv = sum(r.steps for r in ok)
    return dict(requests=int(lat.size), p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), max_s=float(lat.max()), span_s=float(span),
                requests_per_s=float(lat.size / span), matvecs_per_s=float(mv / span),
                failed=sum(r.status == "error" for r in reqs), cancelled=sum(r.status == "cancelled" for r in reqs))


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------

class GpuExecutor(Executor):
    """Plans (3x3 blocks), a Krylov basis of steps+1 vectors and a Hessenberg
    matrix per request; matvecs over `nstreams` streams.

    coeff_fn(n, k) returns the request's complex128 device coefficient array
    (3, 3, 2n_1-1, ...); parity_fn(d) its (3, 3, d) symmetry mask, used when
    `mirrored` (symbols stored mirrored)."""

    def __init__(self, coeff_fn, parity_fn=None, dtype: str = "c64", nstreams: int = 4, mirrored: bool = True,
                 schedule: str = "depth", keep_basis: bool = False, max_ahead: int = 2, admit_workers: int = 3):
        import torch
        from . import _native as N
        from .plan import Plan
        self.torch = torch
        self.N = N
        self.Plan = Plan
        self.coeff_fn = coeff_fn
        self.parity_fn = parity_fn
        self.keep_basis = keep_basis
        if mirrored and parity_fn is None:
            raise ValueError("mirrored storage needs parity_fn")
        self.dtype = dtype
        self.tdt = torch.complex64 if dtype == "c64" else torch.complex128
        self.esz = 8 if dtype == "c64" else 16
        self.mirrored = mirrored
        self.schedule = schedule
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.main = torch.cuda.current_stream()
        # plan creation (coefficients, FP64 symbols) runs on streams of its own,
        # so its completion waits do not drain the other requests' queued steps
        self.admit_stream = torch.cuda.Stream()
        self._scratch = None
        # plans of finished requests by grid, each with the event after its
        # last use, and their device bytes
        self._idle = {}
        self._idle_total = 0
        # server steps queued on the device beyond the one being issued
        self.max_ahead = max_ahead
        self._inflight = []
        self.wait_s = 0.0  # host seconds spent waiting for the device to drain queued steps
        # admissions (coefficients, plan creation or update, basis, start
        # vector) run on worker threads, each with its own stream and Arnoldi
        # scratch, so the server keeps issuing steps meanwhile and several
        # admissions overlap; the idle-plan pool is shared under a lock
        self._pool = cf.ThreadPoolExecutor(max_workers=admit_workers)
        self._lock = threading.Lock()
        self._lanes = queue_mod.Queue()
        for k in range(admit_workers):
            self._lanes.put((self.admit_stream if k == 0 else torch.cuda.Stream(), f"_adm_scratch{k}"))
            setattr(self, f"_adm_scratch{k}", None)

    def bytes_needed(self, req: Request) -> tuple:
        n, d, b = req.n, len(req.n), 3
        s = math.prod(n)
        V = b * s * self.esz
        sym = 9 * math.prod(v + 1 for v in n) * self.esz if self.mirrored else 2 ** d * 9 * s * self.esz
        ws = (d - 1) * V if self.schedule == "depth" else (2 ** d - 2) * V
        resident = sym + ws + (req.steps + 2) * V + (1 << 20)
        transient = 9 * math.prod(2 * v - 1 for v in n) * 16 + math.prod(2 * v for v in n) * 16
        return resident, transient

    @staticmethod
    def _plan_bytes(plan) -> int:
        info = plan.info()
        return int(info["symbol_bytes"] + info["table_bytes"])

    def idle_bytes(self, req: Optional[Request] = None) -> int:
        with self._lock:
            total = self._idle_total
            if req is not None and self._idle.get(tuple(req.n)):
                total -= self._idle[tuple(req.n)][-1][2]
            return total

    def trim(self, req: Optional[Request] = None) -> None:
        keep = tuple(req.n) if req is not None else None
        with self._lock:
            for key, lst in list(self._idle.items()):
                stay = lst[-1:] if key == keep else []
                for plan, ev, nb in lst[:len(lst) - len(stay)]:
                    ev.synchronize()
                    plan.close()
                    self._idle_total -= nb
                self._idle[key] = stay

    def close(self) -> None:
        self._pool.shutdown(wait=True)
        self.trim()

    def admit(self, req: Request) -> dict:
        """Synchronous admission (the work admit_start does on the worker)."""
        slot = self._admit_job(req)
        self.main.wait_event(slot.pop("ready"))
        return slot

    def admit_start(self, req: Request) -> cf.Future:
        return self._pool.submit(self._admit_job, req)

    def _admit_job(self, req: Request) -> dict:
        """Admission on the admission stream: coefficients, a reused plan's
        update (after its last use) or a new plan, the Krylov basis with the
        start vector, and v_0 = b / ||b||. The slot's "ready" event marks the
        end of this work; its first step waits for it on the main stream."""
        lane = self._lanes.get()
        try:
            return self._admit_on(req, *lane)
        finally:
            self._lanes.put(lane)

    def _admit_on(self, req: Request, stream, scratch: str) -> dict:
        torch = self.torch
        n, b = req.n, 3
        with self._lock:
            reuse = self._idle.get(tuple(n))
            entry = reuse.pop() if reuse else None
            if entry is not None:
                self._idle_total -= entry[2]
        with torch.cuda.stream(stream):
            coeffs = self.coeff_fn(n, req.k)
            if entry is not None:
                # the plan's last applies finish before its symbols change
                plan, ev, _ = entry
                stream.wait_event(ev)
                plan.update(coeffs, stream=stream)
            else:
                par = self.parity_fn(len(n)) if self.mirrored else None
                plan = self.Plan(n, b, coeffs, dtype=self.dtype, parity=par, max_nrhs=1, schedule=self.schedule,
                                 stream=stream)
            del coeffs
            vlen = b * math.prod(n)
            basis = torch.empty((req.steps + 1, vlen), dtype=self.tdt, device="cuda")
            # start vector b: complex normal, drawn on the device from the request's seed
            g = torch.Generator(device="cuda").manual_seed(req.seed)
            real = self.tdt.to_real()
            basis[0].copy_(torch.complex(torch.randn(vlen, generator=g, dtype=real, device="cuda"),
                                         torch.randn(vlen, generator=g, dtype=real, device="cuda")))
            # Hessenberg matrix stored by columns: Hc[j] is column j (contiguous);
            # Hc[steps][0] receives ||b||
            Hc = torch.zeros((req.steps + 1, req.steps + 1), dtype=torch.complex128, device="cuda")
            ws = plan.alloc_workspace(1)
            w = torch.empty(vlen, dtype=self.tdt, device="cuda")
            # v_0 = b / ||b|| (an Arnoldi job with an empty basis)
            self._arnoldi([dict(V=basis, m=0, w=basis[0], vout=basis[0], hcol=Hc[req.steps])],
                          stream=stream, scratch=scratch)
            ready = torch.cuda.Event()
            ready.record(stream)
        # the buffers are used on the main stream (and streams joined to it)
        # from now on: freeing them must wait for that work
        for t in (basis, Hc, ws, w):
            if t is not None:
                t.record_stream(self.main)
        return dict(req=req, plan=plan, basis=basis, w=w, Hc=Hc, ws=ws, j=0, shape=(1, b) + tuple(n), ready=ready,
                    # raw pointers for the one-call step (sfft_apply_each)
                    ptr=(plan.handle.value, basis.data_ptr(), vlen * self.esz, w.data_ptr(),
                         ws.data_ptr() if ws is not None else 0, ws.numel() if ws is not None else 0))

    def _arnoldi(self, jobs, stream=None, scratch="_scratch"):
        N = self.N
        arr = (N.ArnoldiJob * len(jobs))()
        for a, jb in zip(arr, jobs):
            a.V = jb["V"].data_ptr()
            a.ldv = jb["V"].shape[1]
            a.m = jb["m"]
            a.w = jb["w"].data_ptr()
            a.vout = jb["vout"].data_ptr()
            a.n = jb["w"].numel()
            a.hcol = jb["hcol"].data_ptr()
        need = C.c_size_t()
        N.check(N.lib.sfft_arnoldi_scratch_size(len(jobs), arr, C.byref(need)), "sfft_arnoldi_scratch_size")
        stream = self.main if stream is None else stream
        buf = getattr(self, scratch)
        if buf is None or buf.numel() < need.value:
            with self.torch.cuda.stream(stream):
                buf = self.torch.empty(max(int(need.value), 1 << 20), dtype=self.torch.uint8, device="cuda")
            setattr(self, scratch, buf)
        code = N.C64 if self.dtype == "c64" else N.C128
        N.check(N.lib.sfft_arnoldi_step_multi(len(jobs), arr, code, C.c_void_p(buf.data_ptr()), buf.numel(),
                                              C.c_void_p(stream.cuda_stream)), "sfft_arnoldi_step_multi")

    def _throttle(self) -> None:
        # at most max_ahead server steps queued behind the one being issued, so
        # a newly admitted request does not wait behind a long queue
        ev = self.torch.cuda.Event()
        ev.record(self.main)
        self._inflight.append(ev)
        t = time.perf_counter()
        while len(self._inflight) > self.max_ahead:
            self._inflight.pop(0).synchronize()
        self.wait_s += time.perf_counter() - t

    def step(self, slots):
        """w = T v_j for every slot in one native call (sfft_apply_each: the
        products spread over forked streams and joined back), then one batched
        Arnoldi step; slots whose product failed are reported and skipped."""
        N = self.N
        k = len(slots)
        plans, xs, ys = (C.c_void_p * k)(), (C.c_void_p * k)(), (C.c_void_p * k)()
        nr, wss, wsb = (C.c_int64 * k)(*([1] * k)), (C.c_void_p * k)(), (C.c_size_t * k)()
        status = (C.c_int * k)()
        for i, s in enumerate(slots):
            if "ready" in s:  # first step after an asynchronous admission
                self.main.wait_event(s.pop("ready"))
            ph, base, vb, wp, wsp, wsn = s["ptr"]
            plans[i], xs[i], ys[i], wss[i], wsb[i] = ph, base + s["j"] * vb, wp, wsp or None, wsn
        N.check(N.lib.sfft_apply_each(k, plans, xs, ys, nr, wss, wsb, C.c_void_p(self.main.cuda_stream), status),
                "sfft_apply_each")
        failures, jobs = [], []
        for i, s in enumerate(slots):
            if status[i] != N.OK:
                failures.append((i, f"{N._status_name(status[i])}"))
                continue
            j = s["j"]
            jobs.append(dict(V=s["basis"], m=j + 1, w=s["w"], vout=s["basis"][j + 1], hcol=s["Hc"][j]))
            s["j"] = j + 1
        if jobs:
            self._arnoldi(jobs)
        self._throttle()
        return failures

    def finish_start(self, slot) -> None:
        torch = self.torch
        host = torch.empty(slot["Hc"].shape, dtype=torch.complex128, pin_memory=True)
        with torch.cuda.stream(self.main):
            host.copy_(slot["Hc"], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.main)
        slot["fin"] = (ev, host)

    def finish_ready(self, slot) -> bool:
        return slot["fin"][0].query() if "fin" in slot else True

    def finish_wait(self, slot) -> None:
        if "fin" in slot:
            slot["fin"][0].synchronize()

    def finish(self, slot) -> dict:
        """GMRES on the finished chain: y = argmin ||beta e_1 - H y|| (a small
        host least-squares problem), x = V_m y on the device; returns H, beta,
        y, the residual estimate ||beta e_1 - H y|| / beta and, when kept, the
        basis and x."""
        torch = self.torch
        req = slot["req"]
        m = req.steps
        if "fin" in slot:
            ev, host = slot["fin"]
            ev.synchronize()
            Hc = host.numpy()
        else:
            self.main.synchronize()
            Hc = slot["Hc"].cpu().numpy()
        H = Hc[:m].T.copy()                      # (m+1, m) upper Hessenberg
        beta = float(Hc[m, 0].real)              # ||b||
        rhs = np.zeros(m + 1, dtype=np.complex128)
        rhs[0] = beta
        y = np.linalg.lstsq(H, rhs, rcond=None)[0]
        res = float(np.linalg.norm(rhs - H @ y) / beta) if beta > 0 else 0.0
        out = dict(H=H, start_norm=beta, y=y, gmres_residual=res)
        if self.keep_basis:
            V = slot["basis"]
            out["basis"] = V.cpu().numpy()
            yd = torch.from_numpy(y).to(device=V.device)
            out["x"] = (V[:m].to(torch.complex128).transpose(0, 1) @ yd).cpu().numpy()
        return out

    def release(self, slot) -> None:
        # keep the plan for the next request on this grid with an event after
        # its last use: the one behind the finished chain's copy (every stream
        # of the request joined the main stream before it), not one at the
        # current end of the main stream, which may hold later steps
        if "fin" in slot:
            ev = slot["fin"][0]
        else:
            ev = self.torch.cuda.Event()
            ev.record(self.main)
        plan = slot["plan"]
        nb = self._plan_bytes(plan)
        with self._lock:
            self._idle.setdefault(tuple(slot["req"].n), []).append((plan, ev, nb))
            self._idle_total += nb
        slot.clear()


class SingleRequestExecutor(GpuExecutor):
    """The plain path: one request at a time, no overlap (used with
    max_active=1), same kernels; typically FP64 and full symbols."""

    def step(self, slots):
        for s in slots:
            if "ready" in s:
                self.main.wait_event(s.pop("ready"))
            s["plan"].apply(s["basis"][s["j"]].view(s["shape"]), s["w"].view(s["shape"]), s["ws"], stream=self.main)
            j = s["j"]
            self._arnoldi([dict(V=s["basis"], m=j + 1, w=s["w"], vout=s["basis"][j + 1], hcol=s["Hc"][j])])
            s["j"] = j + 1
        self._throttle()
        return []
