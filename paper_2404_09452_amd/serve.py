"""Continuous-batching server for DF-J/K requests on one GPU.

A request is one molecule plus a sequence of occupied-orbital matrices (an
SCF-like run): setup once, then one J/K build per matrix.  Requests arrive
over time; the scheduler admits the head of the queue as soon as a slot is
free and its exact device-memory need (known after the Schwarz screening)
fits in the HBM budget.  Every admitted request runs on its own HIP stream,
so setups and builds of different molecules overlap on the device, and
memory is returned to the budget when a request completes.  Latency is
measured from arrival to the completion of the request's last build.

The scheduling logic is independent of the GPU: `Executor` objects do the
work.  `GpuExecutor` drives the library with one stream per request;
`BatchedGpuExecutor` runs the builds of all set-up requests step by step as
batched calls (grouped launches across molecules).
"""
from __future__ import annotations

import dataclasses
import os
import queue
import threading
import time
from typing import Callable, List, Optional

import numpy as np

# Device memory the HIP runtime needs besides the caching allocator's blocks:
# the private (spill) segments of the integral kernels are allocated by the
# runtime per queue when a kernel is dispatched, and a dispatch that finds no
# room aborts the process.  The server keeps this much out of its budget and
# caps torch's allocator below the device size.
RUNTIME_RESERVE_BYTES = 4 << 30
ALLOCATOR_FRACTION = 0.85


def configure_allocator():
    """Allocator settings for serving molecules of very different sizes; call
    before torch first touches the GPU.  Blocks above 512 MB are never split,
    so a finished molecule's workspace returns as whole segments that can be
    released when a larger molecule needs the room (without it, fragmentation
    left cached blocks unusable and large requests failed inside their
    admitted budget).  Returns False (and changes nothing) when the process
    has already initialised the GPU."""
    import torch
    if torch.cuda.is_initialized():
        return False
    os.environ.setdefault("PYTORCH_ALLOC_CONF", "max_split_size_mb:512")
    return True


def default_budget(frac=0.6):
    """An HBM budget: `frac` of the device memory torch may use after the
    allocator cap (pass it to Server with runtime_reserve_bytes)."""
    import torch
    free, total = torch.cuda.mem_get_info()
    return int(frac * min(free, int(ALLOCATOR_FRACTION * total)))


@dataclasses.dataclass
class Request:
    rid: int
    mol: object                 # anything with coords / ao_* / aux_* (workload.Molecule)
    orbitals: List[np.ndarray]  # one (nao, nocc) matrix per build
    arrival: float = 0.0        # seconds after the stream start
    precision: str = "fp64"
    # filled by the server
    admitted: float = float("nan")
    done: float = float("nan")
    bytes_needed: int = 0
    energies: Optional[np.ndarray] = None    # (nbuilds, 2)
    K_last: Optional[np.ndarray] = None
    J_last: Optional[np.ndarray] = None
    error: Optional[str] = None

    @property
    def latency(self):
        return self.done - self.arrival


class Executor:
    """What the server needs from a backend."""

    def prepare(self, req: Request) -> int:
        """Host preparation and screening; returns the device bytes the request needs."""
        raise NotImplementedError

    def run(self, req: Request) -> None:
        """Setup and every build of the request (blocking until finished)."""
        raise NotImplementedError

    def release(self, req: Request) -> None:
        """Free whatever the request holds."""


class GpuExecutor(Executor):
    """Runs requests through the DF-J/K library, one HIP stream per request."""

    def __init__(self, keep_results=True, schwarz_thresh=1e-14, allocator_fraction=ALLOCATOR_FRACTION):
        import torch

        from .dfjk import Plan
        self.torch = torch
        self.Plan = Plan
        self.keep = keep_results
        self.thresh = schwarz_thresh
        self._plans = {}
        # cached blocks of finished molecules must not take the memory the
        # runtime needs for its own allocations (see RUNTIME_RESERVE_BYTES)
        if allocator_fraction is not None:
            torch.cuda.set_per_process_memory_fraction(allocator_fraction)

    def prepare(self, req):
        torch = self.torch
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            plan = self.Plan.from_molecule(req.mol, schwarz_thresh=self.thresh)
            plan.screen(stream=stream)
            nocc = req.orbitals[0].shape[1]
            need = plan.setup_bytes() + plan.build_bytes(nocc, "fp64")
            if req.precision.endswith("_incr"):
                need += plan.build_delta_bytes(nocc, req.precision[:-5])
            elif req.precision != "fp64":
                need += plan.build_bytes(nocc, req.precision)
            need += 4 * plan.nao * plan.nao * 8 + nocc * plan.nao * 8 * len(req.orbitals)
        self._plans[req.rid] = (plan, stream)
        return int(need)

    def run(self, req):
        torch = self.torch
        plan, stream = self._plans[req.rid]
        with torch.cuda.stream(stream):
            plan.setup(stream=stream)
            nao = plan.nao
            J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
            K = torch.empty_like(J)
            Es = torch.empty((len(req.orbitals), 2), dtype=torch.float64, device="cuda")
            Cs = [torch.as_tensor(C, device="cuda") for C in req.orbitals]
            if req.precision.endswith("_incr"):
                # first build in FP64, later ones as increments on it
                K0 = torch.empty_like(J)
                plan.build(C=Cs[0], precision="fp64", out=(J, K0, Es[0]), stream=stream)
                K.copy_(K0)
                for k in range(1, len(Cs)):
                    plan.build_delta(Cs[k], Cs[0], K0, precision=req.precision[:-5], out=(J, K, Es[k]),
                                     stream=stream)
            else:
                for k, Cd in enumerate(Cs):
                    plan.build(C=Cd, precision=req.precision, out=(J, K, Es[k]), stream=stream)
            stream.synchronize()
            req.energies = Es.cpu().numpy()
            if self.keep:
                req.K_last = K.cpu().numpy()
                req.J_last = J.cpu().numpy()

    def release(self, req):
        entry = self._plans.pop(req.rid, None)
        if entry is not None:
            entry[0].close()


class BatchedGpuExecutor(GpuExecutor):
    """Step-level batching of the builds of small molecules.  Each admitted
    request sets up on its own stream as before.  A molecule with fewer than
    `batch_below_nao` AO functions then joins a build loop that, at every
    step, issues the next build of every joined molecule as one batched call
    (grouped K, reduction and energy launches across the molecules, where the
    launch overhead of separate builds would dominate); requests join and
    leave between steps, so one that arrives while others are mid-run rides
    along from its first build.  Larger molecules, whose kernels fill the
    device by themselves, keep building on their own streams, free of the
    steps, overlapping with the batches.  Direct precisions only (fp64, int8,
    int8_fast, fp32, bf16x3)."""

    def __init__(self, keep_results=True, schwarz_thresh=1e-14, allocator_fraction=ALLOCATOR_FRACTION,
                 batch_below_nao=300):
        super().__init__(keep_results, schwarz_thresh, allocator_fraction)
        self.batch_below_nao = batch_below_nao
        from .dfjk import Batch
        self.Batch = Batch
        self._cv = threading.Condition()
        self._joined = []
        self._loop = None
        self._stream = None
        self.steps = 0
        self.batch_sizes = []
        self._arena = None          # batch scratch of the current step

    def run(self, req):
        torch = self.torch
        if req.precision not in ("fp64", "int8", "int8_fast", "fp32", "bf16x3"):
            raise ValueError("the batched executor runs direct builds only")
        plan, stream = self._plans[req.rid]
        if plan.nao >= self.batch_below_nao:
            super().run(req)
            return
        with torch.cuda.stream(stream):
            plan.setup(stream=stream)
            nao = plan.nao
            st = {"req": req, "plan": plan, "k": 0, "done": threading.Event(),
                  "Cs": [torch.as_tensor(C, device="cuda") for C in req.orbitals],
                  "J": torch.empty((nao, nao), dtype=torch.float64, device="cuda"),
                  "Es": torch.empty((len(req.orbitals), 2), dtype=torch.float64, device="cuda")}
            st["K"] = torch.empty_like(st["J"])
        stream.synchronize()
        with self._cv:
            if self._loop is None:
                self._stream = torch.cuda.Stream()
                self._loop = threading.Thread(target=self._build_loop, daemon=True)
                self._loop.start()
            self._joined.append(st)
            self._cv.notify_all()
        st["done"].wait()
        if "error" in st:
            raise RuntimeError(st["error"])
        req.energies = st["Es"].cpu().numpy()
        if self.keep:
            req.K_last = st["K"].cpu().numpy()
            req.J_last = st["J"].cpu().numpy()

    def _build_loop(self):
        torch = self.torch
        while True:
            with self._cv:
                while not self._joined:
                    self._cv.wait()
                group = list(self._joined)
            finished = []
            by_prec = {}
            for st in group:
                by_prec.setdefault(st["req"].precision, []).append(st)
            try:
                with torch.cuda.stream(self._stream):
                    for prec, sts in by_prec.items():
                        plans = [st["plan"] for st in sts]
                        noccs = [st["Cs"][0].shape[1] for st in sts]
                        need = self.Batch.bytes_needed(plans, noccs, prec)
                        # the arena is reused while it is within 25% above this step's need
                        # (which stays within the build scratch the joined requests were
                        # admitted with), else replaced by one of exactly that size
                        if self._arena is None or not need <= self._arena.numel() <= need + need // 4:
                            self._arena = None          # drop the old arena before the new one
                            self._arena = torch.empty(need, dtype=torch.uint8, device="cuda")
                        b = self.Batch(plans, noccs, prec, scratch=self._arena)
                        b.build([st["Cs"][st["k"]] for st in sts],
                                outs=[(st["J"], st["K"], st["Es"][st["k"]]) for st in sts], stream=self._stream)
                        del b
                for st in group:
                    st["k"] += 1
                    if st["k"] == len(st["Cs"]):
                        finished.append(st)
                # steps queue behind one another on the loop's stream (its
                # arena is allocated and reused there, in stream order); the
                # host waits only when a request's results are handed back
                if finished:
                    self._stream.synchronize()
            except Exception as e:  # fail every request of the step, keep serving
                for st in group:
                    st["error"] = repr(e)
                finished = group
            self.steps += 1
            self.batch_sizes.append(len(group))
            with self._cv:
                for st in finished:
                    self._joined.remove(st)
            for st in finished:
                st["done"].set()


class Server:
    """Admission by slots and an HBM byte budget; FIFO order.  The budget
    counts every byte the library and the request's buffers take
    (Executor.prepare); `runtime_reserve_bytes` of it are kept back for the
    HIP runtime's own allocations (kernel spill segments), so requests are
    admitted against hbm_budget_bytes - runtime_reserve_bytes."""

    def __init__(self, executor: Executor, max_active=4, hbm_budget_bytes=64 << 30,
                 clock: Callable[[], float] = time.perf_counter,
                 on_done: Optional[Callable[[Request], None]] = None,
                 runtime_reserve_bytes: int = 0):
        if max_active < 1:
            raise ValueError("max_active must be >= 1")
        self.ex = executor
        self.max_active = max_active
        self.reserve = int(runtime_reserve_bytes)
        self.budget = int(hbm_budget_bytes) - self.reserve
        if self.budget <= 0:
            raise ValueError("the runtime reserve leaves no budget")
        self.clock = clock
        self.in_use = 0
        self.peak_in_use = 0
        self.active = 0
        self.peak_active = 0
        self._cv = threading.Condition()
        self._errors = []
        self.on_done = on_done      # called from the worker thread after each request

    def _worker(self, req):
        try:
            self.ex.run(req)
        except Exception as e:  # reported per request, the server keeps going
            req.error = repr(e)
        finally:
            req.done = self.clock() - self._t0
            self.ex.release(req)
            with self._cv:
                self.in_use -= req.bytes_needed
                self.active -= 1
                self._cv.notify_all()
            if self.on_done is not None:
                self.on_done(req)

    def serve(self, requests: List[Request]) -> List[Request]:
        """Feed `requests` at their arrival times and return them completed."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        arrived = queue.deque()
        threads = []
        self._t0 = self.clock()
        i = 0
        while i < len(pending) or arrived:
            now = self.clock() - self._t0
            while i < len(pending) and pending[i].arrival <= now:
                arrived.append(pending[i])
                i += 1
            if not arrived:
                time.sleep(max(0.0, min(0.002, pending[i].arrival - now)))
                continue
            head = arrived[0]
            if head.bytes_needed == 0:
                try:
                    head.bytes_needed = max(1, self.ex.prepare(head))
                except Exception as e:
                    head.error = repr(e)
                    head.done = self.clock() - self._t0
                    self.ex.release(head)
                    arrived.popleft()
                    continue
                if head.bytes_needed > self.budget:
                    head.error = "needs %d bytes, more than the whole budget %d" % (head.bytes_needed, self.budget)
                    head.done = self.clock() - self._t0
                    self.ex.release(head)
                    arrived.popleft()
                    continue
            with self._cv:
                while not (self.active < self.max_active and self.in_use + head.bytes_needed <= self.budget):
                    self._cv.wait(timeout=0.002)
                    now = self.clock() - self._t0
                    while i < len(pending) and pending[i].arrival <= now:
                        arrived.append(pending[i])
                        i += 1
                self.in_use += head.bytes_needed
                self.active += 1
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                self.peak_active = max(self.peak_active, self.active)
            arrived.popleft()
            head.admitted = self.clock() - self._t0
            th = threading.Thread(target=self._worker, args=(head,), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        return requests


def summarize(requests: List[Request], wall_s: float):
    ok = [r for r in requests if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.array([np.nan])
    builds = sum(len(r.orbitals) for r in ok)
    return {
        "requests": len(requests),
        "failed": len(requests) - len(ok),
        "builds": builds,
        "wall_s": wall_s,
        "builds_per_s": builds / wall_s if wall_s > 0 else float("nan"),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(np.mean(lat)),
        "errors": sorted(set(r.error for r in requests if r.error is not None))[:3],
    }
