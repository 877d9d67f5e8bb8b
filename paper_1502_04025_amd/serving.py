"""Continuous-batching solve server over resident gauge fields.

Requests (a lattice volume, a kappa and 1..n right-hand sides) arrive over time. Every
volume has its gauge field and clover term resident on the GPU and one worker thread
with its own context, HIP stream and solver batch (`sapdd_batch_*`). A worker admits
waiting requests of its volume into free batch slots between FGMRES restart cycles,
steps the batch (one restart cycle for every active slot: all right-hand sides of the
volume in one multi-RHS launch sequence), and hands back every request whose
right-hand sides have all finished. Workers of different volumes run concurrently, so
their kernels overlap on the device.

Admission is by HBM footprint from one shared budget: the resident fields, a cache of
clover inverses per volume and a reserve for kernel scratch are set aside first; every
request then draws the bytes its right-hand sides need (the batch's per-slot memory, plus
the request's sources, solutions and its clover inverse) from what is left, whatever its
volume. Elastic batches commit a slot's memory on first use and keep it after the slot is
taken, so the volume's next request reuses it without remapping anything. A volume gives
its kept memory back only when another volume is waiting for budget and it has no queued
request itself (or is stuck waiting too); the chunks go to the library's pool, from which
the waiting volume's batch maps them, so memory moves to the volumes that have work as
the load shifts without being freed and allocated again (a fresh allocation right after
a large free can stall for seconds while the device clears the freed memory). A request enters when its volume's batch has free slots and the
budget holds its footprint; one that could never fit is rejected at once. A request
that fails (a singular clover term, a non-finite residual) or misses the tolerance within
the iteration cap comes back with its error set, and its slots and bytes are returned.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    id: int
    t_arrival: float  # seconds after the serving clock starts
    vol: int
    kappa: float
    nrhs: int
    seed: int
    # filled by the server
    t_admit: float = math.nan
    t_done: float = math.nan
    slots: list = field(default_factory=list)
    stats: list = field(default_factory=list)
    x: object = None
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class VolumePlan:
    name: str
    field_bytes: int      # resident links + clover (all precisions in use)
    per_rhs_bytes: int    # one slot's solver state, plus the canonical b and x of one RHS
    kappa_bytes: int      # one clover inverse for a new kappa
    capacity: int = 0     # batch slots (address space only in an elastic batch)
    warm_bytes: int = 0   # elastic: the part of per_rhs_bytes a slot keeps after a take


class HbmBudget:
    """One pool of device memory shared by every served volume (thread-safe): `fixed`
    bytes are set aside at start, requests take and give back the rest."""

    def __init__(self, total_bytes: int, fixed_bytes: int = 0):
        self.total = int(total_bytes)
        self.fixed = int(fixed_bytes)
        self.used = int(fixed_bytes)
        self.peak = self.used
        self.lock = threading.Lock()
        self.waiting = {}  # volumes whose next request waits for bytes -> bytes it lacks
        self.running = set()  # names of the workers not yet finished

    def set_waiting(self, name: str, on: bool, short: int = 0) -> None:
        with self.lock:
            if on:
                self.waiting[name] = int(short)
            else:
                self.waiting.pop(name, None)

    def set_running(self, name: str, on: bool) -> None:
        with self.lock:
            (self.running.add if on else self.running.discard)(name)
            if not on:
                self.waiting.pop(name, None)

    def others_running(self, name: str) -> bool:
        with self.lock:
            return bool(self.running - {name})

    def is_waiting(self, name: str) -> bool:
        with self.lock:
            return name in self.waiting

    def others_waiting(self, name: str) -> bool:
        with self.lock:
            return any(k != name for k in self.waiting)

    def others_short(self, name: str) -> int:
        """The most bytes another waiting volume lacks."""
        with self.lock:
            return max((v for k, v in self.waiting.items() if k != name), default=0)

    def try_take(self, n: int) -> bool:
        with self.lock:
            if self.used + n <= self.total:
                self.used += n
                self.peak = max(self.peak, self.used)
                return True
            return False

    def give_back(self, n: int) -> None:
        with self.lock:
            self.used -= n
            assert self.used >= self.fixed

    @property
    def free(self) -> int:
        return self.total - self.used


def plan_budget(plans, budget_bytes: int, max_slots: int = 24, kappa_cache: int = 16, reserve_bytes: int = 0):
    """Set up the shared budget: the reserve (kernel scratch, graphs, allocator slack), the
    fields and a cache of `kappa_cache` clover inverses per volume are set aside; each
    volume's batch gets as many slots as the rest could fill with its requests alone (at
    most max_slots). Returns the HbmBudget; raises if not even one slot fits."""
    fixed = reserve_bytes + sum(p.field_bytes + kappa_cache * p.kappa_bytes for p in plans)
    if fixed >= budget_bytes:
        raise MemoryError(f"budget {budget_bytes} B cannot hold the resident fields ({fixed} B)")
    for p in plans:
        p.capacity = int(min(max_slots, (budget_bytes - fixed - p.kappa_bytes) // p.per_rhs_bytes))
        if p.capacity < 1:
            raise MemoryError(f"budget leaves no slot for volume {p.name}")
    return HbmBudget(budget_bytes, fixed)


def plan_capacity(plans, budget_bytes: int, max_slots: int = 24, kappa_cache: int = 16, reserve_bytes: int = 0):
    """Split an HBM budget into equal fixed slot counts per volume (for batches whose
    memory is allocated at creation): the same reserve as plan_budget, then the same
    number of slots in every volume, at most max_slots. Raises if not even one fits."""
    fixed = reserve_bytes + sum(p.field_bytes + kappa_cache * p.kappa_bytes for p in plans)
    if fixed >= budget_bytes:
        raise MemoryError(f"budget {budget_bytes} B cannot hold the resident fields ({fixed} B)")
    cap = int(min(max_slots, (budget_bytes - fixed) // sum(p.per_rhs_bytes for p in plans)))
    if cap < 1:
        raise MemoryError("budget leaves no slot for every volume")
    for p in plans:
        p.capacity = cap
    return plans


class Admission:
    """Admission of one volume (thread-safe): a request of n right-hand sides needs n free
    slots of the volume's batch and, with a shared budget, n * slot_bytes +
    request_bytes of it.

    With warm_bytes > 0 (an elastic batch that keeps a taken slot's memory) that part of
    a slot is charged once, when the batch first commits it, and stays charged while the
    batch keeps it: a request pays warm_bytes only for the slots beyond those already
    committed. `released(k)` returns the charge of k kept slots the batch has freed."""

    def __init__(self, capacity: int, budget: HbmBudget | None = None, slot_bytes: int = 0,
                 request_bytes: int = 0, warm_bytes: int = 0):
        self.capacity = capacity
        self.free = capacity
        self.budget = budget
        self.slot_bytes = int(slot_bytes)
        self.request_bytes = int(request_bytes)
        self.warm_bytes = int(warm_bytes) if budget is not None else 0
        self.committed = 0  # slots whose warm part the batch holds (in use or kept)
        self.lock = threading.Lock()

    def _cost(self, n: int, new: int) -> int:
        if self.budget is None:
            return 0
        return n * (self.slot_bytes - self.warm_bytes) + new * self.warm_bytes + self.request_bytes

    def cost(self, n: int) -> int:
        """Bytes n right-hand sides cost when none of their slots is kept from before."""
        return self._cost(n, n)

    def fits_ever(self, n: int) -> bool:
        if n > self.capacity:
            return False
        return self.budget is None or self.cost(n) <= self.budget.total - self.budget.fixed

    def kept(self) -> int:
        """Free slots whose memory the batch still holds."""
        with self.lock:
            return self.committed - (self.capacity - self.free) if self.warm_bytes else 0

    def short(self, n: int) -> int:
        """Bytes the budget lacks for n more right-hand sides now."""
        if self.budget is None:
            return 0
        with self.lock:
            new = max(0, self.capacity - self.free + n - self.committed) if self.warm_bytes else n
            return max(0, self._cost(n, new) - self.budget.free)

    def try_take(self, n: int) -> bool:
        with self.lock:
            if n > self.free:
                return False
            new = max(0, self.capacity - self.free + n - self.committed) if self.warm_bytes else n
            if self.budget is not None and not self.budget.try_take(self._cost(n, new)):
                return False
            self.free -= n
            if self.warm_bytes:
                self.committed += new
            return True

    def give_back(self, n: int) -> None:
        with self.lock:
            self.free += n
            assert self.free <= self.capacity
        if self.budget is not None:
            self.budget.give_back(self._cost(n, 0 if self.warm_bytes else n))

    def released(self, k: int) -> None:
        with self.lock:
            self.committed -= k
            assert 0 <= self.committed and self.committed >= self.capacity - self.free
        if self.budget is not None:
            self.budget.give_back(k * self.warm_bytes)


class VolumeWorker(threading.Thread):
    """Serves the requests of one volume with one batch on its own stream.

    `backend` provides make_source(req) -> list of right-hand sides, make_output(req)
    -> list of outputs, and a batch object with add/step/poll/take (the sapdd Batch, or a
    stand-in in host-only tests)."""

    def __init__(self, name, batch, backend, admission: Admission, clock, on_done):
        super().__init__(name=f"serve-{name}", daemon=True)
        self.batch = batch
        self.backend = backend
        self.adm = admission
        self.clock = clock
        self.on_done = on_done
        self.queue = deque()
        self.cv = threading.Condition()
        self.stop_when_idle = False
        self.active = []
        self.cancels = set()
        self.error = None
        self.steps = 0
        self.trims = 0
        # host wall time per phase (admit_io and admit_add are parts of admit)
        self.busy_s = {"admit": 0.0, "admit_io": 0.0, "admit_add": 0.0, "step": 0.0, "harvest": 0.0, "trim": 0.0}

    def submit(self, req: Request):
        with self.cv:
            if not self.adm.fits_ever(req.nrhs):
                req.error = f"request needs {req.nrhs} slots, volume holds {self.adm.capacity}"
                req.t_done = self.clock()
                self.on_done(req)
                return
            self.queue.append(req)
            self.cv.notify()

    def cancel(self, req_id) -> bool:
        """Cancel a request. A waiting one leaves the queue at once; an admitted one gives
        its slots back before the next batch step, its outputs holding the iterate of the
        last completed restart cycle (a resume point: resubmit it as the start vector).
        Returns False if the request is not waiting (admitted, finished or unknown)."""
        with self.cv:
            for q in list(self.queue):
                if q.id == req_id:
                    self.queue.remove(q)
                    q.error = "cancelled"
                    q.t_done = self.clock()
                    self.on_done(q)
                    return True
            self.cancels.add(req_id)
            self.cv.notify()
        return False

    def _cancel_active(self):
        with self.cv:
            ids, self.cancels = self.cancels, set()
        if not ids:
            return
        still = []
        for req in self.active:
            if req.id not in ids:
                still.append(req)
                continue
            req.stats = [self.batch.take(s, out) for s, out in zip(req.slots, req.x)]
            self.adm.give_back(req.nrhs)
            req.error = "cancelled"
            req.t_done = self.clock()
            self.on_done(req)
        self.active = still

    def finish(self):
        with self.cv:
            self.stop_when_idle = True
            self.cv.notify()

    def _trim_if_wanted(self):
        """Give the memory of kept slots back to the budget when another volume waits for
        it and this one has no queued request, or is waiting itself with nothing running
        (kept memory it cannot use now): as many slots as cover what the waiting volume
        lacks, or all of them."""
        budget = self.adm.budget
        if budget is None or not self.adm.warm_bytes or not budget.others_waiting(self.name):
            return
        with self.cv:
            idle = not self.queue
        stuck = not self.active and budget.is_waiting(self.name)
        k = self.adm.kept()
        if k and (idle or stuck):
            short = budget.others_short(self.name)
            give = min(k, max(1, -(-short // self.adm.warm_bytes)))
            t0 = time.perf_counter()
            self.batch.trim(k - give)
            self.adm.released(give)
            self.trims += 1
            self.busy_s["trim"] += time.perf_counter() - t0

    def _admit(self):
        budget = self.adm.budget
        while True:
            with self.cv:
                if not self.queue:
                    if budget is not None:
                        budget.set_waiting(self.name, False)
                    return
                if not self.adm.try_take(self.queue[0].nrhs):
                    if budget is not None:  # waiting for bytes, not for this volume's own slots
                        n = self.queue[0].nrhs
                        budget.set_waiting(self.name, self.adm.free >= n, self.adm.short(n))
                    return
                if budget is not None:
                    budget.set_waiting(self.name, False)
                req = self.queue.popleft()
            req.t_admit = self.clock()
            req.slots = []
            try:
                t0 = time.perf_counter()
                srcs = self.backend.make_source(req)
                req.x = self.backend.make_output(req)
                t1 = time.perf_counter()
                for b in srcs:
                    req.slots.append(self.batch.add(req.kappa, b))
                self.busy_s["admit_io"] += t1 - t0
                self.busy_s["admit_add"] += time.perf_counter() - t1
            except Exception as e:  # this request fails alone: its slots and bytes go back
                for s, out in zip(req.slots, req.x or []):
                    try:
                        self.batch.take(s, out)
                    except Exception:
                        pass
                self.adm.give_back(req.nrhs)
                req.error = f"admission failed: {e}"
                req.t_done = self.clock()
                self.on_done(req)
                continue
            self.active.append(req)

    def _harvest(self):
        still = []
        for req in self.active:
            done = all(self.batch.poll(s)[0] for s in req.slots)
            if not done:
                still.append(req)
                continue
            stats, errs = [], []
            for s, out in zip(req.slots, req.x):
                try:
                    stats.append(self.batch.take(s, out))
                except Exception as e:  # e.g. a non-finite residual in this slot
                    stats.append({"converged": 0, "error": str(e)})
                    errs.append(str(e))
            req.stats = stats
            self.adm.give_back(req.nrhs)
            if errs:
                req.error = "; ".join(errs)
            elif not all(st.get("converged", 1) for st in stats):
                req.error = "not converged within the iteration cap"
            req.t_done = self.clock()
            self.on_done(req)
        self.active = still

    def start(self):
        if self.adm.budget is not None:
            self.adm.budget.set_running(self.name, True)
        super().start()

    def run(self):
        try:
            with self.backend.thread_context():
                self._loop()
                self._leave()
        except Exception as e:  # surfaced by Server.run
            self.error = e
        finally:
            if self.adm.budget is not None:
                self.adm.budget.set_running(self.name, False)

    def _leave(self):
        """A finishing worker can no longer trim on demand, so while other workers still
        run it gives its kept memory back (the last one keeps it for a later run)."""
        budget = self.adm.budget
        k = self.adm.kept()
        if budget is not None and k and budget.others_running(self.name):
            t0 = time.perf_counter()
            self.batch.trim(0)
            self.adm.released(k)
            self.trims += 1
            self.busy_s["trim"] += time.perf_counter() - t0

    def _loop(self):
        while True:
            self._cancel_active()
            self._trim_if_wanted()
            t0 = time.perf_counter()
            self._admit()
            t1 = time.perf_counter()
            self.busy_s["admit"] += t1 - t0
            if self.active:
                self.batch.step()
                self.steps += 1
                t2 = time.perf_counter()
                self._harvest()
                self.busy_s["step"] += t2 - t1
                self.busy_s["harvest"] += time.perf_counter() - t2
                continue
            with self.cv:
                if self.queue:  # waiting for memory another volume holds: no busy spin
                    self.cv.wait(timeout=0.002)
                    continue
                if self.stop_when_idle:
                    return
                self.cv.wait(timeout=0.05)


class Server:
    """Routes a request stream to per-volume workers and records latencies.

    on_result(req), if given, receives every finished request's solutions (req.x) as it
    completes, after which the server lets go of them: a server that kept every answer
    until the end of a long stream would hold it all in device memory outside the
    budget (the solutions of 500 requests over the three volumes are ~640 GB). Without
    on_result the finished requests keep their solutions (tests read them)."""

    def __init__(self, workers, on_result=None):
        self.workers = workers
        self.done = []
        self.lock = threading.Lock()
        self.t0 = None
        self.on_result = on_result

    def clock(self) -> float:
        return time.perf_counter() - self.t0

    def _on_done(self, req):
        if self.on_result is not None:
            self.on_result(req)
            req.x = None
        with self.lock:
            self.done.append(req)

    def run(self, requests, realtime: bool = True, progress=None, every: float = 30.0):
        """Release every request at its arrival time (or all at once if not realtime) and
        wait for all of them. Returns the finished requests. progress(finished, total), if
        given, is called from this thread about every `every` seconds."""
        self.t0 = time.perf_counter()
        last = [self.t0]

        def tick():
            if progress is not None and time.perf_counter() - last[0] >= every:
                last[0] = time.perf_counter()
                with self.lock:
                    n = len(self.done)
                progress(n, len(requests))

        for w in self.workers:
            w.clock = self.clock
            w.on_done = self._on_done
            w.start()
        for req in sorted(requests, key=lambda r: r.t_arrival):
            if realtime:
                while (dt := req.t_arrival - self.clock()) > 0:
                    time.sleep(min(dt, 1.0))
                    tick()
            self.workers[req.vol].submit(req)
        for w in self.workers:
            w.finish()
        for w in self.workers:
            while w.is_alive():
                w.join(timeout=1.0)
                tick()
        errs = [w.error for w in self.workers if w.error is not None]
        if errs:
            raise errs[0]
        return self.done


def summarize(done, wall: float) -> dict:
    ok = [r for r in done if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.array([np.nan])
    rhs = sum(r.nrhs for r in ok)
    return dict(requests=len(ok), rejected=len(done) - len(ok), rhs_solves=rhs,
                solves_per_s=rhs / wall if wall > 0 else float("nan"),
                requests_per_s=len(ok) / wall if wall > 0 else float("nan"),
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(np.mean(lat) * 1e3))


class TorchVolume:
    """GPU resources of one served volume: a stream, a context, the resident field, the
    batch, and seeded Gaussian sources drawn on the device. With elastic=True the batch
    commits a slot's memory only while the slot is in use (its slots cost address space
    otherwise), so volumes can share one HBM budget."""

    def __init__(self, name, dims, block, eps, gauge_seed, csw, capacity, solver_kw, links=None, elastic=False):
        import torch

        import synthetic  # seeded input recipe shared with the tests
        from .sapdd import Context
        self.name = name
        self.dims = tuple(dims)
        self.solver_kw = dict(solver_kw)
        self.elastic = elastic
        self.stream = torch.cuda.Stream()
        self.ctx = Context(0, stream=self.stream)
        u = links if links is not None else synthetic.gauge_field(dims, eps, gauge_seed)
        with torch.cuda.stream(self.stream):
            self.field = self.ctx.load_gauge(u, block)
            self.field.compute_clover(csw)
        self.torch = torch
        self.batch = None
        if capacity:
            self.start(capacity)

    def plan(self) -> VolumePlan:
        """Memory plan of this volume: resident field (and, elastic, the batch's fixed part),
        bytes per slot (the solver's state plus this backend's canonical b and x of one
        right-hand side), per-kappa clover."""
        lx, ly, lz, lt = self.dims
        v = lx * ly * lz * lt
        canon = 2 * v * 12 * 16  # complex128 b and x
        one = self.field.footprint(1, **self.solver_kw)
        per_rhs = self.field.footprint(2, **self.solver_kw) - one
        lo = one - per_rhs
        prec_b = {"f64": 8, "f32": 4, "f16": 2, "f16l": 2}[self.solver_kw.get("prec", "f64")]
        kappa_bytes = v * 72 * prec_b + v * 4
        field_bytes = 2 * v * 72 * 8 + lo
        if self.elastic and self.batch is not None:
            fixed, slot = self.batch.memory()
            return VolumePlan(self.name, field_bytes + fixed, slot + canon, kappa_bytes, warm_bytes=slot)
        return VolumePlan(self.name, field_bytes, per_rhs + canon, kappa_bytes)

    def start(self, capacity: int):
        from .sapdd import Batch
        with self.torch.cuda.stream(self.stream):
            extra = {"elastic": True} if self.elastic else {}
            self.batch = Batch(self.field, capacity, **extra, **self.solver_kw)

    def thread_context(self):
        return self.torch.cuda.stream(self.stream)

    # One tensor per right-hand side, all of one size per volume: torch's caching
    # allocator then reuses its blocks from request to request instead of keeping blocks
    # of every request size (which grew its reserve to tens of GB outside the budget).
    def make_source(self, req):
        torch = self.torch
        lx, ly, lz, lt = self.dims
        g = torch.Generator(device="cuda")
        g.manual_seed(int(req.seed))
        return [torch.view_as_complex(torch.randn((lt, lz, ly, lx, 4, 3, 2), generator=g, dtype=torch.float64,
                                                  device="cuda")) for _ in range(req.nrhs)]

    def make_output(self, req):
        torch = self.torch
        lx, ly, lz, lt = self.dims
        return [torch.empty((lt, lz, ly, lx, 4, 3), dtype=torch.complex128, device="cuda") for _ in range(req.nrhs)]

    def close(self):
        self.batch.close()
        self.field.free()
        self.ctx.close()
