"""Host-side tests of the serving loop: admission by memory budget, continuous batching,
and completion bookkeeping, with an in-memory stand-in for the GPU batch."""
import contextlib
import math

import pytest

from paper_1502_04025_amd import serving as sv


class FakeBatch:
    """A slot holding source b finishes after 2 + b % 4 steps; records which slots shared
    each step."""

    def __init__(self, capacity, need=None):
        self.cap = capacity
        self.slots = {}
        self.steps = []

    @staticmethod
    def need(b):
        return 2 + b % 4

    def add(self, kappa, b):
        free = [s for s in range(self.cap) if s not in self.slots]
        if not free:
            raise RuntimeError("full")
        self.slots[free[0]] = [0, b]
        return free[0]

    def step(self):
        self.steps.append(sorted(self.slots))
        for st in self.slots.values():
            st[0] += 1
        return sum(1 for st in self.slots.values() if st[0] < self.need(st[1]))

    def poll(self, s):
        return self.slots[s][0] >= self.need(self.slots[s][1]), {}

    def take(self, s, out):
        n, b = self.slots.pop(s)
        out.append(b * 2)
        return {"iters": n}


class FakeBackend:
    def thread_context(self):
        return contextlib.nullcontext()

    def make_source(self, req):
        return [req.seed * 10 + i for i in range(req.nrhs)]

    def make_output(self, req):
        return [[] for _ in range(req.nrhs)]


def test_plan_capacity_and_budget_errors():
    plans = [sv.VolumePlan("a", 100, 10, 1), sv.VolumePlan("b", 300, 40, 2)]
    sv.plan_capacity(plans, 400 + 16 * 3 + 5 * 50, max_slots=24)
    assert [p.capacity for p in plans] == [5, 5]
    sv.plan_capacity(plans, 400 + 16 * 3 + 5 * 50, max_slots=24, reserve_bytes=50)
    assert [p.capacity for p in plans] == [4, 4]  # the reserve buys one slot per volume less
    sv.plan_capacity(plans, 10 ** 9, max_slots=24)
    assert plans[0].capacity == 24
    with pytest.raises(MemoryError):
        sv.plan_capacity(plans, 300)
    with pytest.raises(MemoryError):
        sv.plan_capacity(plans, 400 + 16 * 3 + 10)


def test_admission_is_all_or_nothing():
    a = sv.Admission(4)
    assert a.try_take(3) and not a.try_take(2) and a.try_take(1)
    a.give_back(3)
    assert a.free == 3 and not a.fits_ever(5)


def _run(reqs, capacity):
    batch = FakeBatch(capacity)
    w = sv.VolumeWorker("v", batch, FakeBackend(), sv.Admission(capacity), None, None)
    srv = sv.Server([w])
    done = srv.run(reqs, realtime=False)
    return batch, done


def test_continuous_batching_joins_between_steps_and_completes_everything():
    reqs = [sv.Request(i, 0.0, 0, 0.12, n, seed=i) for i, n in enumerate([2, 3, 1, 4, 2])]
    batch, done = _run(reqs, capacity=5)
    assert len(done) == 5 and all(r.error is None for r in done)
    for r in done:  # every right-hand side came back through its own slot
        assert [o[0] for o in r.x] == [2 * (r.seed * 10 + i) for i in range(r.nrhs)]
        assert r.t_done >= r.t_admit >= 0 and not math.isnan(r.latency)
    # the batch never held more than its capacity, and a later request joined a batch
    # that was already running (continuous batching, not run-to-completion)
    assert max(len(s) for s in batch.steps) <= 5
    joined_late = any(set(batch.steps[k + 1]) - set(batch.steps[k]) and set(batch.steps[k])
                      for k in range(len(batch.steps) - 1))
    assert joined_late


def test_oversized_request_is_rejected_not_stuck():
    reqs = [sv.Request(0, 0.0, 0, 0.12, 7, seed=1), sv.Request(1, 0.0, 0, 0.12, 2, seed=2)]
    _, done = _run(reqs, capacity=4)
    bad = [r for r in done if r.error]
    assert len(bad) == 1 and bad[0].id == 0
    s = sv.summarize(done, wall=1.0)
    assert s["requests"] == 1 and s["rejected"] == 1 and s["rhs_solves"] == 2


def test_cancel_waiting_and_admitted_requests():
    """A waiting request leaves the queue; an admitted one gives its slots back between
    steps and returns its current iterates; the others still complete."""
    batch = FakeBatch(2)
    done = []
    w = sv.VolumeWorker("v", batch, FakeBackend(), sv.Admission(2), lambda: 0.0, done.append)
    reqs = [sv.Request(i, 0.0, 0, 0.12, n, seed=i) for i, n in enumerate([2, 2, 1])]
    for r in reqs:
        w.submit(r)
    assert w.cancel(2)  # still waiting: removed at once
    assert done[-1].id == 2 and done[-1].error == "cancelled"
    w._admit()  # request 0 takes both slots, request 1 waits
    assert [r.id for r in w.active] == [0] and [q.id for q in w.queue] == [1]
    w.batch.step()
    assert not w.cancel(0)  # admitted: cancelled before the next step
    w._cancel_active()
    assert done[-1].id == 0 and done[-1].error == "cancelled" and len(done[-1].stats) == 2
    assert w.adm.free == 2 and not batch.slots
    w.finish()
    w._loop()  # request 1 now runs to completion
    assert done[-1].id == 1 and done[-1].error is None
    assert not w.cancel(99)  # unknown ids are ignored


def test_plan_budget_sets_aside_fields_and_sizes_slots():
    plans = [sv.VolumePlan("a", 100, 10, 1), sv.VolumePlan("b", 300, 40, 2)]
    b = sv.plan_budget(plans, 1000, max_slots=24, kappa_cache=16, reserve_bytes=50)
    assert b.fixed == 50 + 100 + 16 + 300 + 32 and b.used == b.fixed
    # each volume could fill the rest alone: (1000 - 498 - kappa) // per_rhs, capped
    assert [p.capacity for p in plans] == [24, (1000 - 498 - 2) // 40]
    with pytest.raises(MemoryError):
        sv.plan_budget(plans, 450)


def test_shared_budget_moves_memory_between_volumes():
    """Two volumes draw from one budget: while volume 0 holds most of it volume 1's request
    waits, and it enters as soon as volume 0 gives its bytes back."""
    budget = sv.HbmBudget(100, fixed_bytes=10)
    a0 = sv.Admission(8, budget, slot_bytes=10, request_bytes=5)
    a1 = sv.Admission(8, budget, slot_bytes=20, request_bytes=5)
    assert a0.fits_ever(8) and not a1.fits_ever(5)  # 5 * 20 + 5 > 90 free at best
    assert a0.try_take(7)                # 75 bytes: used 85
    assert not a1.try_take(1)            # needs 25
    assert a0.free == 1 and a1.free == 8  # a refused request holds nothing
    a0.give_back(7)                      # 75 back: used 10
    assert a1.try_take(3) and budget.used == 75
    assert not a0.try_take(3)            # 35 more would exceed the budget
    assert a0.try_take(1) and budget.used == 90 and budget.peak == 90
    a0.give_back(1)
    a1.give_back(3)
    assert budget.used == budget.fixed


class FailingBatch(FakeBatch):
    """kappa 0.5 makes add raise (a singular clover term); source value 7 makes take raise
    (a non-finite residual); source value 5 finishes unconverged."""

    def add(self, kappa, b):
        if kappa == 0.5:
            raise RuntimeError("singular")
        return super().add(kappa, b)

    def take(self, s, out):
        n, b = self.slots[s]
        if b % 10 == 7:
            self.slots.pop(s)
            raise RuntimeError("non-finite residual")
        st = super().take(s, out)
        st["converged"] = 0 if b % 10 == 5 else 1
        return st


class FailingBackend(FakeBackend):
    def make_source(self, req):
        return [req.seed * 10 + i for i in range(req.nrhs)]


def test_failed_and_unconverged_requests_report_errors_and_return_their_slots():
    """A request whose slot raises on take, one that finishes unconverged, and one whose
    kappa is rejected on admission each come back with an error; the worker keeps serving
    the others, and every slot is free at the end."""
    batch = FailingBatch(4)
    adm = sv.Admission(4)
    w = sv.VolumeWorker("v", batch, FailingBackend(), adm, None, None)
    reqs = [sv.Request(0, 0.0, 0, 0.12, 1, seed=0),       # sources 0: fine
            sv.Request(1, 0.0, 0, 0.12, 2, seed=1),       # sources 10, 11: fine
            sv.Request(2, 0.0, 0, 0.5, 2, seed=2),        # kappa rejected on the first add
            sv.Request(3, 0.0, 0, 0.12, 3, seed=0),       # sources 0, 1, 2 ... fine
            sv.Request(4, 0.0, 0, 0.12, 1, seed=0.5),     # source 5: not converged
            sv.Request(5, 0.0, 0, 0.12, 1, seed=0.7)]     # source 7: take raises
    done = sv.Server([w]).run(reqs, realtime=False)
    err = {r.id: r.error for r in done}
    assert len(done) == 6
    assert err[0] is None and err[1] is None and err[3] is None
    assert "admission failed" in err[2]
    assert err[4] == "not converged within the iteration cap"
    assert "non-finite" in err[5]
    assert adm.free == 4 and not batch.slots
    s = sv.summarize(done, wall=1.0)
    assert s["requests"] == 3 and s["rejected"] == 3


class KeepingBatch(FakeBatch):
    """An elastic stand-in: a slot's memory is committed on first add and kept after take
    until trim; add prefers a slot that still holds memory (as sapdd_batch_add does)."""

    def __init__(self, capacity):
        super().__init__(capacity)
        self.committed = set()
        self.commits = 0
        self.trimmed = []

    def add(self, kappa, b):
        free = [s for s in range(self.cap) if s not in self.slots]
        if not free:
            raise RuntimeError("full")
        kept = [s for s in free if s in self.committed]
        s = kept[0] if kept else free[0]
        if s not in self.committed:
            self.committed.add(s)
            self.commits += 1
        self.slots[s] = [0, b]
        return s

    def trim(self, keep=0):
        idle = sorted(s for s in self.committed if s not in self.slots)
        for s in idle[keep:]:
            self.committed.discard(s)
        self.trimmed.append(len(idle[keep:]))
        return 10 * len(idle[keep:])


def test_kept_slots_are_charged_once():
    """A request that reuses kept slots pays only for its sources and kappa; released()
    returns the kept slots' bytes."""
    budget = sv.HbmBudget(1000, fixed_bytes=100)
    a = sv.Admission(8, budget, slot_bytes=30, request_bytes=5, warm_bytes=20)
    assert a.try_take(3) and budget.used == 100 + 3 * 30 + 5 and a.committed == 3
    a.give_back(3)  # the batch keeps the 3 slots: their warm part stays charged
    assert budget.used == 100 + 3 * 20 and a.kept() == 3
    assert a.try_take(2) and budget.used == 100 + 60 + 2 * 10 + 5  # no new slot memory
    assert a.try_take(2) and a.committed == 4 and a.kept() == 0    # one slot more
    a.give_back(2)
    a.give_back(2)
    assert a.kept() == 4 and budget.used == 100 + 4 * 20
    a.released(4)
    assert budget.used == budget.fixed and a.committed == 0


def test_idle_volume_gives_kept_memory_to_a_waiting_volume():
    """The two requests cannot hold their memory together: whichever volume runs first
    keeps its slots after finishing, the other volume's request waits for those bytes, and
    the first volume (nothing queued) trims them. Every request completes and the budget
    ends with only the memory still kept."""
    budget = sv.HbmBudget(100, fixed_bytes=10)
    b0, b1 = KeepingBatch(8), KeepingBatch(8)
    a0 = sv.Admission(8, budget, slot_bytes=12, request_bytes=0, warm_bytes=10)
    a1 = sv.Admission(8, budget, slot_bytes=12, request_bytes=0, warm_bytes=10)
    w0 = sv.VolumeWorker("v0", b0, FakeBackend(), a0, None, None)
    w1 = sv.VolumeWorker("v1", b1, FakeBackend(), a1, None, None)
    reqs = [sv.Request(0, 0.0, 0, 0.12, 6, seed=1),   # 72 of the 90 free bytes
            sv.Request(1, 0.0, 1, 0.12, 5, seed=2)]   # 60: waits until volume 0 trims
    done = sv.Server([w0, w1]).run(reqs, realtime=False)
    assert sorted(r.id for r in done) == [0, 1] and all(r.error is None for r in done)
    assert w0.trims + w1.trims >= 1 and bool(b0.committed) != bool(b1.committed)
    assert budget.used == budget.fixed + 10 * (len(b0.committed) + len(b1.committed))
    assert budget.peak <= budget.total and not budget.waiting and not budget.running


def test_busy_volume_keeps_its_memory_between_requests():
    """A volume with queued requests reuses its kept slots: each slot is committed once."""
    budget = sv.HbmBudget(1000, fixed_bytes=0)
    b = KeepingBatch(4)
    a = sv.Admission(4, budget, slot_bytes=12, request_bytes=1, warm_bytes=10)
    w = sv.VolumeWorker("v", b, FakeBackend(), a, None, None)
    reqs = [sv.Request(i, 0.0, 0, 0.12, n, seed=i) for i, n in enumerate([3, 4, 2, 4, 1])]
    done = sv.Server([w]).run(reqs, realtime=False)
    assert len(done) == 5 and all(r.error is None for r in done)
    assert b.commits == 4 and w.trims == 0
    assert budget.used == 4 * 10 and a.kept() == 4


def test_idle_volume_trims_only_what_the_waiting_volume_lacks():
    """Volume 0 keeps 6 slots (60 bytes of kept memory); volume 1's request of 3 slots
    lacks 20 bytes of the budget, so volume 0 gives back 2 slots and keeps 4."""
    budget = sv.HbmBudget(100, fixed_bytes=10)
    b0, b1 = KeepingBatch(8), KeepingBatch(8)
    a0 = sv.Admission(8, budget, slot_bytes=10, request_bytes=0, warm_bytes=10)
    a1 = sv.Admission(8, budget, slot_bytes=10, request_bytes=0, warm_bytes=10)
    w0 = sv.VolumeWorker("v0", b0, FakeBackend(), a0, lambda: 0.0, lambda r: None)
    w1 = sv.VolumeWorker("v1", b1, FakeBackend(), a1, lambda: 0.0, lambda r: None)
    w0.submit(sv.Request(0, 0.0, 0, 0.12, 6, seed=1))
    w0._admit()
    while w0.active:
        w0.batch.step()
        w0._harvest()
    assert a0.kept() == 6 and budget.used == 10 + 60
    w1.submit(sv.Request(1, 0.0, 1, 0.12, 5, seed=2))  # needs 50, 30 free: lacks 20
    w1._admit()
    assert [r.id for r in w1.queue] == [1] and budget.waiting == {w1.name: 20}
    w0._trim_if_wanted()
    assert b0.trimmed == [2] and a0.kept() == 4 and budget.used == 10 + 40
    w1._admit()
    assert [r.id for r in w1.active] == [1] and not budget.waiting


class CountingBackend(FakeBackend):
    """Counts the output arrays alive (made and not yet garbage)."""

    def __init__(self):
        import weakref
        self.refs = []
        self.weakref = weakref

    def make_output(self, req):
        class Out(list):
            pass
        outs = [Out() for _ in range(req.nrhs)]
        self.refs += [self.weakref.ref(o) for o in outs]
        return outs

    def alive(self):
        return sum(r() is not None for r in self.refs)


def test_server_hands_results_over_and_lets_go():
    """With on_result the server passes each finished request's solutions on and drops
    them, so a long stream holds only the requests in flight; without it they stay."""
    import gc
    for keep in (False, True):
        be = CountingBackend()
        got = []
        batch = FakeBatch(3)
        w = sv.VolumeWorker("v", batch, be, sv.Admission(3), None, None)
        srv = sv.Server([w], on_result=None if keep else (lambda r: got.append((r.id, [list(o) for o in r.x]))))
        reqs = [sv.Request(i, 0.0, 0, 0.12, 1 + i % 3, seed=i) for i in range(12)]
        done = srv.run(reqs, realtime=False)
        gc.collect()
        assert len(done) == 12 and all(r.error is None for r in done)
        if keep:
            assert be.alive() == sum(r.nrhs for r in reqs) and all(r.x is not None for r in done)
        else:
            assert be.alive() == 0 and all(r.x is None for r in done)
            assert sorted(i for i, _ in got) == list(range(12))
            assert all(xs[j][0] == 2 * (reqs[i].seed * 10 + j) for i, xs in got for j in range(len(xs)))
