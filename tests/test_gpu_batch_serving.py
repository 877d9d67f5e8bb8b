"""GPU tests of the continuous-batching solver and the serving loop.

A right-hand side's solution must be bit-identical whether it is solved alone or in a
batch with others that join and leave at different times (slots are independent and all
reductions have a fixed order), and every solution must reach a true relative residual
<= 1e-10 recomputed by the oracle's operator.
"""
import numpy as np
import pytest

import synthetic
from oracle import wilson

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1502_04025_amd import Context
    stream = torch.cuda.Stream()
    ctx = Context(0, stream=stream)  # a real stream: SAP sweeps replay from HIP graphs
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    u = synthetic.gauge_field(dims, 0.3, 5)
    t = wilson.clover_term(u, 1.0)
    with torch.cuda.stream(stream):
        f = ctx.load_gauge(u, block)
        f.compute_clover(1.0)
    yield dict(ctx=ctx, f=f, u=u, t=t, dims=dims, stream=stream, torch=torch)
    f.free()
    ctx.close()


def oracle_relres(u, t, kappa, x, b):
    return np.linalg.norm(b - wilson.apply_M(u, t, kappa, x)) / np.linalg.norm(b)


def test_batch_join_leave_matches_solo(env):
    from paper_1502_04025_amd import Batch
    torch, f = env["torch"], env["f"]
    b = synthetic.gaussian_source(env["dims"], 3, 31)
    kap = [0.121, 0.125, 0.123]
    with torch.cuda.stream(env["stream"]):
        solo = [f.solve(kap[r], b[r:r + 1].copy(), prec="f16").x[0] for r in range(3)]
        batch = Batch(f, 2, prec="f16")
        s0 = batch.add(kap[0], b[0])
        batch.step()                      # rhs 0 is one cycle ahead
        s1 = batch.add(kap[1], b[1])      # joins a running batch
        xs = {}
        pending = {0: s0, 1: s1}
        while pending:
            batch.step()
            for r, s in list(pending.items()):
                if batch.poll(s)[0]:
                    out = np.empty_like(b[r])
                    st = batch.take(s, out)
                    assert st["converged"]
                    xs[r] = out
                    del pending[r]
                    if r == 0:            # a freed slot is reused by the third rhs
                        pending[2] = batch.add(kap[2], b[2])
        batch.close()
    for r in range(3):
        assert np.array_equal(xs[r], solo[r])
        assert oracle_relres(env["u"], env["t"], kap[r], xs[r], b[r]) <= 1e-10


def test_batch_full_and_graph_equals_direct_launches(env):
    from paper_1502_04025_amd import EFULL, NO_GRAPH, Batch, SapddError
    torch, f = env["torch"], env["f"]
    b = synthetic.gaussian_source(env["dims"], 2, 32)
    with torch.cuda.stream(env["stream"]):
        batch = Batch(f, 1, prec="f32")
        batch.add(0.124, b[0])
        with pytest.raises(SapddError) as e:
            batch.add(0.124, b[1])
        assert e.value.code == EFULL
        batch.close()
        g = f.solve(0.124, b, prec="f32").x
        d = f.solve(0.124, b, prec="f32", flags=NO_GRAPH).x
    assert np.array_equal(g, d)


def test_serving_loop_results_equal_alone(env):
    from paper_1502_04025_amd import serving as sv
    torch = env["torch"]
    vols = [sv.TorchVolume("v0", (8, 8, 8, 8), (4, 4, 4, 4), 0.3, 5, 1.0, 6, dict(prec="f16")),
            sv.TorchVolume("v1", (8, 8, 8, 16), (4, 4, 4, 4), 0.3, 6, 1.0, 6, dict(prec="f16"))]
    reqs = synthetic.serving_requests(10, rate=1e9, seed=33, volumes=[v.dims for v in vols], max_rhs=4)
    reqs = [sv.Request(r["id"], 0.0, r["vol"], r["kappa"], r["nrhs"], r["seed"]) for r in reqs]
    workers = [sv.VolumeWorker(v.name, v.batch, v, sv.Admission(6), None, None) for v in vols]
    done = sv.Server(workers).run(reqs, realtime=False)
    assert len(done) == 10 and all(r.error is None for r in done)
    for r in done:
        v = vols[r.vol]
        with torch.cuda.stream(v.stream):
            bs = v.make_source(r)
            for i in range(r.nrhs):
                alone = v.field.solve(r.kappa, bs[i].unsqueeze(0).contiguous(), prec="f16").x
                torch.cuda.synchronize()
                assert torch.equal(alone[0], r.x[i])
                assert r.stats[i]["converged"] and r.stats[i]["true_relres"] <= 1e-10
    # every served solution reaches 1e-10 by the oracle's own FP64 operator
    fields = {0: ((8, 8, 8, 8), 5), 1: ((8, 8, 8, 16), 6)}
    ops = {}
    for k, (dims, seed) in fields.items():
        u = synthetic.gauge_field(dims, 0.3, seed)
        ops[k] = (u, wilson.clover_term(u, 1.0))
    for r in done:
        u, t = ops[r.vol]
        bs = vols[r.vol].make_source(r)
        for i in range(r.nrhs):
            rel = oracle_relres(u, t, r.kappa, r.x[i].cpu().numpy(), bs[i].cpu().numpy())
            assert rel <= 1e-10, (r.id, i, rel)
    s = sv.summarize(done, wall=max(r.t_done for r in done))
    assert s["requests"] == 10 and s["p99_ms"] >= s["p50_ms"] > 0
    for v in vols:
        v.close()


def test_cancel_and_resume_from_the_taken_iterate(env):
    """Taking an unfinished slot returns the iterate of its last restart cycle; adding it
    back as the start vector finishes the solve (checkpoint and resume)."""
    from paper_1502_04025_amd import Batch
    torch, f = env["torch"], env["f"]
    b = synthetic.gaussian_source(env["dims"], 1, 34)[0]
    with torch.cuda.stream(env["stream"]):
        batch = Batch(f, 1, prec="f32", restart=2)
        s = batch.add(0.124, b)
        batch.step()
        finished, st = batch.poll(s)
        assert not finished and st["iters"] == 2
        x1 = np.empty_like(b)
        batch.take(s, x1)  # cancels the slot
        r1 = oracle_relres(env["u"], env["t"], 0.124, x1, b)
        assert 1e-10 < r1 < 1.0  # a partial solution
        s = batch.add(0.124, b, x0=x1)  # resume
        while batch.step():
            pass
        x2 = np.empty_like(b)
        st2 = batch.take(s, x2)
        batch.close()
    assert st2["converged"]
    assert oracle_relres(env["u"], env["t"], 0.124, x2, b) <= 1e-10


def test_elastic_batch_commits_memory_per_slot(env):
    """An elastic batch holds only its fixed workspaces until slots are admitted, commits
    at most slot_bytes per admitted right-hand side, keeps a taken slot's memory for the
    next add, gives it back on trim, and computes the same bits as a batch allocated
    whole."""
    from paper_1502_04025_amd import Batch
    torch, f = env["torch"], env["f"]
    b = synthetic.gaussian_source(env["dims"], 3, 35)
    kap = [0.121, 0.125, 0.123]
    with torch.cuda.stream(env["stream"]):
        whole = [f.solve(kap[r], b[r:r + 1].copy(), prec="f16").x[0] for r in range(3)]
        batch = Batch(f, 8, elastic=True, prec="f16")
        held0, slot = batch.memory()
        assert slot > 0
        s0 = batch.add(kap[0], b[0])
        held1, _ = batch.memory()
        assert held0 < held1 <= held0 + slot
        s1 = batch.add(kap[1], b[1])
        held2, _ = batch.memory()
        assert held1 < held2 <= held0 + 2 * slot
        xs, pending = {}, {0: s0, 1: s1}
        while pending:
            batch.step()
            for r, s in list(pending.items()):
                if batch.poll(s)[0]:
                    out = np.empty_like(b[r])
                    assert batch.take(s, out)["converged"]
                    xs[r] = out
                    del pending[r]
                    if r == 0:  # the kept slot's memory serves the third right-hand side
                        pending[2] = batch.add(kap[2], b[2])
                        assert pending[2] == s0 and batch.memory()[0] == held2
        assert batch.memory()[0] == held2  # every slot taken, both kept
        assert batch.trim(1) == held2 - held1 and batch.memory()[0] == held1
        assert batch.trim(0) == held1 - held0 and batch.memory()[0] == held0
        assert batch.trim(0) == 0
        batch.close()
    for r in range(3):
        assert np.array_equal(xs[r], whole[r])
        assert oracle_relres(env["u"], env["t"], kap[r], xs[r], b[r]) <= 1e-10


def test_serving_with_one_shared_budget(env):
    """Two volumes with elastic batches draw from one HBM budget too small for both to
    fill their slots at once: every request still completes, bit-identical to its solve
    alone and at 1e-10 by the oracle's operator, and the budget is never exceeded."""
    from paper_1502_04025_amd import serving as sv
    torch = env["torch"]
    kw = dict(prec="f16")
    vols = [sv.TorchVolume("v0", (8, 8, 8, 8), (4, 4, 4, 4), 0.3, 5, 1.0, 8, kw, elastic=True),
            sv.TorchVolume("v1", (8, 8, 8, 16), (4, 4, 4, 4), 0.3, 6, 1.0, 8, kw, elastic=True)]
    plans = [v.plan() for v in vols]
    fixed = sum(p.field_bytes + 4 * p.kappa_bytes for p in plans)
    total = fixed + 6 * max(p.per_rhs_bytes for p in plans) + 2 * max(p.kappa_bytes for p in plans)
    budget = sv.plan_budget(plans, total, max_slots=8, kappa_cache=4)
    reqs = synthetic.serving_requests(12, rate=1e9, seed=36, volumes=[v.dims for v in vols], max_rhs=4)
    reqs = [sv.Request(r["id"], 0.0, r["vol"], r["kappa"], r["nrhs"], r["seed"]) for r in reqs]
    adms = [sv.Admission(p.capacity, budget, p.per_rhs_bytes, p.kappa_bytes, p.warm_bytes) for p in plans]
    assert all(p.warm_bytes > 0 for p in plans)
    workers = [sv.VolumeWorker(v.name, v.batch, v, a, None, None) for v, a in zip(vols, adms)]
    done = sv.Server(workers).run(reqs, realtime=False)
    assert len(done) == 12 and all(r.error is None for r in done)
    assert budget.peak <= budget.total
    # what the budget still charges is exactly the memory the batches keep
    for v, a, p in zip(vols, adms, plans):
        with torch.cuda.stream(v.stream):
            k = a.kept()
            assert v.batch.trim(0) == k * p.warm_bytes
            a.released(k)
    assert budget.used == budget.fixed
    fields = {0: ((8, 8, 8, 8), 5), 1: ((8, 8, 8, 16), 6)}
    ops = {k: (lambda u: (u, wilson.clover_term(u, 1.0)))(synthetic.gauge_field(d, 0.3, s))
           for k, (d, s) in fields.items()}
    for r in done:
        v = vols[r.vol]
        with torch.cuda.stream(v.stream):
            bs = v.make_source(r)
            for i in range(r.nrhs):
                alone = v.field.solve(r.kappa, bs[i].unsqueeze(0).contiguous(), prec="f16").x
                torch.cuda.synchronize()
                assert torch.equal(alone[0], r.x[i])
        u, t = ops[r.vol]
        for i in range(r.nrhs):
            assert oracle_relres(u, t, r.kappa, r.x[i].cpu().numpy(), bs[i].cpu().numpy()) <= 1e-10
    for v in vols:
        v.close()


def test_clover_cache_recycles_buffers_without_stale_values(env):
    """More distinct kappas than the field's 16 cached clover inverses: one SAP call with
    18 of them, then each kappa alone, must give the same bits (a later kappa of a call
    never recycles an earlier one's buffer, and a recycled buffer holds the new kappa's
    inverse); a batch serving 20 kappas in turn, then the first two again, too."""
    from paper_1502_04025_amd import Batch
    torch, f = env["torch"], env["f"]
    kap = [0.1200 + 0.0003 * r for r in range(20)]
    psi = synthetic.gaussian_source(env["dims"], 18, 37)
    with torch.cuda.stream(env["stream"]):
        together = f.sap(np.array(kap[:18]), psi, prec="f16")
        for r in range(18):
            alone = f.sap(kap[r], psi[r:r + 1].copy(), prec="f16")
            assert np.array_equal(alone[0], together[r])
        b = synthetic.gaussian_source(env["dims"], 1, 38)[0]
        batch = Batch(f, 1, prec="f16")
        xs = []
        for k in kap + kap[:2]:
            s = batch.add(k, b)
            while not batch.poll(s)[0]:
                batch.step()
            out = np.empty_like(b)
            assert batch.take(s, out)["converged"]
            xs.append(out)
        batch.close()
    assert np.array_equal(xs[20], xs[0]) and np.array_equal(xs[21], xs[1])
    assert not np.array_equal(xs[0], xs[1])
    assert oracle_relres(env["u"], env["t"], kap[19], xs[19], b) <= 1e-10


def test_trimmed_memory_moves_to_another_elastic_batch(env):
    """Two elastic batches on one field: the first solves, is trimmed (its chunks go to
    the shared pool) and a second one commits that memory for its own solves; every
    solution has the bits of a batch allocated whole, and both batches trim to their
    fixed part."""
    from paper_1502_04025_amd import Batch
    torch, f = env["torch"], env["f"]
    b = synthetic.gaussian_source(env["dims"], 4, 39)
    kap = [0.121, 0.124, 0.122, 0.125]
    with torch.cuda.stream(env["stream"]):
        whole = [f.solve(kap[r], b[r:r + 1].copy(), prec="f16").x[0] for r in range(4)]

        def run(batch, rs):
            out = {}
            slots = {r: batch.add(kap[r], b[r]) for r in rs}
            while any(not batch.poll(s)[0] for s in slots.values()):
                batch.step()
            for r, s in slots.items():
                out[r] = np.empty_like(b[r])
                assert batch.take(s, out[r])["converged"]
            return out

        b1 = Batch(f, 2, elastic=True, prec="f16")
        fixed1 = b1.memory()[0]
        xs = run(b1, [0, 1])
        assert b1.trim(0) > 0 and b1.memory()[0] == fixed1
        b2 = Batch(f, 2, elastic=True, prec="f16")
        fixed2 = b2.memory()[0]
        xs.update(run(b2, [2, 3]))
        xs.update({r + 10: x for r, x in run(b1, [0, 1]).items()})  # b1 commits again, from the pool
        assert b2.trim(0) > 0 and b1.trim(0) > 0
        assert b1.memory()[0] == fixed1 and b2.memory()[0] == fixed2
        b2.close()
        b1.close()
    for r in range(4):
        assert np.array_equal(xs[r], whole[r])
    assert np.array_equal(xs[10], whole[0]) and np.array_equal(xs[11], whole[1])


_SMALL_PIECES = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, {root!r})
import synthetic
from paper_1502_04025_amd import Batch, Context
stream = torch.cuda.Stream()
ctx = Context(0, stream=stream)
dims = (8, 8, 8, 8)
u = synthetic.gauge_field(dims, 0.3, 5)
b = torch.from_numpy(synthetic.gaussian_source(dims, 3, 40)).cuda()
kap = [0.121, 0.124, 0.122]
with torch.cuda.stream(stream):
    f = ctx.load_gauge(u, (4, 4, 4, 4))
    f.compute_clover(1.0)
    whole = Batch(f, 3, prec="f16")
    el = [Batch(f, 3, elastic=True, prec="f16") for _ in range(2)]

    def run(batch, rs):
        slots = {{r: batch.add(kap[r], b[r]) for r in rs}}
        while any(not batch.poll(s)[0] for s in slots.values()):
            batch.step()
        out = {{}}
        for r, s in slots.items():
            out[r] = torch.empty_like(b[r])
            assert batch.take(s, out[r])["converged"]
        torch.cuda.synchronize()
        return out

    ref = run(whole, [0, 1, 2])
    got = run(el[0], [0, 1])
    assert el[0].trim(0) > 0
    got.update(run(el[1], [2]))
    again = run(el[0], [0, 1])
    for r in range(3):
        assert torch.equal(ref[r], got[r]), r
    assert torch.equal(again[0], ref[0]) and torch.equal(again[1], ref[1])
    for x in el + [whole]:
        x.close()
    f.free()
ctx.close()
print("small pieces ok")
"""


def test_elastic_slots_spanning_many_pieces():
    """With 64 KiB pieces every slot field of an 8^4 batch spans many mappings (zero
    fills, packing and the solver kernels cross them): the results keep the bits of a
    batch allocated whole, also after the memory moved to another batch and back. Runs
    in its own process, which reads the piece size from the environment."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, SAPDD_ELASTIC_PIECE_KB="64")
    r = subprocess.run([sys.executable, "-c", _SMALL_PIECES.format(root=root)], env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0 and "small pieces ok" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
