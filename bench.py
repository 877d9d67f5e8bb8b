#!/usr/bin/env python
"""Benchmark: SAP-preconditioned FGMRES solves on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5|c5_f16l|c5_host_io|c2|c2_f64|c3|c3_f64_1rhs|serve|mg]
    python bench.py --sweep          # time to solution over nmr x ncy x domain shape

One step = one complete solve of M x = b for every right-hand side of the workload to a
true relative residual of 1e-10 (SAP preconditioner + FP64 flexible GMRES, every kernel
of the hot path), with b and x resident in HBM. The default workload is the largest
single-GPU configuration: the 48^3 x 96 lattice with 8x4x4x4 domains, 12 Gaussian
right-hand sides solved together, FP16 Schwarz/MR storage, FP64 FGMRES(3) whose true
residual is recomputed at every restart; 4 MR steps per block solve and 8 Schwarz
cycles per preconditioner application.

Printed: one JSON line with RHS solves/s, the roofline of the dominant kernel (the SAP
half-sweep: per-kernel HIP-event times measured on the solve's stream during the timed
steps, HBM traffic from the committed rocprofv3 counters), and as sub-objects: the
block-Dslash bandwidth on 32^3 x 64, the 16^3 x 32 single-RHS solve (FP32 SAP and the
all-FP64 path), the mixed-precision 12-RHS form against plain FP64 single-RHS solves on
32^3 x 64, a bounded serving phase with p50/p99 latency, the two-level multigrid near
the critical kappa, and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# name: (configuration, SAP storage precision, overrides). The MR steps per block solve
# (4, the paper's optimum) and the Schwarz cycles per preconditioner application (8) are
# the time-to-solution optimum of `bench.py --sweep` on this GPU, near-optimal for every
# workload here; the 4^4 parity case keeps the 4 x 5 of its definition.
NCY = 8
WORKLOADS = {
    "c2": ("c2_16x16x16x32_f32", "f32", {"ncy": NCY}),
    "c2_f64": ("c2_16x16x16x32_f32", "f64", {"ncy": NCY}),
    "c3": ("c3_32x32x32x64_f16", "f16", {"ncy": NCY}),
    "c3_f64_1rhs": ("c3_32x32x32x64_f16", "f64", {"nrhs": 1, "source": "gaussian", "ncy": NCY}),
    # 12 RHS of FGMRES(3) on 48^3x96 need ~213 GB of Krylov state; b and x (6 GB) stay
    # resident in HBM beside it. c5_host_io keeps them in host memory instead (staged over
    # PCIe one right-hand side at a time, inside the timed region).
    "c5": ("c5_48x48x48x96_f16", "f16", {"restart": 3, "ncy": NCY}),
    "c5_host_io": ("c5_48x48x48x96_f16", "f16", {"restart": 3, "ncy": NCY, "host_io": True}),
    # the paper's half-precision mode: FP16 links and clover, FP32 Schwarz spinors
    "c5_f16l": ("c5_48x48x48x96_f16", "f16l", {"restart": 3, "ncy": NCY}),
}


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q))


def make_field(ctx, cfg, u=None):
    import synthetic
    if u is None:
        u = synthetic.gauge_field(cfg["dims"], cfg["eps"], cfg["gauge_seed"])
    f = ctx.load_gauge(u, cfg["block"])
    f.compute_clover(cfg["csw"])
    return u, f


def make_source(cfg):
    import synthetic
    if cfg["source"] == "point":
        return synthetic.point_sources(cfg["dims"])[: cfg["nrhs"]].copy()
    return synthetic.gaussian_source(cfg["dims"], cfg["nrhs"], cfg["source_seed"])


def profiled_traffic(entry):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter summaries, or
    None if there is none for the kernel's current sources (changed since the counters
    were taken)."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.txt")):
        for line in open(path):
            if not line.startswith("TRAFFIC "):
                continue
            rec = json.loads(line[len("TRAFFIC "):])
            if rec["entry"] != entry:
                continue
            h = hashlib.sha256()
            for f in rec["sources"]:
                h.update(open(os.path.join(ROOT, f), "rb").read())
            if h.hexdigest()[:16] == rec["source_sha"]:
                return rec["fetch_bytes"] + rec["write_bytes"]
    return None


def sap_kernel_name(cfg, prec):
    """The SAP half-sweep kernel the library launches for this workload: the pair form for
    FP16 links and clover with at least 256 domains of each colour and 256-site domains,
    the split-parity form otherwise (SAPDD_SAP_KERNEL=pair/split forces one)."""
    force = os.environ.get("SAPDD_SAP_KERNEL")
    ndom = int(np.prod(cfg["dims"])) // int(np.prod(cfg["block"]))
    pair = prec in ("f16", "f16l") and ndom // 2 >= 256
    if force in ("pair", "split"):
        pair = force == "pair"
    pair = pair and int(np.prod(cfg["block"])) >= 256
    return "sap_pair_kernel" if pair else "sap_half_kernel"


def roofline_sap(prof, cfg, prec, nmr):
    """Roofline of the SAP half-sweep from the HIP-event times of the timed steps: flops
    and algorithmic bytes per launch (one colour, every right-hand side), both roofs, and
    the HBM traffic per launch that the committed rocprofv3 counters give for this kernel
    and workload."""
    from paper_1502_04025_amd import perfmodel as pm
    k = prof["sap_half"]
    if k["launches"] == 0:
        return None
    V = int(np.prod(cfg["dims"]))
    nrhs = cfg["nrhs_active"]
    avg = k["seconds"] / k["launches"]
    flops = pm.sap_half_flops(cfg["block"], nmr) * V / 2 * nrhs
    byts = pm.sap_half_bytes(cfg["block"], prec, nrhs) * V / 2
    ar = "f64" if prec == "f64" else "f32"
    alu_peak, alu_pub = pm.ALU_PEAK_TFLOPS[ar], pm.ALU_PEAK_PUBLISHED_TFLOPS[ar]
    kname = sap_kernel_name(cfg, prec)
    traffic = profiled_traffic(f"{kname} {'x'.join(map(str, cfg['dims']))} {'x'.join(map(str, cfg['block']))} "
                               f"{prec} nrhs {nrhs}")
    t_alu = flops / (alu_peak * 1e12)
    t_hbm = byts / (pm.HBM_PEAK_GBS * 1e9)
    tflops, gbs = flops / avg / 1e12, byts / avg / 1e9
    # one SAP cycle's data (both colours) below the 256 MB Infinity Cache makes the
    # bandwidth figure a cache one
    resident = bool(2 * byts < 256e6)
    both = dict(alu_TFLOP_s=round(tflops, 3), alu_frac=round(tflops / alu_peak, 4),
                alu_frac_of_published_157=round(tflops / alu_pub, 4),
                mem_GB_s=round(gbs, 1), mem_frac=round(gbs / pm.HBM_PEAK_GBS, 4),
                working_set_bytes=2 * byts, cache_resident=resident)
    common = dict(traffic=traffic, avg_launch_us=round(avg * 1e6, 2), launches=k["launches"],
                  algorithmic_flops_per_launch=flops, algorithmic_bytes_per_launch=byts,
                  traffic_over_algorithmic=round(traffic / byts, 3) if traffic else None, **both)
    if t_alu >= t_hbm:
        return dict(kernel=kname, bound="alu", achieved=round(tflops, 3), peak=alu_peak,
                    unit="TFLOP/s", frac=round(tflops / alu_peak, 4),
                    peak_note=f"FP32 vector peak without packed FP32 (the build disables it); the published "
                              f"{alu_pub} TFLOP/s counts packed FMAs", **common)
    return dict(kernel=kname, bound="cache" if resident else "hbm", achieved=round(gbs, 1),
                peak=pm.HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / pm.HBM_PEAK_GBS, 4), **common)


def dslash_bandwidth(ctx, warm=10, reps=100):
    """Block Dslash on 32^3 x 64 (4^4 domains), FP16 and FP32 storage, device arrays:
    `warm` untimed launches, then `reps` launches each timed by its own HIP-event pair;
    GB/s at the median launch time, with p10/p90."""
    import torch

    import synthetic
    from paper_1502_04025_amd import perfmodel as pm
    cfg = synthetic.CONFIGS["c3_32x32x32x64_f16"]
    u, f = make_field(ctx, cfg)
    del u
    psi = torch.from_numpy(synthetic.gaussian_source(cfg["dims"], 1, 41)).cuda()
    out = torch.empty_like(psi)
    V = int(np.prod(cfg["dims"]))
    res = {}
    for prec, two_row in (("f16", False), ("f32", False), ("f16", True), ("f32", True)):
        for _ in range(warm):  # the first one builds the low-precision copies
            f.apply_block_D(cfg["kappa"], psi, prec=prec, out=out, links12=two_row)
        ts = []
        for _ in range(reps):
            ctx.profile(True, families=["block_dslash"])
            f.apply_block_D(cfg["kappa"], psi, prec=prec, out=out, links12=two_row)
            ts.append(ctx.profile(False)["block_dslash"]["seconds"])
        med, p10, p90 = (float(np.percentile(ts, q)) for q in (50, 10, 90))
        byts = pm.block_dslash_bytes(cfg["block"], prec, links12=two_row) * V
        gbs = byts / med / 1e9
        kname = "dslash_block12_kernel" if two_row else "dslash_block_kernel"
        res[prec + ("_links12" if two_row else "")] = dict(
            GB_s=round(gbs, 1), frac=round(gbs / pm.HBM_PEAK_GBS, 4), median_launch_us=round(med * 1e6, 2),
            p10_us=round(p10 * 1e6, 2), p90_us=round(p90 * 1e6, 2), launches=reps,
            algorithmic_bytes_per_launch=byts, traffic=profiled_traffic(f"{kname} 32x32x32x64 4x4x4x4 {prec}"))
    f.free()
    return dict(kernel="dslash_block_kernel", lattice="32x32x32x64", block=list(cfg["block"]), **res)


def mg_extra(ctx):
    """One Gaussian RHS on the default workload's field at kappa 0.145 (near critical):
    the two-level multigrid of `--workload mg` against SAP alone, one timed solve each
    after a warm-up."""
    import torch

    import synthetic
    from paper_1502_04025_amd import Multigrid
    cfg = dict(synthetic.CONFIGS["c2_16x16x16x32_f32"])
    mc = dict(MG_RUN)
    u, f = make_field(ctx, cfg)
    del u
    b = torch.from_numpy(synthetic.gaussian_source(cfg["dims"], 1, cfg["source_seed"])).cuda()
    x = torch.empty_like(b)
    vecs = synthetic.gaussian_source(cfg["dims"], mc["nvec"], mc["vec_seed"])
    kw = dict(nmr=mc["nmr"], ncy=mc["ncy"], restart=mc["restart"], tol=1e-10, prec=mc["prec"], max_iter=5000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mg = Multigrid(f, mc["kappa"], vecs, setup_iters=mc["setup_iters"], coarse_iters=mc["coarse_iters"],
                   coarse_cycles=mc["coarse_cycles"], nmr=mc["nmr"], ncy=mc["setup_ncy"], prec=mc["prec"],
                   coarse_form=1)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    out = {"workload": f"16x16x16x32, kappa {mc['kappa']}, 1 gaussian RHS (see --workload mg), coarse GMRES "
                       "with one launch per Arnoldi step", "setup_s": round(setup_s, 3)}
    for name, step in (("mg", lambda: mg.solve(b, x=x, **kw)), ("sap_only", lambda: f.solve(mc["kappa"], b, x=x, **kw))):
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = step()
        torch.cuda.synchronize()
        out[name] = {"ms": round(1e3 * (time.perf_counter() - t0), 2), "outer_iters": r.stats[0]["iters"],
                     "converged": bool(r.stats[0]["converged"])}
    mg.close()
    f.free()
    return out


def copy_bandwidth(ctx, nbytes=1 << 31, reps=10):
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    ctx.copy(a.data_ptr(), b.data_ptr(), nbytes)
    ctx.profile(True)
    for _ in range(reps):
        ctx.copy(a.data_ptr(), b.data_ptr(), nbytes)
    p = ctx.profile(False)["copy"]
    return round(2 * nbytes / (p["seconds"] / p["launches"]) / 1e9, 1)


def cpu_baseline(cfg, iters, restarts, nmr, ncy, nrhs):
    """Time the oracle on a bounded sample of the workload: one Schwarz half-sweep (the
    block solves of one colour plus the residual update) and one operator application on
    a 48 x 48 x 24 x 8 lattice drawn by the workload's recipe (same eps, kappa, c_sw and
    domains), scaled per site to the workload's lattice and to the GPU's iteration count
    (every outer iteration = 2 ncy half-sweeps + one operator application, plus one
    operator application per restart), per right-hand side."""
    from threadpoolctl import threadpool_limits

    import synthetic
    from oracle import sap as osap
    from oracle import wilson
    sample = (48, 48, 24, 8) if tuple(cfg["block"]) == (8, 4, 4, 4) else (32, 32, 32, 8)
    vs = int(np.prod(sample))
    scale = int(np.prod(cfg["dims"])) / vs
    with threadpool_limits(1):
        u = synthetic.gauge_field(sample, cfg["eps"], cfg["gauge_seed"], workers=1)
        t = wilson.clover_term(u, cfg["csw"])
        b = synthetic.gaussian_source(sample, 1, cfg["source_seed"], workers=1)[0]
        sysb = osap.BlockSystem(u, t, cfg["kappa"], cfg["block"])
        t0 = time.perf_counter()
        wilson.apply_M(u, t, cfg["kappa"], b)
        t_m = (time.perf_counter() - t0) * scale
        t0 = time.perf_counter()
        delta, _ = sysb.block_solve(b, 0, nmr)
        wilson.apply_M(u, t, cfg["kappa"], delta)
        t_half = (time.perf_counter() - t0) * scale
    t_solve = iters * (2 * ncy * t_half + t_m) + (restarts + 1) * t_m
    model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")), None)
    return dict(value=round(1.0 / t_solve, 8), unit="RHS solves/s", cores=1, kind="oracle",
                host_cores=len(os.sched_getaffinity(0)), cpu_model=model, extrapolated=True,
                sample=f"one Schwarz half-sweep (even-odd MR block solves of colour 0, nmr {nmr}, plus the "
                       f"residual update) and one operator application on a {'x'.join(map(str, sample))} "
                       f"lattice of the same recipe, NumPy FP64 on one core ({t_half / scale:.1f} s and "
                       f"{t_m / scale:.2f} s), scaled by {scale:.0f}x to {'x'.join(map(str, cfg['dims']))} and to "
                       f"{iters} outer iterations x {2 * ncy} half-sweeps per right-hand side "
                       f"({t_solve:.0f} s per solve; the GPU solves {nrhs} together)")


def serving_measure(n_requests, fracs, budget_gb, warm=6, max_slots=24):
    """Serving stream: Poisson arrivals of 1-12 RHS solve requests on resident fields of
    16^3x32, 24^3x48 and 32^3x64 (4^4 domains, FP16 SAP, FP64 FGMRES(16)), kappa uniform
    in [0.120, 0.126], continuous batching per volume. Admission by HBM footprint from one
    shared budget: every volume's batch is elastic (a slot's memory is committed only while
    it is in use) and every request draws its bytes from the budget, whatever its volume.
    A closed loop (every request at t = 0) measures the saturation rate; then n_requests
    arrive at each fraction of it. Returns the saturation run and one run per fraction."""
    import threading

    import torch

    import synthetic
    from paper_1502_04025_amd import serving as sv
    kw = dict(prec="f16", nmr=4, ncy=NCY, restart=16, tol=1e-10)
    vols = [sv.TorchVolume(f"{'x'.join(map(str, d))}", d, (4, 4, 4, 4), 0.3, 14 + i, 1.0, max_slots, kw,
                           elastic=True)
            for i, d in enumerate(synthetic.SERVING_VOLUMES)]
    plans = [v.plan() for v in vols]
    # 16 GB of the budget stay free for kernel scratch, graphs and the caching allocator
    budget = sv.plan_budget(plans, int(budget_gb * 1e9), max_slots=max_slots, reserve_bytes=16 * 10 ** 9)

    # one admission state per volume for the whole run: the memory of kept slots stays
    # charged to the budget from one phase to the next
    adms = [sv.Admission(p.capacity, budget, p.per_rhs_bytes, p.kappa_bytes, p.warm_bytes) for p in plans]

    def serve(reqs, realtime):
        workers = [sv.VolumeWorker(v.name, v.batch, v, a, None, None) for v, a in zip(vols, adms)]
        srv = sv.Server(workers, on_result=lambda req: None)  # the client takes each answer and goes
        budget.peak = budget.used
        # device memory actually free and held by torch's caching allocator, sampled
        # while the phase runs (the budget covers the library's slots and fields)
        mem = dict(free_min=float("inf"), torch_max=0.0)
        stop = threading.Event()

        def sample():
            while not stop.wait(0.05):
                mem["free_min"] = min(mem["free_min"], torch.cuda.mem_get_info()[0])
                mem["torch_max"] = max(mem["torch_max"], torch.cuda.memory_reserved())

        sampler = threading.Thread(target=sample, daemon=True)
        sampler.start()
        t0 = time.perf_counter()
        done = srv.run(reqs, realtime=realtime,
                       progress=lambda n, tot: print(f"# serving: {n}/{tot} requests done", file=sys.stderr, flush=True))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stop.set()
        sampler.join()
        out = sv.summarize(done, wall)
        torch.cuda.empty_cache()
        out["steps"] = [w.steps for w in workers]
        out["trims"] = [w.trims for w in workers]
        out["worker_busy_s"] = [{k: round(v, 3) for k, v in w.busy_s.items()} for w in workers]
        out["budget_peak_gb"] = round(budget.peak / 1e9, 2)
        out["device_free_min_gb"] = round(mem["free_min"] / 1e9, 2)
        out["torch_reserved_max_gb"] = round(mem["torch_max"] / 1e9, 2)
        out["converged"] = all(all(st["converged"] for st in r.stats) for r in done if r.error is None)
        return out

    def stream_of(n, rate, seed):
        rs = synthetic.serving_requests(n, rate=rate, seed=seed, volumes=synthetic.SERVING_VOLUMES)
        return [sv.Request(r["id"], r["t_arrival"] if rate < 1e8 else 0.0, r["vol"], r["kappa"], r["nrhs"],
                           r["seed"]) for r in rs]

    def note(phase, r):
        print(f"# serving {phase}: {r['rhs_solves']} RHS in {r['requests']} requests, {r['solves_per_s']:.2f} RHS/s, "
              f"p50 {r['p50_ms']:.0f} ms, p99 {r['p99_ms']:.0f} ms", file=sys.stderr, flush=True)
        return r

    note("warm-up", serve(stream_of(warm, 1e9, 30), False))  # graphs, clover inverses, slot memory
    sat = note("saturation", serve(stream_of(n_requests, 1e9, 31), False))
    runs = {}
    for frac in fracs:
        rate = frac * sat["requests_per_s"]
        runs[str(frac)] = dict(rate_req_s=round(rate, 4), **note(f"{frac} x saturation",
                                                                   serve(stream_of(n_requests, rate, 32), True)))
    for v in vols:
        v.close()
    return dict(admission="one shared HBM budget, footprint per request (elastic batches)",
                hbm_budget_gb=budget_gb, fixed_gb=round(budget.fixed / 1e9, 2),
                slots_per_volume=[p.capacity for p in plans],
                slot_gb=[round(p.per_rhs_bytes / 1e9, 3) for p in plans], warmup_requests=warm,
                requests_per_phase=n_requests, saturation=sat, poisson=runs)


def run_serving(args):
    import torch
    torch.cuda.init()
    res = serving_measure(args.requests, (0.5, 0.8, 0.95), args.hbm_budget_gb, warm=args.serve_warmup)
    sat = res["saturation"]
    line = {
        "metric": "Dslash HBM GB/s (% peak); SAP-FGMRES solves/s @ rel. residual 1e-10; p50/p99",
        "value": round(sat["solves_per_s"], 4), "unit": "RHS solves/s", "n_gpus": 1,
        "steps": args.requests, "warmup": args.serve_warmup, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16+f64", "data": "synthetic",
        "config": {"workload": "serving stream: Poisson arrivals, volumes 16^3x32 / 24^3x48 / 32^3x64 "
                               "(4^4 domains, links exp(i 0.3 H), c_sw 1), kappa U[0.120,0.126], 1-12 "
                               "Gaussian RHS, FP16 SAP + FP64 FGMRES(16) to 1e-10",
                   "parallelism": "single GPU"},
        **res,
    }
    print(json.dumps(line), flush=True)


def run_sweep(args):
    """Time to solution of the 16^3x32 problem (1 Gaussian RHS, FP32 SAP, FGMRES(16) to
    1e-10) over MR steps per block solve x Schwarz cycles x domain shape: the paper's
    parameter question (4-5 MR steps optimal) on this GPU."""
    import torch

    import synthetic
    from paper_1502_04025_amd import Context
    cfg = dict(synthetic.CONFIGS["c2_16x16x16x32_f32"])
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = Context(0, stream=stream)
    u = synthetic.gauge_field(cfg["dims"], cfg["eps"], cfg["gauge_seed"])
    b = torch.from_numpy(make_source(cfg)).cuda()
    x = torch.empty_like(b)
    grid = []
    for block in [(8, 4, 4, 4), (4, 4, 4, 4)]:
        f = ctx.load_gauge(u, block)
        f.compute_clover(cfg["csw"])
        for nmr in args.sweep_nmr:
            for ncy in args.sweep_ncy:
                def step():
                    return f.solve(cfg["kappa"], b, x=x, nmr=nmr, ncy=ncy, restart=16, tol=1e-10, prec="f32",
                                   max_iter=400, raise_on_noconv=False)
                r = step()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    r = step()
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / args.steps
                st = r.stats[0]
                rec = dict(block=list(block), nmr=nmr, ncy=ncy, ms_per_solve=round(dt * 1e3, 3),
                           solves_per_s=round(1.0 / dt, 2), outer_iters=st["iters"],
                           converged=bool(st["converged"]), true_relres=st["true_relres"])
                grid.append(rec)
                print("# " + json.dumps(rec), flush=True)
        f.free()
    ok = [g for g in grid if g["converged"]]
    best = min(ok, key=lambda g: g["ms_per_solve"]) if ok else None
    print(json.dumps({"sweep": "16x16x16x32, 1 gaussian RHS, FP32 SAP, FGMRES(16) to 1e-10", "steps": args.steps,
                      "best": best, "grid": grid}), flush=True)

# Two-level multigrid workload: the 16^3 x 32 field of the default workload at kappa 0.145,
# near its critical value; 12 Gaussian right-hand sides solved together, and one alone.
# 16 test vectors per aggregate and chirality, 6 set-up smoothing passes with 3 SAP
# cycles each, coarse solves of 3 restart cycles of GMRES(24), SAP smoother of 4 MR steps
# and 2 cycles in FP32 storage. SAP alone runs with the same 4 x 2, its own optimum at this
# kappa (more cycles per application need more outer steps here: 1236 at 4, no
# convergence at 8). Both chosen by sweeps on this GPU.
MG_RUN = dict(kappa=0.145, nrhs=12, nvec=16, setup_iters=6, setup_ncy=3, coarse_iters=24, coarse_cycles=3, nmr=4,
              ncy=2, restart=16, prec="f32", vec_seed=77)


def run_mg(args):
    import torch

    import synthetic
    from paper_1502_04025_amd import Context, Multigrid
    from paper_1502_04025_amd import perfmodel as pm
    cfg = dict(synthetic.CONFIGS["c2_16x16x16x32_f32"])
    mc = dict(MG_RUN)
    cfg["kappa"] = mc["kappa"]
    cfg["nrhs"] = mc["nrhs"]
    cfg["source"] = "gaussian"
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = Context(0, stream=stream)
    u, field = make_field(ctx, cfg)
    b = torch.from_numpy(make_source(cfg)).cuda()
    x = torch.empty_like(b)
    nrhs = b.shape[0]
    vecs = synthetic.gaussian_source(cfg["dims"], mc["nvec"], mc["vec_seed"])
    kw = dict(nmr=mc["nmr"], ncy=mc["ncy"], restart=mc["restart"], tol=1e-10, prec=mc["prec"], max_iter=5000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mg = Multigrid(field, mc["kappa"], vecs, setup_iters=mc["setup_iters"], coarse_iters=mc["coarse_iters"],
                   coarse_cycles=mc["coarse_cycles"], nmr=mc["nmr"], ncy=mc["setup_ncy"], prec=mc["prec"])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0

    def timed(step, steps):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = None
        for _ in range(steps):
            r = step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, r

    t_mg, r_mg = timed(lambda: mg.solve(b, x=x, **kw), args.steps)
    x_mg = x[0].cpu().numpy()
    t_sap, r_sap = timed(lambda: field.solve(mc["kappa"], b, x=x, **kw), args.steps)
    b1, x1 = b[:1].clone(), x[:1].clone()
    mg1 = Multigrid(field, mc["kappa"], vecs, setup_iters=mc["setup_iters"], coarse_iters=mc["coarse_iters"],
                    coarse_cycles=mc["coarse_cycles"], nmr=mc["nmr"], ncy=mc["setup_ncy"], prec=mc["prec"],
                    coarse_form=1)  # one launch per coarse Arnoldi step: the form for a single system
    t_mg1, r_mg1 = timed(lambda: mg1.solve(b1, x=x1, **kw), args.steps)
    mg1.close()
    t_sap1, r_sap1 = timed(lambda: field.solve(mc["kappa"], b1, x=x1, **kw), args.steps)
    # per-family device time of one multi-RHS solve launched without graphs
    ctx.profile(True)
    mg.solve(b, x=x, flags=4, **kw)
    fam = ctx.profile(False)
    from oracle import wilson
    t_or = wilson.clover_term(u, cfg["csw"])
    b0 = b[0].cpu().numpy()
    oracle_relres = float(np.linalg.norm(b0 - wilson.apply_M(u, t_or, mc["kappa"], x_mg)) / np.linalg.norm(b0))
    stats = r_mg.stats
    conv = all(s["converged"] for s in stats)
    napp = fam["mg_coarse"]["launches"]
    t_coarse = fam["mg_coarse"]["seconds"] / max(napp, 1)
    nagg = int(np.prod(cfg["dims"])) // int(np.prod(cfg["block"]))
    cbytes = mc["coarse_cycles"] * pm.mg_coarse_bytes(nagg, 2 * mc["nvec"], mc["coarse_iters"], nrhs)
    line = {
        "metric": "two-level multigrid (SAP smoother) FGMRES RHS solves/s @ rel. residual 1e-10",
        "value": round(nrhs / t_mg, 4),
        "unit": "RHS solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_mg, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"mg_16x16x16x32: {'x'.join(map(str, cfg['dims']))} lattice, "
                               f"{'x'.join(map(str, cfg['block']))} aggregates = Schwarz domains, kappa {mc['kappa']}, "
                               f"c_sw {cfg['csw']}, links exp(i {cfg['eps']} H), {nrhs} gaussian RHS, {mc['nvec']} test "
                               f"vectors, {mc['setup_iters']} set-up smoothing passes (ncy {mc['setup_ncy']}), coarse solve {mc['coarse_cycles']}"
                               f" x GMRES({mc['coarse_iters']}), SAP smoother {mc['prec']} (nmr {mc['nmr']}, "
                               f"ncy {mc['ncy']}), FP64 FGMRES({mc['restart']}) to 1e-10",
                   "parallelism": "single GPU"},
        "mg": {"outer_iters": [s["iters"] for s in stats], "converged": conv,
               "true_relres_max": max(s["true_relres"] for s in stats), "oracle_relres_rhs0": oracle_relres,
               "setup_s": round(setup_s, 4)},
        "sap_only": {"outer_iters": [s["iters"] for s in r_sap.stats], "ms_per_step": round(1e3 * t_sap, 3),
                     "rhs_solves_per_s": round(nrhs / t_sap, 4)},
        "one_rhs": {"mg_coarse_form": 1, "mg_ms": round(1e3 * t_mg1, 3), "mg_iters": r_mg1.stats[0]["iters"],
                    "sap_ms": round(1e3 * t_sap1, 3), "sap_iters": r_sap1.stats[0]["iters"]},
        "kernel_time_one_step_no_graph_s": {k: round(v["seconds"], 6) for k, v in fam.items() if v["launches"]},
        "roofline": {"kernel": "coarse GMRES, one launch = all cycles for all systems (two launches per Arnoldi "
                               "step: mg_cres, mg_cinit, mg_capply, mg_cgs, mg_cfinal, mg_caccum kernels)",
                     "bound": "hbm",
                     "achieved": round(cbytes / t_coarse / 1e9, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(cbytes / t_coarse / 8e12, 4), "traffic": None,
                     "avg_launch_us": round(t_coarse * 1e6, 2), "launches": napp,
                     "algorithmic_bytes_per_launch": cbytes, "cache_resident": True},
    }
    print(json.dumps(line), flush=True)
    mg.close()
    field.free()
    ctx.close()
    if not conv or oracle_relres > 1e-10:
        sys.exit(1)


def timed_solves(field, kappa, b, x, steps, warmup, profile_families=("sap_half",), **kw):
    """warmup untimed solves, then `steps` timed ones (HIP events on the dominant kernel's
    family only); returns (seconds per solve, per-solve latencies, stats, profile)."""
    import torch
    for _ in range(warmup):
        field.solve(kappa, b, x=x, **kw)
    torch.cuda.synchronize()
    ctx = field.ctx
    ctx.profile(True, families=list(profile_families))
    lat, r = [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        r = field.solve(kappa, b, x=x, **kw)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile(False)
    return elapsed / steps, lat, r.stats, prof


def sub_c2(ctx, steps=10, warmup=2):
    """16^3 x 32, 8x4x4x4 domains, one Gaussian right-hand side: FP32 SAP against the
    all-FP64 path (working set inside the Infinity Cache)."""
    import torch

    import synthetic
    cfg = synthetic.CONFIGS["c2_16x16x16x32_f32"]
    _, f = make_field(ctx, cfg)
    b = torch.from_numpy(make_source(cfg)).cuda()
    x = torch.empty_like(b)
    out = {"workload": "16x16x16x32, 8x4x4x4 domains, kappa 0.125, 1 gaussian RHS, FGMRES(16), nmr 4, ncy 8"}
    for prec in ("f32", "f64"):
        t, lat, st, _ = timed_solves(f, cfg["kappa"], b, x, steps, warmup, nmr=4, ncy=NCY, restart=16, tol=1e-10,
                                     prec=prec)
        out[prec] = {"solves_per_s": round(1.0 / t, 3), "ms_per_solve": round(1e3 * t, 3),
                     "p50_ms": round(1e3 * percentile(lat, 50), 3), "p99_ms": round(1e3 * percentile(lat, 99), 3),
                     "outer_iters": st[0]["iters"], "converged": bool(st[0]["converged"])}
    f.free()
    return out


def sub_mixed_vs_fp64(ctx, steps=3, warmup=1):
    """32^3 x 64, 4^4 domains, kappa 0.126: the mixed-precision multi-RHS form (12 point
    sources solved together, FP16 SAP, FP64 FGMRES(16)) against plain FP64 single-RHS
    solves (one Gaussian right-hand side, FP64 SAP), in RHS solves per second."""
    import torch

    import synthetic
    cfg = synthetic.CONFIGS["c3_32x32x32x64_f16"]
    _, f = make_field(ctx, cfg)
    kw = dict(nmr=4, ncy=NCY, restart=16, tol=1e-10)
    b = torch.from_numpy(synthetic.point_sources(cfg["dims"])).cuda()
    x = torch.empty_like(b)
    t12, _, st12, _ = timed_solves(f, cfg["kappa"], b, x, steps, warmup, prec="f16", **kw)
    del b, x
    b1 = torch.from_numpy(synthetic.gaussian_source(cfg["dims"], 1, cfg["source_seed"])).cuda()
    x1 = torch.empty_like(b1)
    t1, _, st1, _ = timed_solves(f, cfg["kappa"], b1, x1, steps, warmup, prec="f64", **kw)
    f.free()
    mixed, plain = 12 / t12, 1 / t1
    return {"workload": "32x32x32x64, 4x4x4x4 domains, kappa 0.126, c_sw 1, links exp(i 0.25 H)",
            "mixed_12rhs_f16": {"rhs_solves_per_s": round(mixed, 3), "s_per_step": round(t12, 4),
                                "outer_iters": [s_["iters"] for s_ in st12],
                                "converged": all(s_["converged"] for s_ in st12)},
            "plain_f64_1rhs": {"rhs_solves_per_s": round(plain, 3), "s_per_step": round(t1, 4),
                               "outer_iters": st1[0]["iters"], "converged": bool(st1[0]["converged"])},
            "speedup": round(mixed / plain, 3)}


EXTRAS = ("dslash", "copy_GB_s", "c2_16x16x16x32", "mixed_vs_fp64_32x32x32x64", "serving", "mg_near_critical")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS) + ["serve", "mg"])
    ap.add_argument("--requests", type=int, default=500, help="serve: requests per arrival rate")
    ap.add_argument("--serve-warmup", type=int, default=50, help="serve: warm-up requests")
    ap.add_argument("--hbm-budget-gb", type=float, default=220.0, help="serve: HBM budget for admission")
    ap.add_argument("--nmr", type=int, default=4, help="MR iterations per block solve")
    ap.add_argument("--ncy", type=int, default=None,
                    help="Schwarz cycles per preconditioner application (default: the workload's)")
    ap.add_argument("--restart", type=int, default=None, help="FGMRES restart length (default: the workload's)")
    ap.add_argument("--deflate", type=int, default=0, help="deflated restarts: harmonic Ritz vectors kept")
    ap.add_argument("--sweep", action="store_true", help="time-to-solution sweep over nmr x ncy x domain shape")
    ap.add_argument("--sweep-nmr", type=int, nargs="+", default=[2, 3, 4, 5, 6, 8])
    ap.add_argument("--sweep-ncy", type=int, nargs="+", default=[2, 3, 4, 5, 6, 8, 12, 16])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the sub-benchmarks")
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma-separated sub-benchmarks to run (default: all of " + ", ".join(EXTRAS) + ")")
    ap.add_argument("--copy-probe", action="store_true",
                    help="with --no-extras: still run the 2 GiB copy kernel (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    unknown = set(args.extras.split(",")) - set(EXTRAS) - {""}
    if unknown:
        ap.error(f"unknown extras: {sorted(unknown)}")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        return run_sweep(args)
    if args.workload == "serve":
        return run_serving(args)
    if args.workload == "mg":
        return run_mg(args)

    import synthetic
    name, prec, over = WORKLOADS[args.workload]
    cfg = dict(synthetic.CONFIGS[name])
    cfg.update(over)
    nmr, tol = args.nmr, 1e-10
    restart = args.restart if args.restart is not None else cfg.get("restart", 16)
    deflate = args.deflate
    ncy = args.ncy if args.ncy is not None else cfg.get("ncy", 5)
    # inputs first: worker processes draw them before this process touches the GPU
    t0 = time.perf_counter()
    u = synthetic.gauge_field(cfg["dims"], cfg["eps"], cfg["gauge_seed"])
    b = make_source(cfg)
    print(f"# inputs {'x'.join(map(str, cfg['dims']))}: {time.perf_counter() - t0:.1f} s", flush=True)

    import torch

    from paper_1502_04025_amd import Context
    torch.cuda.init()
    stream = torch.cuda.Stream()  # a real stream: the SAP sweep replays from HIP graphs
    torch.cuda.set_stream(stream)
    ctx = Context(0, stream=stream)
    _, field = make_field(ctx, cfg, u)
    del u
    if cfg.get("host_io"):
        x = np.empty_like(b)
    else:
        b = torch.from_numpy(b).cuda()
        x = torch.empty_like(b)
    nrhs = b.shape[0]
    cfg["nrhs_active"] = nrhs
    kw = dict(nmr=nmr, ncy=ncy, restart=restart, deflate=deflate, tol=tol, prec=prec)
    t_step, lat, stats, prof = timed_solves(field, cfg["kappa"], b, x, args.steps, args.warmup, **kw)
    # one more step with every kernel family recorded, for the time breakdown
    ctx.profile(True)
    field.solve(cfg["kappa"], b, x=x, **kw)
    prof_all = ctx.profile(False)
    iters = [s_["iters"] for s_ in stats]
    relres = [s_["true_relres"] for s_ in stats]
    ok = all(s_["converged"] for s_ in stats)
    # above 4M sites the oracle's residual recheck (minutes, ~66 GB of host memory) is the
    # job of tests/test_gpu_c5.py
    oracle_relres = None
    if int(np.prod(cfg["dims"])) <= 4_000_000:
        from oracle import wilson
        uo = synthetic.gauge_field(cfg["dims"], cfg["eps"], cfg["gauge_seed"])
        t_or = wilson.clover_term(uo, cfg["csw"])
        x0 = x[0] if isinstance(x, np.ndarray) else x[0].cpu().numpy()
        b0 = b[0] if isinstance(b, np.ndarray) else b[0].cpu().numpy()
        oracle_relres = float(np.linalg.norm(b0 - wilson.apply_M(uo, t_or, cfg["kappa"], x0)) / np.linalg.norm(b0))
        del t_or, uo
    line = {
        "metric": "Dslash HBM GB/s (% peak); SAP-FGMRES solves/s @ rel. residual 1e-10; p50/p99",
        "value": round(nrhs / t_step, 4),
        "unit": "RHS solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32+f64", "f16": "f16+f64", "f16l": "f16/f32+f64"}.get(prec, "f64"),
        "data": "synthetic",
        "config": {"workload": f"{name}: {'x'.join(map(str, cfg['dims']))} lattice, {'x'.join(map(str, cfg['block']))} "
                               f"domains, kappa {cfg['kappa']}, c_sw {cfg['csw']}, links exp(i {cfg['eps']} H), "
                               f"{nrhs} {cfg['source']} RHS solved together, SAP {prec} storage (nmr {nmr}, ncy {ncy}), "
                               f"FP64 FGMRES({restart}){f' with {deflate} deflated vectors' if deflate else ''} "
                               f"to {tol}, b and x {'in host memory' if cfg.get('host_io') else 'resident in HBM'}",
                   "parallelism": "single GPU"},
        "step_latency_ms": {"p50": round(1e3 * percentile(lat, 50), 3), "p99": round(1e3 * percentile(lat, 99), 3)},
        "solve": {"outer_iters": iters, "true_relres": relres, "oracle_relres_rhs0": oracle_relres,
                  "converged": ok},
        "kernel_time_one_step_s": {k: round(v["seconds"], 6) for k, v in prof_all.items() if v["launches"]},
        "roofline": roofline_sap(prof, cfg, prec, nmr),
    }
    field.free()
    del b, x
    torch.cuda.empty_cache()
    if not args.no_extras:
        wanted = set(args.extras.split(","))

        def extra(key, fn):
            if key not in wanted:
                return
            t0 = time.perf_counter()
            try:
                line[key] = fn()
            except Exception as e:  # report, do not hide the main number
                line[key] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()
            print(f"# {key}: {time.perf_counter() - t0:.1f} s", flush=True)
        extra("dslash", lambda: dslash_bandwidth(ctx))
        extra("copy_GB_s", lambda: copy_bandwidth(ctx))
        for key in ("f16", "f32", "f16_links12", "f32_links12"):  # also as a fraction of the copy bandwidth
            if (isinstance(line.get("dslash"), dict) and isinstance(line["dslash"].get(key), dict)
                    and isinstance(line.get("copy_GB_s"), float)):
                line["dslash"][key]["frac_of_copy"] = round(line["dslash"][key]["GB_s"] / line["copy_GB_s"], 4)
        extra("c2_16x16x16x32", lambda: sub_c2(ctx))
        extra("mixed_vs_fp64_32x32x32x64", lambda: sub_mixed_vs_fp64(ctx))
        extra("serving", lambda: serving_measure(40, (0.8,), 200.0, warm=6))
        extra("mg_near_critical", lambda: mg_extra(ctx))
    if args.no_extras and args.copy_probe:
        line["copy_GB_s"] = copy_bandwidth(ctx)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        line["cpu_baseline"] = cpu_baseline(cfg, int(np.mean(iters)), int(np.mean([s_["restarts"] for s_ in stats])),
                                            nmr, ncy, nrhs)
        print(f"# cpu_baseline: {time.perf_counter() - t0:.1f} s", flush=True)
    print(json.dumps(line), flush=True)
    ctx.close()
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
