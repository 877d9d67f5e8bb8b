#!/usr/bin/env python
"""Benchmark: SAP-preconditioned FGMRES solves on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c2_f64|c3]

One step = one complete solve of M x = b to a true relative residual of 1e-10 (SAP
preconditioner + FP64 flexible GMRES, every kernel of the hot path), with b and x
resident in HBM. The default workload is the 16^3 x 32 lattice with 8x4x4x4 domains,
FP32 Schwarz/MR storage and FP64 outer solver, one Gaussian right-hand side.

Printed: one JSON line with solves/s (RHS solves per second), p50/p99 solve latency, the
roofline of the dominant kernel (per-kernel HIP-event times measured on the solve's
stream during the timed steps), the block-Dslash bandwidth on the 32^3 x 64 lattice
(FP16 storage, working set far above the 256 MB Infinity Cache), the all-FP64 path on
the same problem, and the CPU oracle timed on a bounded sample of the same solve.
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

WORKLOADS = {
    "c2": ("c2_16x16x16x32_f32", "f32", None),
    "c2_f64": ("c2_16x16x16x32_f32", "f64", None),
    "c3": ("c3_32x32x32x64_f16", "f16", None),
}


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q))


def make_field(ctx, cfg):
    import synthetic
    u = synthetic.gauge_field(cfg["dims"], cfg["eps"], cfg["gauge_seed"])
    f = ctx.load_gauge(u, cfg["block"])
    f.compute_clover(cfg["csw"])
    return u, f


def make_source(cfg):
    import synthetic
    if cfg["source"] == "point":
        return synthetic.point_sources(cfg["dims"])[: cfg["nrhs"]].copy()
    return synthetic.gaussian_source(cfg["dims"], cfg["nrhs"], cfg["source_seed"])


def roofline_sap(prof, cfg, prec, nmr):
    from paper_1502_04025_amd import perfmodel as pm
    k = prof["sap_half"]
    if k["launches"] == 0:
        return None
    V = int(np.prod(cfg["dims"]))
    avg = k["seconds"] / k["launches"]
    units = V / 2 * cfg["nrhs_active"]  # sites of one colour per launch
    flops = pm.sap_half_flops(cfg["block"], nmr) * units
    byts = pm.sap_half_bytes(cfg["block"], prec) * units
    alu_peak = pm.ALU_PEAK_TFLOPS["f64" if prec == "f64" else "f32"]
    t_alu = flops / (alu_peak * 1e12)
    t_hbm = byts / (pm.HBM_PEAK_GBS * 1e9)
    if t_alu >= t_hbm:
        ach = flops / avg / 1e12
        return dict(kernel="sap_half_kernel", bound="alu", achieved=round(ach, 3), peak=alu_peak,
                    unit="TFLOP/s", frac=round(ach / alu_peak, 4), traffic=None,
                    avg_launch_us=round(avg * 1e6, 2), launches=k["launches"],
                    algorithmic_flops_per_launch=flops, algorithmic_bytes_per_launch=byts)
    ach = byts / avg / 1e9
    return dict(kernel="sap_half_kernel", bound="hbm", achieved=round(ach, 1), peak=pm.HBM_PEAK_GBS,
                unit="GB/s", frac=round(ach / pm.HBM_PEAK_GBS, 4), traffic=None,
                avg_launch_us=round(avg * 1e6, 2), launches=k["launches"],
                algorithmic_flops_per_launch=flops, algorithmic_bytes_per_launch=byts)


def dslash_bandwidth(ctx, reps=20):
    """Block Dslash on 32^3 x 64 (4^4 domains), FP16 and FP32 storage, device arrays."""
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
    for prec in ("f16", "f32"):
        f.apply_block_D(cfg["kappa"], psi, prec=prec, out=out)  # warm (builds the low-precision copies)
        ctx.profile(True)
        for _ in range(reps):
            f.apply_block_D(cfg["kappa"], psi, prec=prec, out=out)
        p = ctx.profile(False)["block_dslash"]
        avg = p["seconds"] / p["launches"]
        byts = pm.block_dslash_bytes(cfg["block"], prec) * V
        gbs = byts / avg / 1e9
        res[prec] = dict(GB_s=round(gbs, 1), frac=round(gbs / pm.HBM_PEAK_GBS, 4), avg_launch_us=round(avg * 1e6, 2),
                         algorithmic_bytes_per_launch=byts)
    f.free()
    return dict(kernel="dslash_block_kernel", lattice="32x32x32x64", block=list(cfg["block"]), **res)


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


def cpu_baseline(cfg, iters, restarts):
    """Time the oracle on a bounded sample: one Schwarz half-sweep and one operator
    application at the full lattice, scaled to one solve with the GPU's iteration count."""
    from threadpoolctl import threadpool_limits

    import synthetic
    from oracle import sap as osap
    from oracle import wilson
    with threadpool_limits(1):
        u = synthetic.gauge_field(cfg["dims"], cfg["eps"], cfg["gauge_seed"])
        t = wilson.clover_term(u, cfg["csw"])
        b = synthetic.gaussian_source(cfg["dims"], 1, cfg["source_seed"])[0]
        sysb = osap.BlockSystem(u, t, cfg["kappa"], cfg["block"])
        t0 = time.perf_counter()
        m = wilson.apply_M(u, t, cfg["kappa"], b)
        t_m = time.perf_counter() - t0
        t0 = time.perf_counter()
        for c in (0, 1):  # one half-sweep = block solves of one colour + residual update
            delta, _ = sysb.block_solve(b, c, 4)
            wilson.apply_M(u, t, cfg["kappa"], delta)
        t_half = (time.perf_counter() - t0) / 2
    del m
    ncy = 5
    t_solve = iters * (2 * ncy * t_half + t_m) + (restarts + 1) * t_m
    return dict(value=round(1.0 / t_solve, 6), unit="solves/s", cores=1, kind="oracle",
                sample=f"two Schwarz half-sweeps (even-odd MR block solves, nmr 4, plus the residual "
                       f"update) and one operator application on the full {'x'.join(map(str, cfg['dims']))} "
                       f"lattice, NumPy FP64 on one core ({t_half:.1f} s per half-sweep, {t_m:.2f} s per "
                       f"operator), scaled to {iters} outer iterations x {2 * ncy} half-sweeps")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the Dslash/copy/FP64 side measurements")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synthetic
    from paper_1502_04025_amd import Context
    from paper_1502_04025_amd import perfmodel as pm

    name, prec, _ = WORKLOADS[args.workload]
    cfg = dict(synthetic.CONFIGS[name])
    nmr, ncy, restart, tol = 4, 5, 16, 1e-10
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = Context(0, stream=stream)
    u, field = make_field(ctx, cfg)
    b = torch.from_numpy(make_source(cfg)).cuda()
    x = torch.empty_like(b)
    nrhs = b.shape[0]
    cfg["nrhs_active"] = nrhs

    def step():
        return field.solve(cfg["kappa"], b, x=x, nmr=nmr, ncy=ncy, restart=restart, tol=tol, prec=prec)

    for _ in range(args.warmup):
        r = step()
    torch.cuda.synchronize()
    ctx.profile(True)
    lat = []
    stats = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        r = step()
        lat.append(time.perf_counter() - ts)
        stats = r.stats
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile(False)
    elapsed = t1 - t0
    solves_per_s = args.steps * nrhs / elapsed
    iters = [s["iters"] for s in stats]
    relres = [s["true_relres"] for s in stats]
    ok = all(s["converged"] for s in stats)

    # oracle check of the last solution's residual (first right-hand side)
    from oracle import wilson
    t_or = wilson.clover_term(u, cfg["csw"])
    x0 = x[0].cpu().numpy()
    b0 = b[0].cpu().numpy()
    oracle_relres = float(np.linalg.norm(b0 - wilson.apply_M(u, t_or, cfg["kappa"], x0)) / np.linalg.norm(b0))
    del t_or

    line = {
        "metric": "Dslash HBM GB/s (% peak); SAP-FGMRES solves/s @ rel. residual 1e-10; p50/p99",
        "value": round(solves_per_s, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == "f32" else ("f16+f64" if prec == "f16" else "f64"),
        "data": "synthetic",
        "config": {"workload": f"{name}: {'x'.join(map(str, cfg['dims']))} lattice, {'x'.join(map(str, cfg['block']))} "
                               f"domains, kappa {cfg['kappa']}, c_sw {cfg['csw']}, links exp(i {cfg['eps']} H), "
                               f"{nrhs} {cfg['source']} RHS, SAP {prec} storage (nmr {nmr}, ncy {ncy}), "
                               f"FP64 FGMRES({restart}) to {tol}",
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(1e3 * percentile(lat, 50), 3), "p99": round(1e3 * percentile(lat, 99), 3)},
        "solve": {"outer_iters": iters, "true_relres": relres, "oracle_relres_rhs0": oracle_relres,
                  "converged": ok},
        "kernel_time_s": {k: round(v["seconds"], 6) for k, v in prof.items() if v["launches"]},
        "roofline": roofline_sap(prof, cfg, prec, nmr),
    }
    if not args.no_extras:
        try:
            line["dslash"] = dslash_bandwidth(ctx)
        except Exception as e:  # report, do not hide the main number
            line["dslash"] = {"error": str(e)}
        line["copy_GB_s"] = copy_bandwidth(ctx)
        if prec != "f64":
            t0 = time.perf_counter()
            n64 = 3
            r64 = None
            for _ in range(n64):
                r64 = field.solve(cfg["kappa"], b, x=x, nmr=nmr, ncy=ncy, restart=restart, tol=tol, prec="f64")
            torch.cuda.synchronize()
            t64 = (time.perf_counter() - t0) / n64
            line["fp64_path"] = {"solves_per_s": round(nrhs / t64, 4),
                                 "outer_iters": [s["iters"] for s in r64.stats]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, int(np.mean(iters)), int(np.mean([s["restarts"] for s in stats])))
    print(json.dumps(line), flush=True)
    field.free()
    ctx.close()
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
