"""The largest benchmark configuration, 48^3 x 96 with 8x4x4x4 domains (12 Gaussian
right-hand sides, FP16 Schwarz storage, FP64 FGMRES(3) with the true residual checked at
every restart), solved on the GPU and checked by the oracle: the oracle's own FP64
operator recomputes |b - M x| / |b| for the first and the last right-hand side.

The oracle needs about 66 GB of host memory here (links, the 12x12 clover term of every
site and a few spinor fields) and about three minutes on one core: the clover term
takes two of them, each operator application forty seconds.
"""
import resource
import time

import numpy as np
import pytest

import synthetic
from oracle import wilson

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.mark.timeout(900)
def test_c5_solution_residual_by_the_oracle():
    import torch
    from paper_1502_04025_amd import Context
    assert torch.cuda.is_available()
    cfg = synthetic.CONFIGS["c5_48x48x48x96_f16"]
    dims = cfg["dims"]
    t0 = time.perf_counter()
    u = synthetic.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    b = synthetic.gaussian_source(dims, cfg["nrhs"], cfg["source_seed"])
    print(f"c5 inputs {time.perf_counter() - t0:.1f} s", flush=True)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = Context(0, stream=stream)
    f = ctx.load_gauge(u, cfg["block"])
    f.compute_clover(cfg["csw"])
    bd = torch.from_numpy(b).cuda()
    xd = torch.empty_like(bd)
    t0 = time.perf_counter()
    res = f.solve(cfg["kappa"], bd, x=xd, nmr=4, ncy=8, restart=3, tol=1e-10, prec="f16")
    torch.cuda.synchronize()
    print(f"c5 solve {time.perf_counter() - t0:.1f} s, iters {[s['iters'] for s in res.stats]}", flush=True)
    assert all(s["converged"] and s["true_relres"] <= 1e-10 for s in res.stats)
    check = (0, cfg["nrhs"] - 1)
    xs = {r: xd[r].cpu().numpy() for r in check}
    del bd, xd
    f.free()
    ctx.close()
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    t = wilson.clover_term(u, cfg["csw"])
    print(f"oracle clover term {time.perf_counter() - t0:.1f} s", flush=True)
    for r in check:
        t0 = time.perf_counter()
        rel = np.linalg.norm(b[r] - wilson.apply_M(u, t, cfg["kappa"], xs[r])) / np.linalg.norm(b[r])
        print(f"rhs {r}: oracle relres {rel:.3e} (library {res.stats[r]['true_relres']:.3e}), "
              f"{time.perf_counter() - t0:.1f} s", flush=True)
        assert rel <= 1e-10
    print(f"host max RSS {resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 1e6:.1f} GB", flush=True)
