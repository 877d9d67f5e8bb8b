"""The largest benchmark configuration, 48^3 x 96 with 8x4x4x4 domains (12 Gaussian
right-hand sides, FP16 Schwarz storage, FP64 FGMRES(3) with the true residual checked at
every restart), solved on the GPU and checked by the oracle: the oracle's own FP64
operator recomputes |b - M x| / |b| for the first and the last right-hand side.

The oracle needs about 66 GB of host memory here (links, the 12x12 clover term of every
site and a few spinor fields) and about three and a half minutes on one core: the clover
term takes two of them, each operator application forty seconds. The check is split
into four tests run in order (solve, clover term, one residual each) so that no single
step stays silent for minutes; they share the arrays through a module-level cache.
"""
import resource
import time

import numpy as np
import pytest

import synthetic
from oracle import wilson

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

CFG = synthetic.CONFIGS["c5_48x48x48x96_f16"]
CHECK = (0, CFG["nrhs"] - 1)
_state = {}


def test_c5_solve_on_the_gpu():
    import torch
    from paper_1502_04025_amd import Context
    assert torch.cuda.is_available()
    dims = CFG["dims"]
    t0 = time.perf_counter()
    u = synthetic.gauge_field(dims, CFG["eps"], CFG["gauge_seed"])
    b = synthetic.gaussian_source(dims, CFG["nrhs"], CFG["source_seed"])
    print(f"c5 inputs {time.perf_counter() - t0:.1f} s", flush=True)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = Context(0, stream=stream)
    f = ctx.load_gauge(u, CFG["block"])
    f.compute_clover(CFG["csw"])
    bd = torch.from_numpy(b).cuda()
    xd = torch.empty_like(bd)
    t0 = time.perf_counter()
    res = f.solve(CFG["kappa"], bd, x=xd, nmr=4, ncy=8, restart=3, tol=1e-10, prec="f16")
    torch.cuda.synchronize()
    print(f"c5 solve {time.perf_counter() - t0:.1f} s, iters {[s['iters'] for s in res.stats]}", flush=True)
    assert all(s["converged"] and s["true_relres"] <= 1e-10 for s in res.stats)
    _state.update(u=u, b={r: b[r] for r in CHECK}, x={r: xd[r].cpu().numpy() for r in CHECK},
                  lib={r: res.stats[r]["true_relres"] for r in CHECK})
    del b, bd, xd
    f.free()
    ctx.close()
    torch.cuda.empty_cache()


def test_c5_oracle_clover_term():
    assert "u" in _state, "the GPU solve did not run"
    t0 = time.perf_counter()
    _state["t"] = wilson.clover_term(_state["u"], CFG["csw"])
    print(f"oracle clover term {time.perf_counter() - t0:.1f} s", flush=True)


@pytest.mark.parametrize("r", CHECK)
def test_c5_residual_by_the_oracle(r):
    assert "t" in _state, "the oracle clover term is missing"
    t0 = time.perf_counter()
    b, x = _state["b"][r], _state["x"][r]
    rel = np.linalg.norm(b - wilson.apply_M(_state["u"], _state["t"], CFG["kappa"], x)) / np.linalg.norm(b)
    print(f"rhs {r}: oracle relres {rel:.3e} (library {_state['lib'][r]:.3e}), {time.perf_counter() - t0:.1f} s, "
          f"host max RSS {resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 1e6:.1f} GB", flush=True)
    assert rel <= 1e-10
    if r == CHECK[-1]:
        _state.clear()
