"""GPU tests of the deflated restarts (flexible GMRES with deflated restarts, Sec. 3.1),
through the C ABI, against the oracle's fgmres_dr.

Deflation recombines the basis, the preconditioned vectors and the Hessenberg matrix at
every full restart; the oracle does the same with a library eigensolver (harmonic Ritz
vectors from eigenvectors, where the library uses sorted Schur vectors of the same
invariant subspace). Both judge convergence on the FP64 true residual.
"""
import numpy as np
import pytest

import synthetic
from oracle import fgmres as ofg
from oracle import sap as osap
from oracle import wilson

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_1502_04025_amd import Context
    c = Context(0)
    yield c
    c.close()


def oracle_relres(u, t, kappa, x, b):
    return np.linalg.norm(b - wilson.apply_M(u, t, kappa, x)) / np.linalg.norm(b)


@pytest.mark.parametrize("nmr,ncy,m,k", [(1, 1, 4, 2), (2, 1, 3, 1), (4, 5, 4, 2)])
def test_deflated_restarts_match_oracle(ctx, nmr, ncy, m, k):
    """The first configuration (4^4, 2^4 blocks, FP64 SAP) with short restarts: same
    iteration count as the oracle (within one) and true residual <= 1e-10."""
    print(f"deflation nmr {nmr} ncy {ncy} m {m} k {k}", flush=True)
    cfg = synthetic.CONFIGS["c1_4x4x4x4_f64"]
    dims, block = cfg["dims"], cfg["block"]
    u = synthetic.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    t = wilson.clover_term(u, cfg["csw"])
    b = synthetic.gaussian_source(dims, 1, cfg["source_seed"])
    f = ctx.load_gauge(u, block)
    f.compute_clover(cfg["csw"])
    res = f.solve(cfg["kappa"], b, nmr=nmr, ncy=ncy, restart=m, deflate=k, tol=1e-10, prec="f64")
    st = res.stats[0]
    assert st["converged"] and st["true_relres"] <= 1e-10
    assert oracle_relres(u, t, cfg["kappa"], res.x[0], b[0]) <= 1e-10
    sysb = osap.BlockSystem(u, t, cfg["kappa"], block)
    _, info = ofg.fgmres_dr(lambda v: wilson.apply_M(u, t, cfg["kappa"], v),
                            lambda v: osap.sap(sysb, v, ncy, nmr), b[0], m=m, k=k, tol=1e-10)
    assert info["converged"]
    assert abs(info["iters"] - st["iters"]) <= 1
    assert st["restarts"] >= 2
    f.free()


def test_deflated_restarts_half_precision_batch(ctx):
    """FP16 SAP with FP64 preconditioned vectors, FGMRES-DR(3, 1), three right-hand sides
    with their own kappa: every one converges (oracle residual <= 1e-10) and is
    bit-identical to its solve alone."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    u = synthetic.gauge_field(dims, 0.3, 5)
    t = wilson.clover_term(u, 1.0)
    b = synthetic.gaussian_source(dims, 3, 41)
    kap = [0.121, 0.125, 0.123]
    f = ctx.load_gauge(u, block)
    f.compute_clover(1.0)
    kw = dict(nmr=2, ncy=2, restart=3, deflate=1, tol=1e-10, prec="f16")
    res = f.solve(kap, b, **kw)
    for r in range(3):
        st = res.stats[r]
        assert st["converged"] and st["restarts"] >= 2
        assert oracle_relres(u, t, kap[r], res.x[r], b[r]) <= 1e-10
        alone = f.solve(kap[r], b[r:r + 1].copy(), **kw)
        assert np.array_equal(alone.x[0], res.x[r])
    f.free()


def test_deflation_parameter_checked(ctx):
    from paper_1502_04025_amd import EINVAL, SapddError
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    u = synthetic.gauge_field(dims, 0.3, 5)
    b = synthetic.gaussian_source(dims, 1, 3)
    f = ctx.load_gauge(u, block)
    f.compute_clover(1.0)
    for k in (-1, 4):
        with pytest.raises(SapddError) as e:
            f.solve(0.12, b, restart=4, deflate=k, prec="f64")
        assert e.value.code == EINVAL
    f.free()


def test_reliable_update_gap_forces_plain_restarts(ctx):
    """The reliable-update gap rule: when a cycle's FP64 true residual exceeds gap times
    the implicit residual the Arnoldi relation carries, the next cycle restarts plainly
    from the true residual and drops the deflated basis. Forcing the rule on every cycle
    (gap 1e-300, any nonzero true residual exceeds it) turns FGMRES-DR(4, 2) into plain
    FGMRES(4): the same iterate bit for bit, one gap restart per cycle after the first
    deflated one. With the default gap (10) the FP64 path never triggers it."""
    cfg = synthetic.CONFIGS["c1_4x4x4x4_f64"]
    dims, block = cfg["dims"], cfg["block"]
    u = synthetic.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    t = wilson.clover_term(u, cfg["csw"])
    b = synthetic.gaussian_source(dims, 1, cfg["source_seed"])
    f = ctx.load_gauge(u, block)
    f.compute_clover(cfg["csw"])
    kw = dict(nmr=2, ncy=1, restart=4, tol=1e-10, prec="f64")
    plain = f.solve(cfg["kappa"], b, deflate=0, **kw)
    forced = f.solve(cfg["kappa"], b, deflate=2, gap=1e-300, **kw)
    normal = f.solve(cfg["kappa"], b, deflate=2, **kw)
    sp, sf, sn = plain.stats[0], forced.stats[0], normal.stats[0]
    assert sp["converged"] and sf["converged"] and sn["converged"]
    assert np.array_equal(plain.x, forced.x)
    assert sf["iters"] == sp["iters"] and sf["restarts"] == sp["restarts"]
    assert sf["gap_restarts"] == sf["restarts"] >= 2
    assert sn["gap_restarts"] == 0 and sp["gap_restarts"] == 0
    assert oracle_relres(u, t, cfg["kappa"], forced.x[0], b[0]) <= 1e-10
    f.free()
