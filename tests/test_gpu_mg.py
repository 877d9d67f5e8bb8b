"""GPU tests of the two-level multigrid with the Schwarz smoother (Sec. 2.6), through the
C ABI, against the oracle's TwoLevel (oracle/mg.py).

The library keeps P and D_c in FP32 and runs the coarse GMRES in FP32 (FP64 sums), so
results agree with the FP64 oracle to the FP32 level: 1e-5 relative on P and D_c, 1e-4 on
the coarse solve and one preconditioner application (a nonlinear map of its input), and
within one outer iteration on full solves, whose true residual the oracle recomputes.
"""
import numpy as np
import pytest

import synthetic
from oracle import fgmres as ofg
from oracle import mg as omg
from oracle import wilson

pytestmark = pytest.mark.gpu

CASES = {  # dims (x, y, z, t), block, nvec
    "2x2x2x2": ((4, 4, 4, 4), (2, 2, 2, 2), 2),
    "4x4x4x4": ((8, 8, 8, 16), (4, 4, 4, 4), 2),
    "8x4x4x4": ((16, 8, 8, 8), (8, 4, 4, 4), 2),
}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_1502_04025_amd import Context
    c = Context(0)
    yield c
    c.close()


def _setup(ctx, dims, block, kappa=0.128, eps=0.3, seed=41, nvec=4):
    u = synthetic.gauge_field(dims, eps, seed)
    t = wilson.clover_term(u, 1.0)
    f = ctx.load_gauge(u, block)
    f.compute_clover(1.0)
    vecs = synthetic.gaussian_source(dims, nvec, seed + 1)
    return u, t, f, vecs


def _fields_from_cols(cols, nvec):
    """The oracle's columns as nvec fields (both chiralities of vector j together)."""
    return np.stack([cols[j] + cols[nvec + j] for j in range(nvec)])


def _dense_from_stencil(st, grid):
    """Expand [Gt,Gz,Gy,Gx,9,K,K] into the dense coarse matrix, summing blocks that
    refer to the same neighbour (block-grid extent 2)."""
    gx, gy, gz, gt = grid
    nagg = gx * gy * gz * gt
    K = st.shape[-1]
    st = st.reshape(nagg, 9, K, K)
    dense = np.zeros((nagg * K, nagg * K), dtype=np.complex128)
    ext = (gx, gy, gz, gt)
    for a in range(nagg):
        g = [a % gx, a // gx % gy, a // (gx * gy) % gz, a // (gx * gy * gz)]
        for d in range(9):
            h = list(g)
            if d:
                mu = (d - 1) // 2
                h[mu] = (h[mu] + (1 if d % 2 else -1)) % ext[mu]
            b = ((h[3] * gz + h[2]) * gy + h[1]) * gx + h[0]
            dense[a * K:(a + 1) * K, b * K:(b + 1) * K] += st[a, d]
    return dense


@pytest.mark.parametrize("name", list(CASES))
def test_prolongator_and_coarse_operator_match_oracle(ctx, name):
    dims, block, nvec = CASES[name]
    print(f"mg P and D_c on {dims} blocks {block} nvec {nvec}", flush=True)
    from paper_1502_04025_amd import Multigrid
    u, t, f, vecs = _setup(ctx, dims, block, nvec=nvec)
    mg = Multigrid(f, 0.128, vecs, setup_iters=0, coarse_iters=4, prec="f64")
    cols = omg.prolongator(list(vecs), block)
    p_ref = _fields_from_cols(cols, nvec)
    p_gpu = mg.prolongator()
    assert np.abs(p_gpu - p_ref).max() <= 1e-6 * np.abs(p_ref).max()
    dc_ref = omg.coarse_dense(u, t, 0.128, cols, block)
    grid = tuple(dims[mu] // block[mu] for mu in range(4))
    dc_gpu = _dense_from_stencil(mg.coarse_operator(), grid)
    assert np.abs(dc_gpu - dc_ref).max() <= 1e-5 * np.abs(dc_ref).max()
    mg.close()
    f.free()


@pytest.fixture(scope="module")
def small(ctx):
    """8^4 lattice, 4^4 aggregates, 4 test vectors smoothed twice by FP64 SAP."""
    from paper_1502_04025_amd import Multigrid
    dims, block, kappa = (8, 8, 8, 8), (4, 4, 4, 4), 0.128
    u, t, f, vecs = _setup(ctx, dims, block, kappa=kappa, seed=43)
    mg = Multigrid(f, kappa, vecs, setup_iters=2, coarse_iters=8, nmr=4, ncy=2, prec="f64")
    tl = omg.TwoLevel(u, t, kappa, block, list(vecs), ncy=2, nmr=4, setup_iters=2, coarse_iters=8)
    yield dict(dims=dims, block=block, kappa=kappa, u=u, t=t, f=f, mg=mg, tl=tl, vecs=vecs)
    mg.close()
    f.free()


def test_setup_smoothing_matches_oracle(small):
    print("mg set-up smoothing", flush=True)
    p_ref = _fields_from_cols(small["tl"].cols, 4)
    p_gpu = small["mg"].prolongator()
    assert np.abs(p_gpu - p_ref).max() <= 1e-5 * np.abs(p_ref).max()


def test_coarse_gmres_matches_oracle(small):
    print("mg coarse GMRES", flush=True)
    tl = small["tl"]
    rng = np.random.default_rng(3)
    shape = (2, 2, 2, 2, 8)
    rhs = np.stack([rng.standard_normal(shape) + 1j * rng.standard_normal(shape) for _ in range(2)])
    got = small["mg"].coarse_solve(rhs)
    for i in range(2):
        ref = omg.gmres_fixed(tl.coarse_apply, rhs[i], 8)
        assert np.linalg.norm(got[i] - ref) <= 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("form", [0, 1])
def test_coarse_gmres_20_steps_matches_oracle(small, form):
    """GMRES(20) on the coarse system in both forms of the Arnoldi step; in the one-launch
    form the steps run with every bound on the basis vectors a step loads (8, 16, 24),
    and the cycle's tail in the last."""
    from paper_1502_04025_amd import Multigrid
    print(f"mg coarse GMRES(20), form {form}", flush=True)
    mg = Multigrid(small["f"], small["kappa"], small["vecs"], setup_iters=2, coarse_iters=20, nmr=4, ncy=2,
                   prec="f64", coarse_form=form)
    try:
        rng = np.random.default_rng(5)
        shape = (2, 2, 2, 2, 8)
        rhs = np.stack([rng.standard_normal(shape) + 1j * rng.standard_normal(shape) for _ in range(2)])
        got = mg.coarse_solve(rhs)
        for i in range(2):
            ref = omg.gmres_fixed(small["tl"].coarse_apply, rhs[i], 20)
            err = np.linalg.norm(got[i] - ref) / np.linalg.norm(ref)
            print(f"  rhs {i}: rel err {err:.2e}", flush=True)
            assert err <= 1e-4
    finally:
        mg.close()


def test_restarted_coarse_solve_and_application_match_oracle(small):
    """Three restart cycles of GMRES(6) on the coarse system, alone and inside one
    preconditioner application."""
    print("mg restarted coarse GMRES", flush=True)
    from paper_1502_04025_amd import Multigrid
    f, kappa = small["f"], small["kappa"]
    vecs = synthetic.gaussian_source(small["dims"], 4, 44)
    mg = Multigrid(f, kappa, vecs, setup_iters=2, coarse_iters=6, coarse_cycles=3, nmr=4, ncy=2, prec="f64")
    tl = omg.TwoLevel(small["u"], small["t"], kappa, small["block"], list(vecs), ncy=2, nmr=4, setup_iters=2,
                      coarse_iters=6, coarse_cycles=3)
    rng = np.random.default_rng(9)
    shape = (2, 2, 2, 2, 8)
    rhs = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))[None]
    got = mg.coarse_solve(rhs)[0]
    ref = tl.coarse_solve(rhs[0])
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
    # the restarts reach further than one cycle of the same length
    one = omg.gmres_fixed(tl.coarse_apply, rhs[0], 6)
    assert np.linalg.norm(rhs[0] - tl.coarse_apply(ref)) < np.linalg.norm(rhs[0] - tl.coarse_apply(one))
    r = synthetic.gaussian_source(small["dims"], 1, 48)
    got = mg.precond(r)[0]
    ref = tl.precond(r[0])
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
    mg.close()


def test_preconditioner_application_matches_oracle(small):
    print("mg one application", flush=True)
    r = synthetic.gaussian_source(small["dims"], 2, 47)
    got = small["mg"].precond(r)
    for i in range(2):
        ref = small["tl"].precond(r[i])
        assert np.linalg.norm(got[i] - ref) <= 1e-4 * np.linalg.norm(ref)


def test_solve_matches_oracle_iterations(small):
    print("mg solve 8^4", flush=True)
    b = synthetic.gaussian_source(small["dims"], 1, 53)
    res = small["mg"].solve(b, nmr=4, ncy=2, restart=8, tol=1e-10, prec="f64")
    st = res.stats[0]
    tl = small["tl"]
    assert st["converged"]
    rel = np.linalg.norm(b[0] - tl.apply_m(res.x[0])) / np.linalg.norm(b[0])
    assert rel <= 1e-10
    _, info = ofg.fgmres(tl.apply_m, tl.precond, b[0], m=8, tol=1e-10)
    assert info["converged"] and abs(info["iters"] - st["iters"]) <= 1


@pytest.mark.parametrize("form", [0, 1])
def test_batch_results_do_not_depend_on_the_batch(small, form):
    """Two right-hand sides solved together give the same bits as each alone, with the
    FP32 smoother and graphs, in both forms of the coarse Arnoldi step."""
    print(f"mg batch independence, form {form}", flush=True)
    from paper_1502_04025_amd import Batch, Multigrid
    b = synthetic.gaussian_source(small["dims"], 2, 59)
    f = small["f"]
    mg = small["mg"] if form == 0 else Multigrid(f, small["kappa"], small["vecs"], setup_iters=2, coarse_iters=8,
                                                 nmr=4, ncy=2, prec="f64", coarse_form=1)
    alone = []
    for i in range(2):
        res = mg.solve(b[i:i + 1], nmr=4, ncy=2, restart=8, tol=1e-10, prec="f32")
        alone.append(res.x[0].copy())
    batch = Batch(f, 2, nmr=4, ncy=2, restart=8, tol=1e-10, prec="f32")
    batch.set_mg(mg)
    slots = [batch.add(small["kappa"], b[i]) for i in range(2)]
    while batch.step():
        pass
    for i, s in enumerate(slots):
        x = np.empty_like(b[i])
        st = batch.take(s, x)
        assert st["converged"]
        np.testing.assert_array_equal(x, alone[i])
    batch.close()
    if form == 1:
        mg.close()


def test_graph_replays_equal_direct_launches(small):
    """The multigrid cycle inside the FGMRES batch replays from HIP graphs (one per slot
    count and Arnoldi step, replayed every cycle); two graph solves in a row and a solve
    without graphs give the same bits."""
    print("mg graphs vs direct", flush=True)
    from paper_1502_04025_amd import NO_GRAPH
    b = synthetic.gaussian_source(small["dims"], 2, 61)
    kw = dict(nmr=4, ncy=2, restart=4, tol=1e-10, prec="f32")
    mg = small["mg"]
    g1 = mg.solve(b, **kw).x.copy()
    g2 = mg.solve(b, **kw).x.copy()
    d = mg.solve(b, flags=NO_GRAPH, **kw)
    assert all(st["converged"] for st in d.stats)
    np.testing.assert_array_equal(g1, g2)
    np.testing.assert_array_equal(g1, d.x)


def test_errors_are_reported(small):
    from paper_1502_04025_amd import Batch, Multigrid, SapddError, EINVAL
    f = small["f"]
    vecs = synthetic.gaussian_source(small["dims"], 3, 61)
    with pytest.raises(SapddError) as e:
        Multigrid(f, 0.128, vecs)  # odd nvec
    assert e.value.code == EINVAL
    with pytest.raises(SapddError):
        Multigrid(f, 0.128, vecs[:2], coarse_iters=25)
    with pytest.raises(SapddError) as e:
        Multigrid(f, 0.128, vecs[:2], coarse_form=2)  # no such form
    assert e.value.code == EINVAL
    batch = Batch(f, 1, nmr=2, ncy=1, restart=4)
    batch.set_mg(small["mg"])
    with pytest.raises(SapddError) as e:
        batch.add(0.12, vecs[0])  # not the multigrid's kappa
    assert e.value.code == EINVAL
    batch.close()


def test_freeing_objects_closes_what_depends_on_them(ctx):
    """Closing a multigrid closes the batches that precondition with it; freeing a field
    closes its batches and multigrid objects (the library needs them gone first)."""
    print("mg close order", flush=True)
    from paper_1502_04025_amd import Batch, Multigrid
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    u, t, f, vecs = _setup(ctx, dims, block, seed=97, nvec=2)
    mg = Multigrid(f, 0.128, vecs, coarse_iters=2, nmr=2, ncy=1, prec="f32")
    batch = Batch(f, 1, nmr=2, ncy=1, restart=4)
    batch.set_mg(mg)
    mg.close()
    assert batch.h is None and mg.h is None
    mg2 = Multigrid(f, 0.128, vecs, coarse_iters=2, nmr=2, ncy=1, prec="f32")
    batch2 = Batch(f, 1, nmr=2, ncy=1, restart=4)
    batch3 = Batch(f, 1, nmr=2, ncy=1, restart=4)
    batch3.set_mg(mg2)
    f.free()
    assert batch2.h is None and batch3.h is None and mg2.h is None and f.h is None


def test_full_size_16x16x16x32_sampled_columns_and_solve(ctx):
    """16^3 x 32 with 8x4^3 aggregates and 8 test vectors: sampled block columns of D_c
    against the oracle's P^H M P e, gamma_5-Hermiticity of the whole stencil, and an FP32
    multigrid solve whose true residual the oracle recomputes."""
    print("mg 16^3x32", flush=True)
    from paper_1502_04025_amd import Multigrid
    dims, block, kappa, nvec = (16, 16, 16, 32), (8, 4, 4, 4), 0.128, 8
    u, t, f, vecs = _setup(ctx, dims, block, kappa=kappa, seed=67, nvec=nvec)
    mg = Multigrid(f, kappa, vecs, setup_iters=0, coarse_iters=12, prec="f32")
    st = mg.coarse_operator()  # [Gt, Gz, Gy, Gx, 9, K, K]
    grid = (2, 4, 4, 8)
    cols = omg.prolongator(list(vecs), block)
    K = 2 * nvec
    gshape = (8, 4, 4, 2)
    rng = np.random.default_rng(7)
    for _ in range(3):  # D_c applied to unit vectors: one block column and its neighbours
        a = tuple(int(rng.integers(n)) for n in gshape)  # [gt, gz, gy, gx]
        k = int(rng.integers(K))
        e = np.zeros(gshape + (K,), dtype=np.complex128)
        e[a + (k,)] = 1.0
        ref = omg.restrict(cols, wilson.apply_M(u, t, kappa, omg.prolong(cols, e, block)), block)
        gt, gz, gy, gx = a
        g = [gx, gy, gz, gt]
        got = np.zeros_like(ref)
        for d in range(9):  # aggregate a's column k reaches a and its neighbours h with D_c(h, a)
            h = list(g)
            if d:
                mu = (d - 1) // 2
                h[mu] = (h[mu] - (1 if d % 2 else -1)) % grid[mu]  # a is h's neighbour d
            got[h[3], h[2], h[1], h[0]] += st[h[3], h[2], h[1], h[0], d, :, k]
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    # gamma_5-Hermiticity: sigma D_c(a, a+mu) sigma = D_c(a+mu, a)^H
    sig = np.concatenate([np.ones(nvec), -np.ones(nvec)])
    flat = st.reshape(-1, 9, K, K)
    for a in range(0, flat.shape[0], 37):
        ga = [a % 2, a // 2 % 4, a // 8 % 4, a // 32]
        for mu in range(1, 4):  # directions with block-grid extent > 2
            h = list(ga)
            h[mu] = (h[mu] + 1) % grid[mu]
            b = ((h[3] * 4 + h[2]) * 4 + h[1]) * 2 + h[0]
            lhs = sig[:, None] * flat[a, 1 + 2 * mu] * sig[None, :]
            assert np.abs(lhs - np.conj(flat[b, 2 + 2 * mu].T)).max() <= 1e-5 * np.abs(flat[a, 0]).max()
    b = synthetic.gaussian_source(dims, 1, 71)
    res = mg.solve(b, nmr=4, ncy=4, restart=16, tol=1e-10, prec="f32")
    assert res.stats[0]["converged"]
    rel = np.linalg.norm(b[0] - wilson.apply_M(u, t, kappa, res.x[0])) / np.linalg.norm(b[0])
    assert rel <= 1e-10
    mg.close()
    f.free()
