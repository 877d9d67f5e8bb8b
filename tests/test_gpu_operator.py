"""GPU parity of the operators (full M, block M_B, clover build) against the oracle.

Tolerances (relative 2-norm error of the output against the oracle's FP64 result on
the same seeded inputs, storage quantisation included): FP64 1e-12, FP32 1e-6, FP16
5e-3.
"""
import numpy as np
import pytest

import synthetic
from oracle import wilson

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "f16": 5e-3}

# lattice, block: several blocks per direction, lattices whose site count is not a
# multiple of the operator's 2048-site launch tile (ragged tail), and all block shapes
CASES = [
    ((4, 4, 4, 4), (2, 2, 2, 2)),
    ((4, 4, 8, 12), (2, 2, 2, 2)),
    ((8, 8, 8, 8), (4, 4, 4, 4)),
    ((8, 8, 16, 8), (4, 4, 4, 4)),
    ((16, 8, 8, 8), (8, 4, 4, 4)),
]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_1502_04025_amd import Context
    c = Context(0)
    yield c
    c.close()


_cache = {}


def setup_case(ctx, dims, block, csw=1.0, eps=0.3, seed=5):
    key = (dims, block, csw, eps, seed)
    if key not in _cache:
        u = synthetic.gauge_field(dims, eps, seed)
        t = wilson.clover_term(u, csw)
        f = ctx.load_gauge(u, block)
        f.compute_clover(csw)
        _cache[key] = (u, t, f)
    return _cache[key]


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_full_operator(ctx, dims, block, prec):
    print(f"full D {dims} {block} {prec}", flush=True)
    u, t, f = setup_case(ctx, dims, block)
    psi = synthetic.gaussian_source(dims, 2, 7)
    out = f.apply_D(0.124, psi, prec=prec)
    for r in range(2):
        ref = wilson.apply_M(u, t, 0.124, psi[r])
        assert relerr(out[r], ref) <= TOL[prec]


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_block_operator(ctx, dims, block, prec):
    print(f"block D {dims} {block} {prec}", flush=True)
    u, t, f = setup_case(ctx, dims, block)
    psi = synthetic.gaussian_source(dims, 1, 8)
    out = f.apply_block_D(0.126, psi, prec=prec)
    ref = wilson.apply_M(u, t, 0.126, psi[0], block=block)
    assert relerr(out[0], ref) <= TOL[prec]


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_block_operator_two_row_links(ctx, dims, block, prec):
    """Links read as their first two rows, the third rebuilt as the conjugate cross
    product: same tolerance against the oracle's M_B as the 18-real links (the field's
    links are special unitary to rounding)."""
    print(f"block D two-row links {dims} {block} {prec}", flush=True)
    u, t, f = setup_case(ctx, dims, block)
    psi = synthetic.gaussian_source(dims, 2, 9)
    out = f.apply_block_D(0.126, psi, prec=prec, links12=True)
    for r in range(2):
        ref = wilson.apply_M(u, t, 0.126, psi[r], block=block)
        assert relerr(out[r], ref) <= TOL[prec]


def test_two_row_links_reject_fp64(ctx):
    from paper_1502_04025_amd import EINVAL, SapddError
    u, t, f = setup_case(ctx, (4, 4, 4, 4), (2, 2, 2, 2))
    with pytest.raises(SapddError) as e:
        f.apply_block_D(0.126, synthetic.gaussian_source((4, 4, 4, 4), 1, 9), prec="f64", links12=True)
    assert e.value.code == EINVAL


def test_loaded_clover_equals_device_built(ctx):
    dims, block = (4, 4, 8, 4), (2, 2, 2, 2)
    u = synthetic.gauge_field(dims, 0.3, 9)
    t = wilson.clover_term(u, 1.7)
    f1 = ctx.load_gauge(u, block)
    f1.compute_clover(1.7)
    f2 = ctx.load_gauge(u, block)
    f2.load_clover(np.ascontiguousarray(t))
    psi = synthetic.gaussian_source(dims, 1, 3)
    a = f1.apply_D(0.12, psi)
    b = f2.apply_D(0.12, psi)
    ref = wilson.apply_M(u, t, 0.12, psi[0])
    assert relerr(a[0], ref) <= 1e-12 and relerr(b[0], ref) <= 1e-12
    f1.free()
    f2.free()


def test_device_pointers_and_special_cases(ctx):
    import torch
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    u, t, f = setup_case(ctx, dims, block)
    psi = synthetic.gaussian_source(dims, 3, 11)
    dpsi = torch.from_numpy(psi).cuda()
    dout = f.apply_D(0.125, dpsi)
    host = f.apply_D(0.125, psi)
    assert np.array_equal(dout.cpu().numpy(), host)  # same kernels, same bits
    # kappa = 0: M = 1 exactly
    ident = f.apply_D(0.0, psi)
    assert np.array_equal(ident, psi)
    # point source with FP16 storage: zero sites (scale 0) stay exactly zero
    pt = synthetic.point_sources(dims)[:2].copy()
    out = f.apply_D(0.125, pt, prec="f16")
    ref = wilson.apply_M(u, t, 0.125, pt[1])
    assert relerr(out[1], ref) <= TOL["f16"]
    far = (4, 4, 4, 4)  # not a neighbour of the origin
    assert np.all(out[1][far[3], far[2], far[1], far[0]] == 0)


def test_operator_deterministic(ctx):
    dims, block = (8, 8, 16, 8), (4, 4, 4, 4)
    u, t, f = setup_case(ctx, dims, block)
    psi = synthetic.gaussian_source(dims, 1, 12)
    a = f.apply_D(0.12, psi, prec="f32")
    b = f.apply_D(0.12, psi, prec="f32")
    assert np.array_equal(a, b)


def test_layout_round_trip_all_precisions(ctx):
    """canonical -> device layout -> canonical through M = 1 (kappa = 0): FP64 exact, FP32
    exactly the float32 rounding of every real, FP16 within 2^-11 of each site's max |value|
    (one scale per site, nearest-even halves)."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    u, t, f = setup_case(ctx, dims, block)
    psi = synthetic.gaussian_source(dims, 2, 13)
    psi[0, 1, 2, 3, 4] *= 1e-30  # a site far below the others: its own scale keeps it
    assert np.array_equal(f.apply_D(0.0, psi, prec="f64"), psi)
    r32 = f.apply_D(0.0, psi, prec="f32")
    want = psi.real.astype(np.float32).astype(np.float64) + 1j * psi.imag.astype(np.float32).astype(np.float64)
    assert np.array_equal(r32, want)
    r16 = f.apply_D(0.0, psi, prec="f16")
    re = np.stack([psi.real, psi.imag], axis=-1).reshape(psi.shape[:5] + (24,))
    err = np.stack([(r16 - psi).real, (r16 - psi).imag], axis=-1).reshape(psi.shape[:5] + (24,))
    scale = np.abs(re).max(axis=-1, keepdims=True)
    assert np.all(np.abs(err) <= 2.0 ** -11 * scale)
    assert np.max(np.abs(err) / scale) > 2.0 ** -14  # the bound is not slack: halves are used
