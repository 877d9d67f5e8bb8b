"""The allocation-free Schwarz entry point (sapdd_sap_noalloc) against sapdd_sap.

Both run the same kernels on the same inputs, so the outputs must agree bit for bit.
Two calls in a row share the device array the entry point works in: the second, on a
smaller lattice with fewer right-hand sides, must not see anything the first left
behind. Sizes beyond the fixed maximum and host pointers are rejected with EINVAL.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_1502_04025_amd import Context
    c = Context(0)
    yield c
    c.close()


def field(ctx, dims, block, seed):
    f = ctx.load_gauge(synthetic.gauge_field(dims, 0.3, seed), block)
    f.compute_clover(1.0)
    return f


@pytest.mark.parametrize("prec", ["f16", "f32", "f64"])
def test_noalloc_equals_sap_twice_second_smaller(ctx, prec):
    import torch
    print(f"noalloc {prec}", flush=True)
    cases = [((16, 8, 8, 16), (8, 4, 4, 4), [0.125, 0.121, 0.125]), ((8, 8, 8, 8), (4, 4, 4, 4), [0.124])]
    for dims, block, kap in cases:  # the second call is smaller: lattice and right-hand sides
        f = field(ctx, dims, block, 71)
        eta = torch.from_numpy(synthetic.gaussian_source(dims, len(kap), 72)).cuda()
        ref = f.sap(np.array(kap), eta, nmr=4, ncy=2, prec=prec)
        out = torch.full_like(eta, float("nan"))
        f.sap_noalloc(np.array(kap), eta, out, nmr=4, ncy=2, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (dims, prec)
        f.free()


def test_noalloc_rejects_beyond_its_limits(ctx):
    import torch
    from paper_1502_04025_amd import EINVAL, SapddError
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    f = field(ctx, dims, block, 73)
    eta = synthetic.gaussian_source(dims, 1, 74)
    with pytest.raises(SapddError) as e:  # host arrays
        f.sap_noalloc(0.124, eta, np.empty_like(eta))
    assert e.value.code == EINVAL
    de = torch.from_numpy(synthetic.gaussian_source(dims, 17, 75)).cuda()
    with pytest.raises(SapddError) as e:  # more right-hand sides than the limit
        f.sap_noalloc(0.124, de, torch.empty_like(de))
    assert e.value.code == EINVAL
    f.free()
    big = (32, 32, 32, 16)  # 524288 sites: the FP64 workspaces exceed 256 MiB
    f = field(ctx, big, (4, 4, 4, 4), 76)
    db = torch.from_numpy(synthetic.gaussian_source(big, 1, 77)).cuda()
    with pytest.raises(SapddError) as e:
        f.sap_noalloc(0.124, db, torch.empty_like(db), prec="f64")
    assert e.value.code == EINVAL and "maximum" in str(e.value)
    f.free()
