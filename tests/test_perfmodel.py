"""The host-side accounting (bytes, flops, load model) against numbers the paper prints."""
import json
import os

import pytest

from paper_1502_04025_amd import perfmodel as pm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_flop_convention():
    assert pm.HOP_FLOPS + pm.CLOVER_FLOPS + pm.COMBINE_FLOPS == GOLD["wilson_clover_flops_per_site"]["value"]


def test_half_storage_saving_of_an_8x4x4x4_domain():
    """Links + clover in half instead of single precision save 456 - 312 = 144 kB per domain."""
    g = GOLD["working_set_8x4x4x4_kB"]
    single = pm.domain_working_set_bytes((8, 4, 4, 4), "f32", "f32", 0)
    half = pm.domain_working_set_bytes((8, 4, 4, 4), "f16", "f32", 0)
    assert (single - half) / 1024 == g["single"] - g["half_links_clover"]


def test_load_model_examples():
    u = GOLD["load_uniform_64x64x64x128_1024_knc"]
    assert round(pm.load(u["domains_per_knc"], u["cores"]), 2) == u["value"]
    n = GOLD["load_nonuniform_t_split"]
    avg = sum(pm.load(d, n["cores"]) for d in n["domains_per_knc"]) / len(n["domains_per_knc"])
    assert round(avg, 2) == n["value"]
    w = GOLD["load_48x48x48x64_64_knc"]
    nd = 1
    for l, b in zip(w["local_volume"], w["block"]):
        nd *= l // b
    assert round(pm.load(nd, w["cores"]), 2) == w["value"]


@pytest.mark.parametrize("block,f", [((2, 2, 2, 2), 0.5), ((4, 4, 4, 4), 0.75), ((8, 4, 4, 4), 0.78125)])
def test_internal_hop_fraction(block, f):
    assert pm.internal_fraction(block) == f


def test_block_dslash_bytes_per_site():
    # f L + C + 2 S at one right-hand side
    assert pm.block_dslash_bytes((4, 4, 4, 4), "f64") == 0.75 * 576 + 576 + 2 * 192
    assert pm.block_dslash_bytes((8, 4, 4, 4), "f16") == 0.78125 * 148 + 148 + 2 * 52


def test_mg_coarse_bytes_one_step():
    """One coarse step over one aggregate with K = 2: the first vector's norm, the stencil
    (9 blocks of 2 x 2 complex FP32), v_0 for the operator, the new vector written, two
    Gram-Schmidt reads of v_0, the new vector read and written by the correction, each
    vector 2 complex FP32 numbers."""
    nc = 2 * 8
    assert pm.mg_coarse_bytes(1, 2, 1) == nc + 9 * 4 * 8 + nc + nc + 2 * nc + 2 * nc
    # two systems share the stencil and double everything else
    assert pm.mg_coarse_bytes(1, 2, 1, 2) == 2 * nc + 9 * 4 * 8 + 2 * (6 * nc)


def test_two_row_link_bytes():
    """4 directions x 12 reals: FP32 192 bytes; FP16 96 bytes plus the 4-byte site scale.
    On 4^4 blocks the block operator then reads 624 (FP32) and 327 (FP16) bytes per site
    instead of 696 and 363."""
    assert pm.LINK12_BYTES == {"f32": 4 * 12 * 4, "f16": 4 * 12 * 2 + 4}
    assert pm.block_dslash_bytes((4, 4, 4, 4), "f32", links12=True) == 0.75 * 192 + 288 + 192
    assert pm.block_dslash_bytes((4, 4, 4, 4), "f16", links12=True) == 0.75 * 100 + 148 + 104
    assert pm.block_dslash_bytes((4, 4, 4, 4), "f32") == 696
