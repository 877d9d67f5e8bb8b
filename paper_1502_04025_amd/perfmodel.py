"""Algorithmic byte and flop counts of the solver's kernels, and the paper's load model.

These are accounting functions (no arithmetic of the method): the bytes a kernel must
move and the flops it must execute per lattice site, used to turn measured kernel times
into roofline fractions, and the domain-to-core load model of the paper.

Flop convention (Sec. 3.7): one Wilson-clover application costs 1848 flops per site,
read here as 1320 for the hopping term (8 hops of 165 flops), 504 for the clover term
(two Hermitian 6x6 blocks) and 24 for combining them.
"""
from __future__ import annotations

WILSON_CLOVER_FLOPS = 1848
HOP_FLOPS = 1320
CLOVER_FLOPS = 504
COMBINE_FLOPS = 24

# bytes per site: spinor (24 reals), links (4 x 18 reals), clover (72 reals); FP16 adds
# one FP32 scale per site to each field
# "f16l" is the Schwarz mode with FP16 links and clover and FP32 spinors
SPINOR_BYTES = {"f64": 192, "f32": 96, "f16": 52, "f16l": 96}
LINK_BYTES = {"f64": 576, "f32": 288, "f16": 148, "f16l": 148}
CLOVER_BYTES = {"f64": 576, "f32": 288, "f16": 148, "f16l": 148}
PSI_BYTES = {"f64": 192, "f32": 96, "f16": 96, "f16l": 96}  # the preconditioner output is FP32 below FP64

# MI355X published peaks (single GPU)
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz; the library is compiled without
# packed FP32 instructions, so FP32 runs at the FP64 vector rate
ALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 78.6}
# the published FP32 vector peak counts packed (two-wide) FP32 FMAs
ALU_PEAK_PUBLISHED_TFLOPS = {"f64": 78.6, "f32": 157.3}


def internal_fraction(block) -> float:
    """Fraction of the 8 nearest-neighbour hops of a site that stay inside its block."""
    return sum((b - 1) / b for b in block) / 4.0


# links stored as their first two rows (4 x 12 reals, FP16 plus a 4-byte site scale)
LINK12_BYTES = {"f32": 192, "f16": 100}


def block_dslash_bytes(block, prec: str, nrhs: int = 1, links12: bool = False) -> float:
    """Block operator M_B: internal links, clover, one spinor read and one written."""
    f = internal_fraction(block)
    lb = LINK12_BYTES[prec] if links12 else LINK_BYTES[prec]
    return f * lb + CLOVER_BYTES[prec] + 2 * nrhs * SPINOR_BYTES[prec]


def block_dslash_flops(block) -> float:
    f = internal_fraction(block)
    return f * HOP_FLOPS + CLOVER_FLOPS + COMBINE_FLOPS


def full_dslash_bytes(prec: str, nrhs: int = 1, in_prec: str | None = None) -> float:
    """Full operator: all links and clover once, one input and one output spinor per RHS."""
    sin = SPINOR_BYTES[in_prec or prec]
    return LINK_BYTES[prec] + CLOVER_BYTES[prec] + nrhs * (sin + SPINOR_BYTES[prec])


def sap_half_bytes(block, prec: str, nrhs: int = 1, nkappa: int = 1) -> float:
    """One Schwarz half-sweep, per site of the swept colour, in the steady state (the
    stored-residual mode), for nrhs right-hand sides solved together: own links plus the
    neighbour-owned face links once, the clover X once per distinct kappa, and per
    right-hand side the stored even-site residual (read and written), the neighbours'
    corrections across the faces, psi read-modify-write and the new correction written."""
    f = internal_fraction(block)
    s = SPINOR_BYTES[prec]
    per_rhs = s / 2 + 8 * (1 - f) * s + 2 * PSI_BYTES[prec] + s + s / 2
    return (1 + (1 - f)) * LINK_BYTES[prec] + nkappa * CLOVER_BYTES[prec] + nrhs * per_rhs


def sap_half_flops(block, nmr: int) -> float:
    """Flops per site of one block solve: nmr MR steps and one more application of the
    in-block operator (split between the right-hand side and the odd-site
    reconstruction), the MR vector algebra (360 flops per even site and step) and the
    gather of the face hops."""
    f = internal_fraction(block)
    return (nmr + 1) * (f * HOP_FLOPS + CLOVER_FLOPS) + 180 * nmr + (1 - f) * HOP_FLOPS


def cgs2_bytes(j: int) -> float:
    """Fused CGS2 at Arnoldi step j (j + 1 basis vectors), FP64 per site: three passes
    read the basis, two of them write w."""
    return 192 * (3 * (j + 1) + 3 + 2)


def domain_working_set_bytes(block, link_clover_prec: str, spinor_prec: str, nspinors: float) -> float:
    """Links + clover + nspinors spinors of one domain (the cache budget of Sec. 3.3)."""
    vb = 1
    for b in block:
        vb *= b
    lc = {"f64": 8, "f32": 4, "f16": 2}[link_clover_prec] * 144
    sp = {"f64": 8, "f32": 4, "f16": 2}[spinor_prec] * 24
    return vb * (lc + nspinors * sp)


def load(n_domains: int, n_cores: int) -> float:
    """Average load x / ceil(x) with x = N_d / (2 N_c) (Sec. 3.5): the domains of one colour
    are spread over the cores in waves, the last wave partly empty."""
    import math
    x = n_domains / (2.0 * n_cores)
    return x / math.ceil(x)


def mg_coarse_bytes(n_agg: int, K: int, k: int, nrhs: int = 1) -> float:
    """Algorithmic bytes of one coarse GMRES cycle of k steps for nrhs systems solved
    together (K coarse dofs per aggregate, FP32 complex, 8 bytes each): per step j the
    stencil (9 K x K blocks per aggregate, shared by all systems) and, per system, v_j for
    the operator, the new vector written, basis vectors 0..j read twice (dot products,
    correction), the new vector read and written again by the correction; the first
    vector of each system read once for its norm."""
    nc = n_agg * K * 8
    stencil = n_agg * 9 * K * K * 8
    total = nrhs * nc
    for j in range(k):
        total += stencil + nrhs * (2 * (j + 1) * nc + 4 * nc)
    return float(total)
