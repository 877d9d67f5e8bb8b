"""Lattice geometry for the oracle (test infrastructure only).

Sites x = (x, y, z, t) on an Lx x Ly x Lz x Lt torus, x fastest (the paper's notation
L_x x L_y x L_z x L_t, Sec. 3.2). Arrays carry the site as four leading axes in the
order [t, z, y, x], so direction mu (0 = x, 1 = y, 2 = z, 3 = t) lives on axis 3 - mu.

Boundary conditions: periodic in x, y, z and antiperiodic in t. The antiperiodic sign
is applied to the hopping term only, as a factor -1 on every hop that wraps around the
time boundary (both directions).

Schwarz blocks (Sec. 3.1, multiplicative Schwarz with the domains checkerboarded as in
Sec. 3.5): block extents B_mu divide L_mu, block coordinate b_mu = floor(x_mu / B_mu),
block colour c = sum_mu b_mu mod 2. Colour 0 is swept first.
"""
from __future__ import annotations

import numpy as np


def axis(mu: int) -> int:
    """Array axis of direction mu for arrays indexed [t, z, y, x, ...]."""
    return 3 - mu


def dims_of(field: np.ndarray):
    """(Lx, Ly, Lz, Lt) of a canonical site-leading array."""
    lt, lz, ly, lx = field.shape[:4]
    return (lx, ly, lz, lt)


def coords(dims):
    """Integer coordinate arrays X[mu][t, z, y, x] = x_mu."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return (x, y, z, t)


def parity(dims) -> np.ndarray:
    """p(x) = sum_mu x_mu mod 2, shape [t, z, y, x]."""
    c = coords(dims)
    return (c[0] + c[1] + c[2] + c[3]) % 2


def shift_fwd(f: np.ndarray, mu: int, antiperiodic: bool = False) -> np.ndarray:
    """g(x) = f(x + mu_hat), times -1 where the hop wraps in t if antiperiodic."""
    g = np.roll(f, -1, axis=axis(mu))
    if antiperiodic and mu == 3:
        g = g.copy()
        g[-1] *= -1.0
    return g


def shift_bwd(f: np.ndarray, mu: int, antiperiodic: bool = False) -> np.ndarray:
    """g(x) = f(x - mu_hat), times -1 where the hop wraps in t if antiperiodic."""
    g = np.roll(f, 1, axis=axis(mu))
    if antiperiodic and mu == 3:
        g = g.copy()
        g[0] *= -1.0
    return g


def block_colour(dims, block) -> np.ndarray:
    """Colour sum_mu floor(x_mu / B_mu) mod 2 of every site, shape [t, z, y, x]."""
    c = coords(dims)
    return sum(c[mu] // block[mu] for mu in range(4)) % 2


def internal_fwd(dims, block, mu: int) -> np.ndarray:
    """True where the hop x -> x + mu_hat stays inside x's block."""
    return (coords(dims)[mu] % block[mu]) != block[mu] - 1


def internal_bwd(dims, block, mu: int) -> np.ndarray:
    """True where the hop x -> x - mu_hat stays inside x's block."""
    return (coords(dims)[mu] % block[mu]) != 0


def block_sum(f: np.ndarray, block) -> np.ndarray:
    """Sum of a per-site array over the sites of each block.

    f has shape [t, z, y, x]; the result has shape [Gt, Gz, Gy, Gx] with G = L / B.
    """
    lx, ly, lz, lt = dims_of(f)
    bx, by, bz, bt = block
    r = f.reshape(lt // bt, bt, lz // bz, bz, ly // by, by, lx // bx, bx)
    return r.sum(axis=(1, 3, 5, 7))


def block_broadcast(g: np.ndarray, block) -> np.ndarray:
    """Inverse of block_sum's shape change: per-block values copied to every site."""
    bx, by, bz, bt = block
    r = np.repeat(g, bt, axis=0)
    r = np.repeat(r, bz, axis=1)
    r = np.repeat(r, by, axis=2)
    return np.repeat(r, bx, axis=3)


def check_blocking(dims, block) -> None:
    """Blocks must tile the lattice, have even extents and form an even block grid."""
    for mu in range(4):
        if block[mu] < 2 or block[mu] % 2:
            raise ValueError(f"block extent {block[mu]} in direction {mu} must be even >= 2")
        if dims[mu] % block[mu]:
            raise ValueError(f"block extent {block[mu]} does not divide {dims[mu]}")
        if (dims[mu] // block[mu]) % 2:
            raise ValueError("the block grid must have an even extent in every direction")
