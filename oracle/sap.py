"""Schwarz alternating procedure with even-odd MR block solves (oracle; test only).

What the paper fixes (Sec. 3.1): the lattice is cut into domains; after reordering,
M = block-diagonal part (hops inside a domain) + remainder (hops between domains); the
preconditioner is the multiplicative Schwarz method, with the domains checkerboarded
so that the N_d / 2 domains of one colour are independent (Sec. 3.5); every domain is
solved approximately by the minimal-residual (MR) method with even-odd
preconditioning. The paper gives no further detail, so the oracle takes these readings:

  * blocks of one colour are solved from the same residual (Jacobi within a colour),
    colour 0 first, then colour 1, and this pair is repeated ncy times;
  * on a block B, M_B = [[A_e, K_eo], [K_oe, A_o]] with K = -kappa * (block hopping);
    the even-site Schur complement Dhat = A_e - K_eo A_o^-1 K_oe is solved by MR;
  * MR starts from zero, takes exactly nmr steps with step length
    alpha = <p, r> / <p, p> (p = Dhat r, <a, b> = sum conj(a) b over the block's even
    sites) and alpha = 0 on a block where <p, p> = 0;
  * the odd sites follow from delta_o = A_o^-1 (rho_o - K_oe delta_e), so the block
    residual becomes (r_MR on even sites, 0 on odd sites);
  * after a colour, every site outside the swept blocks gets rho -= (M delta).

All blocks of a colour are handled at once on full-lattice arrays: the block-restricted
hopping term has no hop between blocks, and the MR scalars are per-block sums.
"""
from __future__ import annotations

import numpy as np

from . import lattice as lat
from .wilson import apply_clover, apply_M, hopping


class BlockSystem:
    """The block-diagonal (Schwarz) part of M for one gauge field, kappa and blocking."""

    def __init__(self, u, t, kappa, block, antiperiodic=True):
        self.u = u
        self.t = t
        self.kappa = float(kappa)
        self.block = tuple(int(b) for b in block)
        self.antiperiodic = antiperiodic
        dims = lat.dims_of(u)
        self.dims = dims
        lat.check_blocking(dims, self.block)
        par = lat.parity(dims)
        self.even = (par == 0)[..., None, None]
        self.odd = (par == 1)[..., None, None]
        self.colour = lat.block_colour(dims, self.block)
        self.a = np.eye(12) + self.kappa * t
        self.ainv = np.linalg.inv(self.a)

    # pieces of M_B
    def k_block(self, psi):
        """K psi = -kappa * (hopping restricted to blocks)."""
        return -self.kappa * hopping(self.u, psi, self.antiperiodic, self.block)

    def schur(self, r_e):
        """Dhat r_e = A_e r_e - K_eo A_o^-1 K_oe r_e (even-site field in, even out)."""
        t_o = self.odd * apply_clover(self.ainv, self.odd * self.k_block(r_e))
        return self.even * (apply_clover(self.a, r_e) - self.k_block(t_o))

    def block_dot(self, a, b):
        """<a, b> per block, broadcast back to every site [t, z, y, x, 1, 1]."""
        s = np.sum(np.conj(a) * b, axis=(-1, -2))
        return lat.block_broadcast(lat.block_sum(s, self.block), self.block)[..., None, None]

    def mr(self, bhat, nmr):
        """nmr minimal-residual steps on Dhat x = bhat in every block, from x = 0."""
        x = np.zeros_like(bhat)
        r = bhat.copy()
        for _ in range(nmr):
            p = self.schur(r)
            pr = self.block_dot(p, r)
            pp = self.block_dot(p, p).real
            alpha = np.where(pp > 0, pr / np.where(pp > 0, pp, 1.0), 0.0)
            x = x + alpha * r
            r = r - alpha * p
        return x, r

    def block_solve(self, rho, colour, nmr):
        """Even-odd MR solve of M_B delta = rho on all blocks of one colour.

        Returns (delta, r_mr): delta is zero outside the colour's blocks, r_mr is the new
        even-site block residual (zero elsewhere).
        """
        inside = (self.colour == colour)[..., None, None]
        rho_e = rho * inside * self.even
        rho_o = rho * inside * self.odd
        bhat = rho_e - self.even * self.k_block(apply_clover(self.ainv, rho_o))
        d_e, r = self.mr(bhat, nmr)
        d_o = self.odd * apply_clover(self.ainv, rho_o - self.odd * self.k_block(d_e))
        return d_e + d_o, r


def sap(sys: BlockSystem, eta, ncy: int, nmr: int, trace=None):
    """psi = SAP(eta): ncy cycles of colour 0 then colour 1 block solves.

    If `trace` is a list, (psi, rho) is appended after every half-sweep.
    """
    psi = np.zeros_like(eta)
    rho = eta.copy()
    for _ in range(ncy):
        for c in (0, 1):
            delta, r_mr = sys.block_solve(rho, c, nmr)
            psi = psi + delta
            inside = (sys.colour == c)[..., None, None]
            m_delta = apply_M(sys.u, sys.t, sys.kappa, delta, sys.antiperiodic)
            rho = np.where(inside, r_mr, rho - m_delta)
            if trace is not None:
                trace.append((psi.copy(), rho.copy()))
    return psi
