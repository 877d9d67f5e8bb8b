"""Two-level aggregation multigrid with the Schwarz procedure as its smoother (oracle;
test infrastructure only).

What the paper fixes (Sec. 2.6, application software): the group's adaptive algebraic
multigrid solver is a Krylov method preconditioned by a multigrid V-cycle, and the
smoother of that cycle is the domain-decomposition preconditioner of Sec. 3.1 (the
Schwarz procedure of `oracle.sap`). It cites the adaptive aggregation method of Frommer,
Kahl, Krieg, Leder and Rottmann for the rest and prints no formula, so the oracle writes
out the standard two-level form of that method with these readings:

  * aggregates are the Schwarz blocks, each split into its two chiralities (spins 0, 1
    with gamma_5 = +1 and spins 2, 3 with gamma_5 = -1), so gamma_5 maps every column
    of the interpolation to plus or minus itself;
  * test vectors: nvec given fields v_j, each smoothed setup_iters times by
    v <- v - SAP(M v) (the smoother applied to M x = 0 from the start v);
  * interpolation P: on every aggregate and chirality s, the restrictions of v_1 ..
    v_nvec orthonormalised by Gram-Schmidt in index order (the Q of a QR factorisation
    whose R has a positive real diagonal); coarse index k = s * nvec + j;
  * coarse operator: the Galerkin product D_c = P^H M P, which couples an aggregate
    only to itself and its eight neighbours;
  * coarse solve: coarse_cycles cycles of restarted GMRES(coarse_iters) from zero on
    D_c e = P^H r (every cycle minimises over the Krylov space of the current residual);
  * preconditioner: B(r) = e + SAP(r - M e) with e = P GMRES(D_c, P^H r), the
    coarse-grid correction followed by one Schwarz application (ncy cycles).

Fields are canonical full-lattice arrays [t, z, y, x, spin, colour]; coarse vectors are
arrays [Gt, Gz, Gy, Gx, K] over the block grid (K = 2 nvec), flattened with x fastest.
"""
from __future__ import annotations

import numpy as np

from . import lattice as lat
from .sap import BlockSystem, sap
from .wilson import apply_M

# spins of the two chiralities (gamma_5 = diag(1, 1, -1, -1) in the oracle's basis)
CHIRAL_SPINS = ((0, 1), (2, 3))


def chiral_part(v: np.ndarray, s: int) -> np.ndarray:
    """The spin components of chirality s of a spinor field (the others set to zero)."""
    out = np.zeros_like(v)
    for sp in CHIRAL_SPINS[s]:
        out[..., sp, :] = v[..., sp, :]
    return out


def aggregate_dot(a: np.ndarray, b: np.ndarray, block) -> np.ndarray:
    """<a, b> = sum conj(a) b over every aggregate (block), shape [Gt, Gz, Gy, Gx]."""
    return lat.block_sum(np.sum(np.conj(a) * b, axis=(-1, -2)), block)


def _spread(g: np.ndarray, block) -> np.ndarray:
    """Per-aggregate values as a factor on every site of a spinor field."""
    return lat.block_broadcast(g, block)[..., None, None]


def prolongator(vecs, block):
    """Columns of P as 2 nvec spinor fields (column s * nvec + j); on every aggregate
    the nvec columns of chirality s are orthonormal and span the chirality-s parts of
    the test vectors there. Modified Gram-Schmidt with one reorthogonalisation pass."""
    nvec = len(vecs)
    cols = [None] * (2 * nvec)
    for s in (0, 1):
        q = []
        for v in vecs:
            w = chiral_part(v, s)
            for _ in range(2):
                for qi in q:
                    w = w - _spread(aggregate_dot(qi, w, block), block) * qi
            nrm = np.sqrt(aggregate_dot(w, w, block).real)
            if np.any(nrm == 0.0):
                raise ValueError("test vectors are linearly dependent on an aggregate")
            q.append(w / _spread(nrm, block))
        cols[s * nvec:(s + 1) * nvec] = q
    return cols


def restrict(cols, r: np.ndarray, block) -> np.ndarray:
    """P^H r as a coarse vector [Gt, Gz, Gy, Gx, K]."""
    return np.stack([aggregate_dot(c, r, block) for c in cols], axis=-1)


def prolong(cols, e: np.ndarray, block) -> np.ndarray:
    """P e for a coarse vector e [Gt, Gz, Gy, Gx, K]."""
    out = np.zeros_like(cols[0])
    for k, c in enumerate(cols):
        out = out + _spread(e[..., k], block) * c
    return out


def coarse_dense(u, t, kappa, cols, block, antiperiodic=True) -> np.ndarray:
    """D_c = P^H M P as a dense (Nd K) x (Nd K) matrix (row/column index = aggregate * K
    + k, aggregates in block-grid order with x fastest), one column per unit vector."""
    gshape = lat.block_sum(np.zeros(u.shape[:4]), block).shape
    nk = len(cols)
    n = int(np.prod(gshape)) * nk
    out = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(gshape + (nk,), dtype=np.complex128)
    flat = e.reshape(-1)
    for col in range(n):
        flat[col] = 1.0
        y = apply_M(u, t, kappa, prolong(cols, e, block), antiperiodic)
        out[:, col] = restrict(cols, y, block).reshape(-1)
        flat[col] = 0.0
    return out


def gmres_fixed(apply_a, rhs: np.ndarray, k: int) -> np.ndarray:
    """k steps of GMRES from zero on A e = rhs (no restart): the e in the Krylov space
    span{rhs, A rhs, .., A^(k-1) rhs} that minimises |rhs - A e|. Arnoldi with modified
    Gram-Schmidt; stops early at an exact breakdown (h_{j+1,j} = 0)."""
    beta = float(np.linalg.norm(rhs))
    if beta == 0.0:
        return np.zeros_like(rhs)
    vs = [rhs / beta]
    h = np.zeros((k + 1, k), dtype=np.complex128)
    steps = 0
    for j in range(k):
        w = apply_a(vs[j])
        for i in range(j + 1):
            h[i, j] = np.vdot(vs[i].reshape(-1), w.reshape(-1))
            w = w - h[i, j] * vs[i]
        h[j + 1, j] = np.linalg.norm(w)
        steps = j + 1
        if h[j + 1, j] == 0.0:
            break
        vs.append(w / h[j + 1, j])
    g = np.zeros(steps + 1, dtype=np.complex128)
    g[0] = beta
    y = np.linalg.lstsq(h[:steps + 1, :steps], g, rcond=None)[0]
    out = np.zeros_like(rhs)
    for i in range(steps):
        out = out + y[i] * vs[i]
    return out


def gmres_restarted(apply_a, rhs: np.ndarray, k: int, cycles: int) -> np.ndarray:
    """cycles cycles of GMRES(k) from zero: e <- e + GMRES_k(A, rhs - A e)."""
    e = np.zeros_like(rhs)
    for _ in range(int(cycles)):
        e = e + gmres_fixed(apply_a, rhs - apply_a(e), k)
    return e


class TwoLevel:
    """The two-level preconditioner for one gauge field, kappa and blocking."""

    def __init__(self, u, t, kappa, block, vecs, ncy=5, nmr=4, setup_iters=0,
                 coarse_iters=16, coarse_cycles=1, antiperiodic=True):
        self.sys = BlockSystem(u, t, kappa, block, antiperiodic)
        self.block = tuple(int(b) for b in block)
        self.ncy, self.nmr, self.coarse_iters = int(ncy), int(nmr), int(coarse_iters)
        self.coarse_cycles = int(coarse_cycles)
        vecs = [np.array(v, dtype=np.complex128) for v in vecs]
        for _ in range(int(setup_iters)):
            vecs = [v - sap(self.sys, self.apply_m(v), self.ncy, self.nmr) for v in vecs]
        self.vecs = vecs
        self.cols = prolongator(vecs, self.block)

    def apply_m(self, psi):
        s = self.sys
        return apply_M(s.u, s.t, s.kappa, psi, s.antiperiodic)

    def coarse_apply(self, e):
        """D_c e = P^H M P e."""
        return restrict(self.cols, self.apply_m(prolong(self.cols, e, self.block)), self.block)

    def coarse_solve(self, rc):
        """The coarse solve: coarse_cycles cycles of GMRES(coarse_iters) on D_c e = rc."""
        return gmres_restarted(self.coarse_apply, rc, self.coarse_iters, self.coarse_cycles)

    def coarse_correction(self, r):
        """P GMRES(D_c, P^H r)."""
        return prolong(self.cols, self.coarse_solve(restrict(self.cols, r, self.block)), self.block)

    def precond(self, r):
        """B(r): coarse-grid correction, then one Schwarz application on the residual."""
        e = self.coarse_correction(r)
        return e + sap(self.sys, r - self.apply_m(e), self.ncy, self.nmr)
