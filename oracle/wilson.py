"""Wilson-clover Dirac operator (oracle; test infrastructure only).

The paper's operator is Wilson-clover (Sec. 3.1) with 1848 flops per site (Sec. 3.7);
it prints no formula, so the oracle writes out the standard kappa-normalised form:

  (M psi)(x) = A(x) psi(x)
               - kappa * sum_mu [ eta_f (1 - gamma_mu) U_mu(x) psi(x + mu)
                                + eta_b (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ]

with eta = -1 on hops across the time boundary (antiperiodic t) and +1 otherwise, and
the Sheikholeslami-Wohlert clover term

  A(x) = 1 + kappa * T(x),   T(x) = -c_sw * sum_{mu<nu} (gamma_mu gamma_nu) (x) Fhat_mu,nu(x)

Fhat_mu,nu = (Q_mu,nu - Q_mu,nu^dag) / 8 with its trace removed, where Q_mu,nu(x) sums
the four plaquettes in the (mu, nu) plane that start and end at x, all traversed in the
same sense (mu first, then nu). Since i*sigma_mu,nu = -gamma_mu gamma_nu for mu != nu,
this is 1 + i kappa c_sw sum_{mu<nu} sigma_mu,nu Fhat_mu,nu, i.e. 2 kappa times the
mass-normalised operator with kappa = 1 / (2 m0 + 8). The clover is built from the
periodic links; the time-boundary sign cancels in every closed loop.

Shapes: links U[t,z,y,x,mu,3,3], spinors psi[t,z,y,x,4,3], clover T[t,z,y,x,12,12]
with row index 3 * spin + colour.
"""
from __future__ import annotations

import numpy as np

from .gamma import GAMMA
from . import lattice as lat


def _dag(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def _colour_mul(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U psi)[s, a] = sum_b U[a, b] psi[s, b] at every site."""
    return np.einsum("...ab,...sb->...sa", u, psi)


def _spin_mul(g: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(g psi)[s, a] = sum_t g[s, t] psi[t, a] at every site."""
    return np.einsum("st,...ta->...sa", g, psi)


def hop_forward(u: np.ndarray, psi: np.ndarray, mu: int, antiperiodic: bool = True):
    """eta_f (1 - gamma_mu) U_mu(x) psi(x + mu) at every site x."""
    chi = _colour_mul(u[..., mu, :, :], lat.shift_fwd(psi, mu, antiperiodic))
    return chi - _spin_mul(GAMMA[mu], chi)


def hop_backward(u: np.ndarray, psi: np.ndarray, mu: int, antiperiodic: bool = True):
    """eta_b (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) at every site x."""
    chi = lat.shift_bwd(_colour_mul(_dag(u[..., mu, :, :]), psi), mu, antiperiodic)
    return chi + _spin_mul(GAMMA[mu], chi)


def hopping(u: np.ndarray, psi: np.ndarray, antiperiodic: bool = True,
            block=None) -> np.ndarray:
    """H psi = sum_mu [forward + backward hop]; with `block`, hops that leave a block
    are dropped (the block-diagonal part of the Schwarz splitting, Sec. 3.1)."""
    dims = lat.dims_of(psi)
    out = np.zeros_like(psi)
    for mu in range(4):
        f = hop_forward(u, psi, mu, antiperiodic)
        b = hop_backward(u, psi, mu, antiperiodic)
        if block is not None:
            f = f * lat.internal_fwd(dims, block, mu)[..., None, None]
            b = b * lat.internal_bwd(dims, block, mu)[..., None, None]
        out += f + b
    return out


def plaquette_leaves(u: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """Q_mu,nu(x): sum of the four (mu, nu) plaquettes based at x, same orientation."""
    um = u[..., mu, :, :]
    un = u[..., nu, :, :]

    def f(m, d):  # m(x + d_hat)
        return lat.shift_fwd(m, d)

    def b(m, d):  # m(x - d_hat)
        return lat.shift_bwd(m, d)

    # x -> x+mu -> x+mu+nu -> x+nu -> x
    l1 = um @ f(un, mu) @ _dag(f(um, nu)) @ _dag(un)
    # x -> x+nu -> x+nu-mu -> x-mu -> x
    l2 = un @ _dag(b(f(um, nu), mu)) @ _dag(b(un, mu)) @ b(um, mu)
    # x -> x-mu -> x-mu-nu -> x-nu -> x
    l3 = _dag(b(um, mu)) @ _dag(b(b(un, mu), nu)) @ b(b(um, mu), nu) @ b(un, nu)
    # x -> x-nu -> x-nu+mu -> x+mu -> x
    l4 = _dag(b(un, nu)) @ b(um, nu) @ f(b(un, nu), mu) @ _dag(um)
    return l1 + l2 + l3 + l4


def field_strength(u: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """Fhat_mu,nu = (Q - Q^dag)/8 with the trace removed (anti-Hermitian, traceless)."""
    q = plaquette_leaves(u, mu, nu)
    f = (q - _dag(q)) / 8.0
    tr = np.trace(f, axis1=-2, axis2=-1)
    return f - (tr / 3.0)[..., None, None] * np.eye(3)


def clover_term(u: np.ndarray, csw: float) -> np.ndarray:
    """T(x) = -c_sw sum_{mu<nu} gamma_mu gamma_nu (x) Fhat_mu,nu(x), shape [...,12,12]."""
    lead = u.shape[:4]
    t = np.zeros(lead + (4, 3, 4, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            g = GAMMA[mu] @ GAMMA[nu]
            f = field_strength(u, mu, nu)
            t += np.einsum("st,...ab->...satb", g, f)
    return (-csw * t).reshape(lead + (12, 12))


def apply_clover(a: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(A psi)(x) with A[...,12,12] acting on the flattened (spin, colour) index."""
    flat = psi.reshape(psi.shape[:4] + (12,))
    return np.einsum("...ij,...j->...i", a, flat).reshape(psi.shape)


def apply_M(u, t, kappa, psi, antiperiodic=True, block=None):
    """M psi = (1 + kappa T) psi - kappa H psi; with `block`, the block-restricted M_B."""
    return psi + kappa * apply_clover(t, psi) - kappa * hopping(u, psi, antiperiodic, block)


def dense_matrix(u, t, kappa, antiperiodic=True, block=None) -> np.ndarray:
    """M as a dense (12 V) x (12 V) matrix, columns = M applied to unit vectors."""
    lead = u.shape[:4]
    n = int(np.prod(lead)) * 12
    cols = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(lead + (4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for j in range(n):
        flat[j] = 1.0
        cols[:, j] = apply_M(u, t, kappa, e, antiperiodic, block).reshape(-1)
        flat[j] = 0.0
    return cols
