"""Pins of the oracle's Dirac operator against facts that do not come from its own code.

Each test checks a closed form, an invariant or a reduction that a plausible mistake
in the oracle (a wrong gamma sign, U instead of U^dag, a missing factor in the clover
normalisation, the time-boundary sign on the wrong hop, a transposed index) breaks.
"""
import itertools

import numpy as np
import pytest

import synthetic
from oracle import gamma, lattice, wilson

G = gamma.GAMMA


def test_clifford_algebra():
    for mu, nu in itertools.product(range(4), repeat=2):
        ac = G[mu] @ G[nu] + G[nu] @ G[mu]
        assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4), atol=0)
    for mu in range(4):
        assert np.allclose(G[mu], G[mu].conj().T)
    assert np.allclose(gamma.GAMMA5, np.diag([1, 1, -1, -1]))


def _free_spectrum(dims, kappa):
    """Closed-form eigenvalues of the free Wilson operator with antiperiodic time."""
    lx, ly, lz, lt = dims
    vals = []
    for n in itertools.product(range(lx), range(ly), range(lz), range(lt)):
        p = [2 * np.pi * n[0] / lx, 2 * np.pi * n[1] / ly, 2 * np.pi * n[2] / lz,
             2 * np.pi * (n[3] + 0.5) / lt]
        re = 1.0 - 2.0 * kappa * sum(np.cos(q) for q in p)
        im = 2.0 * kappa * np.sqrt(sum(np.sin(q) ** 2 for q in p))
        vals += [re + 1j * im] * 6 + [re - 1j * im] * 6
    return np.array(vals)


def _unit_links(dims):
    lx, ly, lz, lt = dims
    u = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    u[..., :, :] = np.eye(3)
    return u


def _match_multisets(a, b, tol):
    a = np.sort_complex(np.round(a, 9))
    b = np.sort_complex(np.round(b, 9))
    return np.max(np.abs(a - b)) < tol


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4)])
def test_free_field_spectrum_dense(dims):
    kappa = 0.11
    u = _unit_links(dims)
    t = wilson.clover_term(u, 1.0)
    assert np.max(np.abs(t)) == 0.0  # flat field: no clover
    m = wilson.dense_matrix(u, t, kappa)
    ev = np.linalg.eigvals(m)
    assert _match_multisets(ev, _free_spectrum(dims, kappa), 1e-9)


def test_free_field_plane_waves_4444():
    """M e^{ipx} u = e^{ipx} (1 - 2k sum cos p + 2ik sum gamma sin p) u, p_t antiperiodic."""
    dims = (4, 4, 4, 4)
    kappa = 0.125
    u = _unit_links(dims)
    t = np.zeros((4, 4, 4, 4, 12, 12), dtype=np.complex128)
    x = lattice.coords(dims)
    rng = np.random.default_rng(3)
    for n in [(0, 0, 0, 0), (1, 0, 2, 3), (3, 1, 1, 0), (2, 2, 2, 1)]:
        p = [2 * np.pi * n[0] / 4, 2 * np.pi * n[1] / 4, 2 * np.pi * n[2] / 4,
             2 * np.pi * (n[3] + 0.5) / 4]
        phase = np.exp(1j * sum(p[mu] * x[mu] for mu in range(4)))
        spin = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = phase[..., None, None] * spin
        mp = (1 - 2 * kappa * sum(np.cos(q) for q in p)) * np.eye(4) \
            + 2j * kappa * sum(G[mu] * np.sin(p[mu]) for mu in range(4))
        expect = phase[..., None, None] * (mp @ spin)
        got = wilson.apply_M(u, t, kappa, psi)
        assert np.max(np.abs(got - expect)) < 1e-13


def _field(dims, eps=0.3, seed=5):
    return synthetic.gauge_field(dims, eps, seed)


def test_clover_hermitian_and_chiral():
    u = _field((4, 4, 4, 4))
    t = wilson.clover_term(u, 1.0)
    assert np.max(np.abs(t - np.conj(np.swapaxes(t, -1, -2)))) < 1e-14
    g5 = np.kron(gamma.GAMMA5, np.eye(3))
    assert np.max(np.abs(t @ g5 - g5 @ t)) < 1e-14
    assert np.max(np.abs(t)) > 1e-2


def test_gamma5_hermiticity():
    dims = (4, 4, 4, 6)
    u = _field(dims)
    t = wilson.clover_term(u, 1.3)
    src = synthetic.gaussian_source(dims, 2, 9)
    phi, psi = src[0], src[1]
    g5 = lambda f: np.einsum("st,...ta->...sa", gamma.GAMMA5, f)  # noqa: E731
    kappa = 0.13
    lhs = np.vdot(phi, g5(wilson.apply_M(u, t, kappa, g5(psi))))
    rhs = np.vdot(wilson.apply_M(u, t, kappa, phi), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(rhs) * 10


def test_gauge_covariance():
    """M[U^Omega] (Omega psi) = Omega M[U] psi, U^Omega_mu(x) = Om(x) U_mu(x) Om(x+mu)^dag."""
    dims = (4, 4, 6, 4)
    u = _field(dims)
    om = synthetic.random_su3(u.shape[:4], 17)
    ug = np.empty_like(u)
    for mu in range(4):
        ug[..., mu, :, :] = om @ u[..., mu, :, :] @ np.conj(
            np.swapaxes(lattice.shift_fwd(om, mu), -1, -2))
    psi = synthetic.gaussian_source(dims, 1, 4)[0]
    kappa, csw = 0.124, 1.0
    t = wilson.clover_term(u, csw)
    tg = wilson.clover_term(ug, csw)
    om_psi = np.einsum("...ab,...sb->...sa", om, psi)
    lhs = wilson.apply_M(ug, tg, kappa, om_psi)
    rhs = np.einsum("...ab,...sb->...sa", om, wilson.apply_M(u, t, kappa, psi))
    assert np.max(np.abs(lhs - rhs)) < 1e-13


@pytest.mark.parametrize("n", [1, 2])
def test_uniform_abelian_flux_clover(n):
    """Constant xy flux phi = 2 pi n / (Lx Ly) in the colour direction T = diag(1,-1,0):
    every site's A = 1 + kappa*T has eigenvalues 1 +- kappa c_sw sin(phi) (x4 each), 1 (x4)."""
    dims = (4, 6, 2, 2)
    lx, ly, lz, lt = dims
    phi = 2 * np.pi * n / (lx * ly)
    tdiag = np.array([1.0, -1.0, 0.0])
    x = lattice.coords(dims)
    u = _unit_links(dims)
    # U_y(x) = exp(i phi x0 T); U_x = exp(-i phi Lx x1 T) on the last x slice
    uy = np.exp(1j * phi * x[0][..., None] * tdiag)
    u[..., 1, :, :] = uy[..., :, None] * np.eye(3)
    ux = np.where((x[0] == lx - 1)[..., None], np.exp(-1j * phi * lx * x[1][..., None] * tdiag),
                  1.0 + 0j)
    u[..., 0, :, :] = ux[..., :, None] * np.eye(3)
    kappa, csw = 0.125, 1.7
    t = wilson.clover_term(u, csw)
    a = np.eye(12) + kappa * t
    ev = np.sort(np.linalg.eigvalsh(a.reshape(-1, 12, 12)), axis=-1)
    s = kappa * csw * np.sin(phi)
    expect = np.sort(np.array([1 + s] * 4 + [1 - s] * 4 + [1.0] * 4))
    assert np.max(np.abs(ev - expect)) < 1e-13


def test_special_cases():
    dims = (4, 4, 4, 4)
    u = _field(dims)
    psi = synthetic.gaussian_source(dims, 1, 2)[0]
    t = wilson.clover_term(u, 1.0)
    assert np.array_equal(wilson.apply_M(u, t, 0.0, psi), psi)  # kappa = 0: M = 1
    assert np.max(np.abs(wilson.clover_term(u, 0.0))) == 0.0  # c_sw = 0: pure Wilson


def test_block_restricted_operator_matches_dense_blocks():
    """M_B is M with every hop between blocks removed: its dense matrix equals M's with
    the entries between different blocks zeroed."""
    dims = (4, 4, 4, 4)
    block = (2, 2, 2, 2)
    u = _field(dims)
    t = wilson.clover_term(u, 1.0)
    m = wilson.dense_matrix(u, t, 0.12)
    mb = wilson.dense_matrix(u, t, 0.12, block=block)
    c = lattice.coords(dims)
    bid = sum((c[mu] // block[mu]) * (10 ** mu) for mu in range(4)).reshape(-1)
    bid = np.repeat(bid, 12)
    same = bid[:, None] == bid[None, :]
    assert np.max(np.abs(mb - np.where(same, m, 0))) == 0.0
    assert np.max(np.abs(np.where(same, 0, m))) > 0  # there are hops between blocks


def test_synthetic_links_are_special_unitary():
    """The two-row link storage of the block operator rebuilds row 2 of every link as the
    conjugate cross product of rows 0 and 1, which holds exactly for special unitary
    matrices; the generator's links satisfy it to rounding (and U U^+ = 1, det U = 1)."""
    u = synthetic.gauge_field((4, 4, 4, 4), 0.3, 5)
    assert np.abs(np.conj(np.cross(u[..., 0, :], u[..., 1, :])) - u[..., 2, :]).max() < 1e-13
    assert np.abs(u @ np.conj(np.swapaxes(u, -1, -2)) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(u) - 1.0).max() < 1e-13
