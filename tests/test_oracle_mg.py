"""Pins of the oracle's two-level multigrid (interpolation, Galerkin coarse operator,
coarse GMRES, two-grid preconditioner).

The paper prints no coarse operator or iteration count for a defined input, so these
pins use what the mathematics fixes: the interpolation against a Householder QR from
the library, the gamma_5-Hermiticity that the Galerkin product inherits from M with
chirality-split aggregates, the nearest-neighbour sparsity of that product, exactness
of the coarse-grid correction when the interpolation is square, GMRES against an
explicit least-squares solve over the Krylov basis, and the fact that the two-grid
preconditioner with an exact coarse solve reproduces any vector of the coarse space.
"""
import numpy as np
import pytest

import synthetic
from oracle import fgmres as fg
from oracle import lattice, mg, sap, wilson


def _field(dims, kappa=0.12, seed=11):
    u = synthetic.gauge_field(dims, 0.3, seed)
    return u, wilson.clover_term(u, 1.0), kappa


def _vecs(dims, n, seed):
    return list(synthetic.gaussian_source(dims, n, seed))


def _aggregate_rows(f, block, g, s):
    """Entries of field f on aggregate g (block-grid coordinates x, y, z, t) and
    chirality s as a flat vector (site-major, then spin, colour)."""
    sl = tuple(slice(g[mu] * block[mu], (g[mu] + 1) * block[mu]) for mu in (3, 2, 1, 0))
    spins = list(mg.CHIRAL_SPINS[s])
    return f[sl][..., spins, :].reshape(-1)


def test_prolongator_is_the_q_of_a_householder_qr():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    vecs = _vecs(dims, 3, 5)
    cols = mg.prolongator(vecs, block)
    nvec = len(vecs)
    for g in [(0, 0, 0, 0), (1, 0, 1, 0), (1, 1, 1, 1)]:
        for s in (0, 1):
            a = np.stack([_aggregate_rows(v, block, g, s) for v in vecs], axis=1)
            q, r = np.linalg.qr(a)
            ph = np.diag(r) / np.abs(np.diag(r))
            q = q * ph[None, :]  # R with a positive real diagonal
            got = np.stack([_aggregate_rows(cols[s * nvec + j], block, g, s) for j in range(nvec)],
                           axis=1)
            np.testing.assert_allclose(got, q, atol=1e-13)
            # the other chirality is zero in every column of chirality s
            for j in range(nvec):
                assert not np.any(_aggregate_rows(cols[s * nvec + j], block, g, 1 - s))


@pytest.fixture(scope="module")
def full_rank():
    """2x2x2x4 lattice, two 2^4 aggregates with 96 test vectors: P is square (unitary).
    (Extents of 2 wrap a hop onto the site's other neighbour; M stays well defined.)"""
    dims, block = (2, 2, 2, 4), (2, 2, 2, 2)
    u, t, kappa = _field(dims)
    vecs = _vecs(dims, 96, 7)
    cols = mg.prolongator(vecs, block)
    dc = mg.coarse_dense(u, t, kappa, cols, block)
    return dict(dims=dims, block=block, u=u, t=t, kappa=kappa, cols=cols, dc=dc)


def _sigma(n_agg, nvec):
    s = np.concatenate([np.ones(nvec), -np.ones(nvec)])
    return np.tile(s, n_agg)


def test_full_rank_coarse_correction_solves_exactly(full_rank):
    f = full_rank
    b = synthetic.gaussian_source(f["dims"], 1, 9)[0]
    rc = mg.restrict(f["cols"], b, f["block"])
    ec = np.linalg.solve(f["dc"], rc.reshape(-1)).reshape(rc.shape)
    x = mg.prolong(f["cols"], ec, f["block"])
    res = b - wilson.apply_M(f["u"], f["t"], f["kappa"], x)
    assert np.linalg.norm(res) / np.linalg.norm(b) < 1e-12


def test_coarse_operator_is_gamma5_hermitian(full_rank):
    f = full_rank
    sig = _sigma(2, 96)
    lhs = sig[:, None] * f["dc"] * sig[None, :]
    np.testing.assert_allclose(lhs, np.conj(f["dc"].T), atol=1e-12)


@pytest.fixture(scope="module")
def long_t():
    """4x4x4x8 lattice, 2^4 aggregates (block grid 2x2x2x4), 2 test vectors."""
    dims, block = (4, 4, 4, 8), (2, 2, 2, 2)
    u, t, kappa = _field(dims, seed=13)
    vecs = _vecs(dims, 2, 17)
    cols = mg.prolongator(vecs, block)
    dc = mg.coarse_dense(u, t, kappa, cols, block)
    return dict(dims=dims, block=block, u=u, t=t, kappa=kappa, cols=cols, dc=dc, vecs=vecs)


def test_coarse_operator_couples_only_neighbouring_aggregates(long_t):
    f = long_t
    gdims = (2, 2, 2, 4)
    nagg, nk = 32, 4
    blocks = f["dc"].reshape(nagg, nk, nagg, nk)

    def gcoord(a):
        return (a % 2, a // 2 % 2, a // 4 % 2, a // 8)

    for a in range(nagg):
        for b in range(nagg):
            ga, gb = gcoord(a), gcoord(b)
            d = [min((ga[mu] - gb[mu]) % gdims[mu], (gb[mu] - ga[mu]) % gdims[mu]) for mu in range(4)]
            near = sum(d) <= 1
            if near:
                assert np.linalg.norm(blocks[a, :, b, :]) > 1e-3
            else:
                assert np.linalg.norm(blocks[a, :, b, :]) == 0.0
    sig = _sigma(nagg, 2)
    np.testing.assert_allclose(sig[:, None] * f["dc"] * sig[None, :], np.conj(f["dc"].T), atol=1e-12)


def test_galerkin_orthogonality_of_the_coarse_correction(long_t):
    f = long_t
    b = synthetic.gaussian_source(f["dims"], 1, 19)[0]
    rc = mg.restrict(f["cols"], b, f["block"])
    ec = np.linalg.solve(f["dc"], rc.reshape(-1)).reshape(rc.shape)
    res = b - wilson.apply_M(f["u"], f["t"], f["kappa"], mg.prolong(f["cols"], ec, f["block"]))
    assert np.abs(mg.restrict(f["cols"], res, f["block"])).max() < 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(res) > 0.1 * np.linalg.norm(b)  # P is far from square here


def test_gmres_fixed_is_the_krylov_least_squares_minimiser():
    rng = np.random.default_rng(3)
    n = 40
    a = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    rhs = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for k in (1, 5, 12):
        e = mg.gmres_fixed(lambda v: a @ v, rhs, k)
        kry = np.stack([np.linalg.matrix_power(a, i) @ rhs for i in range(k)], axis=1)
        q, _ = np.linalg.qr(kry)
        y = np.linalg.lstsq(a @ q, rhs, rcond=None)[0]
        np.testing.assert_allclose(e, q @ y, rtol=0, atol=1e-10 * np.linalg.norm(q @ y))
    e = mg.gmres_fixed(lambda v: a @ v, rhs, n)
    np.testing.assert_allclose(a @ e, rhs, atol=1e-9)


def test_restarted_gmres_minimises_each_cycle_over_its_residual_krylov_space():
    """Cycle c of the restarted solve adds the minimiser of |r - A d| over the Krylov space
    of its starting residual r (an explicit least-squares solve over that basis), and one
    cycle is plain GMRES(k)."""
    rng = np.random.default_rng(4)
    n, k = 30, 4
    a = np.eye(n) * 2 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    rhs = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    op = lambda v: a @ v  # noqa: E731
    np.testing.assert_allclose(mg.gmres_restarted(op, rhs, k, 1), mg.gmres_fixed(op, rhs, k), atol=1e-12)
    e = np.zeros(n, dtype=complex)
    for c in range(1, 4):
        r = rhs - a @ e
        kry = np.stack([np.linalg.matrix_power(a, i) @ r for i in range(k)], axis=1)
        q, _ = np.linalg.qr(kry)
        e = e + q @ np.linalg.lstsq(a @ q, r, rcond=None)[0]
        got = mg.gmres_restarted(op, rhs, k, c)
        np.testing.assert_allclose(got, e, atol=1e-10 * np.linalg.norm(e))
    assert np.linalg.norm(rhs - a @ e) < np.linalg.norm(rhs - a @ mg.gmres_fixed(op, rhs, k))


def test_two_grid_with_exact_coarse_solve_reproduces_the_coarse_space(long_t):
    f = long_t
    tl = mg.TwoLevel(f["u"], f["t"], f["kappa"], f["block"], f["vecs"], ncy=2, nmr=3,
                     coarse_iters=128)
    rng = np.random.default_rng(5)
    shape = (4, 2, 2, 2, 4)  # [Gt, Gz, Gy, Gx, K]
    e = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    pe = mg.prolong(tl.cols, e, f["block"])
    np.testing.assert_allclose(tl.precond(tl.apply_m(pe)), pe, atol=1e-8 * np.abs(pe).max())


def test_setup_smoothing_finds_near_null_vectors():
    """v <- v - SAP(M v) damps the modes SAP resolves well, so |M v| / |v| falls."""
    dims, block = (4, 4, 4, 8), (2, 2, 2, 2)
    u, t, kappa = _field(dims, kappa=0.13)
    v0 = _vecs(dims, 1, 23)
    ratios = []
    for it in (0, 1, 3):
        tl = mg.TwoLevel(u, t, kappa, block, v0, ncy=2, nmr=4, setup_iters=it)
        v = tl.vecs[0]
        ratios.append(np.linalg.norm(tl.apply_m(v)) / np.linalg.norm(v))
    assert ratios[0] > 2 * ratios[1] > 2 * ratios[2]


def test_two_level_fgmres_converges_to_the_true_residual(long_t):
    f = long_t
    b = synthetic.gaussian_source(f["dims"], 1, 31)[0]
    tl = mg.TwoLevel(f["u"], f["t"], f["kappa"], f["block"], f["vecs"], ncy=2, nmr=4, setup_iters=2,
                     coarse_iters=8)
    x, info = fg.fgmres(tl.apply_m, tl.precond, b, m=8, tol=1e-10)
    assert info["converged"]
    assert np.linalg.norm(b - tl.apply_m(x)) / np.linalg.norm(b) <= 1e-10
