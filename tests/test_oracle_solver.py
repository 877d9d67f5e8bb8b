"""Pins of the oracle's MR, Schwarz and FGMRES steps.

The paper prints no iterate, residual history or iteration count for a defined input,
so these pins use closed forms (one MR step, Schwarz theory with exact block solves),
invariants that hold at every step (residual bookkeeping, Arnoldi relation,
orthogonality) and reductions to library routines (dense LU, least squares over an
explicit Krylov basis).
"""
import numpy as np
import pytest

import synthetic
from oracle import fgmres as fg
from oracle import lattice, sap, wilson

DIMS = (4, 4, 4, 4)
BLOCK = (2, 2, 2, 2)


@pytest.fixture(scope="module")
def system():
    u = synthetic.gauge_field(DIMS, 0.3, 11)
    t = wilson.clover_term(u, 1.0)
    return sap.BlockSystem(u, t, 0.12, BLOCK)


@pytest.fixture(scope="module")
def eta():
    return synthetic.gaussian_source(DIMS, 1, 21)[0]


def _blocks(dims, block):
    c = lattice.coords(dims)
    g = [dims[mu] // block[mu] for mu in range(4)]
    bid = ((c[3] // block[3] * g[2] + c[2] // block[2]) * g[1] + c[1] // block[1]) * g[0] \
        + c[0] // block[0]
    return bid


_DENSE = {}


def _dense_block_inverse_apply(system, rho, colour):
    """delta = M_B^-1 rho_B on every block of `colour`, by dense LU per block."""
    key = id(system)
    if key not in _DENSE:
        _DENSE[key] = wilson.dense_matrix(system.u, system.t, system.kappa, block=system.block)
    mb = _DENSE[key]
    bid = np.repeat(_blocks(system.dims, system.block).reshape(-1), 12)
    col = np.repeat(system.colour.reshape(-1), 12)
    r = rho.reshape(-1)
    out = np.zeros_like(r)
    for b in np.unique(bid[col == colour]):
        idx = np.nonzero(bid == b)[0]
        out[idx] = np.linalg.solve(mb[np.ix_(idx, idx)], r[idx])
    return out.reshape(rho.shape)


def test_mr_one_step_closed_form(system, eta):
    bhat = eta * system.even * (system.colour == 0)[..., None, None]
    x, r = system.mr(bhat, 1)
    p = system.schur(bhat)
    # per block: alpha = <p, b>/<p, p>; check on every block separately
    bid = _blocks(DIMS, BLOCK)
    for b in np.unique(bid[system.colour == 0]):
        m = (bid == b)[..., None, None]
        alpha = np.vdot(p * m, bhat * m) / np.vdot(p * m, p * m)
        assert np.max(np.abs(x * m - alpha * bhat * m)) < 1e-14
    # blocks of the other colour have a zero right-hand side and stay at zero
    other = (system.colour == 1)[..., None, None]
    assert np.max(np.abs(x * other)) == 0.0


def test_mr_residual_monotone_and_orthogonal(system, eta):
    bhat = eta * system.even
    bid = _blocks(DIMS, BLOCK)
    prev = None
    for k in range(1, 6):
        x, r = system.mr(bhat, k)
        # residual identity r = bhat - Dhat x
        assert np.max(np.abs(r - (bhat - system.schur(x)))) < 1e-12
        norms = np.array([np.linalg.norm(r * (bid == b)[..., None, None])
                          for b in range(16)])
        if prev is not None:
            assert np.all(norms <= prev * (1 + 1e-12))
            # MR: the new residual is orthogonal to Dhat applied to the previous one
            for b in range(16):
                m = (bid == b)[..., None, None]
                assert abs(np.vdot(system.schur(r_prev) * m, r * m)) < 1e-12 * prev[b] ** 2
        prev = norms
        r_prev = r


def test_even_odd_block_solve_converges_to_dense_lu(system, eta):
    for colour in (0, 1):
        delta, r = system.block_solve(eta, colour, 40)
        exact = _dense_block_inverse_apply(system, eta, colour)
        assert np.linalg.norm(delta - exact) < 1e-9 * np.linalg.norm(exact)


def test_sap_residual_invariant(system, eta):
    """After every half-sweep rho = eta - M psi (exact in exact arithmetic)."""
    trace = []
    sap.sap(system, eta, 3, 4, trace=trace)
    assert len(trace) == 6
    for psi, rho in trace:
        true = eta - wilson.apply_M(system.u, system.t, system.kappa, psi)
        assert np.linalg.norm(rho - true) < 1e-12 * np.linalg.norm(eta)


def test_sap_exact_blocks_schwarz_product(system, eta, monkeypatch):
    """With exact block solves, 1 - M P = [(1 - M K_1)(1 - M K_0)]^ncy (Schwarz theory)."""
    ncy = 3

    def exact_solve(rho, colour, nmr):
        d = _dense_block_inverse_apply(system, rho, colour)
        inside = (system.colour == colour)[..., None, None]
        return d, np.zeros_like(d) * inside

    monkeypatch.setattr(system, "block_solve", exact_solve)
    psi = sap.sap(system, eta, ncy, 0)
    lhs = eta - wilson.apply_M(system.u, system.t, system.kappa, psi)

    mfun = lambda f: wilson.apply_M(system.u, system.t, system.kappa, f)  # noqa: E731
    v = eta.copy()
    for _ in range(ncy):
        for c in (0, 1):
            v = v - mfun(_dense_block_inverse_apply(system, v, c))
    assert np.linalg.norm(lhs - v) < 1e-12 * np.linalg.norm(eta)


def test_sap_large_nmr_approaches_exact_block_sap(system, eta):
    psi_mr = sap.sap(system, eta, 2, 40)
    psi = np.zeros_like(eta)
    rho = eta.copy()
    mfun = lambda f: wilson.apply_M(system.u, system.t, system.kappa, f)  # noqa: E731
    for _ in range(2):
        for c in (0, 1):
            d = _dense_block_inverse_apply(system, rho, c)
            psi = psi + d
            rho = rho - mfun(d)
    assert np.linalg.norm(psi_mr - psi) < 1e-8 * np.linalg.norm(psi)


def _ops(system):
    mfun = lambda f: wilson.apply_M(system.u, system.t, system.kappa, f)  # noqa: E731
    return mfun


def test_fgmres_arnoldi_relation_and_orthonormality(system, eta):
    mfun = _ops(system)
    prec = lambda v: sap.sap(system, v, 2, 3)  # noqa: E731
    rec = {}
    fg.fgmres(mfun, prec, eta, m=6, tol=1e-30, max_iter=6, record=rec)
    v = np.array([x.reshape(-1) for x in rec["V"]]).T
    z = np.array([x.reshape(-1) for x in rec["Z"]]).T
    h = rec["H"]
    # modified Gram-Schmidt loses orthogonality in proportion to how close each new
    # vector is to the span of the previous ones (SAP removes most of the residual), so
    # the bound is loose; a wrong conjugation or projection would give O(1) errors
    assert np.max(np.abs(v.conj().T @ v - np.eye(v.shape[1]))) < 1e-9
    mz = np.array([mfun(x).reshape(-1) for x in rec["Z"]]).T
    assert np.linalg.norm(mz - v @ h) < 1e-12 * np.linalg.norm(mz)


def test_fgmres_identity_preconditioner_is_gmres(system, eta):
    """With P = 1, m steps from x = 0 minimise |b - M x| over span{b, Mb, ..., M^(m-1) b}."""
    mfun = _ops(system)
    m = 5
    x, info = fg.fgmres(mfun, lambda v: v, eta, m=m, tol=1e-30, max_iter=m)
    k = [eta.reshape(-1)]
    for _ in range(m - 1):
        k.append(mfun(k[-1].reshape(eta.shape)).reshape(-1))
    q, _ = np.linalg.qr(np.array(k).T)
    mq = np.array([mfun(q[:, i].reshape(eta.shape)).reshape(-1) for i in range(m)]).T
    c = np.linalg.lstsq(mq, eta.reshape(-1), rcond=None)[0]
    x_ref = (q @ c).reshape(eta.shape)
    assert np.linalg.norm(x - x_ref) < 1e-10 * np.linalg.norm(x_ref)


def test_fgmres_exact_preconditioner_one_step(system, eta):
    mfun = _ops(system)
    mdense = wilson.dense_matrix(system.u, system.t, system.kappa)
    exact = lambda v: np.linalg.solve(mdense, v.reshape(-1)).reshape(v.shape)  # noqa: E731
    x, info = fg.fgmres(mfun, exact, eta, m=16, tol=1e-10)
    assert info["converged"] and info["iters"] == 1


def test_dense_lu_2222_gmres():
    dims = (2, 2, 2, 2)
    u = synthetic.gauge_field(dims, 0.3, 7)
    t = wilson.clover_term(u, 1.0)
    b = synthetic.gaussian_source(dims, 1, 8)[0]
    mfun = lambda f: wilson.apply_M(u, t, 0.12, f)  # noqa: E731
    x, info = fg.fgmres(mfun, lambda v: v, b, m=16, tol=1e-10)
    md = wilson.dense_matrix(u, t, 0.12)
    x_lu = np.linalg.solve(md, b.reshape(-1)).reshape(b.shape)
    cond = np.linalg.cond(md)
    assert info["converged"]
    assert np.linalg.norm(x - x_lu) <= cond * 1e-10 * np.linalg.norm(x_lu)


def test_dense_lu_4444_sap_fgmres(system, eta):
    """The first configuration end to end: 4^4, 2^4 blocks, nmr = 4, ncy = 5, FGMRES(16)."""
    mfun = _ops(system)
    prec = lambda v: sap.sap(system, v, 5, 4)  # noqa: E731
    x, info = fg.fgmres(mfun, prec, eta, m=16, tol=1e-10)
    assert info["converged"] and info["relres"] <= 1e-10
    md = wilson.dense_matrix(system.u, system.t, system.kappa)
    x_lu = np.linalg.solve(md, eta.reshape(-1)).reshape(eta.shape)
    cond = np.linalg.cond(md)
    assert np.linalg.norm(x - x_lu) <= cond * 1e-10 * np.linalg.norm(x_lu)
    # SAP is a strong preconditioner: far fewer iterations than unpreconditioned GMRES
    _, info_id = fg.fgmres(mfun, lambda v: v, eta, m=16, tol=1e-10)
    assert info["iters"] < info_id["iters"]


# ---- flexible GMRES with deflated restarts

def _normal_matrix_with_small_eigenvalues(n=160, small=(1e-3, 2e-3 + 1e-3j, 3e-3, 4e-3 - 5e-4j), seed=5):
    """A = Q diag(lambda) Q^H with a few eigenvalues near 0 and the rest in [1, 3]: restarted
    GMRES stalls on the small ones, deflation removes them."""
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.concatenate([np.array(small, dtype=np.complex128), rng.uniform(1.0, 3.0, n - len(small))])
    return (q * lam) @ q.conj().T, lam


def test_fgmres_dr_without_deflation_is_restarted_fgmres(system, eta):
    """k = 0 restarts from the recursive residual V s instead of the recomputed true
    residual: in exact arithmetic the same vector, so the iterates agree to rounding."""
    mfun = _ops(system)
    prec = lambda v: sap.sap(system, v, 2, 1)  # noqa: E731
    x0, i0 = fg.fgmres(mfun, prec, eta, m=3, tol=1e-9, max_iter=60)
    x1, i1 = fg.fgmres_dr(mfun, prec, eta, m=3, k=0, tol=1e-9, max_iter=60)
    assert i0["converged"] and i1["converged"] and i0["restarts"] > 2
    assert i1["iters"] == i0["iters"]
    assert np.linalg.norm(x1 - x0) <= 1e-7 * np.linalg.norm(x0)


def test_fgmres_dr_arnoldi_relation_after_deflated_restart(system, eta):
    """After deflated restarts the cycle still satisfies M Z = V Hbar with orthonormal V,
    and c holds the residual's coordinates: V c = b - M x at the cycle start."""
    mfun = _ops(system)
    prec = lambda v: sap.sap(system, v, 2, 1)  # noqa: E731
    rec = {}
    x, info = fg.fgmres_dr(mfun, prec, eta, m=4, k=2, tol=1e-30, max_iter=10, record=rec)
    assert info["restarts"] >= 3 and len(rec["theta"]) >= 2
    v = np.array([a.reshape(-1) for a in rec["V"]]).T
    z = np.array([a.reshape(-1) for a in rec["Z"]]).T
    h = rec["H"]
    assert np.max(np.abs(v.conj().T @ v - np.eye(v.shape[1]))) < 1e-9
    mz = np.array([mfun(a).reshape(-1) for a in rec["Z"]]).T
    assert np.linalg.norm(mz - v @ h) < 1e-11 * np.linalg.norm(mz)
    assert np.abs(h[2, 0]) > 0 and np.abs(h[2, 1]) > 0 or h.shape[1] < 2  # dense leading block


def test_fgmres_dr_deflation_finds_small_eigenvalues_and_accelerates():
    """On A = Q diag(lambda) Q^H (identity preconditioner), GMRES-DR(10, 4) converges in a
    fraction of the iterations restarted GMRES(10) needs, and its harmonic Ritz values
    converge to the four small eigenvalues."""
    a, lam = _normal_matrix_with_small_eigenvalues()
    b = np.random.default_rng(6).standard_normal(a.shape[0]) + 0j
    mfun = lambda v: a @ v  # noqa: E731
    ident = lambda v: v  # noqa: E731
    _, plain = fg.fgmres(mfun, ident, b, m=10, tol=1e-10, max_iter=1500)
    rec = {}
    x, dr = fg.fgmres_dr(mfun, ident, b, m=10, k=4, tol=1e-10, max_iter=1500, record=rec)
    assert dr["converged"]
    assert np.linalg.norm(b - a @ x) <= 1e-10 * np.linalg.norm(b) * 1.0001
    assert dr["iters"] * 4 < (plain["iters"] if plain["converged"] else 1500)
    got = np.sort_complex(rec["theta"][-1])
    want = np.sort_complex(lam[:4])
    assert np.max(np.abs(got - want)) < 1e-6
