"""Flexible GMRES(m), restarted and with deflated restarts (oracle; test infrastructure only).

The paper's outer solver is flexible GMRES (with deflated restarts, Sec. 3.1); the
preconditioner it wraps is the Schwarz procedure, which is not a fixed linear map
(its MR step lengths depend on the data), hence the flexible variant. The oracle
implements the plain restarted flexible GMRES of Saad (1993) without deflation:

  restart:  r = b - M x, beta = |r|; stop if beta <= tol |b|; v_1 = r / beta
  step j:   z_j = P(v_j)
            w = M z_j, orthogonalised against v_1..v_j by modified Gram-Schmidt
            h_{j+1,j} = |w|, v_{j+1} = w / h_{j+1,j}
            y_j = argmin |beta e_1 - Hbar_j y| (numpy.linalg.lstsq)
            leave the cycle when that minimum is <= tol |b| or h_{j+1,j} = 0
  update:   x += Z_j y_j; the next restart recomputes the true residual.

fgmres_dr adds the deflated restart of the paper's outer solver (flexible GMRES with
deflated restarts, Sec. 3.1; the restart of Morgan's GMRES-DR in its flexible form,
Giraud, Gratton, Pinel and Vasseur 2010). At the end of a full cycle (m steps,
M Z_m = V_{m+1} Hbar_m, coefficients c of the residual in the basis V_{m+1}):

  y = argmin |c - Hbar_m y|, x += Z_m y, s = c - Hbar_m y   (residual = V_{m+1} s)
  harmonic Ritz pairs of Hbar_m: (H_m + H_m^-H h^H h) g = theta g, with H_m the first m
            rows and h the last row of Hbar_m; G_k = the k vectors of smallest |theta|
  P_{k+1} = orthonormal basis of [[G_k; 0], s]   ((m+1) x (k+1), from a QR
            factorisation; P_k = its first m rows and k columns)
  V_{k+1} <- V_{m+1} P_{k+1},  Z_k <- Z_m P_k,  Hbar_k <- P_{k+1}^H Hbar_m P_k,
  c <- P_{k+1}^H s, and the Arnoldi process continues from step k + 1.

The relation M Z = V Hbar survives the restart because Hbar_m P_k lies in the span of
P_{k+1} (the harmonic Ritz vectors make it so). Convergence is judged on the true
residual b - M x after every cycle; a cycle that ends short of m steps without
converging restarts plainly from that true residual.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def fgmres(apply_m, precond, b, m=16, tol=1e-10, max_iter=2000, x0=None, record=None):
    """Solve M x = b. Returns (x, info) with info = dict(iters, restarts, relres,
    converged, history). `record`, if a dict, receives the last cycle's V, Z, Hbar."""
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else x0.copy()
    iters = 0
    restarts = 0
    history = []
    if bnorm == 0.0:
        return np.zeros_like(b), dict(iters=0, restarts=0, relres=0.0, converged=True,
                                      history=history)
    while True:
        r = b - apply_m(x)
        beta = float(np.linalg.norm(r))
        history.append(beta / bnorm)
        if beta <= tol * bnorm:
            return x, dict(iters=iters, restarts=restarts, relres=beta / bnorm,
                           converged=True, history=history)
        if iters >= max_iter:
            return x, dict(iters=iters, restarts=restarts, relres=beta / bnorm,
                           converged=False, history=history)
        vs = [r / beta]
        zs = []
        h = np.zeros((m + 1, m), dtype=np.complex128)
        y = None
        for j in range(m):
            z = precond(vs[j])
            zs.append(z)
            w = apply_m(z)
            for i in range(j + 1):
                h[i, j] = _dot(vs[i], w)
                w = w - h[i, j] * vs[i]
            h[j + 1, j] = np.linalg.norm(w)
            iters += 1
            rhs = np.zeros(j + 2, dtype=np.complex128)
            rhs[0] = beta
            y = np.linalg.lstsq(h[:j + 2, :j + 1], rhs, rcond=None)[0]
            est = float(np.linalg.norm(rhs - h[:j + 2, :j + 1] @ y))
            if h[j + 1, j] == 0.0:
                break
            vs.append(w / h[j + 1, j])
            if est <= tol * bnorm or iters >= max_iter:
                break
        for i, zi in enumerate(zs):
            x = x + y[i] * zi
        if record is not None:
            record.update(V=vs, Z=zs, H=h[:len(zs) + 1, :len(zs)], beta=beta)
        restarts += 1


def fgmres_dr(apply_m, precond, b, m=16, k=2, tol=1e-10, max_iter=2000, x0=None, record=None):
    """Solve M x = b with FGMRES-DR(m, k). Returns (x, info) as fgmres. `record`, if a
    dict, receives the last cycle's V, Z, Hbar, the coefficient vector c of its start,
    and the harmonic Ritz values of every deflated restart (list `theta`)."""
    assert 0 <= k < m
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else x0.copy()
    iters = 0
    restarts = 0
    history = []
    thetas = []
    if bnorm == 0.0:
        return np.zeros_like(b), dict(iters=0, restarts=0, relres=0.0, converged=True,
                                      history=history)
    r = b - apply_m(x)
    beta = float(np.linalg.norm(r))
    history.append(beta / bnorm)
    if beta <= tol * bnorm:
        return x, dict(iters=0, restarts=0, relres=beta / bnorm, converged=True, history=history)
    vs, zs, j0 = [r / beta], [], 0
    h = np.zeros((m + 1, m), dtype=np.complex128)
    c = np.zeros(m + 1, dtype=np.complex128)
    c[0] = beta
    while True:
        y = None
        for j in range(j0, m):
            z = precond(vs[j])
            zs.append(z)
            w = apply_m(z)
            for i in range(j + 1):
                h[i, j] = _dot(vs[i], w)
                w = w - h[i, j] * vs[i]
            h[j + 1, j] = np.linalg.norm(w)
            iters += 1
            y = np.linalg.lstsq(h[:j + 2, :j + 1], c[:j + 2], rcond=None)[0]
            est = float(np.linalg.norm(c[:j + 2] - h[:j + 2, :j + 1] @ y))
            if h[j + 1, j] == 0.0:
                break
            vs.append(w / h[j + 1, j])
            if est <= tol * bnorm or iters >= max_iter:
                break
        nz = len(zs)
        for i in range(nz):
            x = x + y[i] * zs[i]
        if record is not None:
            record.update(V=list(vs), Z=list(zs), H=h[:nz + 1, :nz].copy(), c=c[:nz + 1].copy(),
                          theta=thetas)
        restarts += 1
        r = b - apply_m(x)
        relres = float(np.linalg.norm(r)) / bnorm
        history.append(relres)
        if relres <= tol:
            return x, dict(iters=iters, restarts=restarts, relres=relres, converged=True, history=history)
        if iters >= max_iter:
            return x, dict(iters=iters, restarts=restarts, relres=relres, converged=False, history=history)
        if nz < m or len(vs) < m + 1:
            beta = relres * bnorm  # short cycle: plain restart from the true residual
            vs, zs, j0 = [r / beta], [], 0
            h[:] = 0
            c[:] = 0
            c[0] = beta
            continue
        hb = h.copy()
        s_res = c - hb @ y
        hm, hrow = hb[:m, :], hb[m:m + 1, :]
        a_h = hm + np.linalg.solve(hm.conj().T, hrow.conj().T @ hrow)
        theta, g = np.linalg.eig(a_h)
        order = np.argsort(np.abs(theta), kind="stable")[:k]
        thetas.append(theta[order])
        p = np.zeros((m + 1, k + 1), dtype=np.complex128)
        p[:m, :k] = g[:, order]
        p[:, k] = s_res
        p = np.linalg.qr(p)[0]
        vs = [sum(p[i, l] * vs[i] for i in range(m + 1)) for l in range(k + 1)]
        zs = [sum(p[i, l] * zs[i] for i in range(m)) for l in range(k)]
        hk = p.conj().T @ hb @ p[:m, :k]
        h[:] = 0
        h[:k + 1, :k] = hk
        cn = p.conj().T @ s_res
        c[:] = 0
        c[:k + 1] = cn
        j0 = k
