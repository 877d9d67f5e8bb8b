"""Flexible GMRES(m) with restarts (oracle; test infrastructure only).

The paper's outer solver is flexible GMRES (with deflated restarts, Sec. 3.1); the
preconditioner it wraps is the Schwarz procedure, which is not a fixed linear map
(its MR step lengths depend on the data), hence the flexible variant. The oracle
implements the plain restarted flexible GMRES of Saad (1993) without deflation:

  restart:  r = b - M x, beta = |r|; stop if beta <= tol |b|; v_1 = r / beta
  step j:   z_j = P(v_j)   (optionally rounded to the precision Z is stored in)
            w = M z_j, orthogonalised against v_1..v_j by modified Gram-Schmidt
            h_{j+1,j} = |w|, v_{j+1} = w / h_{j+1,j}
            y_j = argmin |beta e_1 - Hbar_j y| (numpy.linalg.lstsq)
            leave the cycle when that minimum is <= tol |b| or h_{j+1,j} = 0
  update:   x += Z_j y_j; the next restart recomputes the true residual.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def fgmres(apply_m, precond, b, m=16, tol=1e-10, max_iter=2000, x0=None,
           z_dtype=None, record=None):
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
            if z_dtype is not None:
                z = z.astype(z_dtype).astype(np.complex128)
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
