"""Right-preconditioned flexible GMRES(m) (Saad's FGMRES), FP64, as the outer
solver around the multigrid preconditioner.

Arnoldi by modified Gram-Schmidt, Givens rotations on the Hessenberg matrix,
x0 = 0 unless given.  A cycle ends when the rotated residual estimate falls to
rtol * ||b|| (or after m steps); the iterate is then updated and the true
residual ||b - A x|| decides convergence.  fixed_iters > 0 runs exactly that
many Arnoldi steps (across restarts) and ignores the tolerance.
"""
from __future__ import annotations

import numpy as np


def fgmres(A, b, M, restart: int = 30, rtol: float = 1e-8, max_it: int = 1000,
           x0=None, fixed_iters: int = 0):
    """Returns (x, info) with info = dict(iters, restarts, true_relres, converged, history)."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.astype(np.float64).copy()
    bnorm = np.linalg.norm(b)
    history = []
    iters = 0
    restarts = 0
    if bnorm == 0.0:
        return np.zeros(n), dict(iters=0, restarts=0, true_relres=0.0, converged=True, history=[])
    target = rtol * bnorm
    r = b - A(x)
    beta = np.linalg.norm(r)
    history.append(beta / bnorm)
    converged = beta <= target and fixed_iters == 0
    budget = fixed_iters if fixed_iters > 0 else max_it
    while not converged and iters < budget:
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        j_end = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = A(Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            j_end = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if fixed_iters > 0:
                if iters >= fixed_iters or breakdown:
                    break
            elif abs(g[j + 1]) <= target or iters >= max_it or breakdown:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + Z[:j_end].T @ y
        r = b - A(x)
        beta = np.linalg.norm(r)
        restarts += 1
        if fixed_iters == 0 and beta <= target:
            converged = True
        if beta == 0.0:
            converged = fixed_iters == 0 or iters >= fixed_iters
            break
    relres = np.linalg.norm(b - A(x)) / bnorm
    return x, dict(iters=iters, restarts=restarts, true_relres=relres,
                   converged=bool(relres <= rtol), history=history)
