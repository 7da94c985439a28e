"""Newton iteration of one subinterval and time marching with direct sparse
solves of the Jacobian (TEST INFRASTRUCTURE ONLY).  The residual, Jacobian and
data come from the problem description; the oracle takes the Newton steps
u <- u - J(u)^-1 R(u) until ||R|| <= tol ||F||."""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla

from .smoother import spacetime_matrix


def newton_direct(problem, u0, F, tol=1e-12, max_newton=20):
    u = u0.copy()
    hist = []
    scale = max(np.linalg.norm(F), 1e-300)
    for _ in range(max_newton + 1):
        R = problem.residual(u, F)
        hist.append(np.linalg.norm(R) / scale)
        if hist[-1] <= tol:
            break
        L = problem.hierarchy(u)[-1]
        J = spacetime_matrix(L["rowptr"], L["col"], L["val"], L["n_sdofs"], problem.b)
        u = u - sla.spsolve(J.tocsc(), R)
    return u, hist


def march_direct(problem, v0, n_steps, tol=1e-12, max_newton=20):
    """Solutions of n_steps consecutive subintervals from v(0) = v0."""
    v_prev = v0.copy()
    out = []
    u = np.zeros(problem.fine.mesh.n_sdofs * problem.b)
    for n in range(n_steps):
        F = problem.data(n * problem.tau, v_prev)
        u0 = np.repeat(v_prev, problem.b) if n > 0 else u
        u, hist = newton_direct(problem, u0, F, tol, max_newton)
        out.append((u.copy(), hist))
        v_prev = problem.final_velocity(u)
    return out
