"""Newton iteration and dG(k) time marching around the library's linear
solver: every Newton step solves J(u) du = -R(u) by FGMRES preconditioned
with the Vanka-GMG V-cycle on the device.

The problem object supplies the discretisation: data(t0, v_prev) -> F (the
data and jump terms of the subinterval starting at t0), residual(u, F),
hierarchy(u) -> level list of the Jacobian at u (coarsest first),
final_velocity(u) -> v(t_n^-), and the attributes dim, k, b, tau, fine.mesh.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Solver


def newton(solver: Solver, problem, u0, F, tol=1e-12, max_newton=20, lin_rtol=1e-11,
           fp32=False):
    """u with ||R(u)|| <= tol ||F||; returns (u, residual history, linear iterations)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    hist, lin = [], []
    scale = max(np.linalg.norm(F), 1e-300)
    dev = torch.device("cuda", solver.device)
    for _ in range(max_newton + 1):
        R = problem.residual(u, F)
        hist.append(float(np.linalg.norm(R) / scale))
        if hist[-1] <= tol:
            break
        solver.set_hierarchy(problem.hierarchy(u), problem.dim, problem.k)
        solver.build_cell_inverses(fp32=fp32)
        rhs = torch.from_numpy(-R).to(dev)
        du = torch.zeros_like(rhs)
        info = solver.gmres_solve(rhs, du, restart=30, max_it=1000, rtol=lin_rtol)
        lin.append(info["iters"])
        u += du.cpu().numpy()
    return u, hist, lin


def march(solver: Solver, problem, v0, n_steps, tol=1e-12, max_newton=20, lin_rtol=1e-11,
          fp32=False):
    """Solutions of n_steps consecutive subintervals from v(0) = v0; each
    Newton iteration starts from the previous end value held constant."""
    v_prev = np.array(v0, dtype=np.float64, copy=True)
    out = []
    u = np.zeros(problem.fine.mesh.n_sdofs * problem.b)
    for n in range(n_steps):
        F = problem.data(n * problem.tau, v_prev)
        u0 = np.repeat(v_prev, problem.b) if n > 0 else u
        u, hist, lin = newton(solver, problem, u0, F, tol, max_newton, lin_rtol, fp32)
        out.append(dict(u=u.copy(), residuals=hist, linear_iters=lin))
        v_prev = problem.final_velocity(u)
    return out
