"""Recursive V-cycle (Algorithm 4.1 of the paper), with its garbled lines read as:
residual r_g - J_g d_g; the recursion's result is assigned to d_{g-1}; the
prolongation acts on d_{g-1}; post-smoothing uses the original r_g.
Level 0 (the paper's g = 1) is solved directly; pre-smoothing starts from 0.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .smoother import vanka_sweep


def coarse_inverse(L0):
    """Dense FP64 inverse of the coarsest matrix by LU with partial pivoting."""
    A = L0.J.toarray()
    lu, piv = sla.lu_factor(A)
    return sla.lu_solve((lu, piv), np.eye(A.shape[0]))


def vcycle(olevels, r, nu1: int, nu2: int, omega: float, g: int | None = None, coarse_inv=None):
    """d = MG(r, g): one V(nu1, nu2) cycle from the zero initial guess."""
    if g is None:
        g = len(olevels) - 1
    L = olevels[g]
    if g == 0:
        if coarse_inv is not None:
            return coarse_inv @ r
        return np.linalg.solve(L.J.toarray(), r)
    d = np.zeros_like(r)
    for _ in range(nu1):
        d = vanka_sweep(L, r, d, omega)
    rho = r - L.J @ d
    r_c = L.P.T @ rho
    d_c = vcycle(olevels, r_c, nu1, nu2, omega, g - 1, coarse_inv)
    d = d + L.P @ d_c
    for _ in range(nu2):
        d = vanka_sweep(L, r, d, omega)
    return d
