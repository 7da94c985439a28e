"""Gradient of a linear loss of the solution with respect to the per-cell
viscosity and the inflow amplitude, by the adjoint method, written from the
definitions with direct sparse solves (TEST INFRASTRUCTURE ONLY).

With J(nu) x = b(nu, U), L = q . x, J affine in every nu_c
(dJ/dnu_c = W_tau (x) K_c) and b = U (F_0 + sum_c nu_c F_c):
  J^T lam = q,
  dL/dnu_c = lam . (U F_c - (W_tau (x) K_c) x)  (both restricted to cell c),
  dL/dU    = lam . (F_0 + sum_c nu_c F_c).
Pinned in the tests by central finite differences of L with re-assembled
operators and by L being linear in U.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla


def solve_and_adjoint(J, b, q):
    """x = J^-1 b and lam = J^-T q (one sparse LU, used both ways)."""
    lu = sla.splu(J.tocsc())
    return lu.solve(b), lu.solve(q, trans="T")


def cell_contraction(lam, x, cell_sdofs, b, refs, ref_ptr, ref_idx, ref_w, tw):
    """out[c] = sum_i tw_i lam_{c,i} . K_c x_{c,i}, K_c = sum ref_w refs[ref_idx]."""
    nc = cell_sdofs.shape[0]
    out = np.zeros(nc)
    for c in range(nc):
        K = np.zeros(refs.shape[1:])
        for e in range(ref_ptr[c], ref_ptr[c + 1]):
            K += ref_w[e] * refs[ref_idx[e]]
        sd = cell_sdofs[c].astype(np.int64)
        for i in range(b):
            out[c] += tw[i] * (lam[sd * b + i] @ (K @ x[sd * b + i]))
    return out


def cell_dot(lam, cells, cell_sdofs, b, Fc):
    """out[k] = sum_i lam_{cells[k], i} . Fc[k, :, i]."""
    out = np.zeros(len(cells))
    for kk, c in enumerate(cells):
        sd = cell_sdofs[c].astype(np.int64)
        for i in range(b):
            out[kk] += lam[sd * b + i] @ Fc[kk, :, i]
    return out


def loss_gradient(J, b, q, U, nu, cell_sdofs, kb, refs, ref_ptr, ref_idx, ref_w, tw,
                  F0, in_cells, Fc):
    """(L, dL/dnu (per cell), dL/dU, x, lam) for the time-inner system J x = b."""
    x, lam = solve_and_adjoint(J, b, q)
    L = float(q @ x)
    g = -cell_contraction(lam, x, cell_sdofs, kb, refs, ref_ptr, ref_idx, ref_w, tw)
    g[in_cells] += U * cell_dot(lam, in_cells, cell_sdofs, kb, Fc)
    bh = F0.copy()
    for kk, c in enumerate(in_cells):
        sd = cell_sdofs[c].astype(np.int64)
        for i in range(kb):
            bh[sd * kb + i] += nu[c] * Fc[kk, :, i]
    gU = float(lam @ bh)
    return L, g, gU, x, lam


def transpose_levels(olevels):
    """The hierarchy of J^T: every level matrix transposed, the same cells and
    prolongations, the local inverses recomputed from the transposed blocks
    (the Vanka smoother of J^T); level 0 is solved directly."""
    from .smoother import OracleLevel, build_inverses
    out = [OracleLevel(L.J.T.tocsr(), L.dofs, L.n_st, L.P) for L in olevels]
    return build_inverses(out)
