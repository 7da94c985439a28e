"""Cell-based space-time Vanka smoother (Section 4.2, eqs. (4.3)-(4.6)), literally.

Vectors are time-inner, x[s (k+1) + l] for spatial DoF s and time DoF l.
The cell-local order of J_T is the paper's eq. (4.4): time-major, and within
one time DoF the velocity components (Q2 nodes, lexicographic) then the
pressure modes: local index = l * n_ls + alpha.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def spacetime_matrix(rowptr, col, val, n_sdofs: int, b: int) -> sp.csr_matrix:
    """Global level matrix J as scipy CSR (block (s, s') holds J[(s,i),(s',l)])."""
    bsr = sp.bsr_matrix((np.asarray(val).reshape(-1, b, b), np.asarray(col), np.asarray(rowptr)),
                        shape=(n_sdofs * b, n_sdofs * b))
    return bsr.tocsr()


def cell_dofs(cell_sdofs: np.ndarray, b: int) -> np.ndarray:
    """Global space-time DoFs of every cell in eq. (4.4) order: (n_cells, b * n_ls)."""
    nc, nls = cell_sdofs.shape
    out = np.empty((nc, b * nls), dtype=np.int64)
    for l in range(b):
        out[:, l * nls:(l + 1) * nls] = cell_sdofs.astype(np.int64) * b + l
    return out


def extract_cell_matrix(J: sp.csr_matrix, dofs: np.ndarray) -> np.ndarray:
    """J_T: the submatrix of the global level matrix on the cell's DoFs."""
    return J[dofs][:, dofs].toarray()


class SingularCell(Exception):
    pass


def cell_inverse(JT: np.ndarray) -> np.ndarray:
    """Explicit inverse of J_T through an LU factorisation with partial pivoting."""
    lu, piv = sla.lu_factor(JT, check_finite=True)
    if np.any(np.diag(lu) == 0.0):
        raise SingularCell("zero pivot")
    return sla.lu_solve((lu, piv), np.eye(JT.shape[0]))


@dataclass
class OracleLevel:
    J: sp.csr_matrix
    dofs: np.ndarray             # (n_cells, n_loc) eq. (4.4) order
    n_st: int
    P: sp.csr_matrix | None      # space-time prolongation (fine x coarse), None on level 0
    inv: list | None = None      # list of (n_loc x n_loc) inverses


def prepare_levels(levels, b: int):
    """Oracle view of a hierarchy given as ABI-shaped arrays (index 0 = coarsest).

    levels: sequence of objects/dicts with n_sdofs, rowptr, col, val, cell_sdofs, P.
    """
    out = []
    for L in levels:
        get = (lambda k: L[k]) if isinstance(L, dict) else (lambda k: getattr(L, k))
        ns = int(get("n_sdofs"))
        J = spacetime_matrix(get("rowptr"), get("col"), get("val"), ns, b)
        P = None
        Pt = get("P")
        if Pt is not None:
            prow, pcol, pval = Pt
            n_c = int(np.max(pcol)) + 1 if len(pcol) else 0
            Ps = sp.csr_matrix((pval, pcol, prow), shape=(ns, n_c))
            P = sp.kron(Ps, sp.identity(b), format="csr")   # identity in time
        out.append(OracleLevel(J, cell_dofs(np.asarray(get("cell_sdofs")), b), ns * b, P))
    # coarse column count of P must match the coarser level
    for g in range(1, len(out)):
        Pg = out[g].P
        if Pg.shape[1] != out[g - 1].n_st:
            Pg.resize((out[g].n_st, out[g - 1].n_st))
    return out


def build_inverses(olevels, first_level: int = 1):
    """Pre-compute J_T^-1 of every cell on every smoothed level (g >= 1)."""
    for g in range(first_level, len(olevels)):
        L = olevels[g]
        inv = []
        for T in range(L.dofs.shape[0]):
            try:
                inv.append(cell_inverse(extract_cell_matrix(L.J, L.dofs[T])))
            except SingularCell as e:
                raise SingularCell(f"level {g} cell {T}") from e
        L.inv = inv
    return olevels


def residual(J, r, d):
    """r - J d."""
    return r - J @ d


def vanka_sweep(L: OracleLevel, r, d, omega: float, pressure_rows=None):
    """One Jacobi-type sweep of S_T(d, r) = d_T + omega J_T^-1 (r - J d)_T.

    The global residual is computed once from the pre-sweep iterate; the
    cells are then visited in index order and each one overwrites its DoFs
    with d_old + omega J_T^-1 rho_T, so a DoF shared by several cells keeps
    the value written by the last cell of the loop.

    pressure_rows (ablation of eq. (4.5), not the default reading): a boolean
    mask of the level's pressure DoFs; when given, the residual is formed
    from r_0, the right-hand side with its pressure rows set to zero, as
    eq. (4.5)-(4.6) print it.  The default uses the full r.
    """
    if pressure_rows is not None:
        r = np.where(pressure_rows, 0.0, r)
    rho = residual(L.J, r, d)
    d_old = d
    d_new = d.copy()
    for T in range(L.dofs.shape[0]):
        idx = L.dofs[T]
        c = L.inv[T] @ rho[idx]
        d_new[idx] = d_old[idx] + omega * c
    return d_new


def vanka_sweep_combined(L: OracleLevel, r, d, omega: float, average: bool):
    """Alternative readings of the update of shared DoFs (not the paper's):
    every cell adds omega J_T^-1 rho_T to its DoFs; with average=True the sum
    at a DoF is divided by the number of cells containing it."""
    rho = residual(L.J, r, d)
    acc = np.zeros_like(d)
    mult = np.zeros_like(d)
    for T in range(L.dofs.shape[0]):
        idx = L.dofs[T]
        acc[idx] += omega * (L.inv[T] @ rho[idx])
        mult[idx] += 1.0
    return d + (acc / mult if average else acc)


def extract_cell_matrix_blocks(rowptr, col, val, b: int, sdofs) -> np.ndarray:
    """J_T read directly from the block rows of the level matrix (for single
    cells of large levels): entry (l*n_ls + a, m*n_ls + c) = block(sd[a], sd[c])[l, m];
    a pair absent from the block pattern is a zero block."""
    nls = len(sdofs)
    val = np.asarray(val).reshape(-1, b, b)
    out = np.zeros((b * nls, b * nls))
    for a, s in enumerate(sdofs):
        lo, hi = int(rowptr[s]), int(rowptr[s + 1])
        cols = np.asarray(col[lo:hi])
        for c, t in enumerate(sdofs):
            q = lo + int(np.searchsorted(cols, t))
            if q >= hi or col[q] != t:
                continue
            for l in range(b):
                for m in range(b):
                    out[l * nls + a, m * nls + c] = val[q, l, m]
    return out


def owner_cells(cell_sdofs: np.ndarray, n_sdofs: int) -> np.ndarray:
    """Cell whose update a spatial DoF keeps in the literal loop: the last one
    (highest index) that contains it."""
    own = np.full(n_sdofs, -1, dtype=np.int64)
    for T in range(cell_sdofs.shape[0]):
        own[cell_sdofs[T]] = T
    return own
