"""Assembly of the space-time Oseen Jacobian of one subinterval on one level.

Operator (Problem 3.1 with the semilinear form A_h of eq. (2.5), linearised at
a given convection field b: the Oseen reading, and Nitsche's boundary form of
eq. (2.4) with gamma_1 = gamma_2 = 35):
  velocity-velocity  <(b.grad) v, psi> + nu <grad v, grad psi>
                     - <nu d_n v, psi>_D - <v, nu d_n psi>_D
                     + gamma_1 nu / h <v, psi>_D + gamma_2 / h <v.n, psi.n>_D
  pressure in momentum  -<p, div psi> + <p, psi.n>_D
  continuity            <div v, xi>  - <v.n, xi>_D
on the Dirichlet boundary D = inflow (x = 0) and walls; the outflow x = L
carries no term (do-nothing).  h is the cell extent normal to the face.
In time, block (i, l) of the spatial pair is C[i,l] M + delta_il tau w_i A
(time derivative + jump on the velocity mass M; Radau-exact time integral of A).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import fe
from ._native import lib
from .mesh import Mesh

GAMMA1 = 35.0
GAMMA2 = 35.0


class RefData:
    """Quadrature tables of one spatial dimension (cell and faces)."""

    def __init__(self, dim: int, nq1: int = 4):
        self.dim = dim
        self.pts, self.wts = fe.tensor_rule(dim, nq1)
        self.phi, self.dphi = fe.q2_tab(dim, self.pts)
        self.xi = fe.p1disc_tab(dim, self.pts)
        self.nv = 3 ** dim
        self.faces = {}
        if dim > 1:
            fp, fw = fe.tensor_rule(dim - 1, nq1)
        else:
            fp, fw = np.zeros((1, 0)), np.ones(1)
        for a in range(dim):
            for s in (0, 1):
                pts = np.zeros((fp.shape[0], dim))
                others = [c for c in range(dim) if c != a]
                for j, c in enumerate(others):
                    pts[:, c] = fp[:, j]
                pts[:, a] = float(s)
                phi, dphi = fe.q2_tab(dim, pts)
                xi = fe.p1disc_tab(dim, pts)
                self.faces[(a, s)] = (pts, fw, phi, dphi, xi)


def dirichlet_faces(dim: int):
    """Dirichlet faces (axis, side): inflow x = 0 and all walls; outflow x = L is free."""
    out = [(0, 0)]
    for a in range(1, dim):
        out += [(a, 0), (a, 1)]
    return out


def level_constant_parts(ref: RefData, h):
    """Cell matrices that are the same for every cell of a uniform level.

    Returns dict with Mv (3^d x 3^d velocity mass), Kv (stiffness without nu),
    Bd (dim x (d+1) x 3^d, entries int xi_m d_c phi_j) and the Nitsche face
    pieces per Dirichlet face type.
    """
    d = ref.dim
    h = np.asarray(h, dtype=np.float64)
    vol = float(np.prod(h))
    w = ref.wts * vol
    phi, dphi = ref.phi, ref.dphi / h[None, :, None]
    Mv = np.einsum("q,qi,qj->ij", w, phi, phi)
    Kv = np.einsum("q,qci,qcj->ij", w, dphi, dphi)
    Bd = np.einsum("q,qm,qcj->cmj", w, ref.xi, dphi)
    faces = {}
    for (a, s) in dirichlet_faces(d):
        pts, fw, fphi, fdphi, fxi = ref.faces[(a, s)]
        area = vol / h[a]
        ww = fw * area
        sgn = 2.0 * s - 1.0                     # outward normal = sgn * e_a
        dn = sgn * fdphi[:, a, :] / h[a]        # normal derivative of each phi
        Fm = np.einsum("q,qi,qj->ij", ww, fphi, fphi)
        Fdn = np.einsum("q,qi,qj->ij", ww, fphi, dn)      # int phi_i d_n phi_j
        Fp = np.einsum("q,qm,qj->mj", ww, fxi, fphi)      # int xi_m phi_j
        faces[(a, s)] = dict(Fm=Fm, Fdn=Fdn, Fp=Fp, sgn=sgn, hF=h[a])
    return dict(Mv=Mv, Kv=Kv, Bd=Bd, faces=faces, vol=vol, h=h)


def cell_operators(mesh: Mesh, ref: RefData, const, nu_cell, conv, cells):
    """Spatial Oseen operators Ae (len(cells) x n_ls x n_ls) for a chunk of cells.

    nu_cell: viscosity per cell (array over all cells).  conv(x) -> b at
    physical points x (npts, d).  Row = test function, column = trial function.
    """
    d = mesh.dim
    nv = ref.nv
    nls = mesh.n_ls
    h = const["h"]
    ci = mesh.cell_index()[cells]
    origin = ci * h[None, :]
    nc = len(cells)
    # convection: Conv[e, i, j] = sum_q w |T| phi_i(q) (b(x_q) . grad phi_j(q))
    xq = origin[:, None, :] + ref.pts[None, :, :] * h[None, None, :]      # (nc, nq, d)
    bq = conv(xq.reshape(-1, d)).reshape(nc, -1, d)
    dphi = ref.dphi / h[None, :, None]                                    # (nq, d, nv)
    U = np.einsum("eqc,qcj->eqj", bq, dphi)                               # (nc, nq, nv)
    Wphi = (ref.wts * const["vol"])[:, None] * ref.phi                    # (nq, nv)
    Conv = np.matmul(Wphi.T[None, :, :], U)                               # (nc, nv, nv)
    nu = np.asarray(nu_cell, dtype=np.float64)[cells]
    A = np.zeros((nc, nls, nls))
    pv = d * nv
    for c in range(d):
        sl = slice(c * nv, (c + 1) * nv)
        A[:, sl, sl] = Conv + nu[:, None, None] * const["Kv"][None]
        # momentum row (test comp c, node i), pressure trial m: -int xi_m d_c phi_i
        A[:, sl, pv:] = -const["Bd"][c].T[None]
        # continuity row m, velocity trial comp c node j: +int xi_m d_c phi_j
        A[:, pv:, sl] = const["Bd"][c][None]
    # Nitsche on Dirichlet faces
    for (a, s), F in const["faces"].items():
        on = ci[:, a] == (0 if s == 0 else mesh.n[a] - 1)
        if not np.any(on):
            continue
        idx = np.nonzero(on)[0]
        nu_f = nu[idx][:, None, None]
        vv = -F["Fdn"] - F["Fdn"].T + (GAMMA1 / F["hF"]) * F["Fm"]        # times nu
        for c in range(d):
            sl = slice(c * nv, (c + 1) * nv)
            add = nu_f * vv[None]
            if c == a:
                add = add + (GAMMA2 / F["hF"]) * F["Fm"][None]
                # momentum row comp a, pressure trial m: + int xi_m phi_i n_a
                A[idx, sl, pv:] += F["sgn"] * F["Fp"].T[None]
                # continuity row m, trial comp a: - int xi_m phi_j n_a
                A[idx, pv:, sl] -= F["sgn"] * F["Fp"][None]
            A[np.ix_(idx, np.arange(sl.start, sl.stop), np.arange(sl.start, sl.stop))] += add
    return A


def mass_operator(mesh: Mesh, const):
    """n_ls x n_ls velocity mass (component-diagonal); zero on pressure."""
    nv = 3 ** mesh.dim
    M = np.zeros((mesh.n_ls, mesh.n_ls))
    for c in range(mesh.dim):
        sl = slice(c * nv, (c + 1) * nv)
        M[sl, sl] = const["Mv"]
    return M


def dof_kinds(mesh: Mesh) -> np.ndarray:
    """Kind of each spatial DoF: velocity component 0..dim-1, or dim for pressure."""
    d = mesh.dim
    kind = np.full(mesh.n_sdofs, d, dtype=np.uint8)
    kind[: d * mesh.n_vnodes] = np.tile(np.arange(d, dtype=np.uint8), mesh.n_vnodes)
    return kind


def coupling_table(dim: int, pattern: str) -> np.ndarray:
    """Which kinds couple.  'full': every pair of DoFs sharing a cell.
    'oseen': drop the blocks the Oseen operator leaves structurally zero
    (different velocity components, pressure-pressure)."""
    if pattern == "full":
        return np.ones((dim + 1, dim + 1), dtype=np.uint8)
    if pattern == "oseen":
        t = np.eye(dim + 1, dtype=np.uint8)
        t[:dim, dim] = 1
        t[dim, :dim] = 1
        t[dim, dim] = 0
        return t
    raise ValueError(pattern)


def bsr_pattern(mesh: Mesh, cell_sdofs: np.ndarray, pattern: str = "oseen"):
    """Block-row pattern: pairs of spatial DoFs sharing a cell whose kinds
    couple (sorted columns)."""
    L = lib()
    ns, nc, nls = mesh.n_sdofs, mesh.n_cells, mesh.n_ls
    csd = np.ascontiguousarray(cell_sdofs, dtype=np.int32)
    kind = dof_kinds(mesh)
    table = np.ascontiguousarray(coupling_table(mesh.dim, pattern))
    bound = np.zeros(ns, dtype=np.int64)
    L.stgen_row_bounds(ns, nc, nls, csd.ctypes.data, bound.ctypes.data)
    bptr = np.zeros(ns + 1, dtype=np.int64)
    np.cumsum(bound, out=bptr[1:])
    scratch = np.empty(int(bptr[-1]), dtype=np.int32)
    fill = np.empty(ns, dtype=np.int64)
    rowptr = np.empty(ns + 1, dtype=np.int64)
    L.stgen_pattern(ns, nc, nls, csd.ctypes.data, bptr.ctypes.data, kind.ctypes.data,
                    mesh.dim + 1, table.ctypes.data, scratch.ctypes.data, fill.ctypes.data,
                    rowptr.ctypes.data)
    col = scratch[: int(rowptr[-1])].copy()
    del scratch
    return rowptr, col


def assemble_level(mesh: Mesh, k: int, tau: float, nu_cell, conv, chunk: int = 4096,
                   pattern: str = "oseen"):
    """Space-time block-sparse Jacobian of one level.

    pattern 'oseen' stores only the blocks the Oseen operator can make nonzero;
    'full' stores every pair of DoFs sharing a cell (explicit zeros included).
    Returns dict(rowptr int64, col int32, val float64 (nnzb, b, b), cell_sdofs).
    """
    ref = RefData(mesh.dim)
    const = level_constant_parts(ref, mesh.h)
    Me = mass_operator(mesh, const)
    _, w, C, _ = fe.time_matrices(k)
    b = k + 1
    tw = np.ascontiguousarray(tau * w)
    Ct = np.ascontiguousarray(C)
    csd = mesh.cell_sdofs()
    rowptr, col = bsr_pattern(mesh, csd, pattern)
    nnzb = int(rowptr[-1])
    val = np.zeros((nnzb, b, b))
    colour = mesh.colours()
    L = lib()
    nls = mesh.n_ls
    dropped = np.zeros(1, dtype=np.int64)
    for c0 in range(0, mesh.n_cells, chunk):
        cells = np.arange(c0, min(mesh.n_cells, c0 + chunk))
        Ae = np.ascontiguousarray(cell_operators(mesh, ref, const, nu_cell, conv, cells))
        L.stgen_scatter(nls, b, csd.ctypes.data, c0, len(cells), colour.ctypes.data, 1 << mesh.dim,
                        Ae.ctypes.data, Me.ctypes.data, Ct.ctypes.data, tw.ctypes.data,
                        rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, dropped.ctypes.data)
        if dropped[0]:
            raise RuntimeError(f"pattern '{pattern}' drops {dropped[0]} nonzero entries")
    return dict(rowptr=rowptr, col=col, val=val, cell_sdofs=csd)


def assemble_spatial_factors(mesh: Mesh, nu_cell, conv, rowptr, col, chunk: int = 4096):
    """Spatial factors of the level matrix in its block pattern: every block
    (i, l) of the space-time matrix is C[i, l] M + delta_il tau w_i A, with M
    the velocity mass and A the spatial Oseen operator of the same cells.
    Returns (mval, aval), one value per block of the pattern (rowptr, col)."""
    ref = RefData(mesh.dim)
    const = level_constant_parts(ref, mesh.h)
    Me = mass_operator(mesh, const)
    csd = mesh.cell_sdofs()
    colour = mesh.colours()
    L = lib()
    nls = mesh.n_ls
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    nnzb = int(rp[-1])
    mval = np.zeros(nnzb)
    aval = np.zeros(nnzb)
    dropped = np.zeros(1, dtype=np.int64)
    one, zero = np.ones(1), np.zeros(1)
    Z = np.zeros((nls, nls))
    for c0 in range(0, mesh.n_cells, chunk):
        cells = np.arange(c0, min(mesh.n_cells, c0 + chunk))
        Ae = np.ascontiguousarray(cell_operators(mesh, ref, const, nu_cell, conv, cells))
        Zc = np.zeros_like(Ae)
        # b = 1 scatter: C = 1, tau w = 0 gives M; C = 0, tau w = 1 gives A
        L.stgen_scatter(nls, 1, csd.ctypes.data, c0, len(cells), colour.ctypes.data, 1 << mesh.dim,
                        Zc.ctypes.data, Me.ctypes.data, one.ctypes.data, zero.ctypes.data,
                        rp.ctypes.data, cl.ctypes.data, mval.ctypes.data, dropped.ctypes.data)
        L.stgen_scatter(nls, 1, csd.ctypes.data, c0, len(cells), colour.ctypes.data, 1 << mesh.dim,
                        Ae.ctypes.data, Z.ctypes.data, zero.ctypes.data, one.ctypes.data,
                        rp.ctypes.data, cl.ctypes.data, aval.ctypes.data, dropped.ctypes.data)
        if dropped[0]:
            raise RuntimeError("the block pattern drops nonzero factor entries")
    return mval, aval
