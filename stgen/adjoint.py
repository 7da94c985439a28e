"""Problem data of the differentiation workload (input generation only).

The operator of one level is affine in the viscosity of each cell:
  J(nu) = J_0 + sum_c nu_c (W_tau (x) K_c),   W_tau = diag(tau w_i),
where K_c is the spatial n_ls x n_ls derivative of cell c's element matrix:
the velocity stiffness plus, on each Dirichlet face of the cell, the
viscosity-proportional Nitsche terms (eq. (2.4)): -<d_n v, psi> - <v, d_n psi>
+ gamma_1 / h <v, psi>, all component-diagonal.  K_c is returned as a sum of
shared reference matrices (one for the interior, one per Dirichlet face type).

The right-hand side of a start from rest with a parabolic inflow profile
g = U (prod_a 4 x_a (H_a - x_a) / H_a^2, 0, ...) on x = 0 (zero on the walls)
is U (F_0 + sum_c nu_c F_c): F_c is the viscosity-proportional Nitsche data
term of inflow cell c (-<g, d_n psi> + gamma_1 / h <g, psi>), F_0 the rest
(gamma_2 / h <g.n, psi.n> and the continuity term -<g.n, xi>).

The loss is the weighted outflow flux of the first velocity component over
the subinterval, L(x) = int_{I_n} int_{x = L} w v_1 ds dt with the same
parabolic weight w, a linear functional L(x) = q . x.
"""
from __future__ import annotations

import numpy as np

from . import fe
from .assemble import GAMMA1, GAMMA2, RefData, dirichlet_faces, level_constant_parts
from .mesh import Mesh


def _profile(x, ext, dim):
    """prod over the transverse axes of 4 x_a (H_a - x_a) / H_a^2."""
    w = np.ones(x.shape[0])
    for a in range(1, dim):
        H = ext[a]
        w = w * 4.0 * x[:, a] * (H - x[:, a]) / (H * H)
    return w


def nu_derivative_refs(mesh: Mesh):
    """Reference matrices and their use per cell.

    Returns (refs (R, n_ls, n_ls), ref_ptr (n_cells+1), ref_idx, ref_w): cell c
    has K_c = sum_{e in [ref_ptr[c], ref_ptr[c+1])} ref_w[e] refs[ref_idx[e]].
    refs[0] is the interior stiffness, refs[1 + f] the Nitsche viscosity terms
    of Dirichlet face type f (in the order of dirichlet_faces).
    """
    d = mesh.dim
    ref = RefData(d)
    const = level_constant_parts(ref, mesh.h)
    nv, nls = ref.nv, mesh.n_ls
    faces = dirichlet_faces(d)
    refs = np.zeros((1 + len(faces), nls, nls))
    for c in range(d):
        sl = slice(c * nv, (c + 1) * nv)
        refs[0, sl, sl] = const["Kv"]
        for f, key in enumerate(faces):
            F = const["faces"][key]
            refs[1 + f, sl, sl] = -F["Fdn"] - F["Fdn"].T + (GAMMA1 / F["hF"]) * F["Fm"]
    ci = mesh.cell_index()
    ptr = [0]
    idx, wts = [], []
    for cell in range(mesh.n_cells):
        idx.append(0)
        wts.append(1.0)
        for f, (a, s) in enumerate(faces):
            if ci[cell, a] == (0 if s == 0 else mesh.n[a] - 1):
                idx.append(1 + f)
                wts.append(1.0)
        ptr.append(len(idx))
    return refs, np.array(ptr, np.int32), np.array(idx, np.int32), np.array(wts)


def time_weights(k: int, tau: float):
    """tau w_i of the right-Radau rule (the time factor of every term of A)."""
    _, w, _, _ = fe.time_matrices(k)
    return tau * np.asarray(w, dtype=np.float64)


def inflow_rhs_parts(mesh: Mesh, k: int, tau: float):
    """(F0 global time-inner vector, inflow cells, Fc (n_in, n_ls, b) local
    vectors in the spatial order of eq. (4.4), time-inner) for U = 1."""
    d = mesh.dim
    ref = RefData(d)
    tw = time_weights(k, tau)
    b = k + 1
    h = np.array(mesh.h)
    vol = float(np.prod(h))
    nv = ref.nv
    ci = mesh.cell_index()
    csd = mesh.cell_sdofs()
    origin = ci * h[None, :]
    a, s = 0, 0
    pts, fw, fphi, fdphi, fxi = ref.faces[(a, s)]
    on = np.nonzero(ci[:, a] == 0)[0]
    area = vol / h[a]
    sgn = 2.0 * s - 1.0
    xf = origin[on][:, None, :] + pts[None, :, :] * h[None, None, :]
    gq = _profile(xf.reshape(-1, d), mesh.ext, d).reshape(on.size, -1)   # g_0 at face points
    wphi = (fw * area)[:, None] * fphi
    wdn = (fw * area)[:, None] * (sgn * fdphi[:, a, :] / h[a])
    wxi = (fw * area)[:, None] * fxi
    Fc = np.zeros((on.size, mesh.n_ls, b))
    F0loc = np.zeros((on.size, mesh.n_ls, b))
    sl = slice(a * nv, (a + 1) * nv)     # only the normal component carries data
    nuterm = -np.einsum("eq,qj->ej", gq, wdn) + (GAMMA1 / h[a]) * np.einsum("eq,qj->ej", gq, wphi)
    free = (GAMMA2 / h[a]) * np.einsum("eq,qj->ej", gq * sgn * sgn, wphi)
    pres = -np.einsum("eq,qm->em", gq * sgn, wxi)
    for i in range(b):
        Fc[:, sl, i] = tw[i] * nuterm
        F0loc[:, sl, i] = tw[i] * free
        F0loc[:, d * nv:, i] = tw[i] * pres
    F0 = np.zeros(mesh.n_sdofs * b)
    for i in range(b):
        np.add.at(F0, csd[on].reshape(-1).astype(np.int64) * b + i, F0loc[:, :, i].reshape(-1))
    return F0, on.astype(np.int32), Fc


def physical_rhs(mesh: Mesh, k: int, tau: float, nu_cell, U: float = 1.0):
    """b = U (F0 + sum_c nu_c Fc), time-inner."""
    F0, cells, Fc = inflow_rhs_parts(mesh, k, tau)
    b = k + 1
    out = F0.copy()
    csd = mesh.cell_sdofs()
    nu = np.asarray(nu_cell, dtype=np.float64)
    for i in range(b):
        np.add.at(out, csd[cells].reshape(-1).astype(np.int64) * b + i,
                  (nu[cells][:, None] * Fc[:, :, i]).reshape(-1))
    return U * out


def outflow_loss_vector(mesh: Mesh, k: int, tau: float):
    """q with L(x) = q . x = int_{I_n} int_{x = L} w(y) v_1 ds dt (time-inner)."""
    d = mesh.dim
    ref = RefData(d)
    tw = time_weights(k, tau)
    b = k + 1
    h = np.array(mesh.h)
    vol = float(np.prod(h))
    ci = mesh.cell_index()
    csd = mesh.cell_sdofs()
    origin = ci * h[None, :]
    pts, fw, fphi, _, _ = ref.faces[(0, 1)]
    on = np.nonzero(ci[:, 0] == mesh.n[0] - 1)[0]
    xf = origin[on][:, None, :] + pts[None, :, :] * h[None, None, :]
    wq = _profile(xf.reshape(-1, d), mesh.ext, d).reshape(on.size, -1)
    loc = np.einsum("eq,q,qj->ej", wq, fw * (vol / h[0]), fphi)      # component 0 nodes
    q = np.zeros(mesh.n_sdofs * b)
    nv = ref.nv
    for i in range(b):
        np.add.at(q, csd[on][:, :nv].reshape(-1).astype(np.int64) * b + i,
                  tw[i] * loc.reshape(-1))
    return q


def make_differentiation_problem(n_fine=(256, 64), n_levels=5, k=1, tau=0.01, seed=3000,
                                 U=1.0, nu=None):
    """The differentiation workload: seeded convection (amplitudes drawn
    first), per-cell viscosity nu_c = 1e-3 exp(0.3 z_c) on the finest level
    (coarser levels: mean of the children), the physical right-hand side and
    the outflow loss vector.  nu overrides the drawn viscosity."""
    from .problem import L2D, H2D, L3D, H3D, Convection, Problem, make_hierarchy
    dim = len(n_fine)
    rng = np.random.default_rng(seed)
    ext = (L2D, H2D) if dim == 2 else (L3D, H3D, H3D)
    amps = rng.standard_normal(4) if dim == 2 else rng.standard_normal((4, 3))
    conv = Convection(dim, ext, amps).normalise()
    fine = Mesh(dim, tuple(n_fine), ext)
    if nu is None:
        nu = 1e-3 * np.exp(0.3 * rng.standard_normal(fine.n_cells))
    nu = np.asarray(nu, dtype=np.float64)
    levels = make_hierarchy(dim, n_fine, n_levels, k, tau, 1e-3, conv, ext, nu_cell_fine=nu)
    mesh = levels[-1].mesh
    rhs = physical_rhs(mesh, k, tau, nu, U)
    p = Problem(dim, k, tau, 1e-3, levels, rhs, conv,
                meta=dict(seed=seed, n_fine=tuple(n_fine), n_levels=n_levels, U=U))
    p.nu_cell = nu
    p.loss = outflow_loss_vector(mesh, k, tau)
    return p


def add_cell_derivative(level, cell: int, dnu: float, refs, ref_ptr, ref_idx, ref_w, tw):
    """Block values of the level matrix with cell's viscosity raised by dnu
    (J is affine in nu_c: J + dnu (W_tau (x) K_c)); returns a new val array."""
    val = np.array(level.val, copy=True)
    K = sum(ref_w[e] * refs[ref_idx[e]] for e in range(ref_ptr[cell], ref_ptr[cell + 1]))
    sd = level.cell_sdofs[cell]
    rp, col = level.rowptr, level.col
    W = np.diag(tw)
    for a in range(sd.size):
        r = sd[a]
        cols = col[rp[r]:rp[r + 1]]
        for bb in range(sd.size):
            if K[a, bb] == 0.0:
                continue
            q = rp[r] + np.searchsorted(cols, sd[bb])
            assert q < rp[r + 1] and col[q] == sd[bb]
            val[q] += dnu * K[a, bb] * W
    return val
