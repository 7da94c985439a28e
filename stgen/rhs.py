"""Right-hand side of Problem 3.1 from data (f, g, outflow traction, v(t_{n-1})).

For a velocity test function psi (component c) and time test index i:
  tau w_i [ <f(t_i), psi> + B_D(g(t_i), (psi, 0)) + <t_o(t_i), psi>_outflow ]
  + chi_i(0) <v_prev, psi>
and for a pressure test function xi:
  tau w_i [ <q(t_i), xi> - <g(t_i).n, xi>_D ]
where B_D is Nitsche's form of eq. (2.4), t_o a prescribed outflow traction
(zero for the do-nothing condition) and q a prescribed divergence (zero for
incompressible flow).  The Radau rule integrates these time integrals exactly
for data of degree <= k in time.  Vectors are time-inner, x[s (k+1) + i].
"""
from __future__ import annotations

import numpy as np

from . import fe
from .assemble import GAMMA1, GAMMA2, RefData, dirichlet_faces
from .mesh import Mesh


def assemble_rhs(mesh: Mesh, k: int, tau: float, nu: float, t0: float,
                 f, g, v_prev, traction=None, div=None):
    """f, g, traction: (x (n, d), t) -> (n, d);  v_prev: x -> (n, d);  div: (x, t) -> (n,)."""
    d = mesh.dim
    ref = RefData(d)
    tn, w, _, chi0 = fe.time_matrices(k)
    b = k + 1
    h = np.array(mesh.h)
    vol = float(np.prod(h))
    nv = ref.nv
    csd = mesh.cell_sdofs()
    ci = mesh.cell_index()
    F = np.zeros(mesh.n_sdofs * b)
    origin = ci * h[None, :]
    xq = origin[:, None, :] + ref.pts[None, :, :] * h[None, None, :]
    nc, nq = xq.shape[0], xq.shape[1]
    X = xq.reshape(-1, d)
    Wphi = ref.wts[:, None] * ref.phi * vol                  # (nq, nv)
    Wxi = ref.wts[:, None] * ref.xi * vol                    # (nq, d+1)
    loc = np.zeros((nc, mesh.n_ls, b))
    vp = v_prev(X).reshape(nc, nq, d)
    for i in range(b):
        ti = t0 + tau * tn[i]
        fi = f(X, ti).reshape(nc, nq, d)
        for c in range(d):
            loc[:, c * nv:(c + 1) * nv, i] += tau * w[i] * np.einsum("eq,qj->ej", fi[:, :, c], Wphi)
            loc[:, c * nv:(c + 1) * nv, i] += chi0[i] * np.einsum("eq,qj->ej", vp[:, :, c], Wphi)
        if div is not None:
            qi = div(X, ti).reshape(nc, nq)
            loc[:, d * nv:, i] += tau * w[i] * np.einsum("eq,qm->em", qi, Wxi)
    # boundary terms
    faces = [(fa, fs, "D") for (fa, fs) in dirichlet_faces(d)]
    if traction is not None:
        faces.append((0, 1, "O"))
    for (a, s, kind) in faces:
        pts, fw, fphi, fdphi, fxi = ref.faces[(a, s)]
        on = np.nonzero(ci[:, a] == (0 if s == 0 else mesh.n[a] - 1))[0]
        if on.size == 0:
            continue
        area = vol / h[a]
        sgn = 2.0 * s - 1.0
        xf = origin[on][:, None, :] + pts[None, :, :] * h[None, None, :]
        Xf = xf.reshape(-1, d)
        nf = xf.shape[1]
        wphi = (fw * area)[:, None] * fphi                 # (nf, nv)
        wdn = (fw * area)[:, None] * (sgn * fdphi[:, a, :] / h[a])
        wxi = (fw * area)[:, None] * fxi
        for i in range(b):
            ti = t0 + tau * tn[i]
            fac = tau * w[i]
            if kind == "D":
                gi = g(Xf, ti).reshape(on.size, nf, d)
                for c in range(d):
                    sl = slice(c * nv, (c + 1) * nv)
                    val = -nu * np.einsum("eq,qj->ej", gi[:, :, c], wdn)
                    val += (GAMMA1 * nu / h[a]) * np.einsum("eq,qj->ej", gi[:, :, c], wphi)
                    if c == a:
                        val += (GAMMA2 / h[a]) * np.einsum("eq,qj->ej", gi[:, :, a] * sgn * sgn, wphi)
                    loc[on, sl, i] += fac * val
                loc[on, d * nv:, i] -= fac * np.einsum("eq,qm->em", gi[:, :, a] * sgn, wxi)
            else:
                tr = traction(Xf, ti).reshape(on.size, nf, d)
                for c in range(d):
                    sl = slice(c * nv, (c + 1) * nv)
                    loc[on, sl, i] += fac * np.einsum("eq,qj->ej", tr[:, :, c], wphi)
    # scatter (time-inner)
    for i in range(b):
        np.add.at(F, csd.reshape(-1).astype(np.int64) * b + i, loc[:, :, i].reshape(-1))
    return F


def interpolate(mesh: Mesh, k: int, tau: float, t0: float, v, p_coeffs):
    """Coefficients (time-inner) of a velocity given by nodal values and of a
    pressure given per cell by its Legendre coefficients.

    v: (x (n, d), t) -> (n, d) evaluated at the Q2 nodes and Radau times.
    p_coeffs: (cell origins (nc, d), h, t) -> (nc, d+1) Legendre coefficients.
    """
    d = mesh.dim
    tn, _, _, _ = fe.time_matrices(k)
    b = k + 1
    X = mesh.node_coords()
    U = np.zeros(mesh.n_sdofs * b)
    origin = mesh.cell_origin()
    for i in range(b):
        ti = t0 + tau * tn[i]
        vv = v(X, ti)
        for c in range(d):
            U[(np.arange(mesh.n_vnodes) * d + c) * b + i] = vv[:, c]
        pc = p_coeffs(origin, np.array(mesh.h), ti)
        base = d * mesh.n_vnodes + np.arange(mesh.n_cells) * (d + 1)
        for m in range(d + 1):
            U[(base + m) * b + i] = pc[:, m]
    return U
