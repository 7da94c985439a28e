"""Newton linearisation of the space-time Navier-Stokes system of one
subinterval (input generation for the time-marching workload).

Unknowns: u = (v, p) with the dG(k) Radau-Lagrange basis in time, time-inner
vectors u[s (k+1) + l].  With the linear part of the operator (time
derivative and jump on the velocity mass, viscous, Nitsche and pressure terms
of eqs. (2.4)-(2.5)) J_lin = C (x) M + W_tau (x) A_lin, the residual is

  R(u)_i = (J_lin u)_i + tau sum_{l,m} T[i,l,m] c(v_l, v_m)_i - F_i,
  c(a, w)[psi] = <(a . grad) w, psi>,   T[i,l,m] = int_0^1 chi_i chi_l chi_m,

(the convection term integrated exactly in time) and the Newton Jacobian is

  J(u) = J_lin + tau sum_m T[i,l,m] N(v_m),
  N(w)[psi, phi] = <(w . grad) phi, psi> + <(phi . grad) w, psi>,

whose time blocks are full: the Oseen structure (time-diagonal spatial
operator) is the special case of a time-independent linearisation point.
F holds the data terms (force, Nitsche boundary data, outflow traction) and
the jump term chi_i(0) <v(t_{n-1}^-), psi>.
"""
from __future__ import annotations

import numpy as np

from . import fe
from .assemble import RefData, bsr_pattern, cell_operators, level_constant_parts, mass_operator
from .mesh import Mesh


def time_triple(k: int) -> np.ndarray:
    """T[i, l, m] = int_0^1 chi_i chi_l chi_m dt (Gauss rule exact for degree 3k)."""
    nodes, _, _, _ = fe.time_matrices(k)
    t, w = fe.gauss01(k + 2)
    X = fe.lagrange_eval(nodes, t)
    return np.einsum("q,qi,ql,qm->ilm", w, X, X, X)


class NewtonLevel:
    """Assembly of one level: pattern, linear part, convection operators."""

    def __init__(self, mesh: Mesh, k: int, tau: float, nu: float):
        self.mesh, self.k, self.tau, self.nu = mesh, k, tau, nu
        self.b = k + 1
        self.ref = RefData(mesh.dim)
        self.const = level_constant_parts(self.ref, mesh.h)
        self.Me = mass_operator(mesh, self.const)
        _, w, C, chi0 = fe.time_matrices(k)
        self.C, self.tw, self.chi0 = np.asarray(C), tau * np.asarray(w), np.asarray(chi0)
        self.T = time_triple(k)
        self.csd = mesh.cell_sdofs()
        self.rowptr, self.col = bsr_pattern(mesh, self.csd, "full")
        # block position of every (cell, alpha, beta): the pattern's (row, col)
        # keys are sorted (rows ascending, columns sorted within a row)
        nc, nls, ns = mesh.n_cells, mesh.n_ls, mesh.n_sdofs
        rows = np.repeat(np.arange(ns, dtype=np.int64), np.diff(self.rowptr))
        keys = rows * ns + self.col.astype(np.int64)
        want = self.csd[:, :, None].astype(np.int64) * ns + self.csd[:, None, :].astype(np.int64)
        self.pos = np.searchsorted(keys, want.reshape(-1)).reshape(nc, nls, nls)
        assert np.array_equal(keys[self.pos.reshape(-1)], want.reshape(-1))
        zero = lambda x: np.zeros_like(x)
        nu_cell = np.full(mesh.n_cells, float(nu))
        self.Alin = cell_operators(mesh, self.ref, self.const, nu_cell, zero, np.arange(nc))

    # ------------------------------------------------------------- fields
    def velocity_nodes(self, u: np.ndarray) -> np.ndarray:
        """(n_cells, nv, dim, b) nodal velocity values of each cell and time level."""
        d, nv, b = self.mesh.dim, self.ref.nv, self.b
        U = u.reshape(-1, b)
        out = np.empty((self.mesh.n_cells, nv, d, b))
        for c in range(d):
            out[:, :, c, :] = U[self.csd[:, c * nv:(c + 1) * nv]]
        return out

    def _at_quadrature(self, Vn):
        """Values (nc, nq, d, b) and gradients (nc, nq, d, d, b) [component,
        derivative] of the velocity at the cell quadrature points."""
        h = np.asarray(self.const["h"])
        phi = self.ref.phi                           # (nq, nv)
        dphi = self.ref.dphi / h[None, :, None]      # (nq, d, nv)
        val = np.einsum("qj,ejcl->eqcl", phi, Vn)
        grad = np.einsum("qaj,ejcl->eqcal", dphi, Vn)
        return val, grad

    # ------------------------------------------------------------- pieces
    def convection_vectors(self, Vn):
        """c(v_l, v_m) for every cell and time pair: (nc, nls, b, b) (velocity rows)."""
        d, nv, b = self.mesh.dim, self.ref.nv, self.b
        val, grad = self._at_quadrature(Vn)
        w = self.ref.wts * self.const["vol"]
        # (v_l . grad) v_m, component c: sum_a v_l,a d_a v_m,c
        cv = np.einsum("eqal,eqcam->eqclm", val, grad)
        out = np.zeros((self.mesh.n_cells, self.mesh.n_ls, b, b))
        for c in range(d):
            out[:, c * nv:(c + 1) * nv] = np.einsum("q,qi,eqlm->eilm", w, self.ref.phi, cv[:, :, c])
        return out

    def newton_operators(self, Vn):
        """N(v_m) for every cell and time level: (nc, nls, nls, b)."""
        d, nv, b = self.mesh.dim, self.ref.nv, self.b
        h = np.asarray(self.const["h"])
        val, grad = self._at_quadrature(Vn)
        w = self.ref.wts * self.const["vol"]
        phi = self.ref.phi
        dphi = self.ref.dphi / h[None, :, None]
        out = np.zeros((self.mesh.n_cells, self.mesh.n_ls, self.mesh.n_ls, b))
        # (w . grad) phi_j, same component
        adv = np.einsum("q,qi,eqam,qaj->eijm", w, phi, val, dphi)
        for c in range(d):
            sl = slice(c * nv, (c + 1) * nv)
            out[:, sl, sl, :] += adv
            # (phi e_c' . grad) w, component c: phi_j d_c' w_c
            for cp in range(d):
                slp = slice(cp * nv, (cp + 1) * nv)
                out[:, sl, slp, :] += np.einsum("q,qi,qj,eqm->eijm", w, phi, phi, grad[:, :, c, cp, :])
        return out

    # ------------------------------------------------------------- assembly
    def jacobian(self, u: np.ndarray) -> np.ndarray:
        """Block values (nnzb, b, b) of J(u) in the level's pattern."""
        b = self.b
        Vn = self.velocity_nodes(u)
        N = self.newton_operators(Vn)                        # (nc, a, c, m)
        # local blocks (nc, a, c, i, l)
        loc = np.einsum("il,ac->acil", self.C, self.Me)[None] \
            + np.einsum("i,il,eac->eacil", self.tw, np.eye(b), self.Alin) \
            + self.tau * np.einsum("ilm,eacm->eacil", self.T, N)
        val = np.zeros((int(self.rowptr[-1]), b, b))
        np.add.at(val, self.pos.reshape(-1), loc.reshape(-1, b, b))
        return val

    def residual(self, u: np.ndarray, F: np.ndarray) -> np.ndarray:
        """R(u) (time-inner) for the data vector F."""
        b = self.b
        Vn = self.velocity_nodes(u)
        cvec = self.convection_vectors(Vn)                   # (nc, a, l, m)
        U = u.reshape(-1, b)
        Ul = U[self.csd]                                     # (nc, a, l)
        lin = np.einsum("il,ac,ecl->eai", self.C, self.Me, Ul) \
            + np.einsum("i,eac,eci->eai", self.tw, self.Alin, Ul)
        conv = self.tau * np.einsum("ilm,ealm->eai", self.T, cvec)
        R = np.zeros(self.mesh.n_sdofs * b)
        for i in range(b):
            np.add.at(R, self.csd.reshape(-1).astype(np.int64) * b + i,
                      (lin[:, :, i] + conv[:, :, i]).reshape(-1))
        return R - F

    def jump_term(self, v_prev: np.ndarray) -> np.ndarray:
        """chi_i(0) <v(t_{n-1}^-), psi> for a spatial coefficient vector v_prev
        (velocity entries used; time-inner result)."""
        b = self.b
        loc = np.einsum("ac,ec->ea", self.Me, v_prev[self.csd])
        out = np.zeros(self.mesh.n_sdofs * b)
        for i in range(b):
            np.add.at(out, self.csd.reshape(-1).astype(np.int64) * b + i,
                      self.chi0[i] * loc.reshape(-1))
        return out


def inject(fine: Mesh, coarse: Mesh, u_fine: np.ndarray, b: int) -> np.ndarray:
    """Velocity of a fine space-time vector at the coarse Q2 nodes (each coarse
    node is a fine node); pressure entries zero."""
    d = fine.dim
    Xc = coarse.node_coords()
    hf = np.array(fine.h) / 2.0
    idx = fine.node_id(np.rint(Xc / hf[None, :]).astype(np.int64))
    Uf = u_fine.reshape(-1, b)
    out = np.zeros((coarse.n_sdofs, b))
    for c in range(d):
        out[np.arange(coarse.n_vnodes) * d + c] = Uf[idx * d + c]
    return out.reshape(-1)


class NewtonProblem:
    """A channel hierarchy for the time-marching workload: the Jacobian of
    every level at a given iterate (the iterate's velocity injected to the
    coarser levels), the residual and the data of each subinterval.

    Data: parabolic inflow of amplitude U(t) = U min(1, t / ramp) on x = 0,
    no-slip walls, do-nothing outflow, no force."""

    def __init__(self, dim, n_fine, n_levels, k, tau, nu, U=1.0, ramp=0.1):
        from .problem import L2D, H2D, L3D, H3D
        from .mesh import prolongation
        ext = (L2D, H2D) if dim == 2 else (L3D, H3D, H3D)
        meshes = [Mesh(dim, tuple(n_fine), ext)]
        for _ in range(n_levels - 1):
            meshes.append(meshes[-1].coarsen())
        self.meshes = meshes[::-1]
        self.dim, self.k, self.tau, self.nu, self.b = dim, k, tau, nu, k + 1
        self.U, self.ramp = U, ramp
        self.levels = [NewtonLevel(m, k, tau, nu) for m in self.meshes]
        self.P = [None] + [prolongation(self.meshes[g], self.meshes[g - 1])
                           for g in range(1, len(self.meshes))]

    @property
    def fine(self):
        return self.levels[-1]

    def inflow(self, X, t):
        from .adjoint import _profile
        amp = self.U * min(1.0, t / self.ramp) if self.ramp > 0 else self.U
        out = np.zeros_like(X)
        out[:, 0] = amp * _profile(X, self.meshes[-1].ext, self.dim)
        return out

    def data(self, t0: float, v_prev: np.ndarray) -> np.ndarray:
        """F of the subinterval (t0, t0 + tau] given v(t0^-) (spatial vector)."""
        from .rhs import assemble_rhs
        m = self.meshes[-1]
        zero = lambda X, t: np.zeros_like(X)
        F = assemble_rhs(m, self.k, self.tau, self.nu, t0, zero, self.inflow,
                         lambda X: np.zeros_like(X))
        return F + self.fine.jump_term(v_prev)

    def residual(self, u, F):
        return self.fine.residual(u, F)

    def hierarchy(self, u):
        """Level dicts (coarsest first) of the Jacobian at u."""
        out = []
        vals = [None] * len(self.levels)
        us = [None] * len(self.levels)
        us[-1] = u
        for g in range(len(self.levels) - 1, 0, -1):
            us[g - 1] = inject(self.meshes[g], self.meshes[g - 1], us[g], self.b)
        for g, L in enumerate(self.levels):
            vals[g] = L.jacobian(us[g])
            out.append(dict(n_sdofs=L.mesh.n_sdofs, rowptr=L.rowptr, col=L.col, val=vals[g],
                            cell_sdofs=L.csd, P=self.P[g]))
        return out

    def final_velocity(self, u):
        """v(t_n^-): the last time level (the right end point is a Radau node)."""
        return u.reshape(-1, self.b)[:, -1].copy()
