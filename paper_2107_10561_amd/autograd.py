"""Differentiable space-time solve.

SpaceTimeSolve.apply(nu, U, data, opts) returns x with J(nu) x = b(nu, U) on
the finest level, solved by the library's FGMRES + Vanka-GMG.  Its backward
pass solves the adjoint system J^T lam = dL/dx with the transposed
Vanka-GMG (the stored inverses read transposed) and forms

  dL/dnu_c = -lam_c^T (W_tau (x) K_c) x_c + U lam_c^T F_c,
  dL/dU    = lam^T (F_0 + sum_c nu_c F_c),

for an operator affine in each cell's viscosity, J = J_0 + sum_c nu_c
(W_tau (x) K_c), and a right-hand side b = U (F_0 + sum_c nu_c F_c).  The
right-hand side is assembled on the device (stv_cell_scatter) and the
gradient of every cell in one device pass (stv_cell_gradient).  `data`
describes the problem (attributes below); the hierarchy for a given
viscosity comes from data.build(nu).
"""
from __future__ import annotations

import numpy as np
import torch

from . import Solver


class AdjointData:
    """Problem description for SpaceTimeSolve.

    build(nu) -> list of levels, coarsest first, for the
    per-cell viscosity nu of the finest level; dim, k; refs (R, n_ls, n_ls),
    kptr, kidx, kw (K_c per finest cell), tw (time weights of K_c); F0
    (time-inner vector), in_cells, Fc (n_in, n_ls, k+1): the right-hand side
    for U = 1.
    """

    def __init__(self, build, dim, k, refs, kptr, kidx, kw, tw, F0, in_cells, Fc):
        self.build, self.dim, self.k = build, dim, k
        self.refs, self.kptr, self.kidx, self.kw, self.tw = refs, kptr, kidx, kw, tw
        self.F0, self.in_cells, self.Fc = F0, np.asarray(in_cells, np.int32), Fc

    def fc_rows(self):
        """F_c of the listed cells as rows in the cell-local order alpha*(k+1) + l."""
        return np.ascontiguousarray(self.Fc.reshape(len(self.in_cells), -1))


class SolveOptions:
    def __init__(self, device=0, fp32=False, rtol=1e-10, restart=30, max_it=1000):
        self.device, self.fp32, self.rtol = device, fp32, rtol
        self.restart, self.max_it = restart, max_it
        self.solver = None
        self.last_info = {}
        # the forward call whose hierarchy and inverses the solver holds
        self.loaded = None


class SpaceTimeSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, nu, U, data, opts):
        nu_h = nu.detach().cpu().numpy().astype(np.float64)
        U_h = float(U.detach().cpu())
        levels = data.build(nu_h)
        if opts.solver is None:
            opts.solver = Solver(opts.device)
        s = opts.solver
        s.set_hierarchy(levels, data.dim, data.k)
        s.build_cell_inverses(fp32=opts.fp32, full=True)
        token = object()
        opts.loaded = token
        ctx.token, ctx.nu_h, ctx.fp32 = token, nu_h, opts.fp32
        csd = np.asarray(levels[-1].cell_sdofs)
        dev = torch.device("cuda", opts.device)
        # F0 + sum_c nu_c F_c on the device
        G = s.n_levels - 1
        bh = torch.from_numpy(np.ascontiguousarray(data.F0, dtype=np.float64)).to(dev)
        s.cell_scatter(G, data.in_cells, nu_h[data.in_cells], data.fc_rows(), bh)
        b = U_h * bh
        x = torch.zeros_like(b)
        info = s.gmres_solve(b, x, restart=opts.restart, max_it=opts.max_it, rtol=opts.rtol)
        opts.last_info["forward"] = info
        ctx.save_for_backward(x, bh)
        ctx.data, ctx.opts, ctx.U, ctx.nu_dev, ctx.nu_dtype = data, opts, U_h, nu.device, nu.dtype
        ctx.n_cells = csd.shape[0]
        return x

    @staticmethod
    def backward(ctx, gx):
        x, bh = ctx.saved_tensors
        data, opts, s = ctx.data, ctx.opts, ctx.opts.solver
        if opts.loaded is not ctx.token:
            # another forward has replaced the operator since this one ran:
            # reload J(nu) of this forward before the adjoint solve
            s.set_hierarchy(data.build(ctx.nu_h), data.dim, data.k)
            s.build_cell_inverses(fp32=ctx.fp32, full=True)
            opts.loaded = ctx.token
        lam = torch.zeros_like(x)
        info = s.gmres_solve_transposed(gx.contiguous().to(torch.float64), lam,
                                        restart=opts.restart, max_it=opts.max_it, rtol=opts.rtol)
        opts.last_info["adjoint"] = info
        G = s.n_levels - 1
        # -lam_c^T (W (x) K_c) x_c + U lam_c^T F_c for every cell, one device pass
        grad_nu = torch.empty(ctx.n_cells, dtype=torch.float64, device=x.device)
        s.cell_gradient(G, lam, x, data.refs, data.kptr, data.kidx, data.kw, data.tw, -1.0,
                        data.in_cells, data.fc_rows(), ctx.U, grad_nu)
        gU = s.dot(lam, bh)[0]
        return (grad_nu.to(ctx.nu_dev, ctx.nu_dtype),
                torch.tensor(gU, dtype=torch.float64), None, None)
