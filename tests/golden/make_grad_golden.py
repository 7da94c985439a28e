"""Writes grad_256x64_dG1.txt: the oracle's adjoint gradient of the outflow
loss for the differentiation workload (2d 256x64 cells, 5 levels, dG(1),
tau = 0.01, seed 3000, U = 1), at 200 cells drawn with seed 7 plus the loss
and dL/dU.  Calls only the generator and the oracle (about a minute)."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import adjoint as oadj                # noqa: E402
from oracle.smoother import spacetime_matrix      # noqa: E402
from stgen import adjoint as gadj                 # noqa: E402


def main():
    p = gadj.make_differentiation_problem((256, 64), 5, 1, 0.01, 3000)
    m = p.levels[-1].mesh
    L = p.levels[-1]
    J = spacetime_matrix(L.rowptr, L.col, L.val, L.n_sdofs, p.b)
    refs, ptr, idx, w = gadj.nu_derivative_refs(m)
    F0, cells, Fc = gadj.inflow_rhs_parts(m, p.k, p.tau)
    Lv, g, gU, _, _ = oadj.loss_gradient(J, p.rhs, p.loss, 1.0, p.nu_cell, m.cell_sdofs(), p.b,
                                         refs, ptr, idx, w, gadj.time_weights(p.k, p.tau), F0,
                                         cells, Fc)
    rng = np.random.default_rng(7)
    sample = np.sort(np.concatenate([rng.choice(m.n_cells, 190, replace=False), cells[:10]]))
    sample = np.unique(sample)
    with open(os.path.join(HERE, "grad_256x64_dG1.txt"), "w") as f:
        f.write("# oracle adjoint gradient, 2d 256x64 dG(1) 5 levels, tau 0.01, seed 3000, U 1\n")
        f.write("# written by make_grad_golden.py (generator + oracle only)\n")
        f.write(f"loss {Lv:.17e}\n")
        f.write(f"dL_dU {gU:.17e}\n")
        f.write(f"max_abs_grad {np.abs(g).max():.17e}\n")
        for c in sample:
            f.write(f"{int(c)} {g[c]:.17e}\n")


if __name__ == "__main__":
    main()
