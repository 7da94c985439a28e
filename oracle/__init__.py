"""Plain FP64 CPU oracle of the space-time Vanka-GMG-FGMRES hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the entry module
and the CPU-baseline leg of the benchmark may import this package.  It shares
no code with the HIP library: it reads the same level data (block-sparse
space-time Jacobians, cell->DoF maps, prolongations) and computes everything
again with numpy / scipy, slowly and literally.

Functions and what pins them (tests marked "not gpu"):
  spacetime_matrix, cell_dofs       - pinned by the patch test of the assembly
                                      (J U = F for exact discrete data)
  cell_inverse, build_inverses      - pinned: J_T^-1 J_T = I to 1e-12, every
                                      cell of every smoothed level
  vanka_sweep_combined              - pinned: disjoint cells -> exact solve for both
                                      readings; hand-derived two-cell example
  extract_cell_matrix_blocks        - pinned: equals extract_cell_matrix on C1
  vanka_sweep                       - pinned: one cell, omega = 1 -> exact solve;
                                      disjoint cells -> exact solve; a hand-derived
                                      two-cell overwrite example
  vanka_sweep(pressure_rows=...)    - the eq. (4.5) ablation (r_0 with zeroed pressure
                                      rows): pinned to break the fixed point and the
                                      one-cell exact solve, and to agree with the full-r
                                      sweep when r has zero pressure rows
  coarse_inverse                    - pinned: a hand-inverted 3x3 that needs pivoting
                                      and has a non-symmetric inverse; two-sided
                                      inverse of the coarse Oseen matrix
  vcycle                            - pinned: one level = direct solve; no smoothing
                                      = coarse-grid correction P J_c^-1 P^T r;
                                      linearity in r
  fgmres                            - pinned: identity preconditioner reproduces
                                      scipy's GMRES residual history; minimal
                                      residual over the explicit Krylov space;
                                      restart >= n converges in <= n steps
  The assembled operators these functions read come from the seeded
  generator (stgen), pinned separately: closed-form element and time
  matrices, patch tests, and manufactured-solution convergence rates
  (velocity L2 order 3, pressure L2 order 2) on three nested meshes.
  The cell loop order and the "last update wins" reading (owner = highest
  cell index) are readings of the paper, not fixed by it: parity unpinned by
  the paper for that choice; the hand-derived example pins the implementation
  of the reading.
"""
from .smoother import (spacetime_matrix, cell_dofs, extract_cell_matrix, cell_inverse,
                       build_inverses, residual, vanka_sweep, vanka_sweep_combined,
                       extract_cell_matrix_blocks, owner_cells, OracleLevel, prepare_levels)
from .multigrid import vcycle, coarse_inverse
from .krylov import fgmres

__all__ = ["spacetime_matrix", "cell_dofs", "extract_cell_matrix", "cell_inverse",
           "build_inverses", "residual", "vanka_sweep", "vanka_sweep_combined",
           "extract_cell_matrix_blocks", "owner_cells", "OracleLevel", "prepare_levels",
           "vcycle", "coarse_inverse", "fgmres"]
