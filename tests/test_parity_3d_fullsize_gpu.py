"""Parity of the 3d precision workload at full size: channel 128x24x24,
Q2/P1disc x dG(1) (170 local DoFs per cell), 4 levels, set up exactly as
bench.py times it (spatial factors on every level, autotuned shapes).

Kernels reached: k_spmv_kron (residual from the factors, split lists), the
cell inverses through the complex time-decoupled block (k_inverse_cx<85>,
owned complex rows, FP64 and FP32 store), the sweep on that store
(k_vanka_cx, FP64 and FP32), the transfers (k_csr_lanes, autotuned and every
shape), the coarse inverse of order 10,854 assembled from the complex-pair
block eliminated with complex pivots (k_gj_tour_cx, k_gj_slab_update_cx128),
and FGMRES.
Sampled outputs are compared with the oracle computed one cell at a time, the
coarse solve with a sparse direct solve, FGMRES with a host residual.
"""
import numpy as np
import pytest

from fullsize_common import (bench_solver, check_coarse, check_gmres, check_inverse_rows,
                             check_residual_rows, check_sweep, check_transfers)
from gpu_common import log
from stgen.problem import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bench3d():
    log("[3d-fullsize] generating 3d 128x24x24 dG(1), 4 levels")
    p = make_problem(3, (128, 24, 24), 4, 1, 0.01, 1e-3, 1003)
    log("[3d-fullsize] spatial factors, upload, inverses, autotune")
    s, _ = bench_solver(p)
    yield p, s
    s.close()


def test_3d_residual_from_factors(bench3d):
    p, s = bench3d
    rng = np.random.default_rng(41)
    for g in (len(p.levels) - 1, 1):
        e = check_residual_rows(p, s, g, rng)
        log(f"[3d-fullsize] residual level {g}: max rel err {e:.2e}")


def test_3d_transfers_every_shape(bench3d):
    p, s = bench3d
    worst = check_transfers(p, s, np.random.default_rng(46), shapes=(0, 1, 2, 3, 4, 5))
    log(f"[3d-fullsize] transfers: worst rel err {worst:.2e}")
    assert worst <= 1e-13


@pytest.mark.parametrize("fp32", [False, True])
def test_3d_cell_inverses(bench3d, fp32):
    p, s = bench3d
    if fp32:
        s.build_cell_inverses(fp32=True)
    try:
        rng = np.random.default_rng(42)
        extra = (1023, 1024, 9215, 9216, 40000, 73726)
        worst = check_inverse_rows(p, s, rng, extra, tol=1e-6 if fp32 else 1e-10)
        log(f"[3d-fullsize] inverse rows fp32={fp32}: worst rel err {worst:.2e}")
    finally:
        if fp32:
            s.build_cell_inverses(fp32=False)


@pytest.mark.parametrize("fp32", [False, True])
def test_3d_sweep(bench3d, fp32):
    p, s = bench3d
    if fp32:
        s.build_cell_inverses(fp32=True)
    try:
        rng = np.random.default_rng(43)
        for g in (len(p.levels) - 1, 1):
            e = check_sweep(p, s, g, rng, fp32, n_sdofs=100)
            log(f"[3d-fullsize] sweep fp32={fp32} level {g}: worst err / tolerance {e:.2f}")
    finally:
        if fp32:
            s.build_cell_inverses(fp32=False)


def test_3d_coarse_solve(bench3d):
    p, s = bench3d
    e = check_coarse(p, s, np.random.default_rng(44))
    log(f"[3d-fullsize] coarse solve (order {p.levels[0].n_sdofs * p.b}) rel err {e:.2e}")


@pytest.mark.parametrize("fp32", [False, True])
def test_3d_gmres_reaches_tolerance(bench3d, fp32):
    p, s = bench3d
    if fp32:
        s.build_cell_inverses(fp32=True)
    try:
        it, true = check_gmres(p, s)
        log(f"[3d-fullsize] FGMRES fp32={fp32}: {it} iterations, true relres {true:.2e}")
    finally:
        if fp32:
            s.build_cell_inverses(fp32=False)
