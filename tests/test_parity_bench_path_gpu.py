"""Parity of the exact launch configuration bench.py times on the 2d channel
512x128, dG(2), 6 levels, at full size.

bench.py sets the spatial factors on every level and autotunes the launch
shapes before it times anything.  That routes the path through
  - the residual from the spatial factors (k_spmv_kron, autotuned shape),
  - the time-decoupled cell inverses, one launch per diagonal block of the
    time split on a grid capped beside the coarse chain, so that each
    wavefront strides over ~32 cells (k_inverse_wave<1|2, 21, true>),
  - the sweep on the time-decoupled store, FP64 and FP32 (k_vanka_dec, on the
    autotuned persistent grid),
  - the coarse inverse assembled from the real and the complex-pair blocks of
    order 1,572 eliminated with complex pivots (k_kron_block_dense,
    k_gj_tour_cx, k_gj_slab_update) and applied from the two blocks'
    inverses (k_kron_coarse_gemv).
Every sampled output is compared with the oracle computed one cell at a time
(the oracle's own LU inverse of the extracted J_T), the coarse solve with a
sparse direct solve, and FGMRES with an independent residual on the host.
"""
import numpy as np
import pytest

from fullsize_common import (bench_solver, check_coarse, check_gmres, check_inverse_rows,
                             check_residual_rows, check_sweep, check_transfers)
from gpu_common import log
from stgen.problem import make_problem

pytestmark = pytest.mark.gpu


# ---------------------------------------------------------------- 2d, dG(2)
@pytest.fixture(scope="module")
def bench2d():
    log("[bench-path] generating 2d 512x128 dG(2), 6 levels")
    p = make_problem(2, (512, 128), 6, 2, 0.005, 1e-3, 1002)
    s, stv = bench_solver(p)
    yield p, s
    s.close()


def test_2d_residual_from_factors(bench2d):
    p, s = bench2d
    rng = np.random.default_rng(31)
    for g in (len(p.levels) - 1, 2, 1):
        e = check_residual_rows(p, s, g, rng)
        log(f"[bench-path] 2d residual level {g}: max rel err {e:.2e}")


def test_2d_transfers_every_shape(bench2d):
    """k_csr_lanes on every level pair, both directions: the autotuned shapes
    (0) and each of 1, 2, 4, 8, 16 lanes per row, whole vectors."""
    p, s = bench2d
    worst = check_transfers(p, s, np.random.default_rng(36), shapes=(0, 1, 2, 3, 4, 5))
    log(f"[bench-path] 2d transfers: worst rel err {worst:.2e}")
    assert worst <= 1e-13


def test_2d_decoupled_inverses_every_stride(bench2d):
    """Sampled cells on every level, including cells far past the first
    stride of the capped grid (2,048 wavefronts on 256 compute units)."""
    p, s = bench2d
    rng = np.random.default_rng(32)
    extra = (2047, 2048, 2049, 4095, 4096, 6143, 8192, 16385, 32767, 49151, 65534)
    worst = check_inverse_rows(p, s, rng, extra)
    log(f"[bench-path] 2d decoupled inverse rows: worst rel err {worst:.2e}")


@pytest.mark.parametrize("fp32", [False, True])
def test_2d_decoupled_sweep(bench2d, fp32):
    p, s = bench2d
    if fp32:
        s.build_cell_inverses(fp32=True)
    try:
        rng = np.random.default_rng(33)
        for g in (len(p.levels) - 1, 1):
            e = check_sweep(p, s, g, rng, fp32)
            log(f"[bench-path] 2d sweep fp32={fp32} level {g}: worst err / tolerance {e:.2f}")
    finally:
        if fp32:
            s.build_cell_inverses(fp32=False)


def test_2d_coarse_real_and_pair_blocks(bench2d):
    p, s = bench2d
    e = check_coarse(p, s, np.random.default_rng(34))
    log(f"[bench-path] 2d coarse solve (order {p.levels[0].n_sdofs * p.b}) rel err {e:.2e}")


@pytest.mark.parametrize("fp32", [False, True])
def test_2d_gmres_reaches_tolerance(bench2d, fp32):
    p, s = bench2d
    if fp32:
        s.build_cell_inverses(fp32=True)
    try:
        it, true = check_gmres(p, s)
        log(f"[bench-path] 2d FGMRES fp32={fp32}: {it} iterations, true relres {true:.2e}")
    finally:
        if fp32:
            s.build_cell_inverses(fp32=False)
