"""Launch shapes of the level kernels (the residual's shape,
persistent sweep grids) and the autotuner that picks them: every shape must
reproduce the oracle, and the sweep must not depend on its grid at all."""
import numpy as np
import pytest

import oracle
from gpu_common import log, problem, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_2107_10561_amd as m
    return m


def solver(stv, name):
    p, ol = problem(name)
    s = stv.Solver(0)
    s.set_hierarchy(p.levels, p.dim, p.k)
    s.build_cell_inverses()
    return s, p, ol


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2", "3d_dg1"])
@pytest.mark.parametrize("rows", [1, 2, 3, 4, 6])
def test_residual_rows_per_wavefront(stv, name, rows):
    s, p, ol = solver(stv, name)
    G = len(ol) - 1
    rng = np.random.default_rng(3)
    r, d = rng.standard_normal(ol[G].n_st), rng.standard_normal(ol[G].n_st)
    s.set_launch(G, rows, 0)
    out = to_dev(np.zeros(ol[G].n_st))
    s.residual(G, to_dev(r), to_dev(d), out)
    ref = r - ol[G].J @ d
    assert np.abs(to_host(out) - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2", "3d_dg1"])
@pytest.mark.parametrize("wgs", [1, 3, 64])
def test_persistent_sweep_is_bitwise_equal(stv, name, wgs):
    s, p, ol = solver(stv, name)
    G = len(ol) - 1
    rng = np.random.default_rng(4)
    r, d0 = rng.standard_normal(ol[G].n_st), rng.standard_normal(ol[G].n_st)
    outs = []
    for w in (0, wgs):
        s.set_launch(G, 2, w)
        d = to_dev(d0)
        s.vanka_sweep(G, to_dev(r), d, 2, 0.7)
        outs.append(to_host(d))
    assert np.array_equal(outs[0], outs[1])
    assert relerr(outs[1], oracle.vanka_sweep(ol[G], r, oracle.vanka_sweep(ol[G], r, d0, 0.7), 0.7)) <= 1e-12


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2", "3d_dg1"])
def test_autotuned_solver_matches_oracle(stv, name):
    s, p, ol = solver(stv, name)
    choice = s.autotune()
    log(f"[autotune] {name}: {choice}")
    for g in range(1, len(ol)):
        rows, wgs = choice[g]
        assert 1 <= rows <= 12 and wgs >= 0
        tp, tpt = s.transfer_shapes(g)
        assert 1 <= tp <= 5 and 1 <= tpt <= 5
    rng = np.random.default_rng(6)
    r = rng.standard_normal(ol[-1].n_st)
    d = to_dev(np.zeros(ol[-1].n_st))
    s.vcycle(to_dev(r), d, 2, 2, 0.7)
    assert relerr(to_host(d), oracle.vcycle(ol, r, 2, 2, 0.7)) <= 1e-11
    cinv = oracle.coarse_inverse(ol[0])
    A = lambda v: ol[-1].J @ v
    M = lambda v: oracle.vcycle(ol, v, 2, 2, 0.7, coarse_inv=cinv)
    xf, _ = oracle.fgmres(A, p.rhs, M, restart=30, fixed_iters=6)
    x = to_dev(np.zeros(ol[-1].n_st))
    s.gmres_solve(to_dev(p.rhs), x, restart=30, fixed_iters=6)
    assert relerr(to_host(x), xf) <= 1e-10


def test_set_launch_rejects_bad_shapes(stv):
    s, p, ol = solver(stv, "c1_2d_dg1")
    for args in ((1, 0, 0), (1, 13, 0), (1, 2, -1), (9, 2, 0)):
        with pytest.raises(stv.StvError):
            s.set_launch(*args)


def test_transfer_shapes_reject_bad_arguments(stv):
    s, p, ol = solver(stv, "c1_2d_dg1")
    for args in ((0, 1, 1), (9, 1, 1), (1, 6, 0), (1, 0, -1)):
        with pytest.raises(stv.StvError):
            s.transfer_shapes(*args)
    assert s.transfer_shapes(1, 3, 4) == (3, 4)
    assert s.transfer_shapes(1) == (3, 4)
