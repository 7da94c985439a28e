"""Parity on the 2d channel 512x128, dG(2), 6 levels, FP64 inverses, without
spatial factors: the block residual, the plain sweep and the plain (not
time-decoupled) store; the launch configuration bench.py times is
checked in test_parity_bench_path_gpu.py.  Outputs the oracle computes one by
one, and properties that hold at any size."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from gpu_common import log, relerr, to_dev, to_host
from stgen.problem import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_10561_amd as stv
    log("[fullsize] generating 512x128 dG(2) hierarchy")
    p = make_problem(2, (512, 128), 6, 2, 0.005, 1e-3, 1002)
    s = stv.Solver(0)
    s.set_hierarchy(p.levels, 2, 2)
    s.build_cell_inverses()
    return p, s, stv


def _J(L, b):
    return sp.bsr_matrix((L.val, L.col, L.rowptr), shape=(L.n_sdofs * b,) * 2)


def test_residual_sampled_rows(big):
    p, s, _ = big
    b = p.b
    rng = np.random.default_rng(11)
    for g in (len(p.levels) - 1, 1):
        L = p.levels[g]
        n = L.n_sdofs * b
        r, d = rng.standard_normal(n), rng.standard_normal(n)
        out = to_dev(np.zeros(n))
        s.residual(g, to_dev(r), to_dev(d), out)
        got = to_host(out)
        J = _J(L, b).tocsr()
        rows = np.concatenate([rng.choice(n, 4000, replace=False), [0, n - 1]])
        ref = r[rows] - J[rows] @ d
        assert np.abs(got[rows] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_cell_inverses_sampled_cells(big):
    p, s, _ = big
    b = p.b
    rng = np.random.default_rng(12)
    worst = 0.0
    for g in range(1, len(p.levels)):
        L = p.levels[g]
        own = oracle.owner_cells(L.cell_sdofs, L.n_sdofs)
        nls = L.cell_sdofs.shape[1]
        cells = np.unique(np.concatenate([rng.choice(L.n_cells, 24, replace=False), [0, L.n_cells - 1]]))
        for T in cells:
            JT = oracle.extract_cell_matrix_blocks(L.rowptr, L.col, L.val, b, L.cell_sdofs[T])
            O = oracle.cell_inverse(JT)
            G = s.get_cell_inverse(g, int(T))
            rows = [l * nls + a for l in range(b) for a in range(nls) if own[L.cell_sdofs[T, a]] == T]
            worst = max(worst, np.linalg.norm(G[rows] - O[rows]) / np.linalg.norm(O[rows]))
    log(f"[fullsize] inverse rows worst rel err {worst:.2e}")
    assert worst <= 1e-10


def test_sweep_sampled_dofs(big):
    """d_new[j] = d[j] + omega (J_T^-1 rho_T)[loc(j)] for the last cell T containing j."""
    p, s, _ = big
    b = p.b
    g = len(p.levels) - 1
    L = p.levels[g]
    n = L.n_sdofs * b
    rng = np.random.default_rng(13)
    r, d = rng.standard_normal(n), rng.standard_normal(n)
    dd = to_dev(d)
    s.vanka_sweep(g, to_dev(r), dd, 1, 0.7)
    got = to_host(dd)
    rho = r - _J(L, b) @ d
    own = oracle.owner_cells(L.cell_sdofs, L.n_sdofs)
    nls = L.cell_sdofs.shape[1]
    sdofs = np.unique(np.concatenate([rng.choice(L.n_sdofs, 300, replace=False), [0, L.n_sdofs - 1]]))
    worst = 0.0
    for sd in sdofs:
        T = int(own[sd])
        idx = oracle.cell_dofs(L.cell_sdofs[T:T + 1], b)[0]
        c = oracle.cell_inverse(oracle.extract_cell_matrix_blocks(L.rowptr, L.col, L.val, b,
                                                                   L.cell_sdofs[T])) @ rho[idx]
        a = int(np.nonzero(L.cell_sdofs[T] == sd)[0][0])
        for l in range(b):
            ref = d[sd * b + l] + 0.7 * c[l * nls + a]
            worst = max(worst, abs(got[sd * b + l] - ref) / max(1.0, abs(ref)))
    log(f"[fullsize] sweep worst err {worst:.2e}")
    assert worst <= 1e-11


def test_coarse_solve_full(big):
    p, s, _ = big
    L0 = p.levels[0]
    n = L0.n_sdofs * p.b
    r = np.random.default_rng(14).standard_normal(n)
    x = to_dev(np.zeros(n))
    s.coarse_solve(to_dev(r), x)
    ref = np.linalg.solve(_J(L0, p.b).toarray(), r)
    assert relerr(to_host(x), ref) <= 1e-11


def test_vcycle_linearity_full(big):
    p, s, _ = big
    n = p.levels[-1].n_sdofs * p.b
    rng = np.random.default_rng(15)
    a, c = rng.standard_normal(n), rng.standard_normal(n)
    outs = []
    for v in (a, c, 2.0 * a - 3.0 * c):
        x = to_dev(np.zeros(n))
        s.vcycle(to_dev(v), x, 2, 2, 0.7)
        outs.append(to_host(x))
    assert relerr(outs[2], 2.0 * outs[0] - 3.0 * outs[1]) <= 1e-12


@pytest.mark.parametrize("fp32", [False, True])
def test_gmres_full_reaches_tolerance(big, fp32):
    p, s, stv = big
    L = p.levels[-1]
    n = L.n_sdofs * p.b
    if fp32:
        s.build_cell_inverses(fp32=True)
    x = to_dev(np.zeros(n))
    info = s.gmres_solve(to_dev(p.rhs), x, restart=30, rtol=1e-8)
    xg = to_host(x)
    true = np.linalg.norm(p.rhs - _J(L, p.b) @ xg) / np.linalg.norm(p.rhs)
    log(f"[fullsize] gmres fp32={fp32} iters {info['iters']} true relres {true:.2e}")
    assert info["converged"] and true <= 1e-8
    assert abs(info["true_relres"] - true) <= 1e-3 * true
    if fp32:
        s.build_cell_inverses(fp32=False)
