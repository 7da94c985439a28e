"""Pins of the FP64 oracle against closed forms, special cases and library routines."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle.smoother import OracleLevel, cell_dofs
from stgen.problem import make_problem


@pytest.fixture(scope="module")
def c1():
    p = make_problem(2, (16, 4), 2, 1, 0.01, 1e-3, 1001)
    ol = oracle.prepare_levels(p.levels, p.b)
    oracle.build_inverses(ol)
    return p, ol


def test_cell_inverses_times_blocks_are_identity(c1):
    _, ol = c1
    for g in range(1, len(ol)):
        L = ol[g]
        for T in range(L.dofs.shape[0]):
            JT = oracle.extract_cell_matrix(L.J, L.dofs[T])
            err = np.abs(L.inv[T] @ JT - np.eye(JT.shape[0])).max()
            assert err <= 1e-12, (g, T, err)


def test_cell_dofs_follow_paper_local_order():
    """eq. (4.4): time-major, velocity components then pressure inside a time DoF."""
    csd = np.array([[10, 11, 12]], dtype=np.int32)
    np.testing.assert_array_equal(cell_dofs(csd, 2)[0], [20, 22, 24, 21, 23, 25])


@pytest.mark.parametrize("k", [0, 1, 2])
def test_single_cell_sweep_is_exact_solve(k):
    """On a one-cell mesh the Vanka sweep with omega = 1 solves J d = r exactly."""
    p = make_problem(2, (1, 1), 1, k, 0.01, 1e-3, 7)
    ol = oracle.prepare_levels(p.levels, p.b)
    oracle.build_inverses(ol, first_level=0)
    L = ol[0]
    rng = np.random.default_rng(3)
    r = rng.standard_normal(L.n_st)
    d0 = rng.standard_normal(L.n_st)
    d = oracle.vanka_sweep(L, r, d0, 1.0)
    x = np.linalg.solve(L.J.toarray(), r)
    np.testing.assert_allclose(d, x, rtol=0, atol=1e-12 * np.abs(x).max())


def test_disjoint_cells_sweep_is_exact_solve():
    """Cells that share no DoF: the sweep is a block-Jacobi exact solve
    (pins the gather/scatter indexing over many cells)."""
    rng = np.random.default_rng(5)
    nc, nloc = 7, 6
    perm = rng.permutation(nc * nloc)
    dofs = perm.reshape(nc, nloc)
    J = np.zeros((nc * nloc, nc * nloc))
    for T in range(nc):
        B = rng.standard_normal((nloc, nloc)) + 4 * np.eye(nloc)
        J[np.ix_(dofs[T], dofs[T])] = B
    L = OracleLevel(sp.csr_matrix(J), dofs, nc * nloc, None)
    L.inv = [np.linalg.inv(J[np.ix_(dofs[T], dofs[T])]) for T in range(nc)]
    r = rng.standard_normal(nc * nloc)
    d = oracle.vanka_sweep(L, r, rng.standard_normal(nc * nloc), 1.0)
    np.testing.assert_allclose(d, np.linalg.solve(J, r), atol=1e-12)


def test_two_cell_overwrite_by_hand():
    """Three DoFs, cells {0,1} and {1,2}; J = [[2,1,0],[1,4,1],[0,2,4]].
    Hand computation: J_0^-1 = [[4,-1],[-1,2]]/7, J_1^-1 = [[4,-1],[-2,4]]/14.
    d = (1,0,-1), r = (1,1,1): rho = r - J d = (-1, 1, 5);
    c_0 = J_0^-1 (-1, 1) = (-5/7, 3/7);  c_1 = J_1^-1 (1, 5) = (-1/14, 18/14).
    omega = 1/2, the shared DoF 1 keeps the later cell's update:
    d_new = (1 - 5/14, 0 - 1/28, -1 + 9/14) = (9/14, -1/28, -5/14)."""
    J = np.array([[2., 1, 0], [1, 4, 1], [0, 2, 4]])
    dofs = np.array([[0, 1], [1, 2]])
    L = OracleLevel(sp.csr_matrix(J), dofs, 3, None)
    L.inv = [oracle.cell_inverse(J[np.ix_(c, c)]) for c in dofs]
    d = oracle.vanka_sweep(L, np.ones(3), np.array([1.0, 0.0, -1.0]), 0.5)
    expect = [Fraction(9, 14), Fraction(-1, 28), Fraction(-5, 14)]
    np.testing.assert_allclose(d, [float(e) for e in expect], atol=1e-15)


def test_vcycle_one_level_is_direct_solve(c1):
    _, ol = c1
    r = np.random.default_rng(1).standard_normal(ol[0].n_st)
    np.testing.assert_allclose(oracle.vcycle(ol[:1], r, 2, 2, 0.7),
                               np.linalg.solve(ol[0].J.toarray(), r), atol=1e-12)


def test_vcycle_without_smoothing_is_coarse_correction(c1):
    _, ol = c1
    r = np.random.default_rng(2).standard_normal(ol[1].n_st)
    Jc = ol[0].J.toarray()
    P = ol[1].P.toarray()
    expect = P @ np.linalg.solve(Jc, P.T @ r)
    np.testing.assert_allclose(oracle.vcycle(ol, r, 0, 0, 0.7), expect, atol=1e-11)


def test_vcycle_is_linear(c1):
    _, ol = c1
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal(ol[1].n_st), rng.standard_normal(ol[1].n_st)
    M = lambda r: oracle.vcycle(ol, r, 2, 2, 0.7)
    lhs = M(2.0 * a - 3.0 * b)
    np.testing.assert_allclose(lhs, 2.0 * M(a) - 3.0 * M(b), atol=1e-10 * np.abs(lhs).max())


def test_vcycle_reduces_error_as_smoother(c1):
    """Two-grid error propagation I - M J has spectral radius < 1 on C1."""
    _, ol = c1
    n = ol[1].n_st
    J = ol[1].J.toarray()
    E = np.eye(n) - np.stack([oracle.vcycle(ol, J[:, j], 2, 2, 0.7) for j in range(n)], axis=1)
    assert np.abs(np.linalg.eigvals(E)).max() < 0.5


def test_fgmres_identity_preconditioner_matches_scipy_gmres():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 40)) + 9 * np.eye(40)
    b = rng.standard_normal(40)
    hist = []
    spla.gmres(A, b, rtol=1e-11, restart=7, maxiter=200, callback=hist.append, callback_type="pr_norm")
    _, info = oracle.fgmres(lambda v: A @ v, b, lambda v: v, restart=7, rtol=1e-11)
    n = min(len(hist), info["iters"])
    assert abs(len(hist) - info["iters"]) <= 1
    ours, ref = np.array(info["history"][1:n + 1]), np.array(hist[:n])
    big = ref > 1e-8          # below that, rounding of the two Arnoldi variants shows
    np.testing.assert_allclose(ours[big], ref[big], rtol=1e-8)
    np.testing.assert_allclose(ours, ref, rtol=1e-4)


def test_fgmres_minimal_residual_over_krylov_space():
    """One cycle of j steps minimises ||b - A M y|| over span{b, (AM) b, ...}."""
    rng = np.random.default_rng(8)
    A = rng.standard_normal((30, 30)) + 6 * np.eye(30)
    Mm = np.diag(1.0 + rng.random(30))
    b = rng.standard_normal(30)
    for j in (3, 6, 9):
        x, info = oracle.fgmres(lambda v: A @ v, b, lambda v: Mm @ v, restart=50, fixed_iters=j)
        K = [b]
        for _ in range(j - 1):
            K.append(A @ (Mm @ K[-1]))
        K = np.stack(K, axis=1)
        AMK = A @ Mm @ K
        y = np.linalg.lstsq(AMK, b, rcond=None)[0]
        best = np.linalg.norm(b - AMK @ y)
        np.testing.assert_allclose(np.linalg.norm(b - A @ x), best, rtol=1e-8)


def test_fgmres_converges_within_n_steps():
    rng = np.random.default_rng(9)
    n = 25
    A = rng.standard_normal((n, n)) + 2 * np.eye(n)
    b = rng.standard_normal(n)
    x, info = oracle.fgmres(lambda v: A @ v, b, lambda v: v, restart=n, rtol=1e-12)
    assert info["iters"] <= n and info["converged"]
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9)


def test_fgmres_gmg_solves_c1(c1):
    p, ol = c1
    cinv = oracle.coarse_inverse(ol[0])
    x, info = oracle.fgmres(lambda v: ol[-1].J @ v, p.rhs,
                            lambda r: oracle.vcycle(ol, r, 2, 2, 0.7, coarse_inv=cinv),
                            restart=30, rtol=1e-8)
    assert info["converged"] and info["true_relres"] <= 1e-8
    xd = np.linalg.solve(ol[-1].J.toarray(), p.rhs)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-6


def test_combined_readings_two_cells_by_hand():
    """Same example as the overwrite test.  The additive reading sums both
    damped updates at the shared DoF: 0 + 0.5 (3/7 - 1/14) = 5/28; the averaged
    reading divides that sum by the two cells: 5/56.  Unshared DoFs as before."""
    J = np.array([[2., 1, 0], [1, 4, 1], [0, 2, 4]])
    dofs = np.array([[0, 1], [1, 2]])
    L = OracleLevel(sp.csr_matrix(J), dofs, 3, None)
    L.inv = [oracle.cell_inverse(J[np.ix_(c, c)]) for c in dofs]
    d0 = np.array([1.0, 0.0, -1.0])
    add = oracle.vanka_sweep_combined(L, np.ones(3), d0, 0.5, average=False)
    avg = oracle.vanka_sweep_combined(L, np.ones(3), d0, 0.5, average=True)
    np.testing.assert_allclose(add, [9 / 14, 5 / 28, -5 / 14], atol=1e-15)
    np.testing.assert_allclose(avg, [9 / 14, 5 / 56, -5 / 14], atol=1e-15)


def test_block_extraction_matches_csr_extraction(c1):
    p, ol = c1
    L = p.levels[-1]
    for T in (0, 17, L.n_cells - 1):
        a = oracle.extract_cell_matrix_blocks(L.rowptr, L.col, L.val, p.b, L.cell_sdofs[T])
        np.testing.assert_array_equal(a, oracle.extract_cell_matrix(ol[-1].J, ol[-1].dofs[T]))


def test_coarse_inverse_hand_worked_3x3():
    """A 3x3 matrix whose (0, 0) entry is zero (pivoting needed) and whose
    inverse is not symmetric (a transposed result fails), inverted by hand:
    A = [[0,1,2],[1,0,3],[4,-3,8]], det A = -2,
    A^-1 = adj(A)/det = [[-9/2, 7, -3/2], [-2, 4, -1], [3/2, -2, 1/2]]."""
    A = np.array([[0., 1, 2], [1, 0, 3], [4, -3, 8]])
    L0 = OracleLevel(sp.csr_matrix(A), np.zeros((0, 3), dtype=np.int64), 3, None)
    inv = oracle.coarse_inverse(L0)
    np.testing.assert_allclose(inv, [[-4.5, 7, -1.5], [-2, 4, -1], [1.5, -2, 0.5]], atol=1e-14)


def test_coarse_inverse_is_two_sided_inverse(c1):
    """On the coarsest space-time Oseen matrix of the small channel: the dense
    inverse times J_0 is the identity from both sides."""
    _, ol = c1
    J0 = ol[0].J.toarray()
    inv = oracle.coarse_inverse(ol[0])
    cond = np.linalg.cond(J0, 1)
    n = J0.shape[0]
    assert np.abs(inv @ J0 - np.eye(n)).max() <= 1e-14 * cond
    assert np.abs(J0 @ inv - np.eye(n)).max() <= 1e-14 * cond
    r = np.random.default_rng(9).standard_normal(n)
    np.testing.assert_allclose(oracle.vcycle(ol[:1], r, 2, 2, 0.7, coarse_inv=inv),
                               np.linalg.solve(J0, r), rtol=0, atol=1e-12 * np.abs(inv @ r).max())


def _pressure_rows(p, g):
    """Space-time DoFs of level g that belong to pressure modes (spatial DoFs
    after the dim * N_v velocity DoFs of the numbering)."""
    m = p.levels[g].mesh
    sdof_is_p = np.arange(m.n_sdofs) >= m.dim * m.n_vnodes
    return np.repeat(sdof_is_p, p.b)


def test_zero_pressure_residual_breaks_consistency():
    """Ablation of eq. (4.5): with r_0 (pressure rows of r set to zero) the exact
    solution of J x = r is not a fixed point of the sweep, and the one-cell sweep
    with omega = 1 no longer solves exactly; with the full r (the reading used
    everywhere else) both hold.  This is why the full r is used."""
    p = make_problem(2, (1, 1), 1, 1, 0.01, 1e-3, 7)
    ol = oracle.prepare_levels(p.levels, p.b)
    oracle.build_inverses(ol, first_level=0)
    L = ol[0]
    pr = _pressure_rows(p, 0)
    rng = np.random.default_rng(4)
    r = rng.standard_normal(L.n_st)
    x = np.linalg.solve(L.J.toarray(), r)
    d0 = rng.standard_normal(L.n_st)
    full = oracle.vanka_sweep(L, r, d0, 1.0)
    zero = oracle.vanka_sweep(L, r, d0, 1.0, pressure_rows=pr)
    np.testing.assert_allclose(full, x, atol=1e-12 * np.abs(x).max())
    assert np.abs(zero - x).max() > 1e-3 * np.abs(x).max()
    # on a multi-cell level: x is a fixed point only with the full r
    p2 = make_problem(2, (4, 2), 1, 1, 0.01, 1e-3, 8)
    o2 = oracle.prepare_levels(p2.levels, p2.b)
    oracle.build_inverses(o2, first_level=0)
    L2 = o2[0]
    r2 = rng.standard_normal(L2.n_st)
    x2 = spla.spsolve(L2.J.tocsc(), r2)
    np.testing.assert_allclose(oracle.vanka_sweep(L2, r2, x2, 0.7), x2,
                               atol=1e-12 * np.abs(x2).max())
    moved = oracle.vanka_sweep(L2, r2, x2, 0.7, pressure_rows=_pressure_rows(p2, 0))
    assert np.abs(moved - x2).max() > 1e-3 * np.abs(x2).max()
    # a right-hand side with zero pressure rows makes the two readings agree
    r3 = np.where(_pressure_rows(p2, 0), 0.0, r2)
    np.testing.assert_array_equal(oracle.vanka_sweep(L2, r3, x2, 0.7),
                                  oracle.vanka_sweep(L2, r3, x2, 0.7, pressure_rows=_pressure_rows(p2, 0)))
