"""Parity of the HIP path (through the C ABI) with the FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_common import CASES, log, problem, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

ALL = list(CASES)


@pytest.fixture(scope="module")
def stv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_2107_10561_amd as m
    return m


_solvers = {}


def solver(stv, name, fp32=False, full=False):
    key = (name, fp32, full)
    if key not in _solvers:
        p, _ = problem(name)
        log(f"[setup] {name} fp32={fp32} full={full}")
        s = stv.Solver(0)
        s.set_hierarchy(p.levels, p.dim, p.k)
        s.build_cell_inverses(fp32=fp32, full=full)
        _solvers[key] = s
    return _solvers[key]


@pytest.mark.parametrize("name", ALL)
def test_residual(stv, name):
    p, ol = problem(name)
    s = solver(stv, name)
    rng = np.random.default_rng(1)
    for g in range(len(ol)):
        r = rng.standard_normal(ol[g].n_st)
        d = rng.standard_normal(ol[g].n_st)
        out = to_dev(np.zeros(ol[g].n_st))
        s.residual(g, to_dev(r), to_dev(d), out)
        ref = oracle.residual(ol[g].J, r, d)
        assert np.abs(to_host(out) - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("name", ALL)
def test_cell_inverses_full_rows(stv, name):
    p, ol = problem(name)
    s = solver(stv, name, full=True)
    worst = 0.0
    for g in range(1, len(ol)):
        for T in range(ol[g].dofs.shape[0]):
            G = s.get_cell_inverse(g, T)
            O = ol[g].inv[T]
            worst = max(worst, np.linalg.norm(G - O) / np.linalg.norm(O))
    log(f"[inverse] {name} worst rel Frobenius {worst:.3e}")
    assert worst <= 1e-10


@pytest.mark.parametrize("name", ALL)
def test_cell_inverses_owned_rows(stv, name):
    p, ol = problem(name)
    s = solver(stv, name)
    g = len(ol) - 1
    L = p.levels[g]
    own = oracle.owner_cells(L.cell_sdofs, L.n_sdofs)
    nls = L.cell_sdofs.shape[1]
    for T in (0, L.n_cells // 2, L.n_cells - 1):
        G = s.get_cell_inverse(g, T)
        O = ol[g].inv[T]
        owned_alpha = [a for a in range(nls) if own[L.cell_sdofs[T, a]] == T]
        rows = [l * nls + a for l in range(p.b) for a in owned_alpha]
        other = sorted(set(range(G.shape[0])) - set(rows))
        assert np.all(np.isnan(G[other]))
        assert np.abs(G[rows] - O[rows]).max() <= 1e-10 * np.abs(O).max()


@pytest.mark.parametrize("name", ALL)
@pytest.mark.parametrize("omega", [1.0, 0.7])
def test_one_sweep(stv, name, omega):
    p, ol = problem(name)
    s = solver(stv, name)
    rng = np.random.default_rng(2)
    g = len(ol) - 1
    r = rng.standard_normal(ol[g].n_st)
    d0 = rng.standard_normal(ol[g].n_st)
    dd = to_dev(d0)
    s.vanka_sweep(g, to_dev(r), dd, 1, omega)
    ref = oracle.vanka_sweep(ol[g], r, d0, omega)
    e = relerr(to_host(dd), ref)
    log(f"[sweep] {name} omega={omega} rel err {e:.3e}")
    assert e <= 1e-12


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2", "3d_dg1"])
def test_two_sweeps_fp64_and_fp32(stv, name):
    p, ol = problem(name)
    rng = np.random.default_rng(3)
    g = len(ol) - 1
    r = rng.standard_normal(ol[g].n_st)
    d0 = np.zeros(ol[g].n_st)
    ref = oracle.vanka_sweep(ol[g], r, oracle.vanka_sweep(ol[g], r, d0, 0.7), 0.7)
    for fp32, tol in ((False, 1e-12), (True, 1e-5)):
        s = solver(stv, name, fp32=fp32)
        dd = to_dev(d0)
        s.vanka_sweep(g, to_dev(r), dd, 2, 0.7)
        e = relerr(to_host(dd), ref)
        log(f"[sweep2] {name} fp32={fp32} rel err {e:.3e}")
        assert e <= tol


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2", "3d_dg1"])
@pytest.mark.parametrize("mode", ["pou", "additive"])
def test_combined_modes(stv, name, mode):
    p, ol = problem(name)
    s = solver(stv, name, full=True)
    rng = np.random.default_rng(4)
    g = len(ol) - 1
    r = rng.standard_normal(ol[g].n_st)
    d0 = rng.standard_normal(ol[g].n_st)
    dd = to_dev(d0)
    s.vanka_sweep(g, to_dev(r), dd, 1, 0.7, stv.STV_POU if mode == "pou" else stv.STV_ADDITIVE)
    ref = oracle.vanka_sweep_combined(ol[g], r, d0, 0.7, average=(mode == "pou"))
    assert relerr(to_host(dd), ref) <= 1e-12


@pytest.mark.parametrize("name", ALL)
def test_transfers_and_coarse(stv, name):
    p, ol = problem(name)
    s = solver(stv, name)
    rng = np.random.default_rng(5)
    G = len(ol) - 1
    # every level pair, the default shape (0) and each of 1..16 lanes per row
    for g in range(G, 0, -1):
        kept = s.transfer_shapes(g)
        for t in (0, 1, 2, 3, 4, 5):
            s.transfer_shapes(g, t, t)
            rho = rng.standard_normal(ol[g].n_st)
            rc = to_dev(np.zeros(ol[g - 1].n_st))
            s.restrict(g, to_dev(rho), rc)
            ref = ol[g].P.T @ rho
            assert np.abs(to_host(rc) - ref).max() <= 1e-13 * np.abs(ref).max(), (g, t)
            dc = rng.standard_normal(ol[g - 1].n_st)
            d = rng.standard_normal(ol[g].n_st)
            dd = to_dev(d)
            s.prolongate_add(g, to_dev(dc), dd)
            ref = d + ol[g].P @ dc
            assert np.abs(to_host(dd) - ref).max() <= 1e-13 * np.abs(ref).max(), (g, t)
        s.transfer_shapes(g, *kept)
    r0 = rng.standard_normal(ol[0].n_st)
    x0 = to_dev(np.zeros(ol[0].n_st))
    s.coarse_solve(to_dev(r0), x0)
    ref = np.linalg.solve(ol[0].J.toarray(), r0)
    assert relerr(to_host(x0), ref) <= 1e-11


@pytest.mark.parametrize("name", ALL)
def test_vcycle(stv, name):
    p, ol = problem(name)
    s = solver(stv, name)
    rng = np.random.default_rng(6)
    r = rng.standard_normal(ol[-1].n_st)
    d = to_dev(np.zeros(ol[-1].n_st))
    s.vcycle(to_dev(r), d, 2, 2, 0.7)
    ref = oracle.vcycle(ol, r, 2, 2, 0.7)
    e = relerr(to_host(d), ref)
    log(f"[vcycle] {name} rel err {e:.3e}")
    assert e <= 1e-11


@pytest.mark.parametrize("name", ALL)
def test_gmres_fixed_iterations(stv, name):
    p, ol = problem(name)
    s = solver(stv, name)
    cinv = oracle.coarse_inverse(ol[0])
    A = lambda v: ol[-1].J @ v
    M = lambda v: oracle.vcycle(ol, v, 2, 2, 0.7, coarse_inv=cinv)
    xo, io = oracle.fgmres(A, p.rhs, M, restart=30, rtol=1e-8)
    n = io["iters"]
    xf, _ = oracle.fgmres(A, p.rhs, M, restart=30, fixed_iters=n)
    x = to_dev(np.zeros(ol[-1].n_st))
    info = s.gmres_solve(to_dev(p.rhs), x, restart=30, fixed_iters=n)
    e = relerr(to_host(x), xf)
    log(f"[gmres-fixed] {name} iters {n} rel err {e:.3e}")
    assert info["iters"] == n
    assert e <= 1e-10


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2"])
@pytest.mark.parametrize("mode", ["fixed", "tolerance"])
def test_gmres_restarted(stv, name, mode):
    """FGMRES(3): the cycles restart from the true residual.  The device
    work of a step is enqueued before the previous step's coefficients reach
    the host; the steps a cycle takes, the restarts and the iterate must be
    those of the oracle's FGMRES(3)."""
    p, ol = problem(name)
    s = solver(stv, name)
    cinv = oracle.coarse_inverse(ol[0])
    A = lambda v: ol[-1].J @ v
    M = lambda v: oracle.vcycle(ol, v, 2, 2, 0.7, coarse_inv=cinv)
    x = to_dev(np.zeros(ol[-1].n_st))
    if mode == "fixed":
        xf, _ = oracle.fgmres(A, p.rhs, M, restart=3, fixed_iters=8)
        info = s.gmres_solve(to_dev(p.rhs), x, restart=3, fixed_iters=8)
        e = relerr(to_host(x), xf)
        log(f"[gmres-restart] {name} fixed 8 rel err {e:.3e} restarts {info['restarts']}")
        assert info["iters"] == 8 and e <= 1e-10
    else:
        xo, io = oracle.fgmres(A, p.rhs, M, restart=3, rtol=1e-8)
        info = s.gmres_solve(to_dev(p.rhs), x, restart=3, rtol=1e-8)
        xg = to_host(x)
        true = np.linalg.norm(p.rhs - ol[-1].J @ xg) / np.linalg.norm(p.rhs)
        log(f"[gmres-restart] {name} gpu iters {info['iters']} oracle {io['iters']} relres {true:.2e}")
        assert info["converged"] and true <= 1e-8
        assert abs(info["iters"] - io["iters"]) <= 1


@pytest.mark.parametrize("name", ALL)
def test_gmres_tolerance_mode(stv, name):
    p, ol = problem(name)
    s = solver(stv, name)
    cinv = oracle.coarse_inverse(ol[0])
    xo, io = oracle.fgmres(lambda v: ol[-1].J @ v, p.rhs,
                           lambda v: oracle.vcycle(ol, v, 2, 2, 0.7, coarse_inv=cinv),
                           restart=30, rtol=1e-8)
    x = to_dev(np.zeros(ol[-1].n_st))
    info = s.gmres_solve(to_dev(p.rhs), x, restart=30, rtol=1e-8)
    xg = to_host(x)
    true = np.linalg.norm(p.rhs - ol[-1].J @ xg) / np.linalg.norm(p.rhs)
    log(f"[gmres] {name} gpu iters {info['iters']} oracle {io['iters']} true relres {true:.2e}")
    assert info["converged"] and true <= 1e-8
    assert abs(info["iters"] - io["iters"]) <= 1
    assert abs(info["true_relres"] - true) <= 1e-3 * true + 1e-14   # recomputing a residual near 1e-13 carries ~1e-15 of rounding


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2", "3d_dg1"])
def test_gmres_fp32_inverses_reach_tolerance(stv, name):
    p, ol = problem(name)
    s = solver(stv, name, fp32=True)
    x = to_dev(np.zeros(ol[-1].n_st))
    info = s.gmres_solve(to_dev(p.rhs), x, restart=30, rtol=1e-8)
    xg = to_host(x)
    true = np.linalg.norm(p.rhs - ol[-1].J @ xg) / np.linalg.norm(p.rhs)
    xd = np.linalg.solve(ol[-1].J.toarray(), p.rhs) if ol[-1].n_st < 6000 else None
    log(f"[gmres-fp32] {name} iters {info['iters']} true relres {true:.2e}")
    assert info["converged"] and true <= 1e-8
    if xd is not None:
        s64 = solver(stv, name)
        x64 = to_dev(np.zeros(ol[-1].n_st))
        s64.gmres_solve(to_dev(p.rhs), x64, restart=30, rtol=1e-8)
        e64 = relerr(to_host(x64), xd)
        e32 = relerr(xg, xd)
        log(f"[gmres-fp32] {name} forward error fp32 {e32:.2e} fp64 {e64:.2e}")
        assert e32 <= 2.0 * e64 + 1e-12


def test_solve_is_bitwise_repeatable(stv):
    p, ol = problem("2d_dg2")
    s = solver(stv, "2d_dg2")
    outs = []
    for _ in range(2):
        x = to_dev(np.zeros(ol[-1].n_st))
        s.gmres_solve(to_dev(p.rhs), x, restart=30, rtol=1e-8)
        outs.append(to_host(x))
    assert np.array_equal(outs[0], outs[1])


def test_singular_cell_is_reported(stv):
    from stgen.problem import make_problem
    p = make_problem(2, (8, 2), 2, 1, 0.01, 1e-3, 21)
    L = p.levels[1]
    T = 5
    s0 = int(L.cell_sdofs[T, 20])          # a pressure DoF: it belongs to cell T only
    L.val[L.rowptr[s0]:L.rowptr[s0 + 1]] = 0.0
    s = stv.Solver(0)
    s.set_hierarchy(p.levels, 2, 1)
    with pytest.raises(stv.StvError) as ei:
        s.build_cell_inverses()
    assert ei.value.code == stv.STV_ESINGULAR
    assert ei.value.level == 1 and ei.value.cell == T
    s.close()


def test_nan_rhs_and_max_it(stv):
    p, ol = problem("c1_2d_dg1")
    s = solver(stv, "c1_2d_dg1")
    b = p.rhs.copy()
    b[7] = np.nan
    x = to_dev(np.zeros(ol[-1].n_st))
    with pytest.raises(stv.StvError) as ei:
        s.gmres_solve(to_dev(b), x)
    assert ei.value.code == stv.STV_ENUMERIC
    info = s.gmres_solve(to_dev(p.rhs), x, max_it=1, raise_on_noconv=False)
    assert info["status"] == stv.STV_ENOCONV and info["iters"] == 1 and not info["converged"]


def _solve_case(stv, dim, n, G, k, seed):
    p = make_problem_cached(dim, n, G, k, seed)
    s = stv.Solver(0)
    s.set_hierarchy(p.levels, dim, k)
    s.build_cell_inverses()
    return p, s


_cases = {}


def make_problem_cached(dim, n, G, k, seed):
    from stgen.problem import make_problem
    key = (dim, n, G, k, seed)
    if key not in _cases:
        _cases[key] = make_problem(dim, n, G, k, 0.01, 1e-3, seed)
    return _cases[key]


def test_ragged_cell_counts(stv):
    """6x2 fine / 3x1 coarse: cell and row counts that fill no launch tile."""
    p, s = _solve_case(stv, 2, (6, 2), 2, 1, 31)
    ol = oracle.prepare_levels(p.levels, p.b)
    oracle.build_inverses(ol)
    rng = np.random.default_rng(7)
    r = rng.standard_normal(ol[-1].n_st)
    d0 = rng.standard_normal(ol[-1].n_st)
    dd = to_dev(d0)
    s.vanka_sweep(1, to_dev(r), dd, 1, 0.7)
    assert relerr(to_host(dd), oracle.vanka_sweep(ol[-1], r, d0, 0.7)) <= 1e-12
    x = to_dev(np.zeros(ol[-1].n_st))
    s.vcycle(to_dev(r), x, 2, 2, 0.7)
    assert relerr(to_host(x), oracle.vcycle(ol, r, 2, 2, 0.7)) <= 1e-11
    s.close()


def test_single_level_hierarchy(stv):
    """One level: the V-cycle is the direct coarse solve and GMRES converges at once."""
    p, s = _solve_case(stv, 2, (4, 2), 1, 1, 32)
    J = oracle.prepare_levels(p.levels, p.b)[0].J.toarray()
    x = to_dev(np.zeros(J.shape[0]))
    s.vcycle(to_dev(p.rhs), x, 2, 2, 0.7)
    assert relerr(to_host(x), np.linalg.solve(J, p.rhs)) <= 1e-11
    x = to_dev(np.zeros(J.shape[0]))
    info = s.gmres_solve(to_dev(p.rhs), x)
    assert info["converged"] and info["iters"] <= 2
    s.close()


def test_one_cell_fine_level_is_exact(stv):
    """Smallest hierarchy: 2x2 fine cells over a 1x1 coarse cell, omega = 1."""
    p, s = _solve_case(stv, 2, (2, 2), 2, 1, 33)
    ol = oracle.prepare_levels(p.levels, p.b)
    oracle.build_inverses(ol)
    r = np.random.default_rng(8).standard_normal(ol[-1].n_st)
    x = to_dev(np.zeros(ol[-1].n_st))
    s.vcycle(to_dev(r), x, 1, 1, 1.0)
    assert relerr(to_host(x), oracle.vcycle(ol, r, 1, 1, 1.0)) <= 1e-11
    s.close()


def test_zero_rhs(stv):
    p, ol = problem("c1_2d_dg1")
    s = solver(stv, "c1_2d_dg1")
    x = to_dev(np.ones(ol[-1].n_st))
    info = s.gmres_solve(to_dev(np.zeros(ol[-1].n_st)), x)
    assert info["converged"] and info["iters"] == 0
    assert not np.any(to_host(x))
