"""Dense coarse-level inversion (the direct solve of Algorithm 4.1) through the
C ABI, every elimination schedule, at orders that cover every panel
configuration of the library (up to 8934 unknowns) and ragged padding.
The tournament schedule may take other pivots than partial pivoting: it is
held to the same residual and forward-error bounds.

Expected values: SuperLU applied to the oracle's coarse matrix (a library
routine on the same matrix), and the residual r - J d computed on the CPU."""
import functools

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle
from gpu_common import log, relerr, to_dev, to_host
from stgen import fe as fe_time
from stgen.problem import make_problem, spatial_factors

pytestmark = pytest.mark.gpu

# (dim, cells, k): coarse orders 1572, 4484, 2806 (3d) and 8934
COARSE = {
    "2d_16x4_dg1": (2, (16, 4), 1),
    "2d_24x8_dg1": (2, (24, 8), 1),
    "3d_8x2x2_dg1": (3, (8, 2, 2), 1),
    "2d_32x8_dg2": (2, (32, 8), 2),
}
# real order 36004 of the time-decoupled block (2 n_s, n_s = 18002): past
# 256 tournament workgroups
LARGE = {"2d_80x20_dg1": (2, (80, 20), 1)}


@functools.lru_cache(maxsize=None)
def coarse_case(name):
    dim, n, k = {**COARSE, **LARGE}[name]
    p = make_problem(dim, n, 1, k, 0.01, 1e-3, 7)
    ol = oracle.prepare_levels(p.levels, p.b)
    J = ol[0].J.tocsc()
    lu = sla.splu(J)
    cond = sla.onenormest(J) * sla.onenormest(
        sla.LinearOperator(J.shape, matvec=lu.solve, rmatvec=lambda v: lu.solve(v, trans="T")))
    return p, J, lu, cond


@pytest.fixture(scope="module")
def stv():
    import paper_2107_10561_amd as m
    return m


def solve_on_gpu(stv, p, algo, r):
    s = stv.Solver(0)
    s.set_coarse_algorithm(algo)
    s.set_hierarchy(p.levels, p.dim, p.k)
    s.build_cell_inverses()
    d = to_dev(np.zeros_like(r))
    s.coarse_solve(to_dev(r), d)
    return to_host(d)


@pytest.mark.parametrize("name", list(COARSE))
def test_coarse_inverse_every_schedule(stv, name):
    p, J, lu, cond = coarse_case(name)
    r = np.random.default_rng(21).standard_normal(J.shape[0])
    ref = lu.solve(r)
    out = {}
    for algo in ("panels", "slabs", "tournament"):
        log(f"[coarse] {name} n={J.shape[0]} {algo}")
        d = solve_on_gpu(stv, p, algo, r)
        res = np.linalg.norm(r - J @ d) / np.linalg.norm(r)
        fe = relerr(d, ref)
        log(f"[coarse] {name} {algo} relres {res:.2e} forward {fe:.2e} cond {cond:.1e}")
        assert res <= 1e-11
        assert fe <= 1e-15 * cond * 10
        out[algo] = d
    # the same pivot sequence: the schedules differ only in rounding order
    assert relerr(out["panels"], out["slabs"]) <= 1e-15 * cond * 10


def solve_decoupled_on_gpu(stv, p, algo, r):
    """The coarse solve with the level's spatial factors set: the inverse is
    built from the real forms of the diagonal blocks T_p (x) M + I (x) A of
    the operator in the real Jordan basis of the time matrix (order 2 n_s
    each), eliminated with complex pivots by the tournament schedule."""
    _, w, C, _ = fe_time.time_matrices(p.k)
    s = stv.Solver(0)
    s.set_coarse_algorithm(algo)
    s.set_hierarchy(p.levels, p.dim, p.k)
    m, a = spatial_factors(p.levels[0])
    s.set_kron_factors(0, m, a, np.asarray(C, dtype=np.float64),
                       p.tau * np.asarray(w, dtype=np.float64))
    s.build_cell_inverses()
    d = to_dev(np.zeros_like(r))
    s.coarse_solve(to_dev(r), d)
    return to_host(d)


@pytest.mark.parametrize("name", list(COARSE))
def test_time_decoupled_coarse_inverse_every_schedule(stv, name):
    """Orders 2 n_s = 1572 (two workgroups of 128 complex rows, ragged),
    4484 and 2806 (merge trees of two levels), 5956 (slabs of 128): the same
    residual and forward-error bounds as the whole-matrix elimination, for
    the complex-pivot tournament and for the real schedules on the same real
    form."""
    p, J, lu, cond = coarse_case(name)
    r = np.random.default_rng(22).standard_normal(J.shape[0])
    ref = lu.solve(r)
    for algo in ("tournament", "slabs"):
        log(f"[coarse] {name} decoupled {algo}")
        d = solve_decoupled_on_gpu(stv, p, algo, r)
        res = np.linalg.norm(r - J @ d) / np.linalg.norm(r)
        fe = relerr(d, ref)
        log(f"[coarse] {name} decoupled {algo} relres {res:.2e} forward {fe:.2e} cond {cond:.1e}")
        assert res <= 1e-11
        assert fe <= 1e-15 * cond * 10


@pytest.mark.parametrize("name", list(LARGE))
def test_time_decoupled_coarse_two_level_merge_tree(stv, name):
    """Real order 36004 (padded to 36096): 282 tournament workgroups of 128
    real rows, so the complex tournament's merge tree takes two levels of
    16-list merges (282 -> 18 -> 2 lists for the root), the only case here
    past one level.  Complex tournament only (the real schedules' narrow
    panels would each sweep the 10 GB matrix); the same residual and
    forward-error bounds against SuperLU."""
    p, J, lu, cond = coarse_case(name)
    r = np.random.default_rng(26).standard_normal(J.shape[0])
    ref = lu.solve(r)
    log(f"[coarse] {name} decoupled tournament, order {J.shape[0]}")
    d = solve_decoupled_on_gpu(stv, p, "tournament", r)
    res = np.linalg.norm(r - J @ d) / np.linalg.norm(r)
    fe = relerr(d, ref)
    log(f"[coarse] {name} relres {res:.2e} forward {fe:.2e} cond {cond:.1e}")
    assert res <= 1e-11
    assert fe <= 1e-15 * cond * 10


@pytest.mark.parametrize("name", ["2d_16x4_dg1", "2d_32x8_dg2"])
@pytest.mark.parametrize("algo", ["tournament", "slabs", "panels"])
def test_time_decoupled_coarse_apply_both_directions(stv, name, algo):
    """The time-decoupled coarse inverse is applied from the eliminated blocks
    where the elimination left them: through paired pivot records (complex
    pivots, tournament) or real ones (slabs, panels), forward (coarse solve)
    and transposed (the V-cycle of the transposed one-level hierarchy is
    J^-T r).  dG(1): one complex pair; dG(2): a real eigenvalue and a pair."""
    p, J, lu, cond = coarse_case(name)
    _, w, C, _ = fe_time.time_matrices(p.k)
    s = stv.Solver(0)
    s.set_coarse_algorithm(algo)
    s.set_hierarchy(p.levels, p.dim, p.k)
    m, a = spatial_factors(p.levels[0])
    s.set_kron_factors(0, m, a, np.asarray(C, dtype=np.float64),
                       p.tau * np.asarray(w, dtype=np.float64))
    s.build_cell_inverses(full=True)
    r = np.random.default_rng(23).standard_normal(J.shape[0])
    for trans in (False, True):
        d = to_dev(np.zeros_like(r))
        if trans:
            s.vcycle_transposed(to_dev(r), d)
        else:
            s.coarse_solve(to_dev(r), d)
        d = to_host(d)
        A = J.T if trans else J
        ref = lu.solve(r, trans="T" if trans else "N")
        res = np.linalg.norm(r - A @ d) / np.linalg.norm(r)
        fe = relerr(d, ref)
        log(f"[coarse] {name} {algo} transposed={trans} relres {res:.2e} forward {fe:.2e}")
        assert res <= 1e-11
        assert fe <= 1e-15 * cond * 10
    s.close()


def test_coarse_algorithm_option_rejects_unknown(stv):
    s = stv.Solver(0)
    with pytest.raises(KeyError):
        s.set_coarse_algorithm("lu")
    with pytest.raises(stv.StvError):
        s._check(stv._lib.stv_set_option(s._h, 1, 7))
