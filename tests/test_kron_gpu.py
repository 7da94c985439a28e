"""Level residual from spatial factors (blocks = C[i,l] M + delta_il tau w_i A)
through the C ABI: it must reproduce the block residual and the oracle's
V-cycle and FGMRES; factors that do not reproduce the stored blocks are
rejected; transposed solves keep using the blocks."""
import numpy as np
import pytest

import oracle
from gpu_common import log, problem, relerr, to_dev, to_host
from oracle import adjoint as oadj
from stgen import fe
from stgen.problem import make_problem, spatial_factors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_2107_10561_amd as m
    return m


def time_factors(p):
    _, w, C, _ = fe.time_matrices(p.k)
    return np.asarray(C, dtype=np.float64), p.tau * np.asarray(w, dtype=np.float64)


def kron_solver(stv, p, full=False):
    s = stv.Solver(0)
    s.set_hierarchy(p.levels, p.dim, p.k)
    C, tw = time_factors(p)
    for g, L in enumerate(p.levels):
        m, a = spatial_factors(L)
        s.set_kron_factors(g, m, a, C, tw)
    s.build_cell_inverses(full=full)
    return s


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2", "3d_dg1"])
def test_kron_residual_vcycle_gmres(stv, name):
    p, ol = problem(name)
    s = kron_solver(stv, p)
    G = len(ol) - 1
    rng = np.random.default_rng(12)
    r, d = rng.standard_normal(ol[G].n_st), rng.standard_normal(ol[G].n_st)
    for rows in range(1, 13):   # (lanes per row, blocks per lane) shapes, one or two lists
        s.set_launch(G, rows, 0)
        out = to_dev(np.zeros(ol[G].n_st))
        s.residual(G, to_dev(r), to_dev(d), out)
        ref = r - ol[G].J @ d
        assert np.abs(to_host(out) - ref).max() <= 1e-13 * np.abs(ref).max()
    dd = to_dev(np.zeros(ol[G].n_st))
    s.vcycle(to_dev(r), dd, 2, 2, 0.7)
    assert relerr(to_host(dd), oracle.vcycle(ol, r, 2, 2, 0.7)) <= 1e-11
    cinv = oracle.coarse_inverse(ol[0])
    xf, _ = oracle.fgmres(lambda v: ol[-1].J @ v, p.rhs,
                          lambda v: oracle.vcycle(ol, v, 2, 2, 0.7, coarse_inv=cinv),
                          restart=30, fixed_iters=6)
    x = to_dev(np.zeros(ol[G].n_st))
    s.gmres_solve(to_dev(p.rhs), x, restart=30, fixed_iters=6)
    e = relerr(to_host(x), xf)
    log(f"[kron] {name} fgmres(6) rel err {e:.2e}")
    assert e <= 1e-10


def test_kron_rejects_inconsistent_factors_and_can_be_dropped(stv):
    p, ol = problem("c1_2d_dg1")
    s = stv.Solver(0)
    s.set_hierarchy(p.levels, p.dim, p.k)
    C, tw = time_factors(p)
    m, a = spatial_factors(p.levels[-1])
    bad = m.copy()
    bad[len(bad) // 2] *= 1.001
    with pytest.raises(stv.StvError, match="reproduce"):
        s.set_kron_factors(1, bad, a, C, tw)
    with pytest.raises(stv.StvError, match="reproduce"):
        s.set_kron_factors(1, m, a, C[::-1].copy(), tw)
    s.set_kron_factors(1, m, a, C, tw)
    s.set_kron_factors(1, None, None, None, None)
    s.build_cell_inverses()
    rng = np.random.default_rng(13)
    r, d = rng.standard_normal(ol[1].n_st), rng.standard_normal(ol[1].n_st)
    out = to_dev(np.zeros(ol[1].n_st))
    s.residual(1, to_dev(r), to_dev(d), out)
    ref = r - ol[1].J @ d
    assert np.abs(to_host(out) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_kron_batch(stv):
    specs = [(2, (16, 4), 2, 1, 0.01, 1e-3, 71), (2, (32, 8), 3, 1, 0.01, 3e-3, 72)]
    probs = [make_problem(*sp) for sp in specs]
    s = stv.Solver(0)
    s.set_batch([q.levels for q in probs], 2, 1)
    C, tw = time_factors(probs[0])
    D = s.n_levels
    for g in range(D):
        ms, as_ = [], []
        for q in probs:
            l = g - (D - len(q.levels))
            if l >= 0:
                m, a = spatial_factors(q.levels[l])
                ms.append(m)
                as_.append(a)
        s.set_kron_factors(g, np.concatenate(ms), np.concatenate(as_), C, tw)
    s.build_cell_inverses()
    b = np.concatenate([q.rhs for q in probs])
    x = to_dev(np.zeros_like(b))
    s.gmres_solve(to_dev(b), x, restart=30, fixed_iters=5)
    xh = to_host(x)
    for i, q in enumerate(probs):
        ol = oracle.build_inverses(oracle.prepare_levels(q.levels, q.b))
        cinv = oracle.coarse_inverse(ol[0])
        xf, _ = oracle.fgmres(lambda v: ol[-1].J @ v, q.rhs,
                              lambda v: oracle.vcycle(ol, v, 2, 2, 0.7, coarse_inv=cinv),
                              restart=30, fixed_iters=5)
        _, o, n = s.instance_layout(i)
        assert relerr(xh[o:o + n], xf) <= 1e-10


def test_transposed_solve_ignores_factors(stv):
    p, ol = problem("2d_dg2")
    s = kron_solver(stv, p, full=True)
    olt = oadj.transpose_levels(ol)
    r = np.random.default_rng(14).standard_normal(ol[-1].n_st)
    d = to_dev(np.zeros_like(r))
    s.vcycle_transposed(to_dev(r), d, 2, 2, 0.7)
    assert relerr(to_host(d), oracle.vcycle(olt, r, 2, 2, 0.7)) <= 1e-11


@pytest.mark.parametrize("name", ["2d_dg2", "c1_2d_dg1"])
def test_time_decoupled_coarse_inverse(stv, name):
    """With spatial factors on the coarsest level the coarse inverse is built
    from the diagonal blocks of the operator in the real Jordan basis of the
    time matrix D^-1 C (dG(2): one real eigenvalue and one complex pair;
    dG(1): a single pair), each block in real form of order 2 n_s and
    eliminated with complex pivots.  Both must reproduce the oracle's dense
    inverse, with and without the factors on the coarsest level."""
    p, ol = problem(name)
    s = kron_solver(stv, p)
    rng = np.random.default_rng(21)
    r = rng.standard_normal(ol[0].n_st)
    ref = oracle.coarse_inverse(ol[0]) @ r
    errs = []
    for drop in (False, True):
        if drop:
            s.set_kron_factors(0, None, None, None, None)
            s.build_cell_inverses()
        d = to_dev(np.zeros(ol[0].n_st))
        s.coarse_solve(to_dev(r), d)
        errs.append(relerr(to_host(d), ref))
    log(f"[kron] {name} coarse solve rel err: decoupled {errs[0]:.2e}, whole {errs[1]:.2e}")
    assert max(errs) <= 1e-10


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2"])
def test_time_decoupled_cell_inverses_and_sweeps(stv, name):
    """With spatial factors the owned-row store of a 2d level holds the
    cell inverses time-decoupled: J_T^-1 = (I (x) V) Q^-1 (I (x) W) with
    Q = M_T (x) T + A_T (x) I block diagonal in time, one stored row of
    B * n_loc values per owned spatial DoF (the real block's row, the real
    and imaginary parts of the complex block's row).  The owned rows of J_T^-1
    read back through the C ABI, one and two damped sweeps (FP64 and FP32
    stores) must match the oracle, which inverts J_T directly."""
    p, ol = problem(name)
    g = len(ol) - 1
    L = p.levels[g]
    own = oracle.owner_cells(L.cell_sdofs, L.n_sdofs)
    nls = L.cell_sdofs.shape[1]
    s = kron_solver(stv, p)
    for T in (0, 1, L.n_cells // 2, L.n_cells - 1):
        G = s.get_cell_inverse(g, T)
        O = ol[g].inv[T]
        owned_alpha = [a for a in range(nls) if own[L.cell_sdofs[T, a]] == T]
        rows = [l * nls + a for l in range(p.b) for a in owned_alpha]
        other = sorted(set(range(G.shape[0])) - set(rows))
        assert np.all(np.isnan(G[other]))
        assert np.abs(G[rows] - O[rows]).max() <= 1e-10 * np.abs(O).max()
    rng = np.random.default_rng(31)
    r = rng.standard_normal(ol[g].n_st)
    d0 = rng.standard_normal(ol[g].n_st)
    dd = to_dev(d0)
    s.vanka_sweep(g, to_dev(r), dd, 1, 0.7)
    d1 = to_host(dd)
    e1 = relerr(d1, oracle.vanka_sweep(ol[g], r, d0, 0.7))
    # persistent grids (each wavefront strides over several cells, fetching
    # the next cell's offsets ahead): bitwise the same result
    for w in (1, 3, 64):
        s.set_launch(g, 2, w)
        dd = to_dev(d0)
        s.vanka_sweep(g, to_dev(r), dd, 1, 0.7)
        assert np.array_equal(to_host(dd), d1), w
    s.set_launch(g, 2, 0)
    z = np.zeros(ol[g].n_st)
    ref2 = oracle.vanka_sweep(ol[g], r, oracle.vanka_sweep(ol[g], r, z, 0.7), 0.7)
    errs = []
    for fp32 in (False, True):
        s2 = stv.Solver(0)
        s2.set_hierarchy(p.levels, p.dim, p.k)
        C, tw = time_factors(p)
        for lv, Lv in enumerate(p.levels):
            m, a = spatial_factors(Lv)
            s2.set_kron_factors(lv, m, a, C, tw)
        s2.build_cell_inverses(fp32=fp32)
        dd = to_dev(z)
        s2.vanka_sweep(g, to_dev(r), dd, 2, 0.7)
        errs.append(relerr(to_host(dd), ref2))
    log(f"[kron] {name} decoupled sweeps rel err: one {e1:.2e}, two fp64 {errs[0]:.2e}, "
        f"two fp32 {errs[1]:.2e}")
    assert e1 <= 1e-12 and errs[0] <= 1e-12 and errs[1] <= 1e-5


def test_store_layout_follows_the_build(stv):
    """The inverse store keeps the layout of the build that made it: factors
    set after a build leave the plain owned-row store in use until the next
    build, which stores the time-decoupled rows; dropping the factors and
    rebuilding returns to the plain store.  Every state sweeps like the
    oracle."""
    p, ol = problem("2d_dg2")
    g = len(ol) - 1
    rng = np.random.default_rng(41)
    r, d0 = rng.standard_normal(ol[g].n_st), rng.standard_normal(ol[g].n_st)
    ref = oracle.vanka_sweep(ol[g], r, d0, 0.7)
    s = stv.Solver(0)
    s.set_hierarchy(p.levels, p.dim, p.k)
    s.build_cell_inverses()
    plain = s.level_info(g)["inverse_bytes"]
    C, tw = time_factors(p)
    for lv, Lv in enumerate(p.levels):
        m, a = spatial_factors(Lv)
        s.set_kron_factors(lv, m, a, C, tw)
    sizes = []
    for step in ("factors set, old store", "rebuilt", "dropped, rebuilt"):
        if step == "rebuilt":
            s.build_cell_inverses()
        if step == "dropped, rebuilt":
            for lv in range(len(p.levels)):
                s.set_kron_factors(lv, None, None, None, None)
            s.build_cell_inverses()
        sizes.append(s.level_info(g)["inverse_bytes"])
        dd = to_dev(d0)
        s.vanka_sweep(g, to_dev(r), dd, 1, 0.7)
        assert relerr(to_host(dd), ref) <= 1e-12, step
    assert sizes[0] == plain and sizes[2] == plain
    assert sizes[1] * p.b == plain     # one row per owned spatial DoF instead of k+1
