"""Helpers of the full-size parity tests: a solver set up exactly as bench.py
sets up its timed steps, and sampled comparisons with the oracle computed one
cell at a time.  Inputs come from the seeded generator; expected values from
the oracle (and a sparse direct solve) only."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from gpu_common import log, relerr, to_dev, to_host
from stgen import fe
from stgen.problem import spatial_factors


def _J(L, b):
    return sp.bsr_matrix((np.asarray(L.val).reshape(-1, b, b), L.col, L.rowptr),
                         shape=(L.n_sdofs * b,) * 2)


def bench_solver(p, fp32=False):
    """A solver set up exactly as bench.py sets up its timed steps."""
    import paper_2107_10561_amd as stv
    s = stv.Solver(0)
    s.set_hierarchy(p.levels, p.dim, p.k)
    _, w, C, _ = fe.time_matrices(p.k)
    tw = p.tau * np.asarray(w, dtype=np.float64)
    for g, L in enumerate(p.levels):
        m, a = spatial_factors(L)
        s.set_kron_factors(g, m, a, np.asarray(C), tw)
    s.build_cell_inverses(fp32=fp32)
    shapes = s.autotune()
    log(f"[bench-path] autotuned shapes {shapes}")
    return s, stv


def check_transfers(p, s, rng, shapes=(0,)):
    """Restriction and prolongation between every pair of levels, whole
    vectors, against P^T rho and d + P d_c formed by scipy from the level's own
    CSR prolongation (I_B in time); shape 0 keeps the shapes in force (the
    autotuned ones), 1..5 force 1..16 lanes per row.  Returns the worst
    relative error."""
    import scipy.sparse as sp
    b = p.b
    worst = 0.0
    for g in range(1, len(p.levels)):
        L, Lc = p.levels[g], p.levels[g - 1]
        rp, col, val = L.P
        P = sp.csr_matrix((val, col, rp), shape=(L.n_sdofs, Lc.n_sdofs))
        kept = s.transfer_shapes(g)
        for t in shapes:
            s.transfer_shapes(g, t, t)
            rho = rng.standard_normal((L.n_sdofs, b))
            rc = to_dev(np.zeros(Lc.n_sdofs * b))
            s.restrict(g, to_dev(rho.ravel()), rc)
            ref = (P.T @ rho).ravel()
            worst = max(worst, np.abs(to_host(rc) - ref).max() / np.abs(ref).max())
            dc = rng.standard_normal((Lc.n_sdofs, b))
            d = rng.standard_normal((L.n_sdofs, b))
            dd = to_dev(d.ravel())
            s.prolongate_add(g, to_dev(dc.ravel()), dd)
            ref = (d + P @ dc).ravel()
            worst = max(worst, np.abs(to_host(dd) - ref).max() / np.abs(ref).max())
        s.transfer_shapes(g, *kept)
    return worst


def sample_cells(n_cells, rng, extra=()):
    base = [0, n_cells - 1] + [c for c in extra if c < n_cells]
    pick = rng.choice(n_cells, min(n_cells, 20), replace=False)
    return np.unique(np.concatenate([np.asarray(base, dtype=np.int64), pick]))


def check_inverse_rows(p, s, rng, extra=(), tol=1e-10):
    """Owned rows of sampled cells on every smoothed level against the oracle's
    inverse of the extracted J_T (relative Frobenius error per cell)."""
    b = p.b
    worst = 0.0
    for g in range(1, len(p.levels)):
        L = p.levels[g]
        own = oracle.owner_cells(L.cell_sdofs, L.n_sdofs)
        nls = L.cell_sdofs.shape[1]
        for T in sample_cells(L.n_cells, rng, extra):
            JT = oracle.extract_cell_matrix_blocks(L.rowptr, L.col, L.val, b, L.cell_sdofs[T])
            O = oracle.cell_inverse(JT)
            G = s.get_cell_inverse(g, int(T))
            rows = [l * nls + a for l in range(b) for a in range(nls)
                    if own[L.cell_sdofs[T, a]] == T]
            e = np.linalg.norm(G[rows] - O[rows]) / np.linalg.norm(O[rows])
            worst = max(worst, e)
            assert e <= tol, (g, int(T), e)
    return worst


def check_residual_rows(p, s, g, rng, n_rows=4000):
    L = p.levels[g]
    n = L.n_sdofs * p.b
    r, d = rng.standard_normal(n), rng.standard_normal(n)
    out = to_dev(np.zeros(n))
    s.residual(g, to_dev(r), to_dev(d), out)
    got = to_host(out)
    J = _J(L, p.b).tocsr()
    rows = np.concatenate([rng.choice(n, min(n, n_rows), replace=False), [0, n - 1]])
    ref = r[rows] - J[rows] @ d
    e = np.abs(got[rows] - ref).max() / np.abs(ref).max()
    assert e <= 1e-13, (g, e)
    return e


def check_sweep(p, s, g, rng, fp32, n_sdofs=200):
    """d_new[j] = d[j] + omega (J_T^-1 rho_T)[loc(j)] for the owner T of j.

    FP64 store: |error| <= 1e-11 max(1, |d_new[j]|).  FP32 store: every stored
    value carries a relative rounding of 2^-24, the (time-decoupled) store's
    recombination can amplify it by the condition of the time basis, and the
    row product accumulates n_loc such terms; the bound is therefore taken
    relative to the absolute row sum: |error| <= 5e-5 omega sum_i
    |(J_T^-1)_{ji} rho_i| (n_loc 2^-24 is 3.8e-6 for n_loc = 63 and 1.0e-5 for
    170)."""
    b = p.b
    L = p.levels[g]
    n = L.n_sdofs * b
    r, d = rng.standard_normal(n), rng.standard_normal(n)
    dd = to_dev(d)
    s.vanka_sweep(g, to_dev(r), dd, 1, 0.7)
    got = to_host(dd)
    rho = r - _J(L, b) @ d
    own = oracle.owner_cells(L.cell_sdofs, L.n_sdofs)
    nls = L.cell_sdofs.shape[1]
    sdofs = np.unique(np.concatenate([rng.choice(L.n_sdofs, n_sdofs, replace=False),
                                      [0, L.n_sdofs - 1]]))
    worst = 0.0
    for sd in sdofs:
        T = int(own[sd])
        idx = oracle.cell_dofs(L.cell_sdofs[T:T + 1], b)[0]
        JT = oracle.extract_cell_matrix_blocks(L.rowptr, L.col, L.val, b, L.cell_sdofs[T])
        inv = oracle.cell_inverse(JT)
        c = inv @ rho[idx]
        a = int(np.nonzero(L.cell_sdofs[T] == sd)[0][0])
        for l in range(b):
            j = l * nls + a
            ref = d[sd * b + l] + 0.7 * c[j]
            if fp32:
                scale = 0.7 * np.abs(inv[j] * rho[idx]).sum()
                e = abs(got[sd * b + l] - ref) / scale / 5e-5
            else:
                e = abs(got[sd * b + l] - ref) / max(1.0, abs(ref)) / 1e-11
            worst = max(worst, e)
    assert worst <= 1.0, (g, worst)
    return worst


def check_coarse(p, s, rng):
    L0 = p.levels[0]
    n = L0.n_sdofs * p.b
    r = rng.standard_normal(n)
    x = to_dev(np.zeros(n))
    s.coarse_solve(to_dev(r), x)
    ref = spla.splu(_J(L0, p.b).tocsc()).solve(r)
    e = relerr(to_host(x), ref)
    assert e <= 1e-11, e
    return e


def check_gmres(p, s):
    L = p.levels[-1]
    n = L.n_sdofs * p.b
    x = to_dev(np.zeros(n))
    info = s.gmres_solve(to_dev(p.rhs), x, restart=30, rtol=1e-8)
    xg = to_host(x)
    true = np.linalg.norm(p.rhs - _J(L, p.b) @ xg) / np.linalg.norm(p.rhs)
    assert info["converged"] and true <= 1e-8, (info, true)
    assert abs(info["true_relres"] - true) <= 1e-3 * true
    return info["iters"], true
