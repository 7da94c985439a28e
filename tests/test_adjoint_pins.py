"""Pins of the differentiation workload's data (generator) and of the
oracle's adjoint gradient, on the CPU."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle.smoother import spacetime_matrix
from stgen import adjoint as gadj
from stgen.assemble import assemble_level
from stgen.mesh import Mesh
from stgen.problem import H2D, L2D, Convection
from stgen.rhs import assemble_rhs


def _mesh():
    return Mesh(2, (8, 2), (L2D, H2D))


def test_rhs_split_equals_nitsche_data_terms():
    """Uniform viscosity: U (F0 + nu sum_c Fc) is the Nitsche right-hand side
    of the parabolic inflow (the patch-tested data-term assembly)."""
    m = _mesh()
    nu, U = 2e-3, 1.7
    g = lambda X, t: np.stack([U * gadj._profile(X, m.ext, 2), np.zeros(len(X))], 1)
    ref = assemble_rhs(m, 1, 0.01, nu, 0.0, lambda X, t: np.zeros_like(X), g,
                       lambda X: np.zeros_like(X))
    mine = gadj.physical_rhs(m, 1, 0.01, np.full(m.n_cells, nu), U)
    assert np.abs(ref - mine).max() <= 1e-15 * np.abs(ref).max() * 10


@pytest.mark.parametrize("cell", [0, 3, 9, 15])
def test_nu_derivative_refs_are_the_operator_derivative(cell):
    """J is affine in nu_c: central differences of the assembled operator
    equal W_tau (x) K_c scattered into the cell's blocks."""
    m = _mesh()
    k, tau = 1, 0.01
    conv = Convection(2, m.ext, np.array([0.3, -0.2, 0.5, 0.1])).normalise()
    nuc = 1e-3 * np.exp(0.3 * np.random.default_rng(0).standard_normal(m.n_cells))
    refs, ptr, idx, w = gadj.nu_derivative_refs(m)
    tw = gadj.time_weights(k, tau)
    h = 1e-4
    e = np.zeros(m.n_cells)
    e[cell] = h
    Ap = assemble_level(m, k, tau, nuc + e, conv, pattern="full")
    Am = assemble_level(m, k, tau, nuc - e, conv, pattern="full")
    D = (Ap["val"] - Am["val"]) / (2 * h)
    Kc = sum(w[q] * refs[idx[q]] for q in range(ptr[cell], ptr[cell + 1]))
    csd = m.cell_sdofs()[cell]
    rp, col = Ap["rowptr"], Ap["col"]
    E = np.zeros_like(D)
    for a in range(m.n_ls):
        for b in range(m.n_ls):
            r = csd[a]
            q = rp[r] + np.searchsorted(col[rp[r]:rp[r + 1]], csd[b])
            E[q] += np.diag(tw) * Kc[a, b]
    assert np.abs(D - E).max() <= 1e-11 * np.abs(E).max()


def test_loss_vector_closed_forms():
    """v_1 = 1: L = tau * int_0^H w = tau 2H/3;  v_1 = y: L = tau H^2/3."""
    m = _mesh()
    q = gadj.outflow_loss_vector(m, 1, 0.01)
    X = m.node_coords()
    for f, exact in ((lambda y: np.ones_like(y), 0.01 * 2 * H2D / 3),
                     (lambda y: y, 0.01 * H2D ** 2 / 3)):
        x = np.zeros(m.n_sdofs * 2)
        v = f(X[:, 1])
        for i in range(2):
            x[(np.arange(m.n_vnodes) * 2) * 2 + i] = v
        assert abs(q @ x - exact) <= 1e-14


def _problem(nu=None, U=1.0):
    return gadj.make_differentiation_problem((16, 4), 2, 1, 0.01, 3000, U=U, nu=nu)


def _oracle_grad(p):
    m = p.levels[-1].mesh
    L = p.levels[-1]
    J = spacetime_matrix(L.rowptr, L.col, L.val, L.n_sdofs, 2)
    refs, ptr, idx, w = gadj.nu_derivative_refs(m)
    F0, cells, Fc = gadj.inflow_rhs_parts(m, 1, 0.01)
    return oadj.loss_gradient(J, p.rhs, p.loss, p.meta["U"], p.nu_cell, m.cell_sdofs(), 2, refs,
                              ptr, idx, w, gadj.time_weights(1, 0.01), F0, cells, Fc)


def _loss(nu, U=1.0):
    p = _problem(nu, U)
    L = p.levels[-1]
    J = spacetime_matrix(L.rowptr, L.col, L.val, L.n_sdofs, 2)
    x, _ = oadj.solve_and_adjoint(J, p.rhs, p.loss)
    return p.loss @ x


def test_adjoint_gradient_matches_central_differences():
    p = _problem()
    Lval, g, gU, _, _ = _oracle_grad(p)
    rng = np.random.default_rng(1)
    cells = list(rng.choice(p.levels[-1].n_cells, 8, replace=False)) + [0, 3, 60, 63]
    h = 1e-6
    for c in cells:
        e = np.zeros_like(p.nu_cell)
        e[c] = h
        fd = (_loss(p.nu_cell + e) - _loss(p.nu_cell - e)) / (2 * h)
        assert abs(fd - g[c]) <= 1e-6 * np.abs(g).max(), (c, fd, g[c])
    # L is linear in the inflow amplitude
    assert abs(gU - Lval) <= 1e-12 * abs(Lval)
    assert abs(_loss(p.nu_cell, 2.5) - 2.5 * Lval) <= 1e-12 * abs(Lval)


def test_transposed_hierarchy_special_cases():
    """Vanka-GMG of J^T: a one-level cycle is the direct solve of J^T, and
    the local inverses are the transposes of J's."""
    import oracle
    from stgen.problem import make_problem
    p = make_problem(2, (8, 2), 2, 1, 0.01, 1e-3, 5)
    ol = oracle.build_inverses(oracle.prepare_levels(p.levels, p.b))
    olt = oadj.transpose_levels(ol)
    for T in (0, 5, 15):
        assert np.allclose(olt[1].inv[T], ol[1].inv[T].T, rtol=1e-12, atol=1e-12 * np.abs(ol[1].inv[T]).max())
    r = np.random.default_rng(2).standard_normal(ol[0].n_st)
    d = oracle.vcycle(olt[:1], r, 2, 2, 0.7)
    assert np.linalg.norm(ol[0].J.T @ d - r) <= 1e-12 * np.linalg.norm(r) * 1e3
