"""Pins of the Newton linearisation / time-marching inputs and of the oracle's
Newton iteration, on the CPU."""
import numpy as np
import pytest

from oracle.newton import march_direct, newton_direct
from oracle.smoother import spacetime_matrix
from stgen import fe
from stgen.mesh import Mesh
from stgen.newton import NewtonLevel, NewtonProblem, inject, time_triple
from stgen.problem import H2D, L2D
from stgen.rhs import assemble_rhs, interpolate


@pytest.mark.parametrize("k", [1, 2])
def test_time_triple_closed_forms(k):
    """sum_m T[i,l,m] = int chi_i chi_l = w_i delta_il; T is symmetric."""
    T = time_triple(k)
    _, w, _, _ = fe.time_matrices(k)
    assert np.allclose(T.sum(axis=2), np.diag(w), atol=1e-15)
    assert np.allclose(T, T.transpose(1, 0, 2)) and np.allclose(T, T.transpose(2, 1, 0))


@pytest.mark.parametrize("k", [1, 2])
def test_jacobian_is_the_residual_derivative(k):
    """R is quadratic: central differences of R equal J(u) d to rounding."""
    m = Mesh(2, (8, 2), (L2D, H2D))
    NL = NewtonLevel(m, k, 0.05, 1e-2)
    rng = np.random.default_rng(k)
    b = k + 1
    u = 0.3 * rng.standard_normal(m.n_sdofs * b)
    F = rng.standard_normal(m.n_sdofs * b)
    J = spacetime_matrix(NL.rowptr, NL.col, NL.jacobian(u), m.n_sdofs, b)
    d = rng.standard_normal(u.size)
    h = 1e-5
    fd = (NL.residual(u + h * d, F) - NL.residual(u - h * d, F)) / (2 * h)
    assert np.abs(J @ d - fd).max() <= 1e-9 * np.abs(fd).max()


def test_jacobian_time_blocks_are_full():
    """A time-dependent linearisation point couples different time levels
    through the convection term (beyond the time-derivative coupling)."""
    m = Mesh(2, (8, 2), (L2D, H2D))
    NL = NewtonLevel(m, 1, 0.05, 1e-2)
    u = np.zeros(m.n_sdofs * 2)
    u[0::2] = 0.0
    u[1::2] = np.random.default_rng(3).standard_normal(m.n_sdofs)     # v at t_1 only
    val = NL.jacobian(u)
    lin = NL.jacobian(np.zeros_like(u))
    diff = val - lin
    assert np.abs(diff[:, 0, 1]).max() > 1e-6 and np.abs(diff[:, 1, 0]).max() > 1e-6


def _patch():
    """v = (1 + t y, 1/2), p = x: divergence free, f = d_t v + (v.grad) v + grad p."""
    vf = lambda X, t: np.stack([1 + t * X[:, 1], 0.5 * np.ones(len(X))], 1)
    f = lambda X, t: np.stack([X[:, 1] + 0.5 * t + 1, np.zeros(len(X))], 1)
    tr = lambda X, t: np.stack([-X[:, 0], np.zeros(len(X))], 1)   # nu d_n v - p n at x = L

    def pco(origin, h, t):
        c = np.zeros((len(origin), 3))
        c[:, 0] = origin[:, 0] + h[0] / 2
        c[:, 1] = h[0] / (2 * np.sqrt(3))
        return c
    return vf, f, tr, pco


class _OneLevel:
    def __init__(self, NL):
        self.NL, self.b = NL, NL.b

    def residual(self, u, F):
        return self.NL.residual(u, F)

    def hierarchy(self, u):
        return [dict(n_sdofs=self.NL.mesh.n_sdofs, rowptr=self.NL.rowptr, col=self.NL.col,
                     val=self.NL.jacobian(u), cell_sdofs=self.NL.csd, P=None)]


def test_navier_stokes_patch_is_reproduced_by_newton_marching():
    """A solution in the discrete space (Q1 velocity linear in time, P1
    pressure) is reproduced exactly over three subintervals: the residual of
    its interpolant vanishes and the Newton iteration returns it."""
    m = Mesh(2, (8, 2), (L2D, H2D))
    k, tau, nu = 1, 0.05, 1e-2
    NL = NewtonLevel(m, k, tau, nu)
    vf, f, tr, pco = _patch()
    v_prev = interpolate(m, 0, 1.0, 0.0, lambda X, t: vf(X, 0.0),
                         lambda o, h, t: np.zeros((len(o), 3))).reshape(-1)
    u = np.zeros(m.n_sdofs * 2)
    prob = _OneLevel(NL)
    for n in range(3):
        t0 = n * tau
        F = assemble_rhs(m, k, tau, nu, t0, f, vf, lambda X: np.zeros_like(X), traction=tr)
        F += NL.jump_term(v_prev)
        ust = interpolate(m, k, tau, t0, vf, pco)
        assert np.abs(NL.residual(ust, F)).max() <= 1e-14 * np.abs(F).max() * 10
        u, hist = newton_direct(prob, u, F, tol=1e-13)
        assert np.abs(u - ust).max() <= 1e-10 * np.abs(ust).max()
        v_prev = u.reshape(-1, 2)[:, -1].copy()


def test_injection_reproduces_coarse_functions():
    fine = Mesh(2, (16, 4), (L2D, H2D))
    coarse = fine.coarsen()
    q = lambda X: np.stack([X[:, 0] ** 2 - X[:, 1], X[:, 0] * X[:, 1]], 1)

    def vec(M):
        out = np.zeros(M.n_sdofs * 2)
        V = q(M.node_coords())
        for c in range(2):
            for l in range(2):
                out[(np.arange(M.n_vnodes) * 2 + c) * 2 + l] = V[:, c]
        return out
    assert np.array_equal(inject(fine, coarse, vec(fine), 2), vec(coarse))


def test_oracle_marching_converges_quadratically():
    prob = NewtonProblem(2, (16, 4), 2, 1, 0.05, 1e-2)
    out = march_direct(prob, np.zeros(prob.fine.mesh.n_sdofs), 2, tol=1e-12)
    for u, hist in out:
        assert hist[-1] <= 1e-12 and len(hist) <= 8
        # quadratic tail: each step squares the error (up to a constant)
        assert hist[-2] <= 1e-4 or len(hist) <= 3
