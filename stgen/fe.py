"""Reference-element data of the Q2 / P1disc x dG(k) discretisation.

Spaces (Section 2.3 of the paper, definition of V_h and Q_h with r = 2):
  * velocity: continuous Q2 Lagrange on tensor-product cells, nodes {0, 1/2, 1}
    per direction, numbered lexicographically with x fastest;
  * pressure: discontinuous P1 with the L2-orthonormal Legendre basis of the
    reference cell [0,1]^d (Remark 4.1): 1, sqrt3(2x-1), sqrt3(2y-1)[, sqrt3(2z-1)].
Time (Section 3, eq. (3.1)): Lagrange basis at the k+1 right Gauss-Radau nodes
of the reference interval (0, 1], whose last node is the end point.

Everything here is input generation: bases, quadrature and the exact time
matrices used to assemble the level operators.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly

SQRT3 = np.sqrt(3.0)


# ---------------------------------------------------------------- quadrature
def gauss01(n: int = 4):
    """n-point Gauss-Legendre rule mapped to [0, 1]."""
    t, w = npleg.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def tensor_rule(dim: int, n: int = 4):
    """Tensor-product Gauss rule on [0,1]^dim; points (nq, dim), x fastest."""
    x1, w1 = gauss01(n)
    grids = np.meshgrid(*([x1] * dim), indexing="ij")
    wg = np.meshgrid(*([w1] * dim), indexing="ij")
    # 'ij' indexing makes the first axis slowest; reverse so that x is fastest
    pts = np.stack([g.transpose(tuple(reversed(range(dim)))).ravel() for g in grids], axis=1)
    wts = np.prod(np.stack([g.transpose(tuple(reversed(range(dim)))).ravel() for g in wg], axis=1), axis=1)
    return pts, wts


# ---------------------------------------------------------------- 1d Q2 basis
def q2_1d(x):
    """Values of the three 1d quadratic Lagrange functions at nodes 0, 1/2, 1."""
    x = np.asarray(x, dtype=np.float64)
    return np.stack([2.0 * (x - 0.5) * (x - 1.0), -4.0 * x * (x - 1.0), 2.0 * x * (x - 0.5)], axis=-1)


def dq2_1d(x):
    x = np.asarray(x, dtype=np.float64)
    return np.stack([4.0 * x - 3.0, -8.0 * x + 4.0, 4.0 * x - 1.0], axis=-1)


def q2_nodes(dim: int):
    """Local Q2 node multi-indices (a, b[, c]) in lexicographic order, x fastest."""
    idx = np.array(np.meshgrid(*([np.arange(3)] * dim), indexing="ij"))
    idx = idx.reshape(dim, -1).T  # first axis slowest
    return idx[:, ::-1].copy()    # columns (a=x, b=y, c=z) with x fastest


def q2_tab(dim: int, pts):
    """phi[q, node] and reference gradients dphi[q, axis, node] at points (nq, dim)."""
    nodes = q2_nodes(dim)
    v = [q2_1d(pts[:, a]) for a in range(dim)]   # (nq, 3) each
    dv = [dq2_1d(pts[:, a]) for a in range(dim)]
    nq, nn = pts.shape[0], nodes.shape[0]
    phi = np.ones((nq, nn))
    for a in range(dim):
        phi *= v[a][:, nodes[:, a]]
    dphi = np.ones((nq, dim, nn))
    for g in range(dim):
        for a in range(dim):
            dphi[:, g, :] *= (dv[a] if a == g else v[a])[:, nodes[:, a]]
    return phi, dphi


def p1disc_tab(dim: int, pts):
    """Legendre P1 pressure basis xi[q, m], m = 0..dim, orthonormal on [0,1]^dim."""
    cols = [np.ones(pts.shape[0])] + [SQRT3 * (2.0 * pts[:, a] - 1.0) for a in range(dim)]
    return np.stack(cols, axis=1)


def n_local_spatial(dim: int) -> int:
    """Local spatial DoFs of one cell: dim * 3^dim velocity + (dim + 1) pressure.

    The pressure count is dim P_{r-1} = binom(d + r - 1, r - 1) = d + 1 for r = 2.
    """
    return dim * 3 ** dim + dim + 1


# ---------------------------------------------------------------- time (dG(k))
def radau_right(k: int):
    """Nodes and weights of the (k+1)-point right Gauss-Radau rule on (0, 1].

    The nodes on [-1, 1] are the roots of P_k - P_{k+1}; the end point is one.
    Weights integrate the Lagrange polynomials exactly.
    """
    if k == 0:
        return np.array([1.0]), np.array([1.0])
    c = np.zeros(k + 2)
    c[k] = 1.0
    c[k + 1] = -1.0
    r = np.sort(np.real(npleg.legroots(c)))
    t = 0.5 * (r + 1.0)
    t[-1] = 1.0
    w = np.array([_integrate01(_lagrange(t, i)) for i in range(k + 1)])
    return t, w


def _lagrange(nodes, i):
    """Power-series coefficients of the i-th Lagrange polynomial on nodes."""
    p = np.array([1.0])
    for j, tj in enumerate(nodes):
        if j != i:
            p = nppoly.polymul(p, np.array([-tj, 1.0]) / (nodes[i] - tj))
    return p


def _integrate01(p):
    P = nppoly.polyint(p)
    return nppoly.polyval(1.0, P) - nppoly.polyval(0.0, P)


def time_matrices(k: int):
    """Exact reference time matrices of dG(k) with the Radau-Lagrange basis.

    Returns (nodes, weights, C, chi0) where
      C[i, l] = int_0^1 chi_l'(t) chi_i(t) dt + chi_l(0) chi_i(0)  (i = test),
      chi0[i] = chi_i(0).
    The time mass int chi_l chi_i = w_i delta_il because the rule is exact
    for degree 2k and the basis interpolates at its nodes.
    """
    t, w = radau_right(k)
    b = k + 1
    L = [_lagrange(t, i) for i in range(b)]
    C = np.zeros((b, b))
    chi0 = np.array([nppoly.polyval(0.0, L[i]) for i in range(b)])
    for i in range(b):
        for l in range(b):
            C[i, l] = _integrate01(nppoly.polymul(nppoly.polyder(L[l]), L[i])) + chi0[l] * chi0[i]
    return t, w, C, chi0


def lagrange_eval(nodes, t):
    """chi_i(t) for all i at points t: array (len(t), len(nodes))."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.stack([nppoly.polyval(t, _lagrange(nodes, i)) for i in range(len(nodes))], axis=1)
