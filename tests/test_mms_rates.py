"""Manufactured-solution convergence rates of the assembled space-time operator.

Pins the assembly (Section 2.3: Q2 velocity / P1disc pressure, Nitsche's
boundary form eq. (2.4) with its penalty scale gamma/h, the semilinear form
eq. (2.5) at a frozen convection field; Problem 3.1 in time) where the
patch test cannot: smooth, non-polynomial data, so that quadrature of the
data and the h-scaling of the Nitsche terms decide the error.  Expected
orders for this pair of spaces: velocity L2 error O(h^3), pressure L2 error
O(h^2).  The exact solution is of degree <= k in time, which dG(k) with the
exact initial value integrates without time error, so the observed order is
the spatial one.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import sympy as sy

from stgen import fe
from stgen.assemble import assemble_level
from stgen.mesh import Mesh
from stgen.problem import Convection
from stgen.rhs import assemble_rhs

EXT = (2.2, 0.41)


def _manufactured(k, nu, conv):
    """Divergence-free velocity from a stream function times a polynomial in
    time of degree k; smooth pressure; the data f, the outflow traction
    (nu d_x v - p e_x at x = L) and the exact fields as numpy callables."""
    x, y, t = sy.symbols("x y t")
    T = sum((sy.Rational(1, 2) - sy.Rational(j, 5)) * t ** j for j in range(k + 1)) + 1
    psi = sy.sin(2 * x + sy.Rational(1, 2)) * sy.cos(5 * y + sy.Rational(1, 3)) / 3
    v = [sy.diff(psi, y) * T, -sy.diff(psi, x) * T]
    p = sy.cos(3 * x) * sy.sin(4 * y + 1) * (1 - t / 3)
    X = (x, y)
    lam = lambda e: sy.lambdify((x, y, t), e, "numpy")
    dv = [[lam(sy.diff(v[c], X[a])) for a in range(2)] for c in range(2)]
    lap = [lam(sy.diff(v[c], x, 2) + sy.diff(v[c], y, 2)) for c in range(2)]
    dvt = [lam(sy.diff(v[c], t)) for c in range(2)]
    dp = [lam(sy.diff(p, X[a])) for a in range(2)]
    vf = [lam(v[c]) for c in range(2)]
    pf = lam(p)

    def bcast(fn, P, tt):
        return np.broadcast_to(fn(P[:, 0], P[:, 1], tt), (P.shape[0],)).astype(np.float64)

    def f(P, tt):
        b = conv(P)
        out = np.zeros((P.shape[0], 2))
        for c in range(2):
            out[:, c] = bcast(dvt[c], P, tt) - nu * bcast(lap[c], P, tt) + bcast(dp[c], P, tt)
            for a in range(2):
                out[:, c] += b[:, a] * bcast(dv[c][a], P, tt)
        return out

    def vel(P, tt):
        return np.stack([bcast(vf[c], P, tt) for c in range(2)], axis=1)

    def traction(P, tt):
        out = np.stack([nu * bcast(dv[c][0], P, tt) for c in range(2)], axis=1)
        out[:, 0] -= bcast(pf, P, tt)
        return out

    return f, vel, (lambda P, tt: bcast(pf, P, tt)), traction


def _l2_errors(m, U, k, tau, t0, vel, pres):
    """L2(Omega) errors of velocity and pressure at every Radau node of the
    subinterval (6-point Gauss rule per direction on every cell)."""
    d, b = 2, k + 1
    tn, _, _, _ = fe.time_matrices(k)
    pts, wts = fe.tensor_rule(d, 6)
    phi, _ = fe.q2_tab(d, pts)
    xi = fe.p1disc_tab(d, pts)
    h = np.array(m.h)
    vol = float(np.prod(h))
    csd = m.cell_sdofs().astype(np.int64)
    X = (m.cell_origin()[:, None, :] + pts[None, :, :] * h[None, None, :]).reshape(-1, d)
    nv = 9
    ev, ep = [], []
    for i in range(b):
        ti = t0 + tau * tn[i]
        loc = U[csd * b + i]                                   # (nc, n_ls)
        vh = np.stack([loc[:, c * nv:(c + 1) * nv] @ phi.T for c in range(d)], axis=2).reshape(-1, d)
        ph = (loc[:, d * nv:] @ xi.T).reshape(-1)
        w = np.tile(wts * vol, m.n_cells)
        ev.append(np.sqrt(np.sum(w * np.sum((vh - vel(X, ti)) ** 2, axis=1))))
        ep.append(np.sqrt(np.sum(w * (ph - pres(X, ti)) ** 2)))
    return max(ev), max(ep)


def _solve_errors(n, k, nu, tau, t0, conv):
    m = Mesh(2, n, EXT)
    f, vel, pres, traction = _manufactured(k, nu, conv)
    A = assemble_level(m, k, tau, np.full(m.n_cells, nu), conv)
    b = k + 1
    J = sp.bsr_matrix((A["val"], A["col"], A["rowptr"]), shape=(m.n_sdofs * b,) * 2).tocsc()
    F = assemble_rhs(m, k, tau, nu, t0, f, vel, lambda P: vel(P, t0), traction, None)
    U = spla.spsolve(J, F)
    return _l2_errors(m, U, k, tau, t0, vel, pres)


@pytest.mark.parametrize("k", [1, 2])
def test_mms_spatial_rates(k):
    """Observed orders on three nested meshes: velocity ~3, pressure ~2."""
    nu, tau, t0 = 0.05, 0.1, 0.2
    conv = Convection(2, EXT, np.random.default_rng(41).standard_normal(4)).normalise()
    meshes = [(8, 2), (16, 4), (32, 8)]
    errs = [_solve_errors(n, k, nu, tau, t0, conv) for n in meshes]
    ev = np.array([e[0] for e in errs])
    ep = np.array([e[1] for e in errs])
    rv = np.log2(ev[:-1] / ev[1:])
    rp = np.log2(ep[:-1] / ep[1:])
    print(f"k={k} velocity errors {ev} rates {rv}; pressure errors {ep} rates {rp}")
    assert rv[-1] >= 2.7 and rv[-1] <= 3.4, rv
    assert rp[-1] >= 1.8 and rp[-1] <= 2.4, rp
    assert np.all(np.diff(ev) < 0) and np.all(np.diff(ep) < 0)
