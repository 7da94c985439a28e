"""Pins of the seeded problem generator (the assembled level operators)."""
import numpy as np
import pytest
import scipy.sparse as sp

from polyfield import Poly, momentum_data, vec_eval
from stgen import fe
from stgen.assemble import RefData, assemble_level, level_constant_parts, cell_operators
from stgen.mesh import Mesh, prolongation
from stgen.rhs import assemble_rhs, interpolate

GOLD = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _read_radau():
    s6 = np.sqrt(6.0)
    out, cur, rows = {}, None, []
    for line in open(f"{GOLD}/radau_iia.txt"):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("k="):
            if cur is not None:
                out[cur] = np.array(rows)
            cur, rows = int(line[2:]), []
        else:
            rows.append([eval(t, {"sqrt6": s6}) for t in line.split()])
    out[cur] = np.array(rows)
    return out


@pytest.mark.parametrize("k", [0, 1, 2])
def test_time_matrices_are_radau_iia(k):
    t, w, C, chi0 = fe.time_matrices(k)
    A = _read_radau()[k]
    np.testing.assert_allclose(np.linalg.inv(np.diag(1.0 / w) @ C), A, atol=1e-13)
    assert t[-1] == 1.0
    np.testing.assert_allclose(w.sum(), 1.0, atol=1e-15)


def test_time_matrix_k1_closed_form():
    _, w, C, _ = fe.time_matrices(1)
    np.testing.assert_allclose(w, [0.75, 0.25], atol=1e-15)
    np.testing.assert_allclose(C, [[9 / 8, 3 / 8], [-9 / 8, 5 / 8]], atol=1e-14)


def test_radau_stability_function():
    """For y' = -lam y one dG(k) step reproduces the Radau IIA stability
    function (the (k, k+1) Pade approximant of exp(-z))."""
    z = 0.7
    pade = {0: 1 / (1 + z), 1: (1 - z / 3) / (1 + 2 * z / 3 + z * z / 6),
            2: (1 - 2 * z / 5 + z * z / 20) / (1 + 3 * z / 5 + 3 * z * z / 20 + z ** 3 / 60)}
    for k in range(3):
        _, w, C, chi0 = fe.time_matrices(k)
        # (C + z W) Y = chi0 * y0, end value = Y[-1] (last node is t = 1)
        Y = np.linalg.solve(C + z * np.diag(w), chi0 * 1.0)
        np.testing.assert_allclose(Y[-1], pade[k], rtol=1e-13)


def test_q2_1d_closed_form():
    lines = [l.split() for l in open(f"{GOLD}/q2_1d.txt") if l.strip() and not l.startswith("#")]
    M30 = np.array(lines[1:4], dtype=float)
    K3 = np.array(lines[5:8], dtype=float)
    h = 0.37
    x, w = fe.gauss01(4)
    phi, dphi = fe.q2_1d(x), fe.dq2_1d(x)
    M = h * np.einsum("q,qi,qj->ij", w, phi, phi)
    K = np.einsum("q,qi,qj->ij", w, dphi, dphi) / h
    np.testing.assert_allclose(M, h / 30 * M30, atol=1e-15)
    np.testing.assert_allclose(K, K3 / (3 * h), atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_tensor_mass_and_pressure_orthonormal(dim):
    h = (0.3, 0.2, 0.25)[:dim]
    const = level_constant_parts(RefData(dim), h)
    x, w = fe.gauss01(4)
    m1 = [hh * np.einsum("q,qi,qj->ij", w, fe.q2_1d(x), fe.q2_1d(x)) for hh in h]
    M = m1[0]
    for a in range(1, dim):
        M = np.kron(m1[a], M)      # x fastest
    np.testing.assert_allclose(const["Mv"], M, atol=1e-15)
    ref = RefData(dim)
    Mp = np.einsum("q,qm,qn->mn", ref.wts, ref.xi, ref.xi) * np.prod(h)
    np.testing.assert_allclose(Mp, np.prod(h) * np.eye(dim + 1), atol=1e-15)


def test_sizes_closed_forms():
    for line in open(f"{GOLD}/paper_sizes.txt"):
        if line.startswith("#") or not line.strip():
            continue
        dim, k, nloc, nbytes = map(int, line.split())
        assert (k + 1) * fe.n_local_spatial(dim) == nloc
        assert nloc * nloc * 8 == nbytes
    for n in [(16, 4), (5, 3)]:
        m = Mesh(2, n, (2.2, 0.41))
        assert m.n_sdofs == 2 * (2 * n[0] + 1) * (2 * n[1] + 1) + 3 * n[0] * n[1]
    assert Mesh(2, (16, 4), (2.2, 0.41)).n_sdofs * 2 == 1572


def _patch(dim, n, k, nu, bconst, v, p, tau=0.1, t0=0.3):
    ext = (2.2, 0.41) if dim == 2 else (2.5, 0.41, 0.41)
    m = Mesh(dim, n, ext)
    conv = lambda X: np.tile(np.array(bconst)[None, :], (X.shape[0], 1))
    A = assemble_level(m, k, tau, np.full(m.n_cells, nu), conv)
    bb = k + 1
    J = sp.bsr_matrix((A["val"], A["col"], A["rowptr"]), shape=(m.n_sdofs * bb, m.n_sdofs * bb))
    f = momentum_data(v, p, bconst, nu, dim)
    div = v[0].d(0)
    for a in range(1, dim):
        div = div + v[a].d(a)
    vf = vec_eval(v)

    def traction(X, t):
        out = np.stack([nu * v[c].d(0)(X, t) for c in range(dim)], axis=1)
        out[:, 0] -= p(X, t)
        return out

    F = assemble_rhs(m, k, tau, nu, t0, vec_eval(f), vf, lambda X: vf(X, t0), traction,
                     lambda X, t: div(X, t))

    def pco(origin, h, t):
        cols = [p(origin + h[None, :] / 2, t)]
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = 1
            cols.append((p(origin + e[None, :], t) - p(origin, t)) * h[a] / (2 * np.sqrt(3)))
        return np.stack(cols, axis=1)

    U = interpolate(m, k, tau, t0, vf, pco)
    return np.abs(J @ U - F).max() / np.abs(F).max()


V2 = [Poly({(2, 1, 0): 1.0, (0, 2, 0): -0.5, (1, 1, 1): 1.0, (1, 0, 1): 1.0}, 3),
      Poly({(1, 2, 0): -1.0, (2, 0, 0): 1.0, (0, 2, 1): 1.0, (2, 1, 1): -0.5}, 3)]
P2 = Poly({(0, 0, 0): 1.0, (1, 0, 0): 2.0, (0, 1, 0): -1.0, (1, 0, 1): 0.5, (0, 1, 1): 1.0}, 3)


@pytest.mark.parametrize("k", [1, 2])
def test_patch_2d(k):
    """Galerkin consistency: the interpolant of an exact discrete solution
    (Q2 velocity, global P1 pressure, degree <= k+1 in time) satisfies J U = F."""
    assert _patch(2, (4, 2), k, 0.1, (0.7, -0.4), V2, P2) < 1e-13
    v = [V2[0] + Poly({(1, 1, k + 1): 0.3}, 3), V2[1]]
    assert _patch(2, (4, 2), k, 0.05, (0.7, -0.4), v, P2) < 1e-13


def test_patch_2d_detects_time_degree_k_plus_2():
    v = [V2[0] + Poly({(1, 1, 3): 0.3}, 3), V2[1]]
    assert _patch(2, (4, 2), 1, 0.1, (0.7, -0.4), v, P2) > 1e-9


def test_patch_3d():
    w = [Poly({(2, 1, 0, 0): 1.0, (0, 1, 2, 0): -0.5, (1, 1, 1, 1): 1.0}, 4),
         Poly({(1, 2, 1, 0): -1.0, (0, 0, 2, 1): 1.0}, 4),
         Poly({(1, 0, 2, 0): 0.5, (0, 2, 1, 1): 1.0, (0, 0, 0, 0): 0.3}, 4)]
    p = Poly({(0, 0, 0, 0): 1.0, (1, 0, 0, 0): 2.0, (0, 1, 0, 0): -1.0, (0, 0, 1, 1): 0.7}, 4)
    assert _patch(3, (2, 2, 2), 1, 0.1, (0.7, -0.4, 0.2), w, p) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_stokes_structure(dim):
    """b = 0: symmetric Nitsche makes the velocity block symmetric positive
    definite and the pressure couplings negative transposes (Bt / -B)."""
    n = (4, 2) if dim == 2 else (2, 2, 2)
    m = Mesh(dim, n, (2.2, 0.41) if dim == 2 else (2.5, 0.41, 0.41))
    A = assemble_level(m, 0, 1.0, np.full(m.n_cells, 0.01), lambda X: np.zeros_like(X))
    J = sp.bsr_matrix((A["val"], A["col"], A["rowptr"]), shape=(m.n_sdofs, m.n_sdofs)).toarray()
    nvel = dim * m.n_vnodes
    # remove the (symmetric) mass part C M: with k = 0, C = 1, tau w = 1
    ref = RefData(dim)
    Avv = J[:nvel, :nvel]
    np.testing.assert_allclose(Avv, Avv.T, atol=1e-13)
    assert np.linalg.eigvalsh(Avv).min() > 0
    np.testing.assert_allclose(J[:nvel, nvel:], -J[nvel:, :nvel].T, atol=1e-14)
    np.testing.assert_allclose(J[nvel:, nvel:], 0.0, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_prolongation_reproduces_coarse_functions(dim):
    n = (4, 2) if dim == 2 else (2, 2, 2)
    ext = (2.2, 0.41) if dim == 2 else (2.5, 0.41, 0.41)
    fm = Mesh(dim, tuple(2 * c for c in n), ext)
    cm = Mesh(dim, n, ext)
    rp, col, val = prolongation(fm, cm)
    P = sp.csr_matrix((val, col, rp), shape=(fm.n_sdofs, cm.n_sdofs))
    # a global Q2 polynomial per component and a global P1 pressure
    nvar = dim + 1
    vq = [Poly({tuple([2] * dim + [0]): 1.0, tuple([1] + [0] * (dim - 1) + [0]): 0.5}, nvar),
          Poly({tuple([0] + [2] + [0] * (dim - 2) + [0]): -1.0, tuple([1] * dim + [0]): 2.0}, nvar)]
    vq += [Poly({tuple([1] * dim + [0]): 1.0}, nvar)] * (dim - 2)
    pq = Poly({tuple([0] * nvar): 0.3, tuple([1] + [0] * dim): -1.0, tuple([0, 1] + [0] * (dim - 1)): 2.0}, nvar)
    vf = vec_eval(vq)

    def pco(origin, h, t):
        cols = [pq(origin + h[None, :] / 2, t)]
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = 1
            cols.append((pq(origin + e[None, :], t) - pq(origin, t)) * h[a] / (2 * np.sqrt(3)))
        return np.stack(cols, axis=1)

    Uf = interpolate(fm, 0, 1.0, 0.0, vf, pco)
    Uc = interpolate(cm, 0, 1.0, 0.0, vf, pco)
    np.testing.assert_allclose(P @ Uc, Uf, atol=1e-13)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (3, 1)])
def test_oseen_pattern_drops_only_zero_blocks(dim, k):
    """The compact pattern stores the same operator as the full cell-pair pattern."""
    from stgen.problem import Convection
    n = (4, 2) if dim == 2 else (2, 2, 2)
    ext = (2.2, 0.41) if dim == 2 else (2.5, 0.41, 0.41)
    m = Mesh(dim, n, ext)
    rng = np.random.default_rng(0)
    conv = Convection(dim, ext, rng.standard_normal(4) if dim == 2 else rng.standard_normal((4, 3)))
    nu = np.full(m.n_cells, 1e-3)
    mats = []
    for pat in ("full", "oseen"):
        A = assemble_level(m, k, 0.01, nu, conv, pattern=pat)
        mats.append(sp.bsr_matrix((A["val"], A["col"], A["rowptr"]),
                                  shape=(m.n_sdofs * (k + 1),) * 2).toarray())
    np.testing.assert_array_equal(mats[0], mats[1])
    full = assemble_level(m, k, 0.01, nu, conv, pattern="full")
    comp = assemble_level(m, k, 0.01, nu, conv, pattern="oseen")
    assert comp["rowptr"][-1] < 0.75 * full["rowptr"][-1]
