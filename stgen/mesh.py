"""Structured axis-aligned channel meshes, DoF numbering and level transfers.

Cells are numbered lexicographically with x fastest; this numbering is also the
loop order of the cell-based smoother.  Spatial degrees of freedom of a level:
  * velocity: Q2 node n (lexicographic over the (2 n_x + 1) x ... node grid,
    x fastest), component c  ->  sdof = n * dim + c;
  * pressure: cell e, Legendre mode m  ->  sdof = dim * N_v + e * (dim + 1) + m.
The cell-local spatial order is component-major over the lexicographic Q2
nodes, followed by the pressure modes (the spatial part of eq. (4.4)).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .fe import SQRT3, q2_1d, q2_nodes, n_local_spatial


@dataclass
class Mesh:
    dim: int
    n: tuple          # cells per axis (n_x, n_y[, n_z])
    ext: tuple        # domain extents (L, H[, H])

    @property
    def h(self):
        return tuple(e / c for e, c in zip(self.ext, self.n))

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.n))

    @property
    def node_dims(self):
        return tuple(2 * c + 1 for c in self.n)

    @property
    def n_vnodes(self) -> int:
        return int(np.prod(self.node_dims))

    @property
    def n_sdofs(self) -> int:
        return self.dim * self.n_vnodes + (self.dim + 1) * self.n_cells

    @property
    def n_ls(self) -> int:
        return n_local_spatial(self.dim)

    def coarsen(self) -> "Mesh":
        assert all(c % 2 == 0 for c in self.n)
        return Mesh(self.dim, tuple(c // 2 for c in self.n), self.ext)

    def cell_index(self):
        """(n_cells, dim) integer cell coordinates, x fastest."""
        grids = np.meshgrid(*[np.arange(c) for c in reversed(self.n)], indexing="ij")
        return np.stack([g.ravel() for g in reversed(grids)], axis=1)

    def cell_origin(self):
        return self.cell_index() * np.array(self.h)

    def node_id(self, ijk):
        """Linear node id of integer node coordinates (..., dim)."""
        nd = self.node_dims
        nid = ijk[..., self.dim - 1].astype(np.int64)
        for a in range(self.dim - 2, -1, -1):
            nid = nid * nd[a] + ijk[..., a]
        return nid

    def cell_sdofs(self) -> np.ndarray:
        """(n_cells, n_ls) int32 global spatial DoFs in cell-local order."""
        d = self.dim
        ci = self.cell_index()                           # (nc, d)
        nodes = q2_nodes(d)                              # (3^d, d)
        gnode = self.node_id(2 * ci[:, None, :] + nodes[None, :, :])   # (nc, 3^d)
        vel = [gnode * d + c for c in range(d)]
        pres = d * self.n_vnodes + np.arange(self.n_cells)[:, None] * (d + 1) + np.arange(d + 1)[None, :]
        return np.concatenate(vel + [pres], axis=1).astype(np.int32)

    def colours(self) -> np.ndarray:
        """Cell parity colour; cells of one colour share no degree of freedom."""
        ci = self.cell_index()
        col = np.zeros(self.n_cells, dtype=np.uint8)
        for a in range(self.dim):
            col |= ((ci[:, a] & 1) << a).astype(np.uint8)
        return col

    def node_coords(self):
        """(N_v, dim) physical coordinates of the Q2 nodes."""
        nd = self.node_dims
        grids = np.meshgrid(*[np.arange(c) for c in reversed(nd)], indexing="ij")
        ijk = np.stack([g.ravel() for g in reversed(grids)], axis=1)
        return ijk * (np.array(self.h) / 2.0)


def prolongation(fine: Mesh, coarse: Mesh):
    """Spatial prolongation (fine x coarse CSR) for a uniformly refined pair.

    Velocity: nodal interpolation of the coarse Q2 functions at the fine nodes
    (1d weights at the quarter points of a coarse cell: 3/8, 3/4, -1/8).
    Pressure: the coarse P1 function of the parent restricted to a child,
    re-expanded in the child's Legendre basis:
      p0_f = p0 + sqrt3 (o_x - 1/2) p1 + sqrt3 (o_y - 1/2) p2 [+ z],  pa_f = pa / 2.
    The time factor is the identity (same time basis on every level).
    Returns (rowptr int32, col int32, val float64), columns sorted per row.
    """
    d = fine.dim
    assert coarse.dim == d and all(f == 2 * c for f, c in zip(fine.n, coarse.n))
    # 1d stencils: fine node f -> 3 (coarse node, weight) slots (zero-padded)
    sc, sw = [], []
    for nc_cells in coarse.n:
        f = np.arange(4 * nc_cells + 1)
        cidx = np.zeros((f.size, 3), dtype=np.int64)
        wts = np.zeros((f.size, 3))
        even = f % 2 == 0
        cidx[even, 0] = f[even] // 2
        wts[even, 0] = 1.0
        odd = ~even
        cell = np.minimum(f[odd] // 4, nc_cells - 1)
        xh = (f[odd] - 4 * cell) / 4.0
        cidx[odd] = 2 * cell[:, None] + np.arange(3)[None, :]
        wts[odd] = q2_1d(xh)
        sc.append(cidx)
        sw.append(wts)
    fnd = fine.node_dims
    grids = np.meshgrid(*[np.arange(c) for c in reversed(fnd)], indexing="ij")
    fijk = np.stack([g.ravel() for g in reversed(grids)], axis=1)       # (Nvf, d)
    combos = q2_nodes(d)                                                 # (3^d, d) slot indices
    cn_ijk = np.stack([sc[a][fijk[:, a]][:, combos[:, a]] for a in range(d)], axis=-1)  # (Nvf, 3^d, d)
    w = np.ones((fijk.shape[0], combos.shape[0]))
    for a in range(d):
        w *= sw[a][fijk[:, a]][:, combos[:, a]]
    cn = coarse.node_id(cn_ijk)                                          # (Nvf, 3^d)
    keep = w != 0.0
    fn_rep = np.broadcast_to(np.arange(fijk.shape[0])[:, None], w.shape)[keep]
    cn_k, w_k = cn[keep], w[keep]
    R, Cc, V = [], [], []
    for c in range(d):
        R.append(fn_rep * d + c)
        Cc.append(cn_k * d + c)
        V.append(w_k)
    # pressure
    fci = fine.cell_index()
    par = fci // 2
    off = fci - 2 * par
    ce = _cell_id_vec(coarse, par)
    cb = d * coarse.n_vnodes + ce * (d + 1)
    fb = d * fine.n_vnodes + np.arange(fine.n_cells) * (d + 1)
    R.append(fb); Cc.append(cb); V.append(np.ones(fine.n_cells))
    for a in range(d):
        R.append(fb); Cc.append(cb + 1 + a); V.append(SQRT3 * (off[:, a] - 0.5))
        R.append(fb + 1 + a); Cc.append(cb + 1 + a); V.append(np.full(fine.n_cells, 0.5))
    R = np.concatenate(R).astype(np.int64)
    Cc = np.concatenate(Cc).astype(np.int64)
    V = np.concatenate(V)
    order = np.lexsort((Cc, R))
    R, Cc, V = R[order], Cc[order], V[order]
    rowptr = np.zeros(fine.n_sdofs + 1, dtype=np.int64)
    np.add.at(rowptr, R + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr.astype(np.int32), Cc.astype(np.int32), V.astype(np.float64)


def _cell_id_vec(mesh: Mesh, ijk):
    cid = ijk[:, mesh.dim - 1].astype(np.int64)
    for a in range(mesh.dim - 2, -1, -1):
        cid = cid * mesh.n[a] + ijk[:, a]
    return cid
