"""Seeded synthetic channel-flow hierarchies (the workloads of the solver).

Readings of the paper used here (it runs the DFG cylinder benchmarks, which
these channel problems stand in for):
  * Oseen linearisation at a frozen, smooth, divergence-free convection field
    with b.n = 0 on the boundary, rescaled to max |b| = 1 on a sample grid;
    2d: b = curl of a stream function sum_m a_m sin(p_m pi x/L) sin(q_m pi y/H);
    3d: b = curl of a vector potential sum_m a_m sin sin sin, a_m in R^3;
  * right-hand side: seeded N(0,1) per space-time DoF, drawn in the paper's
    time-major order (eq. (3.6)) and stored time-inner, x[s (k+1) + l];
  * level g is the uniform coarsening by 2 per axis of level g+1; level 0 is
    the coarsest and is solved directly.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .assemble import assemble_level
from .mesh import Mesh, prolongation

L2D, H2D = 2.2, 0.41
L3D, H3D = 2.5, 0.41
MODES2D = [(1, 1), (2, 1), (1, 2), (3, 1)]
MODES3D = [(1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2)]


@dataclass
class Convection:
    dim: int
    ext: tuple
    amps: np.ndarray           # (4,) in 2d, (4, 3) in 3d
    scale: float = 1.0

    def raw(self, x):
        x = np.asarray(x, dtype=np.float64)
        if self.dim == 2:
            L, H = self.ext
            bx = np.zeros(x.shape[0]); by = np.zeros(x.shape[0])
            for a, (p, q) in zip(self.amps, MODES2D):
                kx, ky = p * np.pi / L, q * np.pi / H
                sx, cx = np.sin(kx * x[:, 0]), np.cos(kx * x[:, 0])
                sy, cy = np.sin(ky * x[:, 1]), np.cos(ky * x[:, 1])
                bx += a * sx * ky * cy          # d psi / dy
                by -= a * kx * cx * sy          # -d psi / dx
            return np.stack([bx, by], axis=1)
        L, H, W = self.ext
        b = np.zeros((x.shape[0], 3))
        for a, (p, q, r) in zip(self.amps, MODES3D):
            k = np.array([p * np.pi / L, q * np.pi / H, r * np.pi / W])
            s = np.sin(k[None, :] * x)
            c = np.cos(k[None, :] * x)
            S = s[:, 0] * s[:, 1] * s[:, 2]
            # gradient of S
            g = np.stack([k[0] * c[:, 0] * s[:, 1] * s[:, 2],
                          k[1] * s[:, 0] * c[:, 1] * s[:, 2],
                          k[2] * s[:, 0] * s[:, 1] * c[:, 2]], axis=1)
            # curl(a S) = grad S x a
            b += np.cross(g, a[None, :])
            del S
        return b

    def __call__(self, x):
        return self.scale * self.raw(x)

    def normalise(self):
        if self.dim == 2:
            g = np.meshgrid(np.linspace(0, self.ext[0], 257), np.linspace(0, self.ext[1], 65), indexing="ij")
        else:
            g = np.meshgrid(np.linspace(0, self.ext[0], 129), np.linspace(0, self.ext[1], 33),
                            np.linspace(0, self.ext[2], 33), indexing="ij")
        pts = np.stack([a.ravel() for a in g], axis=1)
        m = np.max(np.linalg.norm(self.raw(pts), axis=1))
        self.scale = 1.0 / m if m > 0 else 1.0
        return self


@dataclass
class Level:
    mesh: Mesh
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray           # (nnzb, b, b)
    cell_sdofs: np.ndarray    # (n_cells, n_ls)
    P: tuple | None = None    # (rowptr, col, val) fine x coarse spatial, None on level 0
    nu_cell: np.ndarray | None = None   # viscosity per cell the level was assembled with
    conv: object = None                  # convection field of the assembly

    @property
    def n_sdofs(self):
        return self.mesh.n_sdofs

    @property
    def n_cells(self):
        return self.mesh.n_cells


@dataclass
class Problem:
    dim: int
    k: int
    tau: float
    nu: float
    levels: list              # Level, index 0 = coarsest
    rhs: np.ndarray           # time-inner, finest level
    conv: Convection | None = None
    meta: dict = field(default_factory=dict)

    @property
    def b(self):
        return self.k + 1


def time_major_to_inner(x_tm: np.ndarray, n_s: int, b: int) -> np.ndarray:
    """x_tm[l * n_s + s] -> x_ti[s * b + l]."""
    return np.ascontiguousarray(x_tm.reshape(b, n_s).T).reshape(-1)


def time_inner_to_major(x_ti: np.ndarray, n_s: int, b: int) -> np.ndarray:
    return np.ascontiguousarray(x_ti.reshape(n_s, b).T).reshape(-1)


def make_hierarchy(dim, n_fine, n_levels, k, tau, nu, conv, ext=None, nu_cell_fine=None):
    """Assemble every level of the hierarchy (index 0 = coarsest)."""
    if ext is None:
        ext = (L2D, H2D) if dim == 2 else (L3D, H3D, H3D)
    meshes = [Mesh(dim, tuple(n_fine), tuple(ext))]
    for _ in range(n_levels - 1):
        meshes.append(meshes[-1].coarsen())
    meshes = meshes[::-1]
    levels = []
    nu_c = None
    # per-cell viscosity: finest given, coarser = mean of the children
    nus = [None] * n_levels
    if nu_cell_fine is not None:
        nus[-1] = np.asarray(nu_cell_fine, dtype=np.float64)
        for g in range(n_levels - 2, -1, -1):
            fm, cm = meshes[g + 1], meshes[g]
            fci = fm.cell_index() // 2
            cid = fci[:, dim - 1].astype(np.int64)
            for a in range(dim - 2, -1, -1):
                cid = cid * cm.n[a] + fci[:, a]
            s = np.zeros(cm.n_cells)
            np.add.at(s, cid, nus[g + 1])
            nus[g] = s / (2 ** dim)
    for g, m in enumerate(meshes):
        nu_c = nus[g] if nus[g] is not None else np.full(m.n_cells, float(nu))
        A = assemble_level(m, k, tau, nu_c, conv)
        P = prolongation(m, meshes[g - 1]) if g > 0 else None
        levels.append(Level(m, A["rowptr"], A["col"], A["val"], A["cell_sdofs"], P, nu_c, conv))
    return levels


def spatial_factors(level: Level):
    """(mval, aval) of a level: its blocks are C[i, l] M + delta_il tau w_i A."""
    from .assemble import assemble_spatial_factors
    return assemble_spatial_factors(level.mesh, level.nu_cell, level.conv, level.rowptr, level.col)


CONFIGS = {
    # name: (dim, finest cells, levels, k, tau, nu, seed)
    "C1": (2, (16, 4), 2, 1, 0.01, 1e-3, 1001),
    "C2": (2, (512, 128), 6, 2, 0.005, 1e-3, 1002),
    "C3": (3, (128, 24, 24), 4, 1, 0.01, 1e-3, 1003),
}


def make_problem(dim, n_fine, n_levels, k, tau, nu, seed, nu_cell_fine=None):
    """Seeded problem: amplitudes first, then the N(0,1) right-hand side."""
    rng = np.random.default_rng(seed)
    ext = (L2D, H2D) if dim == 2 else (L3D, H3D, H3D)
    amps = rng.standard_normal(4) if dim == 2 else rng.standard_normal((4, 3))
    conv = Convection(dim, ext, amps).normalise()
    levels = make_hierarchy(dim, n_fine, n_levels, k, tau, nu, conv, ext, nu_cell_fine)
    n_s = levels[-1].n_sdofs
    b = k + 1
    rhs_tm = rng.standard_normal(b * n_s)
    rhs = time_major_to_inner(rhs_tm, n_s, b)
    return Problem(dim, k, tau, nu, levels, rhs, conv,
                   meta=dict(seed=seed, n_fine=tuple(n_fine), n_levels=n_levels))


def make_config(name: str, **over):
    dim, n, G, k, tau, nu, seed = CONFIGS[name]
    n = over.get("n_fine", n)
    G = over.get("n_levels", G)
    return make_problem(dim, n, G, k, tau, nu, seed)


def batched_instance(j: int):
    """Instance j of the batched workload: size drawn from four finest grids,
    viscosity uniform in [5e-4, 5e-3], tau = 0.01, coarsened to 8x2 or 12x3."""
    rng = np.random.default_rng(2000 + j)
    choice = int(rng.integers(0, 4))
    n = [(32, 8), (64, 16), (96, 24), (128, 32)][choice]
    nu = float(rng.uniform(5e-4, 5e-3))
    G = {0: 3, 1: 4, 2: 4, 3: 5}[choice]
    return make_problem(2, n, G, 1, 0.01, nu, 2000 + j)
