"""Batched hierarchies through the C ABI: several independent instances of
different sizes and level counts packed into one block-diagonal hierarchy.
Every instance must reproduce, on its own segment, what the oracle computes
for that instance alone (V-cycle, fixed-iteration FGMRES, tolerance mode),
and what the library computes for it as a single hierarchy."""
import functools

import numpy as np
import pytest

import oracle
from gpu_common import log, relerr, to_dev, to_host
from stgen.problem import make_problem

pytestmark = pytest.mark.gpu

# (dim, cells, levels, k, tau, nu, seed): mixed sizes and level counts,
# a one-level instance (solved directly on the finest packed level)
MIXED = [
    (2, (16, 4), 2, 1, 0.01, 1e-3, 41),
    (2, (32, 8), 3, 1, 0.01, 2e-3, 42),
    (2, (8, 2), 1, 1, 0.01, 1e-3, 43),
    (2, (24, 8), 3, 1, 0.01, 5e-4, 44),
    (2, (16, 4), 2, 1, 0.01, 4e-3, 45),
]
MIXED_3D = [
    (3, (8, 2, 2), 2, 1, 0.01, 1e-3, 46),
    (3, (4, 2, 2), 1, 1, 0.01, 2e-3, 47),
]


@functools.lru_cache(maxsize=None)
def instances(name):
    specs = {"mixed2d": MIXED, "mixed3d": MIXED_3D}[name]
    out = []
    for spec in specs:
        p = make_problem(*spec)
        ol = oracle.prepare_levels(p.levels, p.b)
        oracle.build_inverses(ol)
        out.append((p, ol))
    return out


@pytest.fixture(scope="module")
def stv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_2107_10561_amd as m
    return m


def batch_solver(stv, name, fp32=False):
    inst = instances(name)
    s = stv.Solver(0)
    s.set_batch([p.levels for p, _ in inst], inst[0][0].dim, inst[0][0].k)
    s.build_cell_inverses(fp32=fp32)
    return s, inst


def pack(s, vecs):
    out = np.zeros(s.n_st[-1])
    for i, v in enumerate(vecs):
        _, o, n = s.instance_layout(i)
        assert n == v.size
        out[o:o + n] = v
    return out


def unpack(s, x, i):
    _, o, n = s.instance_layout(i)
    return x[o:o + n]


@pytest.mark.parametrize("name", ["mixed2d", "mixed3d"])
def test_batch_layout(stv, name):
    s, inst = batch_solver(stv, name)
    off = 0
    for i, (p, ol) in enumerate(inst):
        nl, o, n = s.instance_layout(i)
        assert nl == len(p.levels) and o == off and n == ol[-1].n_st
        off += n
    assert off == s.n_st[-1]


@pytest.mark.parametrize("name", ["mixed2d", "mixed3d"])
def test_batch_vcycle_matches_oracle_per_instance(stv, name):
    s, inst = batch_solver(stv, name)
    rng = np.random.default_rng(7)
    rs = [rng.standard_normal(ol[-1].n_st) for _, ol in inst]
    d = to_dev(np.zeros(s.n_st[-1]))
    s.vcycle(to_dev(pack(s, rs)), d, 2, 2, 0.7)
    dh = to_host(d)
    for i, (p, ol) in enumerate(inst):
        ref = oracle.vcycle(ol, rs[i], 2, 2, 0.7)
        e = relerr(unpack(s, dh, i), ref)
        log(f"[batch-vcycle] {name} instance {i} levels {len(ol)} rel err {e:.2e}")
        assert e <= 1e-11


@pytest.mark.parametrize("name", ["mixed2d", "mixed3d"])
def test_batch_gmres_fixed_iterations(stv, name):
    s, inst = batch_solver(stv, name)
    n = 6
    b = pack(s, [p.rhs for p, _ in inst])
    x = to_dev(np.zeros(s.n_st[-1]))
    info = s.gmres_solve(to_dev(b), x, restart=30, fixed_iters=n)
    xh = to_host(x)
    assert info["iters"] == n
    for i, (p, ol) in enumerate(inst):
        cinv = oracle.coarse_inverse(ol[0])
        xf, _ = oracle.fgmres(lambda v: ol[-1].J @ v, p.rhs,
                              lambda v: oracle.vcycle(ol, v, 2, 2, 0.7, coarse_inv=cinv),
                              restart=30, fixed_iters=n)
        e = relerr(unpack(s, xh, i), xf)
        log(f"[batch-gmres-fixed] {name} instance {i} rel err {e:.2e}")
        assert e <= 1e-10
        assert s.instance_info(i)["iters"] == n


@pytest.mark.parametrize("name", ["mixed2d", "mixed3d"])
def test_batch_gmres_tolerance_mode(stv, name):
    s, inst = batch_solver(stv, name)
    b = pack(s, [p.rhs for p, _ in inst])
    x = to_dev(np.zeros(s.n_st[-1]))
    info = s.gmres_solve(to_dev(b), x, restart=30, rtol=1e-8)
    xh = to_host(x)
    assert info["converged"]
    for i, (p, ol) in enumerate(inst):
        cinv = oracle.coarse_inverse(ol[0])
        _, io = oracle.fgmres(lambda v: ol[-1].J @ v, p.rhs,
                              lambda v: oracle.vcycle(ol, v, 2, 2, 0.7, coarse_inv=cinv),
                              restart=30, rtol=1e-8)
        xi = unpack(s, xh, i)
        true = np.linalg.norm(p.rhs - ol[-1].J @ xi) / np.linalg.norm(p.rhs)
        ii = s.instance_info(i)
        log(f"[batch-gmres] {name} instance {i} iters {ii['iters']} (oracle {io['iters']}) "
            f"true {true:.2e}")
        assert ii["converged"] and true <= 1e-8
        assert abs(ii["iters"] - io["iters"]) <= 1
        assert abs(ii["true_relres"] - true) <= 1e-3 * true + 1e-14   # recomputing a residual near 1e-13 carries ~1e-15 of rounding


def test_batch_equals_single_instances(stv):
    s, inst = batch_solver(stv, "mixed2d")
    b = pack(s, [p.rhs for p, _ in inst])
    x = to_dev(np.zeros(s.n_st[-1]))
    s.gmres_solve(to_dev(b), x, restart=30, rtol=1e-8)
    xh = to_host(x)
    for i, (p, ol) in enumerate(inst):
        s1 = stv.Solver(0)
        s1.set_hierarchy(p.levels, p.dim, p.k)
        s1.build_cell_inverses()
        x1 = to_dev(np.zeros(ol[-1].n_st))
        info = s1.gmres_solve(to_dev(p.rhs), x1, restart=30, rtol=1e-8)
        e = relerr(unpack(s, xh, i), to_host(x1))
        log(f"[batch-vs-single] instance {i} rel diff {e:.2e}")
        assert info["iters"] == s.instance_info(i)["iters"]
        assert e <= 1e-10


def test_batch_fp32_inverses(stv):
    s64, inst = batch_solver(stv, "mixed2d")
    s32, _ = batch_solver(stv, "mixed2d", fp32=True)
    b = pack(s64, [p.rhs for p, _ in inst])
    x64 = to_dev(np.zeros(s64.n_st[-1]))
    x32 = to_dev(np.zeros(s64.n_st[-1]))
    s64.gmres_solve(to_dev(b), x64, restart=30, rtol=1e-8)
    info = s32.gmres_solve(to_dev(b), x32, restart=30, rtol=1e-8)
    assert info["converged"]
    h64, h32 = to_host(x64), to_host(x32)
    for i, (p, ol) in enumerate(inst):
        xt = np.linalg.solve(ol[-1].J.toarray(), p.rhs)
        e64 = relerr(unpack(s64, h64, i), xt)
        e32 = relerr(unpack(s64, h32, i), xt)
        log(f"[batch-fp32] instance {i} forward error fp64 {e64:.2e} fp32 {e32:.2e}")
        assert e32 <= 2.0 * e64 + 1e-12


def test_batch_residual_and_sweep_on_packed_level(stv):
    s, inst = batch_solver(stv, "mixed2d")
    G = s.n_levels - 1
    rng = np.random.default_rng(9)
    rs = [rng.standard_normal(ol[-1].n_st) for _, ol in inst]
    ds = [rng.standard_normal(ol[-1].n_st) for _, ol in inst]
    out = to_dev(np.zeros(s.n_st[G]))
    s.residual(G, to_dev(pack(s, rs)), to_dev(pack(s, ds)), out)
    oh = to_host(out)
    for i, (p, ol) in enumerate(inst):
        ref = rs[i] - ol[-1].J @ ds[i]
        got = unpack(s, oh, i)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # one sweep: smoothed instances follow the oracle, the one-level
    # instance (no cells) keeps its iterate
    dd = to_dev(pack(s, ds))
    s.vanka_sweep(G, to_dev(pack(s, rs)), dd, 1, 0.7)
    dh = to_host(dd)
    for i, (p, ol) in enumerate(inst):
        got = unpack(s, dh, i)
        if len(ol) == 1:
            assert np.array_equal(got, ds[i])
        else:
            assert relerr(got, oracle.vanka_sweep(ol[-1], rs[i], ds[i], 0.7)) <= 1e-12


def test_batch_rejects_bad_instance(stv):
    inst = instances("mixed2d")
    levels = [p.levels for p, _ in inst]
    bad = [dict(n_sdofs=L.n_sdofs, rowptr=L.rowptr, col=L.col, val=L.val,
                cell_sdofs=L.cell_sdofs, P=L.P) for L in levels[1]]
    bad[-1]["cell_sdofs"] = bad[-1]["cell_sdofs"].copy()
    bad[-1]["cell_sdofs"][0, 0] = 10 ** 8
    s = stv.Solver(0)
    with pytest.raises(stv.StvError, match="instance 1"):
        s.set_batch([levels[0], bad] + levels[2:], 2, 1)
