"""The V-cycle replayed from a captured HIP graph must give exactly the eager
result: every replay (with eager work and synchronisations between the
replays), after a change of the cycle parameters, after the inverses are
rebuilt, and inside FGMRES, for a single hierarchy and for a batch."""
import numpy as np
import pytest

import oracle
from gpu_common import log, problem, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_2107_10561_amd as m
    return m


def solver(stv, name, graph):
    p, ol = problem(name)
    s = stv.Solver(0)
    s.set_hierarchy(p.levels, p.dim, p.k)
    s.build_cell_inverses()
    s.set_graph(graph)
    return s, p, ol


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2", "3d_dg1"])
def test_graph_replays_equal_eager(stv, name):
    sg, p, ol = solver(stv, name, True)
    se, _, _ = solver(stv, name, False)
    rng = np.random.default_rng(11)
    n = ol[-1].n_st
    for rep in range(4):
        r = to_dev(rng.standard_normal(n))
        dg = to_dev(np.zeros(n))
        de = to_dev(np.zeros(n))
        sg.vcycle(r, dg, 2, 2, 0.7)
        se.vcycle(r, de, 2, 2, 0.7)       # eager work between the replays
        a, b = to_host(dg), to_host(de)
        log(f"[graph] {name} replay {rep}: max diff {np.abs(a - b).max():.1e}")
        assert np.array_equal(a, b)
    # new cycle parameters: recaptured
    r = to_dev(rng.standard_normal(n))
    dg, de = to_dev(np.zeros(n)), to_dev(np.zeros(n))
    sg.vcycle(r, dg, 1, 3, 1.0)
    se.vcycle(r, de, 1, 3, 1.0)
    assert np.array_equal(to_host(dg), to_host(de))
    # rebuilt inverses: recaptured, and still the oracle's cycle
    sg.build_cell_inverses(fp32=False)
    rh = rng.standard_normal(n)
    dg = to_dev(np.zeros(n))
    sg.vcycle(to_dev(rh), dg, 2, 2, 0.7)
    assert relerr(to_host(dg), oracle.vcycle(ol, rh, 2, 2, 0.7)) <= 1e-11


@pytest.mark.parametrize("name", ["c1_2d_dg1", "2d_dg2"])
def test_graph_gmres_equals_eager(stv, name):
    sg, p, ol = solver(stv, name, True)
    se, _, _ = solver(stv, name, False)
    xg = to_dev(np.zeros(ol[-1].n_st))
    xe = to_dev(np.zeros(ol[-1].n_st))
    ig = sg.gmres_solve(to_dev(p.rhs), xg, restart=30, rtol=1e-8)
    ie = se.gmres_solve(to_dev(p.rhs), xe, restart=30, rtol=1e-8)
    assert ig["iters"] == ie["iters"] and ig["converged"]
    assert np.array_equal(to_host(xg), to_host(xe))
    # a second solve replays the same graph
    xg2 = to_dev(np.zeros(ol[-1].n_st))
    sg.gmres_solve(to_dev(p.rhs), xg2, restart=30, rtol=1e-8)
    assert np.array_equal(to_host(xg2), to_host(xe))


def test_graph_batch_gmres_equals_eager(stv):
    from stgen.problem import make_problem
    specs = [(2, (16, 4), 2, 1, 0.01, 1e-3, 61), (2, (32, 8), 3, 1, 0.01, 3e-3, 62),
             (2, (8, 2), 1, 1, 0.01, 1e-3, 63)]
    probs = [make_problem(*sp) for sp in specs]
    b = np.concatenate([q.rhs for q in probs])
    out = []
    for graph in (True, False):
        s = stv.Solver(0)
        s.set_batch([q.levels for q in probs], 2, 1)
        s.build_cell_inverses(fp32=True)
        s.set_graph(graph)
        x = to_dev(np.zeros_like(b))
        info = s.gmres_solve(to_dev(b), x, restart=30, rtol=1e-8)
        assert info["converged"]
        out.append(to_host(x))
    assert np.array_equal(out[0], out[1])
