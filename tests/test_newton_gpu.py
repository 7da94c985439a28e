"""Newton linearisation at a time-dependent point and dG(1) time marching
with the library's FGMRES + Vanka-GMG as the linear solver (full time blocks
in every level matrix): the marched solutions equal the oracle's (direct
solves of the same Newton systems), FP64- and FP32-stored inverses."""
import functools

import numpy as np
import pytest

from gpu_common import log, relerr
from oracle.newton import march_direct
from stgen.newton import NewtonProblem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_2107_10561_amd as m
    return m


@functools.lru_cache(maxsize=None)
def setup(n, G):
    prob = NewtonProblem(2, n, G, 1, 0.05, 1e-2)
    ref = march_direct(prob, np.zeros(prob.fine.mesh.n_sdofs), 3, tol=1e-12)
    return prob, ref


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("shape", [((16, 4), 2), ((32, 8), 3)])
def test_marching_matches_oracle(stv, shape, fp32):
    from paper_2107_10561_amd.newton import march
    prob, ref = setup(*shape)
    s = stv.Solver(0)
    out = march(s, prob, np.zeros(prob.fine.mesh.n_sdofs), 3, tol=1e-12, lin_rtol=1e-11,
                fp32=fp32)
    for n, (o, (uo, ho)) in enumerate(zip(out, ref)):
        e = relerr(o["u"], uo)
        log(f"[newton] {shape} fp32={fp32} step {n}: newton residuals "
            f"{['%.1e' % h for h in o['residuals']]}, linear iterations {o['linear_iters']}, "
            f"rel diff to oracle {e:.2e}")
        assert o["residuals"][-1] <= 1e-12
        assert e <= 1e-9
