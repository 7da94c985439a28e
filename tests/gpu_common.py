"""Shared fixtures of the GPU parity tests: problems, oracle state, device
helpers.  Inputs come from the seeded generator; expected values from the
oracle only."""
import functools
import sys

import numpy as np

import oracle
from stgen.problem import make_problem

# name -> (dim, finest cells, levels, k, tau, nu, seed)
CASES = {
    "c1_2d_dg1": (2, (16, 4), 2, 1, 0.01, 1e-3, 1001),
    "2d_dg2": (2, (32, 8), 3, 2, 0.005, 1e-3, 1002),
    "2d_dg0": (2, (16, 4), 2, 0, 0.01, 1e-3, 11),
    "3d_dg0": (3, (8, 2, 2), 2, 0, 0.01, 1e-3, 12),
    "3d_dg1": (3, (8, 2, 2), 2, 1, 0.01, 1e-3, 1003),
}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def problem(name):
    dim, n, G, k, tau, nu, seed = CASES[name]
    p = make_problem(dim, n, G, k, tau, nu, seed)
    ol = oracle.prepare_levels(p.levels, p.b)
    oracle.build_inverses(ol)
    return p, ol


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
