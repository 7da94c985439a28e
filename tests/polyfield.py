"""Tiny exact polynomial fields in (x, y[, z], t) for manufactured-data tests."""
from __future__ import annotations

import numpy as np


class Poly:
    """Polynomial as {exponent tuple (px, py[, pz], pt): coefficient}."""

    def __init__(self, terms: dict, nvar: int):
        self.t = {tuple(k): float(v) for k, v in terms.items() if v != 0.0}
        self.nvar = nvar

    def __call__(self, X, t):
        X = np.atleast_2d(X)
        out = np.zeros(X.shape[0])
        for e, c in self.t.items():
            term = np.full(X.shape[0], c)
            for a in range(self.nvar - 1):
                if e[a]:
                    term = term * X[:, a] ** e[a]
            if e[-1]:
                term = term * t ** e[-1]
            out += term
        return out

    def d(self, var: int) -> "Poly":
        out = {}
        for e, c in self.t.items():
            if e[var] > 0:
                ne = list(e)
                ne[var] -= 1
                out[tuple(ne)] = out.get(tuple(ne), 0.0) + c * e[var]
        return Poly(out, self.nvar)

    def __add__(self, o: "Poly") -> "Poly":
        out = dict(self.t)
        for e, c in o.t.items():
            out[e] = out.get(e, 0.0) + c
        return Poly(out, self.nvar)

    def scale(self, s: float) -> "Poly":
        return Poly({e: s * c for e, c in self.t.items()}, self.nvar)


def momentum_data(v, p, b, nu, dim):
    """f = d_t v + (b.grad) v - nu lap v + grad p, for polynomial v (list), p, constant b."""
    T = dim  # index of t
    f = []
    for c in range(dim):
        fc = v[c].d(T)
        for a in range(dim):
            fc = fc + v[c].d(a).scale(b[a])
            fc = fc + v[c].d(a).d(a).scale(-nu)
        fc = fc + p.d(c)
        f.append(fc)
    return f


def vec_eval(polys):
    return lambda X, t: np.stack([q(X, t) for q in polys], axis=1)
