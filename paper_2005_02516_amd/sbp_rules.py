"""Writes sbp_rules.json: quadrature rules on the reference triangle for the DG-SBP scheme of
Section 3 (traditional SBP operators obtained from the hybridized ones).

Section 3.1 asks of such a rule: positive weights; exactness for polynomials of degree
2N-1; boundary nodes that form, identically on every face, a face rule exact to degree 2N.
Its node sets are shown only as figures, so the rules here are derived from those
conditions.  Each has the N+1 Gauss-Legendre points of every edge among its nodes (face
rule exact to degree 2N+1) and a few interior orbits; all nodes come in orbits of the
triangle's symmetry group, and the weights and interior positions solve the moment
equations int_T r^a s^b = sum_i w_i r_i^a s_i^b (a + b <= 2N-1, exact rational right-hand
sides):

  N | nodes | boundary             | interior
  1 |   6   | 2 GL points per edge | none
  2 |  10   | 3 GL points per edge | centroid
  3 |  18   | 4 GL points per edge | two 3-point orbits (a one-parameter family: the member
    |       |                      | with the largest smallest weight is taken)
  4 |  22   | 5 GL points per edge | centroid + two 3-point orbits

This module is an input generator: nothing in it evaluates the scheme.  Run it to rewrite
the JSON (python -m paper_2005_02516_amd.sbp_rules); tests check the stored rules against
the Section 3.1 conditions.
"""
from __future__ import annotations

import itertools
import json
import os
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "sbp_rules.json")


def monomial_integral(a: int, b: int) -> Fraction:
    """Exact integral of r^a s^b over the triangle (-1,-1), (1,-1), (-1,1):
    int_{-1}^{1} s^b ((-s)^(a+1) - (-1)^(a+1)) / (a+1) ds."""
    tot = Fraction(0)
    # s^b * (-1)^(a+1) s^(a+1) / (a+1)  and  - s^b (-1)^(a+1) / (a+1)
    def int_pow(p):        # int_{-1}^{1} s^p ds
        return Fraction(0) if p % 2 else Fraction(2, p + 1)
    sgn = (-1) ** (a + 1)
    tot += Fraction(sgn, a + 1) * int_pow(a + b + 1)
    tot -= Fraction(sgn, a + 1) * int_pow(b)
    return tot


def _rs(l1, l2, l3):
    """Barycentric (of v1=(-1,-1), v2=(1,-1), v3=(-1,1)) to (r, s)."""
    return -l1 + l2 - l3, -l1 - l2 + l3


def _orbit(bary):
    pts = sorted(set(itertools.permutations(bary)))
    return [_rs(*p) for p in pts]


def _gauss_legendre(n):
    return np.polynomial.legendre.leggauss(n)


def _layout(N, x):
    """Nodes and weights from the unknowns x = (orbit weights..., interior positions...)."""
    t, _ = _gauss_legendre(N + 1)
    bnd = [ti for ti in t if ti > -1e-14]                 # one representative per edge orbit
    interior = {1: [], 2: ["c"], 3: ["3", "3"], 4: ["c", "3", "3"]}[N]
    nw = len(bnd) + len(interior)
    w, pos = x[:nw], list(x[nw:])
    nodes, weights = [], []
    for ti, wi in zip(bnd, w):
        l1, l2 = (1 - ti) / 2, (1 + ti) / 2
        o = _orbit((l1, l2, 0.0)) if abs(ti) > 1e-14 else _orbit((0.5, 0.5, 0.0))
        nodes += o
        weights += [wi] * len(o)
    for kind, wi in zip(interior, w[len(bnd):]):
        if kind == "c":
            o = [_rs(1 / 3, 1 / 3, 1 / 3)]
        else:
            a = pos.pop(0)
            o = _orbit((a, a, 1 - 2 * a))
        nodes += o
        weights += [wi] * len(o)
    return np.array(nodes), np.array(weights), nw


def _residual(N, x):
    P, W, _ = _layout(N, x)
    mons = [(a, d - a) for d in range(2 * N) for a in range(d + 1)]
    return np.array([np.sum(W * P[:, 0] ** a * P[:, 1] ** b) - float(monomial_integral(a, b)) for a, b in mons])


def derive(N: int, seed: int = 0):
    from scipy.optimize import least_squares
    t, _ = _gauss_legendre(N + 1)
    nb = len([ti for ti in t if ti > -1e-14])
    interior = {1: [], 2: ["c"], 3: ["3", "3"], 4: ["c", "3", "3"]}[N]
    nw, npos = nb + len(interior), sum(1 for k in interior if k == "3")
    rng = np.random.default_rng(seed)
    sols = []
    for _ in range(400):
        x0 = np.concatenate([rng.uniform(0.01, 0.3, nw), np.sort(rng.uniform(0.02, 0.48, npos))])
        lo = np.concatenate([np.full(nw, 1e-8), np.full(npos, 1e-3)])
        hi = np.concatenate([np.full(nw, 2.0), np.full(npos, 0.5 - 1e-3)])
        r = least_squares(lambda x: _residual(N, x), x0, bounds=(lo, hi), xtol=1e-15, ftol=1e-15, gtol=1e-15)
        if np.abs(_residual(N, r.x)).max() < 1e-14:
            sols.append(r.x)
    if not sols:
        raise RuntimeError(f"no rule found for N={N}")
    # the member with the largest smallest weight (unique for N=1, 2, 4; N=3 has a family)
    best = max(sols, key=lambda x: _layout(N, x)[1].min())
    P, W, _ = _layout(N, best)
    return P, W


def write(path: str = PATH):
    out = {}
    for N in (1, 2, 3, 4):
        P, W = derive(N)
        out[str(N)] = {"r": [float(v) for v in P[:, 0]], "s": [float(v) for v in P[:, 1]],
                       "w": [float(v) for v in W]}
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def load(N: int):
    """The stored rule of degree N: (r, s, w) arrays."""
    with open(PATH) as fh:
        d = json.load(fh)[str(N)]
    return np.array(d["r"]), np.array(d["s"]), np.array(d["w"])


if __name__ == "__main__":
    rules = write()
    for N, d in rules.items():
        print(N, len(d["w"]), "min weight", min(d["w"]))
