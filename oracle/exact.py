"""Exact rational oracle for tiny graphs.

Two independent exact methods:

* ``resistance_cramer``: ground u instead of g (the result does not depend on the
  ground, Section IV-A). Then R_uv = (L_u^{-1})_vv, and by Cramer's rule
  R_uv = det(L_G without rows/cols u, v) / det(L_G without row/col u).
* ``edge_resistances_trees``: Kirchhoff's matrix-tree view. For an edge e,
  w_e R_e equals the weighted fraction of spanning trees that contain e,
  where a tree's weight is the product of its edge conductances.

Conductances are converted with ``Fraction(float)``, which is exact, so the
results are exact rationals of the given binary inputs; ``to_float`` rounds
them correctly to FP64.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def _laplacian_fraction(n, eu, ev, w):
    L = [[Fraction(0)] * n for _ in range(n)]
    for a, b, x in zip(np.asarray(eu).tolist(), np.asarray(ev).tolist(), np.asarray(w).tolist()):
        if a == b:
            continue
        f = Fraction(x)
        L[a][a] += f
        L[b][b] += f
        L[a][b] -= f
        L[b][a] -= f
    return L


def det_fraction(M) -> Fraction:
    """Determinant by Gaussian elimination over the rationals."""
    A = [row[:] for row in M]
    n = len(A)
    det = Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if A[r][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            A[c], A[p] = A[p], A[c]
            det = -det
        piv = A[c][c]
        det *= piv
        for r in range(c + 1, n):
            if A[r][c] != 0:
                f = A[r][c] / piv
                for k in range(c, n):
                    A[r][k] -= f * A[c][k]
    return det


def _minor(L, drop):
    keep = [i for i in range(len(L)) if i not in drop]
    return [[L[i][j] for j in keep] for i in keep]


def resistance_cramer(g, u: int, v: int) -> Fraction:
    if u == v:
        return Fraction(0)
    L = _laplacian_fraction(g.n, g.eu, g.ev, g.w)
    num = det_fraction(_minor(L, {u, v})) if g.n > 2 else Fraction(1)
    den = det_fraction(_minor(L, {u}))
    return num / den


def edge_resistances_trees(g) -> list:
    """R_e for every edge of g by enumerating spanning trees (n <= 7 or so)."""
    n, m = g.n, g.m
    eu = np.asarray(g.eu).tolist()
    ev = np.asarray(g.ev).tolist()
    w = [Fraction(x) for x in np.asarray(g.w).tolist()]
    total = Fraction(0)
    with_e = [Fraction(0)] * m
    for sub in itertools.combinations(range(m), n - 1):
        parent = list(range(n))

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x

        ok = True
        for e in sub:
            a, b = find(eu[e]), find(ev[e])
            if a == b:
                ok = False
                break
            parent[a] = b
        if not ok:
            continue
        tw = Fraction(1)
        for e in sub:
            tw *= w[e]
        total += tw
        for e in sub:
            with_e[e] += tw
    return [with_e[e] / (w[e] * total) if eu[e] != ev[e] else Fraction(0) for e in range(m)]


def to_float(x: Fraction) -> float:
    """Correctly rounded FP64 value (Python's int/int division rounds correctly)."""
    return x.numerator / x.denominator
