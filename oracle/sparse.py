"""Sparse per-pair oracle: R_uv = b^T L_r^{-1} b for sampled pairs at any size (eq 2 / eq 15).

The grounded Laplacian is reordered with the oracle's own coordinate nested
dissection (``coordinate_nd``; written for the oracle only), factored by SciPy's
SuperLU with diagonal pivoting, and every solve is refined with a residual
evaluated in extended precision (``numpy.longdouble``). Small graphs without
coordinates use SuperLU's own minimum-degree ordering instead.

This follows the paper's accuracy protocol, which measures against direct
per-query solves (Section V-A), but uses an independent factorization.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .laplacian import laplacian_sparse, grounded_sparse, reduced_index


def _neighbours(indptr, indices, nodes):
    starts = indptr[nodes]
    lens = indptr[nodes + 1] - starts
    tot = int(lens.sum())
    if tot == 0:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64)
    owner = np.repeat(np.arange(nodes.shape[0]), lens)
    offs = np.arange(tot) - np.repeat(np.cumsum(lens) - lens, lens)
    return owner, indices[starts[owner] + offs]


def coordinate_nd(A: sp.spmatrix, coords: np.ndarray, leaf: int = 48) -> np.ndarray:
    """Nested dissection by coordinate bisection; returns perm with new -> old.

    A node set is split at the median of its widest coordinate; the separator is
    the set of nodes on the low side with a neighbour on the high side. Order:
    low part, high part, separator (each part recursively).
    """
    A = A.tocsr()
    N = A.shape[0]
    indptr = A.indptr.astype(np.int64)
    indices = A.indices.astype(np.int64)
    side = np.full(N, -1, dtype=np.int8)
    out = []
    stack = [("split", np.arange(N, dtype=np.int64))]
    while stack:
        kind, S = stack.pop()
        if kind == "emit":
            out.append(S)
            continue
        if S.shape[0] <= leaf:
            key = np.lexsort(coords[S].T[::-1])
            out.append(S[key])
            continue
        C = coords[S]
        spread = C.max(axis=0) - C.min(axis=0)
        ax = int(np.argmax(spread))
        if spread[ax] <= 0:
            out.append(S)
            continue
        med = np.median(C[:, ax])
        low = C[:, ax] <= med
        if low.all() or not low.any():
            low = C[:, ax] < med
            if low.all() or not low.any():
                out.append(S)
                continue
        Alow, Bhigh = S[low], S[~low]
        side[Alow] = 0
        side[Bhigh] = 1
        owner, nb = _neighbours(indptr, indices, Alow)
        cut = side[nb] == 1
        in_sep = np.zeros(Alow.shape[0], dtype=bool)
        in_sep[owner[cut]] = True
        sep = Alow[in_sep]
        Arest = Alow[~in_sep]
        side[S] = -1
        stack.append(("emit", sep[np.lexsort(coords[sep].T[::-1])] if sep.shape[0] else sep))
        stack.append(("split", Bhigh))
        stack.append(("split", Arest))
    perm = np.concatenate(out) if out else np.zeros(0, dtype=np.int64)
    assert perm.shape[0] == N
    return perm


class SparseOracle:
    """Factor L_r once, then answer pairs b^T L_r^{-1} b with refined solves."""

    def __init__(self, g, ordering: str = "auto", refine: int = 2, leaf: int = 48):
        self.g = g
        self.refine = refine
        L = laplacian_sparse(g.n, g.eu, g.ev, g.w)
        Ar = grounded_sparse(L, g.ground)
        Ar_ld = grounded_sparse(laplacian_sparse(g.n, g.eu, g.ev, g.w, dtype=np.longdouble), g.ground)
        self.ridx = reduced_index(g.n, g.ground)
        N = Ar.shape[0]
        if ordering == "auto":
            ordering = "nd" if (g.coords is not None and N > 4000) else "mmd"
        self.ordering = ordering
        if ordering == "nd":
            keep = np.concatenate([np.arange(g.ground), np.arange(g.ground + 1, g.n)])
            perm = coordinate_nd(Ar, g.coords[keep], leaf=leaf)
        else:
            perm = np.arange(N)
        self.perm = perm
        self.iperm = np.empty(N, dtype=np.int64)
        self.iperm[perm] = np.arange(N)
        Ap = Ar[perm][:, perm].tocsc()
        self.A = Ap
        self.A_ld = Ar_ld[perm][:, perm].tocsr()
        spec = "NATURAL" if ordering == "nd" else "MMD_AT_PLUS_A"
        self.lu = spla.splu(Ap, permc_spec=spec, diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))

    def _rows(self, x):
        r = self.ridx[np.asarray(x, dtype=np.int64)]
        return np.where(r >= 0, self.iperm[np.maximum(r, 0)], -1)

    def resistances(self, qu, qv, block: int = 16) -> np.ndarray:
        qu = np.asarray(qu, dtype=np.int64)
        qv = np.asarray(qv, dtype=np.int64)
        ru, rv = self._rows(qu), self._rows(qv)
        q = qu.shape[0]
        N = self.A.shape[0]
        out = np.zeros(q, dtype=np.float64)
        for s in range(0, q, block):
            e = min(q, s + block)
            k = e - s
            B = np.zeros((N, k), dtype=np.float64)
            cols = np.arange(k)
            a, b = ru[s:e], rv[s:e]
            same = qu[s:e] == qv[s:e]
            ma = (a >= 0) & ~same
            mb = (b >= 0) & ~same
            B[a[ma], cols[ma]] += 1.0
            B[b[mb], cols[mb]] -= 1.0
            X = self.lu.solve(B).astype(np.longdouble)
            Bl = B.astype(np.longdouble)
            for _ in range(self.refine):
                res = Bl - self.A_ld @ X
                X = X + self.lu.solve(res.astype(np.float64)).astype(np.longdouble)
            out[s:e] = np.sum(Bl * X, axis=0).astype(np.float64)
        return out
