"""Oracles that take a factor as DATA: LSolve per pair and dense implicit columns.

TEST INFRASTRUCTURE ONLY (see the package docstring). Both functions read a
factorisation ``A = P L_r P^T = L D L^T`` (unit lower ``L`` in compressed
columns, pivots ``D``, elimination order ``perm``) that is handed to them as
arrays -- the library's exported factor, or one the tests build with LAPACK.
Nothing here factors a matrix or shares code with the library.

* ``resistances_lsolve`` is the paper's accuracy protocol (Section V-A: the
  error is measured against a direct triangular-solve ("LSolve") answer):
  for each pair, ``y = L^{-1} P (e_u - e_v)`` by a sparse unit-lower
  triangular solve, then ``R = sum_j y_j^2 / D_j``. With ``Z = D^{-1/2} L^{-1}``
  this is ``||Z P (e_u - e_v)||^2`` (Section II-A eq 3 with the square root of
  ``D`` folded in; eq 12), so it evaluates the same expression the implicit
  sweep evaluates, but by explicit substitution.
* ``implicit_columns`` forms ``Z = D^{-1/2} L^{-1}`` densely (small N), the
  matrix whose columns the implicit sweep produces along elimination-tree
  paths (Section III-C eq 11; Lemma 3 states that the implicit rows equal
  triangular substitution). Column ``i`` of ``Z`` is nonzero only on the root
  path of ``i`` (Lemma 1), so ``depth_columns`` rewrites it depth-indexed:
  ``zcol[i][d] = Z[a_d(i), i]`` with ``a_d(i)`` the ancestor at depth ``d+1``
  (root depth 1).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def unit_lower(N: int, colptr, rowidx, Lx) -> sp.csr_matrix:
    """Sparse unit-lower L (explicit ones on the diagonal) from its strict-lower CSC arrays."""
    colptr = np.asarray(colptr, dtype=np.int64)
    rowidx = np.asarray(rowidx, dtype=np.int64)
    Lx = np.asarray(Lx, dtype=np.float64)
    cols = np.repeat(np.arange(N, dtype=np.int64), np.diff(colptr))
    rows = np.concatenate([rowidx, np.arange(N, dtype=np.int64)])
    cols = np.concatenate([cols, np.arange(N, dtype=np.int64)])
    vals = np.concatenate([Lx, np.ones(N)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def _positions(n: int, ground: int, perm) -> np.ndarray:
    """Original id -> elimination position (ground -> -1)."""
    perm = np.asarray(perm, dtype=np.int64)
    pos = np.full(n, -1, dtype=np.int64)
    pos[perm] = np.arange(perm.shape[0])
    pos[ground] = -1
    return pos


def resistances_lsolve(n: int, ground: int, perm, L: sp.spmatrix, D, qu, qv, block: int = 64) -> np.ndarray:
    """R for each pair (qu[k], qv[k]) of original ids by LSolve on the given factor."""
    D = np.asarray(D, dtype=np.float64)
    N = D.shape[0]
    pos = _positions(n, ground, perm)
    qu = np.asarray(qu, dtype=np.int64)
    qv = np.asarray(qv, dtype=np.int64)
    L = sp.csr_matrix(L)
    out = np.zeros(qu.shape[0])
    for s in range(0, qu.shape[0], block):
        e = min(qu.shape[0], s + block)
        B = np.zeros((N, e - s))
        for c, (a, b) in enumerate(zip(qu[s:e].tolist(), qv[s:e].tolist())):
            if a == b:
                continue  # e_u - e_u = 0: R = 0
            if pos[a] >= 0:
                B[pos[a], c] += 1.0
            if pos[b] >= 0:
                B[pos[b], c] -= 1.0
        Y = spla.spsolve_triangular(L, B, lower=True, unit_diagonal=True)
        Y = np.asarray(Y).reshape(N, e - s)
        out[s:e] = np.sum(Y * Y / D[:, None], axis=0)
    return out


def implicit_columns(L: sp.spmatrix, D) -> np.ndarray:
    """Dense Z = D^{-1/2} L^{-1} (N up to a few thousand)."""
    D = np.asarray(D, dtype=np.float64)
    N = D.shape[0]
    Y = la.solve_triangular(np.asarray(sp.csr_matrix(L).todense()), np.eye(N), lower=True, unit_diagonal=True)
    return Y / np.sqrt(D)[:, None]


def depth_columns(Z: np.ndarray, parent, nodes) -> np.ndarray:
    """zcol[k][d] = Z[a_d(i), i] for i = nodes[k]; rows padded with zeros to the tree height."""
    parent = np.asarray(parent, dtype=np.int64)
    N = parent.shape[0]
    depth = np.zeros(N, dtype=np.int64)
    for i in range(N - 1, -1, -1):  # parents have larger indices
        depth[i] = 1 if parent[i] < 0 else depth[parent[i]] + 1
    h = int(depth.max()) if N else 0
    out = np.zeros((len(nodes), h))
    for k, i in enumerate(nodes):
        j = int(i)
        while j >= 0:
            out[k, depth[j] - 1] = Z[j, i]
            j = int(parent[j])
    return out


def ldlt_dense(A: np.ndarray):
    """Unit-lower L and D of a dense SPD matrix via LAPACK Cholesky (C = L D^{1/2}).

    Used by the tests to hand the factor-based oracles a factor that does not
    come from the library.
    """
    C = la.cholesky(A, lower=True)
    d = np.diag(C).copy()
    return C / d[None, :], d * d
