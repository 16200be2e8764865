"""Symbolic structures from their definitions (Section III-A/B, Lemma 1, Definition 2, Algorithm 3).

Given a graph and an elimination order ``perm`` (perm[i] = original id of the
node eliminated i-th; the ground is not in it), everything here is uniquely
determined, so the product's exported structures must match bit for bit:

* the structural pattern of the factor L of A = P L_r P^T, by boolean symbolic
  elimination (dense, small N) or by row subtrees of the elimination tree;
* the elimination tree: parent(i) = min{k > i : L_ki != 0};
* node depth (root depth 1) and ``first(j)``, the smallest index in subtree(j);
* fundamental supernodes: columns i and i+1 share a supernode iff
  parent(i) = i+1, node i+1 has exactly one child and colcount(i) = colcount(i+1)+1
  (colcount includes the diagonal);
* the reach set S_j of row j in the factor graph H (Definition 2: an edge
  i -> k whenever L_ik != 0, i > k), by the augmented DFS of Algorithm 3, which
  also counts the in-degrees d_k inside S_j.

An elimination tree is called postordered here when every subtree occupies the
contiguous index range [first(j), j]; the canonical postorder visits children
in ascending index.
"""
from __future__ import annotations

import sys

import numpy as np
import scipy.sparse as sp


def permuted_pattern(g, perm) -> sp.csr_matrix:
    """Boolean lower triangle (diagonal included) of P L_r P^T as CSR."""
    perm = np.asarray(perm, dtype=np.int64)
    N = g.n - 1
    assert perm.shape[0] == N
    pos = np.full(g.n, -1, dtype=np.int64)
    pos[perm] = np.arange(N)
    a = pos[np.asarray(g.eu, dtype=np.int64)]
    b = pos[np.asarray(g.ev, dtype=np.int64)]
    keep = (a >= 0) & (b >= 0) & (a != b)
    a, b = a[keep], b[keep]
    rows = np.concatenate([np.maximum(a, b), np.arange(N)])
    cols = np.concatenate([np.minimum(a, b), np.arange(N)])
    M = sp.coo_matrix((np.ones(rows.shape[0], dtype=np.int8), (rows, cols)), shape=(N, N)).tocsr()
    M.sum_duplicates()
    M.data[:] = 1
    return M


def symbolic_elimination_dense(Alow: sp.spmatrix) -> np.ndarray:
    """Dense boolean factor pattern: eliminating column k couples every pair of its lower rows."""
    N = Alow.shape[0]
    L = np.asarray(Alow.todense(), dtype=bool)
    L = np.tril(L | L.T)
    for k in range(N):
        idx = np.nonzero(L[k + 1:, k])[0] + k + 1
        if idx.shape[0] > 1:
            L[np.ix_(idx, idx)] = True  # only the lower half is ever read again
    return np.tril(L)


def etree_from_dense_pattern(L: np.ndarray) -> np.ndarray:
    N = L.shape[0]
    parent = np.full(N, -1, dtype=np.int64)
    for i in range(N):
        below = np.nonzero(L[i + 1:, i])[0]
        if below.shape[0]:
            parent[i] = i + 1 + below[0]
    return parent


def etree_liu(Alow: sp.spmatrix) -> np.ndarray:
    """Elimination tree by Liu's ancestor-walking algorithm, without path compression."""
    A = sp.csr_matrix(Alow)
    N = A.shape[0]
    parent = np.full(N, -1, dtype=np.int64)
    for k in range(N):
        for i in A.indices[A.indptr[k]:A.indptr[k + 1]].tolist():
            if i >= k:
                continue
            r = i
            while parent[r] != -1 and parent[r] != k:
                r = parent[r]
            if parent[r] == -1 and r != k:
                parent[r] = k
    return parent


def factor_pattern(Alow: sp.spmatrix, parent: np.ndarray):
    """Strict-lower pattern of L by row subtrees: row k holds every node on the
    etree paths from i (A_ki != 0, i < k) up to, not including, k.

    Returns (colptr int64[N+1], rowidx int32[nnz]) with rows sorted in each column.
    """
    A = sp.csr_matrix(Alow)
    N = A.shape[0]
    cols = [[] for _ in range(N)]
    mark = np.full(N, -1, dtype=np.int64)
    for k in range(N):
        mark[k] = k
        for i in A.indices[A.indptr[k]:A.indptr[k + 1]].tolist():
            while i < k and mark[i] != k:
                cols[i].append(k)
                mark[i] = k
                i = parent[i]
    colptr = np.zeros(N + 1, dtype=np.int64)
    colptr[1:] = np.cumsum([len(c) for c in cols])
    rowidx = np.array([r for c in cols for r in c], dtype=np.int32)
    return colptr, rowidx


def dense_to_csc(L: np.ndarray):
    N = L.shape[0]
    colptr = [0]
    rows = []
    for i in range(N):
        r = np.nonzero(L[i + 1:, i])[0] + i + 1
        rows.extend(r.tolist())
        colptr.append(len(rows))
    return np.array(colptr, dtype=np.int64), np.array(rows, dtype=np.int32)


def depths(parent: np.ndarray) -> np.ndarray:
    N = parent.shape[0]
    d = np.zeros(N, dtype=np.int64)
    for i in range(N - 1, -1, -1):  # parents have larger indices
        d[i] = 1 if parent[i] < 0 else d[parent[i]] + 1
    return d


def subtree_first(parent: np.ndarray) -> np.ndarray:
    N = parent.shape[0]
    first = np.arange(N, dtype=np.int64)
    for i in range(N):
        p = parent[i]
        if p >= 0 and first[i] < first[p]:
            first[p] = first[i]
    return first


def subtree_sizes(parent: np.ndarray) -> np.ndarray:
    N = parent.shape[0]
    size = np.ones(N, dtype=np.int64)
    for i in range(N):
        if parent[i] >= 0:
            size[parent[i]] += size[i]
    return size


def is_postordered(parent: np.ndarray) -> bool:
    first = subtree_first(parent)
    size = subtree_sizes(parent)
    return bool(np.all(first == np.arange(parent.shape[0]) - size + 1))


def canonical_postorder(parent: np.ndarray) -> np.ndarray:
    """post[new] = old; children visited in ascending index, roots in ascending index."""
    N = parent.shape[0]
    children = [[] for _ in range(N)]
    roots = []
    for i in range(N):
        (children[parent[i]] if parent[i] >= 0 else roots).append(i)
    out = []
    for r in roots:
        stack = [(r, 0)]
        while stack:
            v, c = stack.pop()
            if c < len(children[v]):
                stack.append((v, c + 1))
                stack.append((children[v][c], 0))
            else:
                out.append(v)
    return np.array(out, dtype=np.int64)


def fundamental_supernodes(parent: np.ndarray, colptr: np.ndarray) -> np.ndarray:
    """snptr[s]..snptr[s+1]-1 are the columns of supernode s."""
    N = parent.shape[0]
    nchild = np.zeros(N, dtype=np.int64)
    for i in range(N):
        if parent[i] >= 0:
            nchild[parent[i]] += 1
    cc = np.diff(colptr) + 1  # with the diagonal
    snptr = [0]
    for i in range(N - 1):
        join = parent[i] == i + 1 and nchild[i + 1] == 1 and cc[i] == cc[i + 1] + 1
        if not join:
            snptr.append(i + 1)
    snptr.append(N)
    return np.array(snptr, dtype=np.int64)


def row_lists(colptr: np.ndarray, rowidx: np.ndarray, N: int):
    """rows[i] = sorted k < i with L_ik != 0 (the out-edges of i in the factor graph H)."""
    rows = [[] for _ in range(N)]
    for c in range(N):
        for r in rowidx[colptr[c]:colptr[c + 1]].tolist():
            rows[r].append(c)
    return rows


def reach_alg3(rows, j: int):
    """Algorithm 3: DFS from j over H's edges i -> k (L_ik != 0), counting in-degrees.

    Returns (sorted reach set S_j, dict k -> in-degree d_k counted inside S_j).
    """
    vis = set()
    d = {}
    sys.setrecursionlimit(max(10000, sys.getrecursionlimit()))
    stack = [(j, iter(rows[j]))]
    vis.add(j)
    while stack:
        i, it = stack[-1]
        k = next(it, None)
        if k is None:
            stack.pop()
            continue
        d[k] = d.get(k, 0) + 1
        if k not in vis:
            vis.add(k)
            stack.append((k, iter(rows[k])))
    return sorted(vis), d
