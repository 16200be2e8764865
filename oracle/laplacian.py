"""Graph Laplacian and grounding (Section II-A, eq 1).

L_G = D - W = sum over edges (i, j) of w_ij (1_i - 1_j)(1_i - 1_j)^T. A self-loop
contributes a zero matrix; parallel edges add. Grounding node g deletes its row
and column, leaving the reduced Laplacian L_r (SPD for a connected graph).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def laplacian_dense(n: int, eu, ev, w, dtype=np.float64) -> np.ndarray:
    """Dense L_G, built term by term from eq 1.

    With ``dtype=np.longdouble`` the diagonal sums keep 64 mantissa bits, which
    the refinement steps use as the (near-)exact matrix.
    """
    L = np.zeros((n, n), dtype=dtype)
    for a, b, x in zip(np.asarray(eu).tolist(), np.asarray(ev).tolist(), np.asarray(w).tolist()):
        if a == b:
            continue  # (1_a - 1_a) = 0
        x = dtype(x)
        L[a, a] += x
        L[b, b] += x
        L[a, b] -= x
        L[b, a] -= x
    return L


def laplacian_sparse(n: int, eu, ev, w, dtype=np.float64) -> sp.csr_matrix:
    """Sparse L_G (duplicates summed), same terms as ``laplacian_dense``."""
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64).astype(dtype)
    keep = eu != ev
    eu, ev, w = eu[keep], ev[keep], w[keep]
    rows = np.concatenate([eu, ev, eu, ev])
    cols = np.concatenate([eu, ev, ev, eu])
    vals = np.concatenate([w, w, -w, -w])
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


def reduced_index(n: int, g: int) -> np.ndarray:
    """Map original id -> row of L_r (the ground maps to -1)."""
    r = np.arange(n, dtype=np.int64)
    r[g + 1:] -= 1
    r[g] = -1
    return r


def grounded_dense(L: np.ndarray, g: int) -> np.ndarray:
    keep = np.array([i for i in range(L.shape[0]) if i != g], dtype=np.int64)
    return L[np.ix_(keep, keep)]


def grounded_sparse(L: sp.spmatrix, g: int) -> sp.csc_matrix:
    n = L.shape[0]
    keep = np.concatenate([np.arange(g), np.arange(g + 1, n)])
    return L.tocsr()[keep][:, keep].tocsc()


def incidence_columns(n: int, g: int, qu, qv) -> np.ndarray:
    """Dense (n-1) x q matrix whose column k is e_u - e_v restricted to L_r's rows (eq 4)."""
    r = reduced_index(n, g)
    qu = np.asarray(qu, dtype=np.int64)
    qv = np.asarray(qv, dtype=np.int64)
    B = np.zeros((n - 1, qu.shape[0]), dtype=np.float64)
    for k, (a, b) in enumerate(zip(qu.tolist(), qv.tolist())):
        if a == b:
            continue
        if r[a] >= 0:
            B[r[a], k] += 1.0
        if r[b] >= 0:
            B[r[b], k] -= 1.0
    return B
