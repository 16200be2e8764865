"""Dense oracle: R_uv = b^T L_r^{-1} b with b = e_u - e_v (Section II-A eq 2, Section IV-A eq 15).

``resistances`` factors the dense grounded Laplacian with LAPACK Cholesky,
solves for all query right-hand sides at once and refines once with an
extended-precision residual. ``resistances_pinv`` is the independent
pseudo-inverse form the paper also states (Section IV-A):
R_uv = L+_uu + L+_vv - 2 L+_uv, independent of the ground.
Intended for n up to a few thousand.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

from .laplacian import laplacian_dense, grounded_dense, incidence_columns


def resistances(g, qu, qv, refine: int = 2) -> np.ndarray:
    n = g.n
    L_ld = laplacian_dense(n, g.eu, g.ev, g.w, dtype=np.longdouble)
    Lr_ld = grounded_dense(L_ld, g.ground)
    Lr = Lr_ld.astype(np.float64)
    B = incidence_columns(n, g.ground, qu, qv)
    cho = la.cho_factor(Lr, lower=True, check_finite=True)
    X = la.cho_solve(cho, B).astype(np.longdouble)
    if refine:
        # residual against the extended-precision matrix: the FP64 diagonal sums
        # are themselves rounded, and the refinement removes that perturbation
        Lr_ld = sp.csr_matrix(Lr_ld)
        for _ in range(refine):
            res = B.astype(np.longdouble) - Lr_ld @ X
            X = X + la.cho_solve(cho, res.astype(np.float64)).astype(np.longdouble)
    R = np.sum(B.astype(np.longdouble) * X, axis=0)
    return R.astype(np.float64)


def resistances_pinv(g, qu, qv) -> np.ndarray:
    L = laplacian_dense(g.n, g.eu, g.ev, g.w)
    P = np.linalg.pinv(L, hermitian=True)
    qu = np.asarray(qu, dtype=np.int64)
    qv = np.asarray(qv, dtype=np.int64)
    R = P[qu, qu] + P[qv, qv] - 2.0 * P[qu, qv]
    R[qu == qv] = 0.0
    return R


def grounded_inverse(g) -> np.ndarray:
    """Dense L_r^{-1} (rows/cols in reduced order): R_ug = (L_r^{-1})_uu (eq 4, t = g case)."""
    L = laplacian_dense(g.n, g.eu, g.ev, g.w)
    Lr = grounded_dense(L, g.ground)
    cho = la.cho_factor(Lr, lower=True)
    return la.cho_solve(cho, np.eye(Lr.shape[0]))
