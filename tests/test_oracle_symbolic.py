"""Pins for the oracle's symbolic structures (Lemma 1, Definition 2, Theorems 1-2, Algorithm 3).

Two independent constructions of the factor pattern and elimination tree are
compared (dense boolean elimination versus Liu's etree plus row subtrees), and
hand-derived textbook patterns are checked from ``tests/golden``.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as la

import synth
from oracle import symbolic, laplacian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_perm(g, seed):
    rng = np.random.default_rng(seed)
    ids = np.array([x for x in range(g.n) if x != g.ground])
    return rng.permutation(ids)


GRAPHS = [
    lambda: synth.random_connected(40, extra=60, seed=1),
    lambda: synth.grid_unit(7, 6),
    lambda: synth.pdn_multilayer(side=6, layers=3, seed=2, long_frac=0.02),
    lambda: synth.random_tree(50, seed=3),
]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("seed", [0, 1])
def test_two_pattern_constructions_agree(gi, seed):
    g = GRAPHS[gi]()
    perm = _random_perm(g, seed)
    A = symbolic.permuted_pattern(g, perm)
    Ld = symbolic.symbolic_elimination_dense(A)
    p_dense = symbolic.etree_from_dense_pattern(Ld)
    p_liu = symbolic.etree_liu(A)
    assert np.array_equal(p_dense, p_liu)
    cp1, ri1 = symbolic.dense_to_csc(Ld)
    cp2, ri2 = symbolic.factor_pattern(A, p_liu)
    assert np.array_equal(cp1, cp2) and np.array_equal(ri1, ri2)


def test_numeric_factor_pattern_within_symbolic():
    # Lemma 1 / Theorem 2: nonzeros of L^{-1} lie in the etree ancestor relation;
    # and for positive conductances every symbolic entry of L is numerically nonzero.
    g = synth.random_connected(45, extra=70, seed=7)
    perm = _random_perm(g, 3)
    A = symbolic.permuted_pattern(g, perm)
    parent = symbolic.etree_liu(A)
    Lpat = symbolic.symbolic_elimination_dense(A)
    Lg = laplacian.laplacian_dense(g.n, g.eu, g.ev, g.w)
    P = Lg[np.ix_(perm, perm)]
    C = la.cholesky(P, lower=True)
    assert np.array_equal(np.abs(C) > 1e-300, Lpat)
    Z = la.solve_triangular(C, np.eye(C.shape[0]), lower=True)
    N = C.shape[0]
    anc = np.zeros((N, N), dtype=bool)
    for k in range(N):
        j = k
        while j >= 0:
            anc[j, k] = True
            j = parent[j]
    assert np.all(anc[np.abs(Z) > 0])


def test_alg3_reach_is_subtree_range_after_postorder():
    g = synth.grid_unit(8, 7)
    perm0 = _random_perm(g, 5)
    A0 = symbolic.permuted_pattern(g, perm0)
    post = symbolic.canonical_postorder(symbolic.etree_liu(A0))
    perm = perm0[post]
    A = symbolic.permuted_pattern(g, perm)
    parent = symbolic.etree_liu(A)
    assert symbolic.is_postordered(parent)
    cp, ri = symbolic.factor_pattern(A, parent)
    rows = symbolic.row_lists(cp, ri, A.shape[0])
    first = symbolic.subtree_first(parent)
    for j in range(A.shape[0]):
        S, d = symbolic.reach_alg3(rows, j)
        assert S == list(range(first[j], j + 1))
        # in-degree of k inside S_j counts the H-edges i -> k with i in S_j
        for k, dk in d.items():
            assert dk == sum(1 for i in S if k in rows[i])


def test_golden_textbook_patterns():
    with open(os.path.join(GOLDEN, "symbolic_textbook.json")) as f:
        cases = json.load(f)
    for case in cases:
        n = case["n"]
        g = synth.Graph(n=n, eu=np.array(case["eu"], np.int32), ev=np.array(case["ev"], np.int32),
                        w=np.ones(len(case["eu"])), ground=case["ground"])
        perm = np.array(case["perm"])
        A = symbolic.permuted_pattern(g, perm)
        parent = symbolic.etree_liu(A)
        cp, ri = symbolic.factor_pattern(A, parent)
        assert parent.tolist() == case["parent"], case["name"]
        assert cp.tolist() == case["colptr"], case["name"]
        assert ri.tolist() == case["rowidx"], case["name"]
        assert symbolic.fundamental_supernodes(parent, cp).tolist() == case["snptr"], case["name"]
        assert symbolic.depths(parent).tolist() == case["depth"], case["name"]
        if "postorder" in case:
            # children visited in ascending index (the tie-break that makes the
            # renumbered tree unique); hand-derived visiting order and ids
            post = symbolic.canonical_postorder(parent)
            assert post.tolist() == case["postorder"], case["name"]
            assert perm[post].tolist() == case["postorder_ids"], case["name"]


def _postorder_descending(parent):
    """A plausible mistake: children visited in descending index."""
    N = parent.shape[0]
    children = [[] for _ in range(N)]
    roots = []
    for i in range(N):
        (children[parent[i]] if parent[i] >= 0 else roots).append(i)
    out = []

    def visit(v):
        for c in sorted(children[v], reverse=True):
            visit(c)
        out.append(v)
    for r in roots:
        visit(r)
    return np.array(out, dtype=np.int64)


def test_planted_descending_postorder_is_caught(monkeypatch):
    monkeypatch.setattr(symbolic, "canonical_postorder", _postorder_descending)
    with pytest.raises(AssertionError):
        test_golden_textbook_patterns()
