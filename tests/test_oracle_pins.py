"""Pins for the CPU oracle: closed forms, exact arithmetic, Foster's theorem and invariants.

The oracle evaluates the definition R_uv = b^T L_r^{-1} b (Section II-A eq 2,
Section IV-A eq 15). Nothing here re-types that formula: each expected value
comes from an independent fact (a closed form of network theory, exact
rational arithmetic, a theorem), chosen so that a dropped term, a wrong sign or
index, or a transposed operand in the oracle fails at least one test.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import dense, sparse, exact

REL = 1e-13


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tree_edges_are_inverse_conductance(seed):
    g = synth.random_tree(60, seed=seed, wlog=3.0, ground=seed % 60)
    R = dense.resistances(g, g.eu, g.ev)
    assert _rel(R, 1.0 / g.w) < REL


def test_path_series_sum():
    w = 10.0 ** np.linspace(-2, 2, 30)
    g = synth.path_graph(31, w=w, ground=5)
    qu = np.zeros(31, dtype=np.int32)
    qv = np.arange(31, dtype=np.int32)
    R = dense.resistances(g, qu, qv)
    expect = [math.fsum(1.0 / w[:k]) for k in range(31)]
    assert R[0] == 0.0
    assert _rel(R[1:], expect[1:]) < REL


def test_parallel_edges_combine():
    # three parallel edges between 0 and 1 plus a pendant; a self-loop is ignored
    g = synth.Graph(n=3, eu=np.array([0, 0, 0, 1, 2], np.int32), ev=np.array([1, 1, 1, 2, 2], np.int32),
                    w=np.array([1.0, 2.5, 0.5, 3.0, 7.0]), ground=2)
    R = dense.resistances(g, np.array([0, 1, 0]), np.array([1, 2, 2]))
    assert _rel(R, [1 / 4.0, 1 / 3.0, 1 / 4.0 + 1 / 3.0]) < REL


@pytest.mark.parametrize("n", [3, 7, 20])
def test_complete_graph(n):
    g = synth.complete_graph(n, ground=n - 1)
    R = dense.resistances(g, g.eu, g.ev)
    assert _rel(R, np.full(g.m, 2.0 / n)) < REL


@pytest.mark.parametrize("n", [5, 12, 31])
def test_cycle_hop_distance(n):
    g = synth.cycle_graph(n, ground=3)
    qu = np.zeros(n, dtype=np.int32)
    qv = np.arange(n, dtype=np.int32)
    R = dense.resistances(g, qu, qv)
    expect = np.array([k * (n - k) / n for k in range(n)])
    assert R[0] == 0.0
    assert _rel(R[1:], expect[1:]) < REL


@pytest.mark.parametrize("k", [4, 9, 16])
def test_torus2d_edges(k):
    g = synth.torus2d(k, ground=k + 1)
    R = dense.resistances(g, g.eu, g.ev)
    assert _rel(R, np.full(g.m, (k * k - 1) / (2.0 * k * k))) < REL


def test_torus3d_edges():
    g = synth.torus3d(5, ground=7)
    R = dense.resistances(g, g.eu, g.ev)
    n = g.n
    assert _rel(R, np.full(g.m, (n - 1) / (3.0 * n))) < REL


@pytest.mark.parametrize("d", [2, 4, 7])
def test_hypercube_edges(d):
    g = synth.hypercube(d, ground=1)
    R = dense.resistances(g, g.eu, g.ev)
    assert _rel(R, np.full(g.m, (2 ** d - 1) / (d * 2 ** (d - 1)))) < REL


@pytest.mark.parametrize("a,b", [(1, 5), (3, 4), (6, 9)])
def test_complete_bipartite_edges(a, b):
    g = synth.complete_bipartite(a, b, ground=a)
    R = dense.resistances(g, g.eu, g.ev)
    assert _rel(R, np.full(g.m, (a + b - 1) / (a * b))) < REL


def _grid_spectral(a, b, pairs):
    """Unit grid P_a x P_b: R_uv = sum over modes (p,q) != (0,0) of (phi(u)-phi(v))^2 / lambda.

    The path Laplacian's eigenvectors are DCT-II cosines, cos(pi p (x+1/2)/a),
    with eigenvalues 4 sin^2(pi p / 2a); the grid is their Kronecker sum.
    """
    out = []
    cx = [math.sqrt((1.0 if p == 0 else 2.0) / a) for p in range(a)]
    cy = [math.sqrt((1.0 if q == 0 else 2.0) / b) for q in range(b)]
    for u, v in pairs:
        uy, ux = divmod(u, a)
        vy, vx = divmod(v, a)
        terms = []
        for p in range(a):
            for q in range(b):
                if p == 0 and q == 0:
                    continue
                lam = 4 * math.sin(math.pi * p / (2 * a)) ** 2 + 4 * math.sin(math.pi * q / (2 * b)) ** 2
                fu = cx[p] * math.cos(math.pi * p * (ux + 0.5) / a) * cy[q] * math.cos(math.pi * q * (uy + 0.5) / b)
                fv = cx[p] * math.cos(math.pi * p * (vx + 0.5) / a) * cy[q] * math.cos(math.pi * q * (vy + 0.5) / b)
                terms.append((fu - fv) ** 2 / lam)
        out.append(math.fsum(terms))
    return np.array(out)


def test_grid_spectral_closed_form():
    a, b = 9, 6
    g = synth.grid_unit(a, b, ground=0)
    rng = np.random.default_rng(0)
    pairs = [(int(x), int(y)) for x, y in rng.integers(0, a * b, size=(40, 2)) if x != y]
    pairs += list(zip(g.eu.tolist()[:20], g.ev.tolist()[:20]))
    R = dense.resistances(g, [p[0] for p in pairs], [p[1] for p in pairs])
    assert _rel(R, _grid_spectral(a, b, pairs)) < 1e-12


# ---------------------------------------------------------------- exact arithmetic

def test_exact_small_textbook_values():
    # unit triangle: 2/3 per edge; unit square with one diagonal (Wheatstone-like)
    g = synth.complete_graph(3)
    assert exact.resistance_cramer(g, 0, 1) == Fraction(2, 3)
    sq = synth.Graph(n=4, eu=np.array([0, 1, 2, 3, 0], np.int32), ev=np.array([1, 2, 3, 0, 2], np.int32),
                     w=np.ones(5))
    # opposite corners 1-3 of a unit square with diagonal 0-2: series-parallel reduction gives 1
    assert exact.resistance_cramer(sq, 1, 3) == Fraction(1)
    # diagonal edge 0-2: two 2-ohm paths in parallel with 1 ohm: 1/(1+1/2+1/2) = 1/2
    assert exact.resistance_cramer(sq, 0, 2) == Fraction(1, 2)


@pytest.mark.parametrize("seed", range(6))
def test_cramer_equals_spanning_tree_enumeration(seed):
    g = synth.random_connected(6, extra=4, seed=seed, dyadic=True, multi=True)
    trees = exact.edge_resistances_trees(g)
    for e in range(g.m):
        assert exact.resistance_cramer(g, int(g.eu[e]), int(g.ev[e])) == trees[e]


@pytest.mark.parametrize("seed", range(8))
def test_dense_matches_exact(seed):
    g = synth.random_connected(11, extra=12, seed=100 + seed, wlog=2.0, ground=seed % 11)
    rng = np.random.default_rng(seed)
    qu = rng.integers(0, g.n, 25)
    qv = rng.integers(0, g.n, 25)
    R = dense.resistances(g, qu, qv)
    ex = [exact.to_float(exact.resistance_cramer(g, int(a), int(b))) for a, b in zip(qu, qv)]
    for r, e in zip(R, ex):
        if e == 0.0:
            assert r == 0.0
        else:
            assert abs(r - e) / e < 1e-14


# ---------------------------------------------------------------- theorems and invariants

@pytest.mark.parametrize("seed", range(4))
def test_foster_theorem(seed):
    g = synth.random_connected(150, extra=300, seed=seed, wlog=3.0, multi=True)
    R = dense.resistances(g, g.eu, g.ev)
    assert abs(math.fsum(g.w * R) - (g.n - 1)) < 1e-10 * g.n


def test_ground_independence_and_pinv():
    g = synth.random_connected(80, extra=150, seed=9)
    rng = np.random.default_rng(1)
    qu, qv = rng.integers(0, 80, 60), rng.integers(0, 80, 60)
    R0 = dense.resistances(g, qu, qv)
    g2 = synth.Graph(n=g.n, eu=g.eu, ev=g.ev, w=g.w, ground=41)
    assert _rel(R0[qu != qv], dense.resistances(g2, qu, qv)[qu != qv]) < 1e-12
    Rp = dense.resistances_pinv(g, qu, qv)
    assert _rel(R0[qu != qv], Rp[qu != qv]) < 1e-10


def test_dyadic_scaling_is_exact():
    g = synth.random_connected(60, extra=90, seed=4)
    R = dense.resistances(g, g.eu, g.ev)
    R8 = dense.resistances(g.scaled(8.0), g.eu, g.ev)
    assert _rel(R8 * 8.0, R) < 1e-14


def test_edge_bounds():
    g = synth.random_connected(120, extra=200, seed=5)
    R = dense.resistances(g, g.eu, g.ev)
    wr = g.w * R
    assert np.all(wr > 0) and np.all(wr <= 1 + 1e-14)


# ---------------------------------------------------------------- sparse oracle

@pytest.mark.parametrize("seed", range(3))
def test_sparse_matches_dense(seed):
    g = synth.random_connected(300, extra=500, seed=20 + seed, wlog=3.0, ground=seed)
    rng = np.random.default_rng(seed)
    qu = np.concatenate([g.eu, rng.integers(0, g.n, 100)])
    qv = np.concatenate([g.ev, rng.integers(0, g.n, 100)])
    Rd = dense.resistances(g, qu, qv)
    Rs = sparse.SparseOracle(g).resistances(qu, qv)
    nz = Rd > 0
    assert np.all(Rs[~nz] == 0.0)
    assert _rel(Rs[nz], Rd[nz]) < 1e-13


def test_sparse_nd_torus_closed_form():
    k = 96
    g = synth.torus2d(k, ground=17)
    so = sparse.SparseOracle(g, ordering="nd")
    sel = np.arange(0, g.m, 37)
    R = so.resistances(g.eu[sel], g.ev[sel])
    assert _rel(R, np.full(sel.shape[0], (k * k - 1) / (2.0 * k * k))) < 1e-13


def test_coordinate_nd_is_permutation():
    g = synth.pdn_multilayer(side=40, layers=4, seed=3)
    from oracle.laplacian import laplacian_sparse, grounded_sparse
    A = grounded_sparse(laplacian_sparse(g.n, g.eu, g.ev, g.w), 0)
    perm = sparse.coordinate_nd(A, g.coords[1:])
    assert np.array_equal(np.sort(perm), np.arange(g.n - 1))


def test_sparse_nd_pendant_probes_on_pdn():
    base = synth.pdn_multilayer(side=60, layers=4, seed=11)
    g, probes = synth.add_pendants(base, 40, seed=2)
    so = sparse.SparseOracle(g, ordering="nd")
    R = so.resistances(g.eu[probes], g.ev[probes])
    assert _rel(R, 1.0 / g.w[probes]) < 1e-13
