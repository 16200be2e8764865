"""Pins for the factor-based oracles (LSolve per pair, dense implicit columns)
and for ``dense.grounded_inverse`` (the node-to-ground form of eq 4).

Each function is checked against values fixed by the mathematics, not by
itself: tree closed forms, exact rational Cramer determinants, the identity
``Z^T Z = L_r^{-1}`` (Section II-A eq 3), Foster's theorem, and the structure
the paper proves for the implicit rows (Lemma 1, Theorem 2: the row of node j
in ``L^{-1}`` is nonzero exactly on the subtree of j). Planted mistakes in each
function must make one of these fail. The factors handed to the oracles come
from LAPACK here; the library's own exported factor is checked the same way
in ``test_library_factor_through_lsolve``.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dense, exact, factor, laplacian, symbolic


# --------------------------------------------------------------- helpers

def _tree_ground_paths(g):
    """For a tree: parent pointers towards the ground and resistance to the ground."""
    adj = [[] for _ in range(g.n)]
    for a, b, x in zip(g.eu.tolist(), g.ev.tolist(), g.w.tolist()):
        adj[a].append((b, x))
        adj[b].append((a, x))
    par = [-1] * g.n
    dist = [0.0] * g.n
    seen = [False] * g.n
    seen[g.ground] = True
    order = [g.ground]
    for v in order:
        for u, x in adj[v]:
            if not seen[u]:
                seen[u] = True
                par[u] = v
                dist[u] = dist[v] + 1.0 / x
                order.append(u)
    return par, dist


def _tree_shared_resistance(par, dist, u, v):
    """Resistance of the part that the paths u -> ground and v -> ground share."""
    anc = set()
    x = u
    while x >= 0:
        anc.add(x)
        x = par[x]
    x = v
    while x not in anc:
        x = par[x]
    return dist[x]


def _factor_of(g, perm):
    """Unit-lower L (sparse) and D of P L_r P^T from LAPACK (not from the library)."""
    L = laplacian.laplacian_dense(g.n, g.eu, g.ev, g.w)
    pos = laplacian.reduced_index(g.n, g.ground)
    Ar = L[np.ix_(perm, perm)]
    Ld, D = factor.ldlt_dense(Ar)
    import scipy.sparse as sp
    return sp.csr_matrix(np.tril(Ld)), D, pos


def _perm(g, seed):
    ids = np.array([x for x in range(g.n) if x != g.ground])
    return np.random.default_rng(seed).permutation(ids)


# --------------------------------------------------------------- grounded_inverse

def test_grounded_inverse_tree_closed_form():
    # (L_r^{-1})_uv is the resistance of the shared part of the two paths to
    # the ground (series rule on a tree; for u = v it is R_ug)
    g = synth.random_tree(25, seed=4, wlog=2.0, ground=6)
    G = dense.grounded_inverse(g)
    par, dist = _tree_ground_paths(g)
    r = laplacian.reduced_index(g.n, g.ground)
    for u in range(g.n):
        for v in range(g.n):
            if u == g.ground or v == g.ground:
                continue
            want = _tree_shared_resistance(par, dist, u, v)
            assert abs(G[r[u], r[v]] - want) <= 1e-12 * max(1.0, want)


@pytest.mark.parametrize("seed", [1, 2])
def test_grounded_inverse_diagonal_is_exact_node_to_ground(seed):
    g = synth.random_connected(9, extra=9, seed=seed, dyadic=True, ground=3)
    G = dense.grounded_inverse(g)
    r = laplacian.reduced_index(g.n, g.ground)
    tr = 0
    for u in range(g.n):
        if u == g.ground:
            continue
        ex = exact.resistance_cramer(g, u, g.ground)
        tr += ex
        assert abs(G[r[u], r[u]] - exact.to_float(ex)) <= 1e-13 * exact.to_float(ex)
    # sum over nodes of R_ug = trace(L_r^{-1})
    assert abs(np.trace(G) - exact.to_float(tr)) <= 1e-13 * exact.to_float(tr)


def test_grounded_inverse_gives_edge_resistances():
    # R_uv = G_uu + G_vv - 2 G_uv (eq 2 with e_g = 0); Foster's theorem on top
    g = synth.random_connected(60, extra=90, seed=5, wlog=2.0, ground=11)
    G = dense.grounded_inverse(g)
    r = laplacian.reduced_index(g.n, g.ground)

    def ent(a, b):
        return 0.0 if (r[a] < 0 or r[b] < 0) else G[r[a], r[b]]
    R = np.array([ent(a, a) + ent(b, b) - 2 * ent(a, b) for a, b in zip(g.eu.tolist(), g.ev.tolist())])
    assert abs(math.fsum(g.w * R) - (g.n - 1)) <= 1e-11 * g.n
    assert np.max(np.abs(R - dense.resistances(g, g.eu, g.ev)) / R) <= 1e-11


# --------------------------------------------------------------- LSolve on a factor (O6)

@pytest.mark.parametrize("seed", [0, 1])
def test_lsolve_tree_edges(seed):
    g = synth.random_tree(40, seed=seed + 8, wlog=2.0, ground=5)
    perm = _perm(g, seed)
    L, D, _ = _factor_of(g, perm)
    R = factor.resistances_lsolve(g.n, g.ground, perm, L, D, g.eu, g.ev)
    # a random order on a tree fills in, and conductances spanning four
    # decades make the dense factor lose a few digits: the contract gate
    assert np.max(np.abs(R * g.w - 1.0)) <= 1e-10


def test_lsolve_complete_graph_and_ground_pairs():
    g = synth.complete_graph(10, ground=4)
    perm = _perm(g, 3)
    L, D, _ = _factor_of(g, perm)
    R = factor.resistances_lsolve(g.n, g.ground, perm, L, D, g.eu, g.ev)
    assert np.max(np.abs(R - 2.0 / 10)) <= 1e-13
    # pairs with the ground, self pairs
    R2 = factor.resistances_lsolve(g.n, g.ground, perm, L, D, [4, 0, 7, 4], [0, 4, 7, 4])
    assert np.allclose(R2[:2], 2.0 / 10, rtol=1e-13, atol=0) and R2[2] == 0.0 and R2[3] == 0.0


@pytest.mark.parametrize("seed", [3, 4])
def test_lsolve_matches_exact_rational(seed):
    g = synth.random_connected(9, extra=10, seed=seed, dyadic=True, ground=2)
    perm = _perm(g, seed)
    L, D, _ = _factor_of(g, perm)
    qu, qv = np.array([0, 1, 5, 8, 2]), np.array([7, 6, 3, 2, 4])
    R = factor.resistances_lsolve(g.n, g.ground, perm, L, D, qu, qv)
    ex = np.array([exact.to_float(exact.resistance_cramer(g, int(a), int(b))) for a, b in zip(qu, qv)])
    assert np.max(np.abs(R - ex) / ex) <= 1e-13


# --------------------------------------------------------------- dense implicit columns (O5)

def test_implicit_columns_gram_is_grounded_inverse():
    # Z^T Z = L^{-T} D^{-1} L^{-1} = (P L_r P^T)^{-1}
    g = synth.random_connected(50, extra=80, seed=6, wlog=2.0, ground=9)
    perm = _perm(g, 2)
    L, D, r = _factor_of(g, perm)
    Z = factor.implicit_columns(L, D)
    G = dense.grounded_inverse(g)
    rp = r[perm]
    assert np.max(np.abs(Z.T @ Z - G[np.ix_(rp, rp)])) <= 1e-12 * np.max(np.abs(G))


def test_implicit_rows_structure_after_postorder():
    # Lemma 1 / Theorem 2 and the sign structure of a grounded Laplacian: with
    # Y = L^{-1} (unit), Y_jj = 1, 0 <= Y_ji <= 1, and Y_ji > 0 exactly for i in
    # subtree(j) = [first(j), j] once the tree is postordered
    g = synth.grid_unit(9, 8, ground=3)
    perm0 = _perm(g, 7)
    A0 = symbolic.permuted_pattern(g, perm0)
    perm = perm0[symbolic.canonical_postorder(symbolic.etree_liu(A0))]
    parent = symbolic.etree_liu(symbolic.permuted_pattern(g, perm))
    first = symbolic.subtree_first(parent)
    L, D, _ = _factor_of(g, perm)
    Z = factor.implicit_columns(L, D)
    Y = Z * np.sqrt(D)[:, None]
    N = Y.shape[0]
    assert np.allclose(np.diag(Y), 1.0, rtol=0, atol=1e-14)
    assert Y.min() >= -1e-15 and Y.max() <= 1.0 + 1e-13
    for j in range(N):
        sup = np.nonzero(np.abs(Y[j]) > 1e-300)[0]
        assert sup.tolist() == list(range(first[j], j + 1))
    # depth-indexed columns: the diagonal sits at depth - 1, and the squared
    # column sums are the diagonal of L_r^{-1} in elimination order
    nodes = [0, N // 2, N - 1]
    zc = factor.depth_columns(Z, parent, nodes)
    dep = symbolic.depths(parent)
    G = dense.grounded_inverse(g)
    r = laplacian.reduced_index(g.n, g.ground)
    for k, i in enumerate(nodes):
        assert zc[k, dep[i] - 1] == Z[i, i] and np.all(zc[k, dep[i]:] == 0)
        gi = G[r[perm[i]], r[perm[i]]]
        assert abs(np.sum(zc[k] ** 2) - gi) <= 1e-12 * gi


# --------------------------------------------------------------- planted mistakes

def _lsolve_without_d(n, ground, perm, L, D, qu, qv, block=64):
    return factor.resistances_lsolve(n, ground, perm, L, np.ones_like(np.asarray(D)), qu, qv, block)


def _lsolve_forward_product(n, ground, perm, L, D, qu, qv, block=64):
    # y = L b instead of L^{-1} b
    D = np.asarray(D)
    pos = np.full(n, -1)
    pos[np.asarray(perm)] = np.arange(len(perm))
    out = []
    for a, b in zip(np.asarray(qu).tolist(), np.asarray(qv).tolist()):
        x = np.zeros(D.shape[0])
        if a != b:
            if a != ground:
                x[pos[a]] += 1
            if b != ground:
                x[pos[b]] -= 1
        y = L @ x
        out.append(np.sum(y * y / D))
    return np.array(out)


def _lsolve_ignores_perm(n, ground, perm, L, D, qu, qv, block=64):
    ids = np.array([x for x in range(n) if x != ground])
    return factor.resistances_lsolve(n, ground, ids, L, D, qu, qv, block)


def _columns_transposed(L, D):
    return factor.implicit_columns(L, D).T


def _grounded_inverse_no_shift(g):
    # grounds by deleting the last row/column instead of the ground's
    L = laplacian.laplacian_dense(g.n, g.eu, g.ev, g.w)
    return np.linalg.inv(L[:-1, :-1])


def _factor_pins_hold():
    ok = True
    g = synth.random_tree(30, seed=9, wlog=2.0, ground=5)
    perm = _perm(g, 0)
    L, D, _ = _factor_of(g, perm)
    R = factor.resistances_lsolve(g.n, g.ground, perm, L, D, g.eu, g.ev)
    ok &= bool(np.max(np.abs(R * g.w - 1.0)) <= 1e-10)
    g = synth.random_connected(40, extra=60, seed=6, wlog=2.0, ground=9)
    perm = _perm(g, 2)
    L, D, r = _factor_of(g, perm)
    Z = factor.implicit_columns(L, D)
    G = dense.grounded_inverse(g)
    rp = r[perm]
    ok &= bool(np.max(np.abs(Z.T @ Z - G[np.ix_(rp, rp)])) <= 1e-12 * np.max(np.abs(G)))
    gt = synth.random_tree(25, seed=4, wlog=2.0, ground=6)
    Gt = dense.grounded_inverse(gt)
    par, dist = _tree_ground_paths(gt)
    rt = laplacian.reduced_index(gt.n, gt.ground)
    for u in range(gt.n):
        if u != gt.ground:
            ok &= bool(abs(Gt[rt[u], rt[u]] - dist[u]) <= 1e-12 * max(1.0, dist[u]))
    return ok


def test_unmutated_factor_oracles_pass():
    assert _factor_pins_hold()


@pytest.mark.parametrize("target,attr,bad", [
    (factor, "resistances_lsolve", _lsolve_without_d),
    (factor, "resistances_lsolve", _lsolve_forward_product),
    (factor, "resistances_lsolve", _lsolve_ignores_perm),
    (factor, "implicit_columns", _columns_transposed),
    (dense, "grounded_inverse", _grounded_inverse_no_shift),
])
def test_planted_factor_mistake_is_caught(monkeypatch, target, attr, bad):
    monkeypatch.setattr(target, attr, bad)
    try:
        held = _factor_pins_hold()
    except Exception:
        held = False
    assert not held
