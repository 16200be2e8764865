"""GPU parity of the implicit sweep against the CPU oracle (through the C ABI).

Tolerance: the acceptance bar is a relative error of at most 1e-10 per
resistance (the paper's accuracy level, Section V-B); the FP64 noise floor of
two independent solvers is about 1e-15, so the tests also report the observed
maximum. Expected values come from ``oracle`` only (computed here, or stored
in ``tests/golden`` by ``tests/golden/make_golden.py``).
"""
import json
import math
import os

import numpy as np
import pytest

import synth
import paper_2606_31535_amd as P
from oracle import dense, sparse

pytestmark = pytest.mark.gpu
TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def dev(hip_device):
    d = P.peers_device_open(0)
    yield d
    P.peers_device_close(d)


def _factor(dev, g, **kw):
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords, **kw)
    f = P.peers_factor_upload(dev, h)
    return h, f


def _all_edges(dev, g, **kw):
    h, f = _factor(dev, g, **kw)
    try:
        R = np.full(g.m, np.nan)
        P.peers_query_all_edges(f, R)
        return R
    finally:
        P.peers_factor_release(f)
        P.peers_graph_destroy(h)


def _relerr(R, Ro):
    nz = Ro != 0
    assert np.all(R[~nz] == 0.0)
    return float(np.max(np.abs(R[nz] - Ro[nz]) / Ro[nz])) if nz.any() else 0.0


def test_c1_mesh_all_edges_vs_dense_oracle(dev):
    g = synth.mesh2d()
    R = _all_edges(dev, g)
    Ro = dense.resistances(g, g.eu, g.ev)
    err = _relerr(R, Ro)
    print(f"C1 max rel err {err:.3e}")
    assert err <= TOL
    assert abs(math.fsum(g.w * R) - (g.n - 1)) <= TOL * (g.n - 1)


@pytest.mark.parametrize("seed", [1, 2])
def test_random_graphs_vs_dense_oracle(dev, seed):
    g = synth.random_connected(1500, 3000, seed=seed, wlog=2.0, multi=True, ground=seed * 7)
    R = _all_edges(dev, g)
    err = _relerr(R, dense.resistances(g, g.eu, g.ev))
    print(f"random seed {seed} max rel err {err:.3e}")
    assert err <= TOL


def test_tree_edges_exact_inverse_conductance(dev):
    g = synth.random_tree(5000, seed=3, wlog=2.0, ground=17)
    R = _all_edges(dev, g)
    assert _relerr(R, 1.0 / g.w) <= TOL


def test_torus_every_edge_closed_form(dev):
    k = 128
    g = synth.torus2d(k, ground=5)
    R = _all_edges(dev, g)
    err = _relerr(R, np.full(g.m, (k * k - 1) / (2.0 * k * k)))
    print(f"torus {k} max rel err {err:.3e}")
    assert err <= TOL


def test_pdn_with_pendant_probes_and_sample(dev):
    base = synth.pdn_multilayer(side=96, layers=4, seed=21)
    g, probes = synth.add_pendants(base, 200, seed=4)
    R = _all_edges(dev, g)
    assert _relerr(R[probes], 1.0 / g.w[probes]) <= TOL
    rng = np.random.default_rng(5)
    sel = rng.choice(g.m, 300, replace=False)
    Ro = sparse.SparseOracle(g, ordering="nd").resistances(g.eu[sel], g.ev[sel])
    err = _relerr(R[sel], Ro)
    print(f"pdn96 sample max rel err {err:.3e}")
    assert err <= TOL
    assert abs(math.fsum(g.w * R) - (g.n - 1)) <= TOL * (g.n - 1)


def test_edge_cases(dev):
    # two nodes; parallel edges and self-loops; ground as a cut node (forest)
    g = synth.Graph(n=2, eu=np.array([0], np.int32), ev=np.array([1], np.int32), w=np.array([4.0]), ground=1)
    assert _all_edges(dev, g).tolist() == [0.25]
    g = synth.Graph(n=4, eu=np.array([0, 0, 1, 2, 2, 3], np.int32), ev=np.array([1, 1, 1, 3, 1, 0], np.int32),
                    w=np.array([1.0, 3.0, 9.0, 2.0, 0.5, 0.25]), ground=2)
    R = _all_edges(dev, g)
    Ro = dense.resistances(g, g.eu, g.ev)
    assert R[2] == 0.0
    assert _relerr(R, Ro) <= TOL
    g = synth.star_graph(40, ground=0)  # grounding the centre leaves 39 one-node trees
    R = _all_edges(dev, g)
    assert _relerr(R, np.ones(39)) <= TOL
    base = synth.path_graph(30)
    g = synth.Graph(n=30, eu=base.eu, ev=base.ev, w=base.w, ground=15)  # cut node ground
    assert _relerr(_all_edges(dev, g), np.ones(29)) <= TOL


def test_pair_queries_ancestor_and_ground(dev):
    g = synth.mesh2d(24, 20, seed=9)
    h, f = _factor(dev, g)
    try:
        n = g.n
        qu = np.concatenate([g.eu, np.arange(n), np.arange(n), [3, 5]]).astype(np.int32)
        qv = np.concatenate([g.ev, np.full(n, g.ground), np.arange(n), [3, 5]]).astype(np.int32)
        R = np.full(qu.shape[0], np.nan)
        P.peers_query(f, qu, qv, R)
        Ro = dense.resistances(g, qu, qv)
        assert _relerr(R, Ro) <= TOL
        with pytest.raises(P.PeersError) as ei:
            P.peers_query(f, np.array([0], np.int32), np.array([n], np.int32), np.zeros(1))
        assert ei.value.status == -2
    finally:
        P.peers_factor_release(f)
        P.peers_graph_destroy(h)


def test_general_pairs_vs_dense_oracle(dev):
    # pairs of every kind: non-ancestor pairs (split at the lowest common
    # ancestor), ancestor pairs, ground pairs and self pairs, on a mesh and on
    # an unstructured graph (graph ordering, no coordinates)
    for g in (synth.mesh2d(24, 20, seed=9), synth.random_connected(900, 2500, seed=21, wlog=1)):
        rng = synth.rng_for(77)
        k = 1500
        qu = rng.integers(0, g.n, k).astype(np.int32)
        qv = rng.integers(0, g.n, k).astype(np.int32)
        qv[:20] = g.ground
        qv[20:30] = qu[20:30]
        h, f = _factor(dev, g)
        try:
            R = np.full(k, np.nan)
            P.peers_query(f, qu, qv, R)
            Ro = dense.resistances(g, qu, qv)
            err = _relerr(R, Ro)
            print(f"{g.name}: {k} random pairs, max rel err {err:.3e}")
            assert err <= TOL
            # a request of a few pairs sweeps only their subtrees and returns
            # the same bits as inside the large request
            sel = np.array([3, 50, 400, 999, 1400])
            Rs = np.full(len(sel), np.nan)
            P.peers_query(f, qu[sel], qv[sel], Rs)
            assert np.array_equal(Rs.view(np.int64), R[sel].view(np.int64))
        finally:
            P.peers_factor_release(f)
            P.peers_graph_destroy(h)


def test_general_pairs_pdn_vs_sparse_oracle(dev):
    g = synth.pdn_multilayer(side=60, layers=4, seed=7, long_frac=0.002)
    rng = synth.rng_for(78)
    k = 300
    qu = rng.integers(0, g.n, k).astype(np.int32)
    qv = rng.integers(0, g.n, k).astype(np.int32)
    h, f = _factor(dev, g)
    try:
        R = np.full(k, np.nan)
        P.peers_query(f, qu, qv, R)
    finally:
        P.peers_factor_release(f)
        P.peers_graph_destroy(h)
    Ro = sparse.SparseOracle(g).resistances(qu, qv)
    err = _relerr(R, Ro)
    print(f"pdn 14400: {k} random pairs, max rel err {err:.3e}")
    assert err <= TOL


def test_device_output_and_determinism(dev):
    import torch
    g = synth.pdn_multilayer(side=64, layers=4, seed=3)
    h, f = _factor(dev, g)
    try:
        Rd = torch.empty(g.m, dtype=torch.float64, device="cuda")
        P.peers_query_all_edges(f, Rd, flags=P.PEERS_SYNC)
        torch.cuda.synchronize()
        R1 = Rd.cpu().numpy().copy()
        R2 = np.empty(g.m)
        P.peers_query_all_edges(f, R2)
        assert np.array_equal(R1.view(np.int64), R2.view(np.int64))
    finally:
        P.peers_factor_release(f)
        P.peers_graph_destroy(h)


def test_wide_store_addressing_same_bits(dev):
    # stores beyond 4 GB are addressed with 64-bit offsets; forcing that form on
    # a small factor must give the same bits as the 32-bit form
    g = synth.pdn_multilayer(side=48, layers=4, seed=21)
    R32 = _all_edges(dev, g)
    R64 = _all_edges(dev, g, store_offsets_64=True)
    assert np.array_equal(R32.view(np.int64), R64.view(np.int64))
    Ro = sparse.SparseOracle(g).resistances(g.eu[:200], g.ev[:200])
    assert _relerr(R64[:200], Ro) <= TOL


def test_scaling_by_four_is_bit_exact(dev):
    # Z = D^{-1/2} L^{-1}: scaling every conductance by 4 scales D by 4 and
    # D^{-1/2} by exactly 1/2 (sqrt is correctly rounded), L and the ordering
    # not at all, so every R scales by exactly 1/4.
    g = synth.pdn_multilayer(side=40, layers=4, seed=12)
    R = _all_edges(dev, g)
    R4 = _all_edges(dev, g.scaled(4.0))
    assert np.array_equal((R4 * 4.0).view(np.int64), R.view(np.int64))


def test_ground_change_and_relabel(dev):
    g = synth.pdn_multilayer(side=40, layers=4, seed=13)
    R = _all_edges(dev, g)
    g2 = synth.Graph(n=g.n, eu=g.eu, ev=g.ev, w=g.w, ground=g.n // 2, coords=g.coords)
    assert _relerr(_all_edges(dev, g2), R) <= TOL
    perm = synth.rng_for(3).permutation(g.n)
    assert _relerr(_all_edges(dev, g.relabeled(perm)), R) <= TOL


def _golden(cfg):
    path = os.path.join(GOLDEN, f"{cfg}_edges.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as fh:
        d = json.load(fh)
    return np.array(d["edges"]), np.array([float(x) for x in d["R"]])


@pytest.mark.parametrize("cfg,gen", [("C2", synth.pdn_two_layer), ("C3", synth.pdn_multilayer)])
def test_full_size_pdn_sampled_and_foster(dev, cfg, gen):
    g = gen()
    R = _all_edges(dev, g)
    edges, Ro = _golden(cfg)
    err = _relerr(R[edges], Ro)
    foster = math.fsum(g.w * R) - (g.n - 1)
    wr = g.w * R
    print(f"{cfg}: sampled max rel err {err:.3e} on {len(edges)} edges; Foster residual {foster:.3e}; "
          f"max w*R {wr.max():.17g}")
    assert err <= TOL
    assert abs(foster) <= TOL * (g.n - 1)
    assert np.all(wr > 0) and np.all(wr <= 1 + 1e-12)
