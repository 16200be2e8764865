"""Node-to-ground resistances for every node (eq 4 with t = g).

R_ug = (L_r^{-1})_uu, so the oracle's dense grounded inverse (pinned in
test_oracle_factor.py against exact rationals and tree closed forms) gives
every value on small graphs, and its trace gives the sum over nodes. At full
size the stored oracle sample (tests/golden/<cfg>_ground.json, sparse
per-pair solves) pins sampled nodes, and every edge must satisfy the
triangle inequalities of the resistance metric with the two node-to-ground
values of its endpoints.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
import paper_2606_31535_amd as P
from oracle import dense, laplacian

pytestmark = pytest.mark.gpu
TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def dev(hip_device):
    d = P.peers_device_open(0)
    yield d
    P.peers_device_close(d)


def _to_ground(dev, g, also_edges=False):
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords)
    f = P.peers_factor_upload(dev, h)
    try:
        R = np.full(g.n, np.nan)
        P.peers_query_all_to_ground(f, R)
        R2 = np.full(g.n, np.nan)
        P.peers_query_all_to_ground(f, R2)  # the resident plan, second call
        assert np.array_equal(R.view(np.int64), R2.view(np.int64))
        Re = None
        if also_edges:
            Re = np.full(g.m, np.nan)
            P.peers_query_all_edges(f, Re)
        # the same pairs through the general pair path give the same bits
        ids = np.arange(g.n, dtype=np.int32)
        Rp = np.full(g.n, np.nan)
        P.peers_query(f, ids, np.full(g.n, g.ground, np.int32), Rp)
        assert np.array_equal(R.view(np.int64), Rp.view(np.int64))
        return R, Re
    finally:
        P.peers_factor_release(f)
        P.peers_graph_destroy(h)


@pytest.mark.parametrize("name,gen", [
    ("mesh32", lambda: synth.mesh2d()),
    ("random", lambda: synth.random_connected(1500, 3000, seed=3, wlog=2.0, ground=11)),
    ("rgg", lambda: synth.rgg_knn(2500, seed=40013, ground=7)),
    ("pdn", lambda: synth.pdn_multilayer(side=20, layers=4, seed=6, long_frac=0.005)),
])
def test_every_node_vs_dense_inverse_and_trace(dev, name, gen):
    g = gen()
    R, _ = _to_ground(dev, g)
    G = dense.grounded_inverse(g)
    r = laplacian.reduced_index(g.n, g.ground)
    keep = r >= 0
    ref = np.zeros(g.n)
    ref[keep] = np.diag(G)[r[keep]]
    assert R[g.ground] == 0.0
    err = float(np.max(np.abs(R[keep] - ref[keep]) / ref[keep]))
    tr_err = abs(math.fsum(R) - math.fsum(np.diag(G))) / math.fsum(np.diag(G))
    print(f"{name}: max rel err {err:.3e}, sum vs trace(L_r^-1) {tr_err:.3e}")
    assert err <= TOL
    assert tr_err <= TOL


def test_tree_closed_form(dev):
    g = synth.random_tree(4000, seed=12, wlog=2.0, ground=33)
    R, _ = _to_ground(dev, g)
    # resistance to the ground along the unique path (series rule)
    adj = [[] for _ in range(g.n)]
    for a, b, x in zip(g.eu.tolist(), g.ev.tolist(), g.w.tolist()):
        adj[a].append((b, x))
        adj[b].append((a, x))
    dist = np.full(g.n, -1.0)
    dist[g.ground] = 0.0
    order = [g.ground]
    for v in order:
        for u, x in adj[v]:
            if dist[u] < 0:
                dist[u] = dist[v] + 1.0 / x
                order.append(u)
    nz = dist > 0
    assert np.max(np.abs(R[nz] - dist[nz]) / dist[nz]) <= TOL


@pytest.mark.parametrize("cfg,gen", [("C2", synth.pdn_two_layer), ("C3", synth.pdn_multilayer)])
def test_full_size_sample_and_metric_inequalities(dev, cfg, gen):
    g = gen()
    R, Re = _to_ground(dev, g, also_edges=True)
    with open(os.path.join(GOLDEN, f"{cfg}_ground.json")) as fh:
        d = json.load(fh)
    nodes = np.array(d["nodes"])
    Ro = np.array([float(x) for x in d["R"]])
    err = float(np.max(np.abs(R[nodes] - Ro) / Ro))
    # every edge: |R_ug - R_vg| <= R_uv <= R_ug + R_vg (resistance is a metric)
    u, v = g.eu.astype(np.int64), g.ev.astype(np.int64)
    slack = 1e-12 * (R[u] + R[v])
    assert np.all(Re <= R[u] + R[v] + slack)
    assert np.all(np.abs(R[u] - R[v]) <= Re + slack)
    others = np.ones(g.n, bool)
    others[g.ground] = False
    assert np.all(R[others] > 0) and R[g.ground] == 0.0
    print(f"{cfg}: {len(nodes)} sampled nodes, max rel err {err:.3e}; sum of R_ug {math.fsum(R):.6e}")
    assert err <= TOL
