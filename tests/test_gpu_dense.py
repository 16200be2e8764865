"""The dense sums of the rows above bottom subtrees against the plain sweep.

A query whose lower endpoint u lies in a bottom subtree S gets its rows above
S as ||Z[rows, U_S] w||^2 on the matrix cores (w = B_S e_u - B_S e_v, or
- e_v for v in U_S, or B_S e_u for the ground; B_S = -L_{U_S,S} L_SS^{-1}),
and the sweep sums only the rows from S on. The graph option sweep_only
turns this off, so the sweep sums every row (eq 12 as the paper states it).
Both forms must agree to the FP64 noise floor, and a query's result must not
depend on the other queries of its plan (the form is chosen per query from
the factor and the query alone), which the served and batched forms rely on.
The oracle comparisons of the same queries are in test_gpu_parity.py.
"""
import numpy as np
import pytest

import synth
import paper_2606_31535_amd as P

pytestmark = pytest.mark.gpu
NOISE = 1e-13  # FP64 summation-order differences on these graphs


@pytest.fixture(scope="module")
def dev(hip_device):
    d = P.peers_device_open(0)
    yield d
    P.peers_device_close(d)


@pytest.fixture(scope="module")
def pdn(dev):
    g = synth.pdn_multilayer(side=200, layers=4, seed=31)
    out = {}
    for name, kw in (("dense", {}), ("sweep", {"sweep_only": True})):
        h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords, **kw)
        out[name] = (h, P.peers_factor_upload(dev, h))
    yield g, out
    for h, f in out.values():
        P.peers_factor_release(f)
        P.peers_graph_destroy(h)


def _rel(a, b):
    nz = b != 0
    assert np.array_equal(a == 0, b == 0)
    return float(np.max(np.abs(a[nz] - b[nz]) / b[nz]))


def test_all_edges_dense_vs_sweep(pdn):
    g, fs = pdn
    R = {}
    for name, (h, f) in fs.items():
        R[name] = np.full(g.m, np.nan)
        P.peers_query_all_edges(f, R[name], flags=P.PEERS_PROFILE)
        tm = P.peers_factor_timings(fs[name][1])
        print(name, "bottom launches", tm["bottom_launches"], "bottom ms", round(tm["bottom_ms"], 3))
        if name == "dense":
            assert tm["bottom_launches"] > 1  # the dense groups ran
    err = _rel(R["dense"], R["sweep"])
    print(f"all edges: dense vs sweep max rel diff {err:.3e}")
    assert err <= NOISE


def test_ground_and_mixed_pairs_dense_vs_sweep(pdn):
    g, fs = pdn
    rng = np.random.default_rng(7)
    k = 30000
    e = rng.integers(0, g.m, k)
    u = np.concatenate([g.eu[e], rng.integers(0, g.n, k // 4), np.arange(0, g.n, 97)])
    v = np.concatenate([g.ev[e], rng.integers(0, g.n, k // 4), np.full(len(range(0, g.n, 97)), g.ground)])
    R = {}
    for name, (h, f) in fs.items():
        R[name] = np.full(len(u), np.nan)
        P.peers_query(f, u.astype(np.int32), v.astype(np.int32), R[name])
    err = _rel(R["dense"], R["sweep"])
    print(f"mixed pairs: dense vs sweep max rel diff {err:.3e}")
    assert err <= NOISE
    Rg = {}
    for name, (h, f) in fs.items():
        Rg[name] = np.full(g.n, np.nan)
        P.peers_query_all_to_ground(f, Rg[name])
    err = _rel(Rg["dense"], Rg["sweep"])
    print(f"node to ground: dense vs sweep max rel diff {err:.3e}")
    assert err <= NOISE


def test_result_independent_of_other_queries(pdn):
    """A query gets the same bits alone and among others of every kind."""
    g, fs = pdn
    f = fs["dense"][1]
    rng = np.random.default_rng(11)
    e = rng.integers(0, g.m, 2000)
    u0, v0 = g.eu[e].astype(np.int32), g.ev[e].astype(np.int32)
    alone = np.full(len(u0), np.nan)
    P.peers_query(f, u0, v0, alone)
    # the same edges among random pairs (non-ancestor pairs stage columns
    # and keep their subtrees' sweeps at full height) and ground pairs
    ru, rv = rng.integers(0, g.n, 20000), rng.integers(0, g.n, 20000)
    u = np.concatenate([ru[:10000], u0, ru[10000:], np.arange(0, g.n, 13)]).astype(np.int32)
    v = np.concatenate([rv[:10000], v0, rv[10000:], np.full(len(range(0, g.n, 13)), g.ground)]).astype(np.int32)
    mix = np.full(len(u), np.nan)
    P.peers_query(f, u, v, mix)
    got = mix[10000:10000 + len(u0)]
    assert np.array_equal(got.view(np.int64), alone.view(np.int64))
    # and the same as the all-edge plan's bits for those edges
    R = np.full(g.m, np.nan)
    P.peers_query_all_edges(f, R)
    assert np.array_equal(R[e].view(np.int64), alone.view(np.int64))
