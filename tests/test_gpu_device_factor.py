"""Numeric L D L^T on the device against the host factorization and the oracle.

A graph created with numeric_on_device has its factor formed on the GPU by
its first upload. The exported factor must reproduce the grounded Laplacian
(||P L_r P^T - L D L^T|| / ||L_r|| < 1e-13, D > 0), agree entry by entry with
the host factorization (both form each entry from same-signed sums, so the
two differ only in summation order: relative differences of a few ulps), be
the same bits on every run, and give resistances within the 1e-10 gate of the
oracle: the dense oracle on small graphs, the stored oracle samples at full
size (edges and node-to-ground).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

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


def _both(dev, g):
    """Host-factor graph, device-factor graph (uploaded), its factor handle."""
    hh = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords)
    hd = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords, numeric_on_device=True)
    with pytest.raises(P.PeersError) as e:
        P.peers_graph_export_factor(hd)
    assert e.value.status == -12
    f = P.peers_factor_upload(dev, hd)
    return hh, hd, f


def _close(dev, hh, hd, f):
    P.peers_factor_release(f)
    P.peers_graph_destroy(hh)
    P.peers_graph_destroy(hd)


GRAPHS = {
    "mesh32": lambda: synth.mesh2d(),
    "random": lambda: synth.random_connected(1500, 3000, seed=2, wlog=2.0, multi=True, ground=5),
    "rgg": lambda: synth.rgg_knn(3000, seed=40021, ground=3),
    "pdn": lambda: synth.pdn_multilayer(side=24, layers=4, seed=5, long_frac=0.005),
    "tree": lambda: synth.random_tree(2000, seed=6, wlog=2.0, ground=9),
    "star": lambda: synth.star_graph(300, ground=0),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_device_factor_small(dev, name):
    g = GRAPHS[name]()
    hh, hd, f = _both(dev, g)
    try:
        ex = P.peers_graph_export_symbolic(hd)
        Lx, D = P.peers_graph_export_factor(hd)
        Lh, Dh = P.peers_graph_export_factor(hh)
        st = P.peers_graph_stats_get(hd)
        assert st["t_numeric"] > 0
        # same ordering and pattern on both sides; values within a few ulps
        assert np.array_equal(P.peers_graph_export_symbolic(hh)["rowidx"], ex["rowidx"])
        assert np.all(D > 0)
        dL = np.max(np.abs(Lx - Lh) / np.maximum(np.abs(Lh), 1e-300)) if len(Lx) else 0.0
        dD = np.max(np.abs(D - Dh) / Dh)
        print(f"{name}: device vs host factor: L {dL:.2e}, D {dD:.2e}; t_numeric {st['t_numeric'] * 1e3:.2f} ms")
        assert dL <= 1e-12 and dD <= 1e-12
        # the factor reproduces the grounded Laplacian
        N = g.n - 1
        cols = np.repeat(np.arange(N), np.diff(ex["colptr"]))
        L = sp.csc_matrix((Lx, (ex["rowidx"], cols)), shape=(N, N)) + sp.eye(N)
        Ar = laplacian.grounded_sparse(laplacian.laplacian_sparse(g.n, g.eu, g.ev, g.w), g.ground)
        pos = laplacian.reduced_index(g.n, g.ground)[ex["perm"]]
        Ap = Ar[pos][:, pos]
        res = abs(L @ sp.diags(D) @ L.T - Ap).max() / abs(Ap).max()
        assert res < 1e-13
        # resistances from the device-formed factor
        R = np.full(g.m, np.nan)
        P.peers_query_all_edges(f, R)
        Ro = dense.resistances(g, g.eu, g.ev)
        nz = Ro > 0
        assert np.all(R[~nz] == 0.0)
        assert np.max(np.abs(R[nz] - Ro[nz]) / Ro[nz]) <= TOL
        # the same bits on a second device factorization
        h2 = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords, numeric_on_device=True)
        f2 = P.peers_factor_upload(dev, h2)
        L2, D2 = P.peers_graph_export_factor(h2)
        P.peers_factor_release(f2)
        P.peers_graph_destroy(h2)
        assert np.array_equal(L2.view(np.int64), Lx.view(np.int64)) and np.array_equal(D2.view(np.int64), D.view(np.int64))
    finally:
        _close(dev, hh, hd, f)


@pytest.mark.parametrize("cfg,gen", [("C2", synth.pdn_two_layer), ("C3", synth.pdn_multilayer)])
def test_device_factor_full_size(dev, cfg, gen):
    g = gen()
    hd = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords, numeric_on_device=True)
    f = P.peers_factor_upload(dev, hd)
    try:
        st = P.peers_graph_stats_get(hd)
        Lx, D = P.peers_graph_export_factor(hd)
        assert np.all(D > 0) and np.all(Lx <= 0)
        R = np.full(g.m, np.nan)
        P.peers_query_all_edges(f, R)
        with open(os.path.join(GOLDEN, f"{cfg}_edges.json")) as fh:
            d = json.load(fh)
        e = np.array(d["edges"])
        Ro = np.array([float(x) for x in d["R"]])
        err = float(np.max(np.abs(R[e] - Ro) / Ro))
        Rg = np.full(g.n, np.nan)
        P.peers_query_all_to_ground(f, Rg)
        with open(os.path.join(GOLDEN, f"{cfg}_ground.json")) as fh:
            d = json.load(fh)
        nodes = np.array(d["nodes"])
        Rgo = np.array([float(x) for x in d["R"]])
        errg = float(np.max(np.abs(Rg[nodes] - Rgo) / Rgo))
        print(f"{cfg}: device t_numeric {st['t_numeric'] * 1e3:.1f} ms; edges max rel err {err:.2e}, "
              f"node-to-ground {errg:.2e}")
        assert err <= TOL and errg <= TOL
    finally:
        P.peers_factor_release(f)
        P.peers_graph_destroy(hd)


def test_concurrent_uploads_of_one_device_factor_graph(dev):
    # two threads upload the same numeric_on_device graph at once: the uploads
    # run one at a time, the first forms the factor and the second reuses it;
    # both factors give the same bits
    import threading
    g = synth.pdn_multilayer(side=40, layers=3, seed=5)
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords, numeric_on_device=True)
    fs, errs = [None, None], []

    def up(i):
        try:
            fs[i] = P.peers_factor_upload(dev, h)
        except Exception as e:  # reported below
            errs.append(e)

    ts = [threading.Thread(target=up, args=(i,)) for i in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    try:
        assert not errs, errs
        Rs = []
        for f in fs:
            R = np.full(g.m, np.nan)
            P.peers_query_all_edges(f, R)
            Rs.append(R)
        assert np.array_equal(Rs[0].view(np.int64), Rs[1].view(np.int64))
        Ro = dense.resistances(g, g.eu, g.ev)
        assert float(np.max(np.abs(Rs[0] - Ro) / Ro)) <= TOL
        Lx, D = P.peers_graph_export_factor(h)
        assert np.all(D > 0)
    finally:
        for f in fs:
            if f is not None:
                P.peers_factor_release(f)
        P.peers_graph_destroy(h)
