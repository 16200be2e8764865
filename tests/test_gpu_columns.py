"""The sweep's intermediate values on the GPU: columns of Z = D^{-1/2} L^{-1}.

The sweep never stores Z; for checking, ``peers_factor_export_columns`` runs
a sweep that keeps the requested columns (top-store columns, and staged
bottom-subtree columns) and copies them out depth-indexed. They are compared
entry by entry with the oracle's dense triangular inverse of the library's
own exported factor (the factor enters as data), which isolates the sweep's
error from the factor's (Lemma 3: the implicit rows equal triangular
substitution). Every term of the recurrence is nonnegative for a grounded
Laplacian, so each entry carries a small relative error; the bound used is
1e-12 per entry, with exact zeros past each column's depth.
"""
import numpy as np
import pytest

import synth
import paper_2606_31535_amd as P
from oracle import factor

pytestmark = pytest.mark.gpu
RTOL = 1e-12


@pytest.fixture(scope="module")
def dev(hip_device):
    d = P.peers_device_open(0)
    yield d
    P.peers_device_close(d)


def _check_columns(dev, g, nodes=None):
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords)
    try:
        st = P.peers_graph_stats_get(h)
        ex = P.peers_graph_export_symbolic(h)
        Lx, D = P.peers_graph_export_factor(h)
        f = P.peers_factor_upload(dev, h)
        try:
            N = g.n - 1
            pos = np.full(g.n, -1)
            pos[ex["perm"]] = np.arange(N)
            if nodes is None:
                nodes = np.array([x for x in range(g.n) if x != g.ground], dtype=np.int32)
            h_ld = st["height"] + 5
            Zg = P.peers_factor_export_columns(f, nodes, h_ld)
        finally:
            P.peers_factor_release(f)
    finally:
        P.peers_graph_destroy(h)
    L = factor.unit_lower(N, ex["colptr"], ex["rowidx"], Lx)
    Z = factor.implicit_columns(L, D)
    zc = factor.depth_columns(Z, ex["parent"], pos[nodes])
    ref = np.zeros_like(Zg)
    ref[:, :zc.shape[1]] = zc
    assert np.all((Zg == 0) == (ref == 0)), "support differs"
    nz = ref != 0
    err = float(np.max(np.abs(Zg[nz] - ref[nz]) / np.abs(ref[nz])))
    print(f"{g.name}: {len(nodes)} columns, height {st['height']}, max entry rel err {err:.3e}")
    assert err <= RTOL
    return err


def test_mesh_every_column(dev):
    _check_columns(dev, synth.mesh2d())


def test_random_graph_every_column(dev):
    # tall elimination tree: most nodes are top-tree (chain) nodes
    _check_columns(dev, synth.random_connected(1500, 3000, seed=4, wlog=2.0, ground=3))


def test_pdn_selected_columns(dev):
    g = synth.pdn_multilayer(side=20, layers=4, seed=9, long_frac=0.005)
    rng = np.random.default_rng(5)
    nodes = rng.choice(np.arange(1, g.n, dtype=np.int32), size=300, replace=False)
    _check_columns(dev, g, nodes)


def test_export_errors(dev):
    g = synth.mesh2d(8, 8)
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords)
    f = P.peers_factor_upload(dev, h)
    try:
        hgt = P.peers_graph_stats_get(h)["height"]
        with pytest.raises(P.PeersError) as e:
            P.peers_factor_export_columns(f, [g.ground], hgt)
        assert e.value.status == -1
        with pytest.raises(P.PeersError) as e:
            P.peers_factor_export_columns(f, [g.n], hgt)
        assert e.value.status == -2
        with pytest.raises(P.PeersError) as e:
            P.peers_factor_export_columns(f, [1], hgt - 1)
        assert e.value.status == -1
    finally:
        P.peers_factor_release(f)
        P.peers_graph_destroy(h)
