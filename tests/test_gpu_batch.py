"""Batched form: many factors in one captured launch sequence.

Every result must be bit-identical to the same query on the factor alone
(the per-factor path is itself checked against the oracle in
test_gpu_parity.py); one graph of the batch is also checked against the
dense oracle directly.
"""
import numpy as np
import pytest

import synth
import paper_2606_31535_amd as P
from oracle import dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev(hip_device):
    d = P.peers_device_open(0)
    yield d
    P.peers_device_close(d)


@pytest.fixture(scope="module")
def batch(dev):
    # graphs of uneven size and shape: random geometric graphs (the batched
    # workload's family) and two small PDN meshes
    graphs = [synth.rgg_knn(n, seed=40000 + i) for i, n in enumerate([2000, 3500, 2600, 5200, 2100, 4100])]
    graphs += [synth.pdn_multilayer(side=40, layers=3, seed=5), synth.mesh2d(30, 17, seed=8)]
    hs, fs = [], []
    for g in graphs:
        h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords)
        hs.append(h)
        fs.append(P.peers_factor_upload(dev, h))
    yield graphs, fs
    for f in fs:
        P.peers_factor_release(f)
    for h in hs:
        P.peers_graph_destroy(h)


def _bits(x):
    return np.asarray(x).view(np.int64)


def test_all_edge_batch_matches_single_calls(dev, batch):
    graphs, fs = batch
    alone = []
    for g, f in zip(graphs, fs):
        R = np.full(g.m, np.nan)
        P.peers_query_all_edges(f, R)
        alone.append(R)
    outs = [np.full(g.m, np.nan) for g in graphs]
    P.peers_batch_query(dev, fs, [None] * len(fs), [None] * len(fs), outs)
    info = P.peers_batch_last_info(dev)
    print("batch info", info)
    assert info["factors"] == len(fs) and info["graph_reused"] == 0
    assert 0 <= info["schedule"] < info["candidates"]
    assert all(t > 0 for t in info["candidate_ms"])
    for a, b in zip(alone, outs):
        assert np.array_equal(_bits(a), _bits(b))
    # the second call replays the captured graph
    outs2 = [np.full(g.m, np.nan) for g in graphs]
    P.peers_batch_query(dev, fs, [None] * len(fs), [None] * len(fs), outs2)
    # host outputs go through each factor's result buffer, so the key is the same
    assert P.peers_batch_last_info(dev)["graph_reused"] == 1
    for a, b in zip(alone, outs2):
        assert np.array_equal(_bits(a), _bits(b))
    g = graphs[-1]
    Ro = dense.resistances(g, g.eu, g.ev)
    assert float(np.max(np.abs(outs[-1] - Ro) / Ro)) <= 1e-10


def test_device_outputs_and_replay(dev, batch):
    import torch
    graphs, fs = batch
    outs = [torch.empty(g.m, dtype=torch.float64, device="cuda") for g in graphs]
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        P.peers_batch_query(dev, fs, [None] * len(fs), [None] * len(fs), outs, flags=P.PEERS_SYNC)
        torch.cuda.synchronize()
        assert P.peers_batch_last_info(dev)["graph_reused"] == (1 if rep else 0)
        for g, f, o in zip(graphs, fs, outs):
            R = np.full(g.m, np.nan)
            P.peers_query_all_edges(f, R)
            assert np.array_equal(_bits(R), _bits(o.cpu().numpy()))


def test_mixed_pairs_and_edges(dev, batch):
    graphs, fs = batch
    qus, qvs, outs, alone = [], [], [], []
    for i, (g, f) in enumerate(zip(graphs, fs)):
        if i % 2:
            qus.append(None)
            qvs.append(None)
            outs.append(np.full(g.m, np.nan))
            R = np.full(g.m, np.nan)
            P.peers_query_all_edges(f, R)
        else:
            rng = synth.rng_for(500 + i)
            k = 300 + 50 * i
            u = rng.integers(0, g.n, k).astype(np.int32)
            v = rng.integers(0, g.n, k).astype(np.int32)
            v[:5] = g.ground
            v[5:8] = u[5:8]
            qus.append(u)
            qvs.append(v)
            outs.append(np.full(k, np.nan))
            R = np.full(k, np.nan)
            P.peers_query(f, u, v, R)
        alone.append(R)
    P.peers_batch_query(dev, fs, qus, qvs, outs)
    for a, b in zip(alone, outs):
        assert np.array_equal(_bits(a), _bits(b))
    g = graphs[0]
    Ro = dense.resistances(g, qus[0], qvs[0])
    nz = Ro > 0
    assert np.all(outs[0][~nz] == 0)
    assert float(np.max(np.abs(outs[0][nz] - Ro[nz]) / Ro[nz])) <= 1e-10


def test_batch_errors(dev, batch):
    graphs, fs = batch
    with pytest.raises(P.PeersError) as ei:
        P.peers_batch_query(dev, [fs[0], fs[0]], [None, None], [None, None],
                            [np.zeros(graphs[0].m), np.zeros(graphs[0].m)])
    assert ei.value.status == -1
    with pytest.raises(P.PeersError) as ei:
        P.peers_batch_query(dev, [fs[1]], [np.array([0, graphs[1].n], np.int32)], [np.array([1, 2], np.int32)],
                            [np.zeros(2)])
    assert ei.value.status == -2


def test_batch_with_wide_store_factor(dev, batch):
    # one factor with 64-bit store offsets switches the group's bottom step to
    # the 64-bit form; every factor must still give its single-call bits
    graphs, fs = batch
    g = synth.pdn_multilayer(side=24, layers=3, seed=31)
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords, store_offsets_64=True)
    f = P.peers_factor_upload(dev, h)
    try:
        gs = graphs[:3] + [g]
        sub = fs[:3] + [f]
        alone = []
        for x, fx in zip(gs, sub):
            R = np.full(x.m, np.nan)
            P.peers_query_all_edges(fx, R)
            alone.append(R)
        outs = [np.full(x.m, np.nan) for x in gs]
        P.peers_batch_query(dev, sub, [None] * len(sub), [None] * len(sub), outs)
        for a, b in zip(alone, outs):
            assert np.array_equal(_bits(a), _bits(b))
        Ro = dense.resistances(g, g.eu, g.ev)
        assert float(np.max(np.abs(outs[-1] - Ro) / Ro)) <= 1e-10
    finally:
        P.peers_factor_release(f)
        P.peers_graph_destroy(h)


def test_schedule_memo_by_structure(dev, batch):
    # other factor handles of the same graphs (a fresh upload of each) have the
    # batch's structure signature: the new batch takes the remembered schedule
    # without timing, and still gives every factor's single-call bits
    graphs, fs = batch
    outs = [np.full(g.m, np.nan) for g in graphs]
    P.peers_batch_query(dev, fs, [None] * len(fs), [None] * len(fs), outs)
    first = P.peers_batch_last_info(dev)
    hs, fs2 = [], []
    try:
        for g in graphs:
            h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords)
            hs.append(h)
            fs2.append(P.peers_factor_upload(dev, h))
        outs2 = [np.full(g.m, np.nan) for g in graphs]
        P.peers_batch_query(dev, fs2, [None] * len(fs2), [None] * len(fs2), outs2)
        info = P.peers_batch_last_info(dev)
        print("memo", first["signature"], info["signature"], info["schedule_name"])
        assert info["graph_reused"] == 0 and info["schedule_cached"] == 1
        assert info["signature"] == first["signature"] and info["schedule"] == first["schedule"]
        for f, g, o in zip(fs2, graphs, outs2):
            R = np.full(g.m, np.nan)
            P.peers_query_all_edges(f, R)
            assert np.array_equal(_bits(R), _bits(o))
        # a batch of another structure is timed
        outs3 = [np.full(g.m, np.nan) for g in graphs[:3]]
        P.peers_batch_query(dev, fs2[:3], [None] * 3, [None] * 3, outs3)
        info3 = P.peers_batch_last_info(dev)
        assert info3["signature"] != first["signature"] and info3["schedule_cached"] == 0
    finally:
        for f in fs2:
            P.peers_factor_release(f)
        for h in hs:
            P.peers_graph_destroy(h)
