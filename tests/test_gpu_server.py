"""Served form: continuous batching over resident factors.

Each request's result must be the same bits as the same pairs run alone
through peers_query (itself checked against the oracle in
test_gpu_parity.py), whatever other requests share its batches.
"""
import threading

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
def factors(dev):
    graphs = [synth.pdn_multilayer(side=s, layers=4, seed=1002 + s) for s in (24, 40, 64)]
    graphs.append(synth.rgg_knn(3000, seed=40007))
    graphs.append(synth.mesh2d(20, 20, seed=3))
    hs = [P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords) for g in graphs]
    fs = [P.peers_factor_upload(dev, h) for h in hs]
    yield graphs, fs
    for f in fs:
        P.peers_factor_release(f)
    for h in hs:
        P.peers_graph_destroy(h)


def _requests(graphs, count, seed):
    rng = synth.rng_for(seed)
    out = []
    for k in range(count):
        gi = int(rng.integers(0, len(graphs)))
        g = graphs[gi]
        size = int(min(3000, np.floor(np.exp(rng.uniform(0, np.log(3001))))))
        ne = int(round(0.8 * size))
        e = rng.integers(0, g.m, ne)
        u = np.concatenate([g.eu[e], rng.integers(0, g.n, size - ne)]).astype(np.int32)
        v = np.concatenate([g.ev[e], rng.integers(0, g.n, size - ne)]).astype(np.int32)
        out.append((gi, u, v))
    return out


def test_results_same_alone_and_in_the_mix(dev, factors):
    graphs, fs = factors
    reqs = _requests(graphs, 120, seed=901)
    alone = []
    for gi, u, v in reqs:
        R = np.full(len(u), np.nan)
        P.peers_query(fs[gi], u, v, R)
        alone.append(R)
    srv = P.peers_server_start(dev, max_batch_pairs=20000, max_wait_us=300, streams=2)
    outs = [np.full(len(u), np.nan) for _, u, _ in reqs]
    tickets = [None] * len(reqs)
    keep = []

    def submit(idx):
        for i in idx:
            gi, u, v = reqs[i]
            t, k = P.peers_server_submit(srv, fs[gi], u, v, outs[i])
            tickets[i] = t
            keep.append(k)

    th = [threading.Thread(target=submit, args=(range(j, len(reqs), 2),)) for j in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for t in tickets:
        st, res = P.peers_server_wait(srv, t, -1)
        assert st == 0 and res == 0
    stats = P.peers_server_stats_get(srv)
    P.peers_server_stop(srv)
    print("server stats", stats)
    assert stats["completed"] == len(reqs) and stats["rejected"] == 0
    assert 1 <= stats["batches"] < len(reqs)  # requests were batched together
    assert 0 < stats["p50_us"] <= stats["p99_us"] <= stats["max_us"]
    for a, b in zip(alone, outs):
        assert np.array_equal(a.view(np.int64), b.view(np.int64))
    # one request checked against the dense oracle directly
    i = next(k for k, r in enumerate(reqs) if r[0] == 4)
    gi, u, v = reqs[i]
    Ro = dense.resistances(graphs[gi], u, v)
    nz = Ro > 0
    assert np.all(outs[i][~nz] == 0)
    assert float(np.max(np.abs(outs[i][nz] - Ro[nz]) / Ro[nz])) <= 1e-10


def test_server_errors_and_stop_drains(dev, factors):
    graphs, fs = factors
    srv = P.peers_server_start(dev)
    g = graphs[0]
    with pytest.raises(P.PeersError) as ei:
        P.peers_server_submit(srv, fs[0], np.array([0, g.n], np.int32), np.array([1, 1], np.int32), np.zeros(2))
    assert ei.value.status == -2
    st, _ = P.peers_server_wait(srv, 987654321, 0)
    assert st == -1
    # stop() finishes what was submitted
    outs, ts, keep = [], [], []
    for k in range(10):
        u = g.eu[k * 10:(k + 1) * 10].astype(np.int32)
        v = g.ev[k * 10:(k + 1) * 10].astype(np.int32)
        outs.append(np.full(10, np.nan))
        t, kk = P.peers_server_submit(srv, fs[0], u, v, outs[-1])
        ts.append(t)
        keep.append(kk)
    P.peers_server_stop(srv)
    R = np.full(g.m, np.nan)
    P.peers_query_all_edges(fs[0], R)
    for k in range(10):
        assert np.array_equal(outs[k].view(np.int64), R[k * 10:(k + 1) * 10].view(np.int64))


def _big_request(g, size, seed):
    rng = synth.rng_for(seed)
    ne = int(0.8 * size)
    e = rng.integers(0, g.m, ne)
    u = np.concatenate([g.eu[e], rng.integers(0, g.n, size - ne)]).astype(np.int32)
    v = np.concatenate([g.ev[e], rng.integers(0, g.n, size - ne)]).astype(np.int32)
    return u, v


def test_hot_factor_in_overlapping_batches(dev, factors):
    # every request on one factor: batches of the same factor run on both
    # streams at once and must still give each request its lone result
    graphs, fs = factors
    g, f = graphs[2], fs[2]
    reqs = [_big_request(g, 4000, 300 + k) for k in range(24)]
    alone = []
    for u, v in reqs:
        R = np.empty(len(u))
        P.peers_query(f, u, v, R)
        alone.append(R)
    srv = P.peers_server_start(dev, max_batch_pairs=4000, max_wait_us=50, streams=2)
    outs = [np.full(len(u), np.nan) for u, _ in reqs]
    keep, tickets = [], []
    for (u, v), o in zip(reqs, outs):
        t, k = P.peers_server_submit(srv, f, u, v, o)
        tickets.append(t)
        keep.append(k)
    for t in tickets:
        st, res = P.peers_server_wait(srv, t, -1)
        assert st == 0 and res == 0
    stats = P.peers_server_stats_get(srv)
    P.peers_server_stop(srv)
    assert stats["batches"] >= 12
    for a, b in zip(alone, outs):
        assert np.array_equal(a.view(np.int64), b.view(np.int64))


def test_busy_when_queue_full(dev, factors):
    graphs, fs = factors
    g, f = graphs[2], fs[2]
    srv = P.peers_server_start(dev, max_batch_pairs=50000, queue_capacity=1, streams=1)
    u, v = _big_request(g, 50000, 17)
    outs, tickets, busy = [], [], 0
    try:
        for k in range(200):
            o = np.full(len(u), np.nan)
            try:
                t, _ = P.peers_server_submit(srv, f, u, v, o)
            except P.PeersError as e:
                assert e.status == -9  # BUSY
                busy += 1
                continue
            outs.append(o)
            tickets.append(t)
        assert busy > 0, "a queue of one request never overflowed"
        for t in tickets:
            st, res = P.peers_server_wait(srv, t, -1)
            assert st == 0 and res == 0
        stats = P.peers_server_stats_get(srv)
        assert stats["rejected"] == busy
    finally:
        P.peers_server_stop(srv)
    R = np.empty(len(u))
    P.peers_query(f, u, v, R)
    for o in outs:
        assert np.array_equal(o.view(np.int64), R.view(np.int64))


def test_timeout_and_cancel(dev, factors):
    graphs, fs = factors
    g, f = graphs[2], fs[2]
    srv = P.peers_server_start(dev, max_batch_pairs=60000, streams=1)
    reqs = [_big_request(g, 60000, 40 + k) for k in range(6)]
    outs = [np.full(60000, np.nan) for _ in reqs]
    keep, tickets = [], []
    for (u, v), o in zip(reqs, outs):
        t, k = P.peers_server_submit(srv, f, u, v, o)
        tickets.append(t)
        keep.append(k)
    # the last request is behind five others on one stream: not finished
    st, _ = P.peers_server_wait(srv, tickets[-1], 0)
    assert st == -11  # TIMEOUT, the request stays live
    P.peers_server_cancel(srv, tickets[-1])
    st, res = P.peers_server_wait(srv, tickets[-1], -1)
    assert st == 0 and res in (-10, 0)
    if res == -10:
        assert np.all(np.isnan(outs[-1])), "a cancelled request's output was written"
    for t in tickets[:-1]:
        st, res = P.peers_server_wait(srv, t, -1)
        assert st == 0 and res == 0
    with pytest.raises(P.PeersError):
        P.peers_server_cancel(srv, 123456789)
    P.peers_server_stop(srv)
    R = np.empty(60000)
    u, v = reqs[0]
    P.peers_query(f, u, v, R)
    assert np.array_equal(outs[0].view(np.int64), R.view(np.int64))


def test_over_budget_upload_leaves_nothing(hip_device):
    g = synth.pdn_multilayer(side=40, layers=4, seed=77)
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords)
    d = P.peers_device_open(0, 1 << 20)
    try:
        with pytest.raises(P.PeersError) as e:
            P.peers_factor_upload(d, h)
        assert e.value.status == -7
        assert P.peers_device_usage(d)[0] == 0
    finally:
        P.peers_device_close(d)
        P.peers_graph_destroy(h)


def test_request_too_large_for_idle_device_and_queued_admission(hip_device):
    g = synth.pdn_multilayer(side=64, layers=4, seed=78)
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords)
    reqs = [_big_request(g, 100000, 500 + k) for k in range(6)]
    # arena of one such batch, measured on an unconstrained device
    d0 = P.peers_device_open(0)
    f0 = P.peers_factor_upload(d0, h)
    srv = P.peers_server_start(d0, max_batch_pairs=100000, streams=1)
    o = np.empty(100000)
    t, k = P.peers_server_submit(srv, f0, reqs[0][0], reqs[0][1], o)
    assert P.peers_server_wait(srv, t, -1) == (0, 0)
    arena = P.peers_server_stats_get(srv)["arena_bytes"]
    P.peers_server_stop(srv)
    alone = []
    for u, v in reqs:
        R = np.empty(len(u))
        P.peers_query(f0, u, v, R)
        alone.append(R)
    P.peers_factor_release(f0)
    P.peers_device_close(d0)
    assert arena > (1 << 20)
    try:
        # a budget that holds the factor and one batch arena but not two
        d = P.peers_device_open(0)
        f = P.peers_factor_upload(d, h)
        base = P.peers_device_usage(d)[0]
        P.peers_device_set_budget(d, base + arena + arena // 2)
        srv = P.peers_server_start(d, max_batch_pairs=100000, streams=2)
        outs = [np.full(100000, np.nan) for _ in reqs]
        keep, tickets = [], []
        for (u, v), o in zip(reqs, outs):
            t, k = P.peers_server_submit(srv, f, u, v, o)
            tickets.append(t)
            keep.append(k)
        for t in tickets:
            assert P.peers_server_wait(srv, t, -1) == (0, 0)  # queued, never refused
        stats = P.peers_server_stats_get(srv)
        print("queued admission", stats)
        assert stats["memory_waits"] >= 1 and stats["rejected"] == 0
        for a, b in zip(alone, outs):
            assert np.array_equal(a.view(np.int64), b.view(np.int64))
        P.peers_server_stop(srv)
        assert P.peers_device_usage(d)[0] == base  # the arenas went back to the budget
        # a budget with no room for even one arena: the request fails alone,
        # and nothing stays reserved
        P.peers_device_set_budget(d, base + (1 << 16))
        with pytest.raises(P.PeersError) as e:
            P.peers_device_set_budget(d, base - 1)
        assert e.value.status == -7
        srv = P.peers_server_start(d, streams=2)
        o = np.full(100000, np.nan)
        t, k = P.peers_server_submit(srv, f, reqs[1][0], reqs[1][1], o)
        assert P.peers_server_wait(srv, t, -1) == (0, -7)
        assert np.all(np.isnan(o))
        P.peers_server_stop(srv)
        assert P.peers_device_usage(d)[0] == base
        P.peers_factor_release(f)
        P.peers_device_close(d)
    finally:
        P.peers_graph_destroy(h)
