"""peers_query_noalloc: the entry point that allocates no device memory.

Two calls in a row, the second with a smaller input, on host and on device
outputs, must give exactly the bits of peers_query on the same pairs (which
the parity tests check against the oracle). The library's device usage does
not move, and a request larger than the fixed scratch array is refused.
"""
import numpy as np
import pytest

import synth
import paper_2606_31535_amd as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup(hip_device):
    d = P.peers_device_open(0)
    g = synth.pdn_multilayer(side=100, layers=4, seed=91, long_frac=0.002)
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords)
    f = P.peers_factor_upload(d, h)
    yield d, g, f
    P.peers_factor_release(f)
    P.peers_graph_destroy(h)
    P.peers_device_close(d)


def _pairs(g, size, seed):
    rng = np.random.default_rng(seed)
    ne = int(0.8 * size)
    e = rng.integers(0, g.m, ne)
    u = np.concatenate([g.eu[e], rng.integers(0, g.n, size - ne), [0, 5]]).astype(np.int32)
    v = np.concatenate([g.ev[e], rng.integers(0, g.n, size - ne), [7, 5]]).astype(np.int32)
    return u, v


def test_noalloc_matches_peers_query_twice(setup):
    import torch
    d, g, f = setup
    cases = []
    for size, seed in ((3000, 1), (400, 2)):   # the second call is smaller
        u, v = _pairs(g, size, seed)
        ref = np.empty(len(u))
        P.peers_query(f, u, v, ref)
        cases.append((u, v, ref))
    torch.cuda.synchronize()
    used0 = P.peers_device_usage(d)[0]
    free0 = None
    for u, v, ref in cases:
        got = np.full(len(u), np.nan)
        P.peers_query_noalloc(f, u, v, got)
        assert np.array_equal(got.view(np.int64), ref.view(np.int64))
        gd = torch.full((len(u),), float("nan"), dtype=torch.float64, device="cuda")
        P.peers_query_noalloc(f, u, v, gd)
        torch.cuda.synchronize()
        assert np.array_equal(gd.cpu().numpy().view(np.int64), ref.view(np.int64))
        del gd
        # nothing reserved by the library
        assert P.peers_device_usage(d)[0] == used0
        # nothing taken from the device after the first call (which brings
        # the fixed scratch array into the device's memory)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        free = torch.cuda.mem_get_info()[0]
        if free0 is None:
            free0 = free
        assert free >= free0 - (4 << 20)


def test_noalloc_all_edges_through_pairs(setup):
    # every edge as a pair: a plan that reads every chain (the unpruned path)
    d, g, f = setup
    R = np.empty(g.m)
    P.peers_query_all_edges(f, R)
    got = np.full(g.m, np.nan)
    P.peers_query_noalloc(f, g.eu.astype(np.int32), g.ev.astype(np.int32), got)
    assert np.array_equal(got.view(np.int64), R.view(np.int64))


def test_noalloc_refuses_oversized_request(setup):
    d, g, f = setup
    rng = np.random.default_rng(9)
    u = rng.integers(0, g.n, 400000).astype(np.int32)
    v = rng.integers(0, g.n, 400000).astype(np.int32)
    with pytest.raises(P.PeersError) as e:
        P.peers_query_noalloc(f, u, v, np.empty(400000))
    assert e.value.status == -7
    # and the entry point still works afterwards
    u, v = _pairs(g, 100, 3)
    ref = np.empty(len(u))
    P.peers_query(f, u, v, ref)
    got = np.empty(len(u))
    P.peers_query_noalloc(f, u, v, got)
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))
