"""The Python binding validates buffers before any pointer reaches the library.

Outputs must be contiguous 1-D float64 of exactly the length the call writes;
node ids are converted to int32 on the host (ids that do not fit are refused)
and must already be contiguous int32 when given as tensors. A wrong buffer
would otherwise be written past its end (device or host memory) or read as
the wrong type. These checks run before the library is called, so a fake
factor handle is enough and no GPU is needed.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2606_31535_amd as P


@pytest.fixture
def fake_factor(monkeypatch):
    h = C.c_void_p(0x1000)
    monkeypatch.setitem(P._FACTOR_EDGES, h.value, 10)

    class NoLib:
        def __getattr__(self, name):
            raise AssertionError(f"the library was called ({name}) with a buffer the binding should refuse")
    monkeypatch.setattr(P, "_lib", NoLib())
    return h


@pytest.mark.parametrize("bad", [
    np.zeros(10, np.float32),            # wrong dtype
    np.zeros(9),                         # short
    np.zeros(11),                        # long
    np.zeros(20)[::2],                   # strided view
    np.zeros((10, 1)),                   # 2-D
    torch.zeros(10, dtype=torch.float32),
    torch.zeros(9, dtype=torch.float64),
    torch.zeros(20, dtype=torch.float64)[::2],
])
def test_all_edge_output_refused(fake_factor, bad):
    with pytest.raises(ValueError):
        P.peers_query_all_edges(fake_factor, bad)


def test_pair_query_checks(fake_factor):
    qu = np.array([0, 1, 2], np.int64)
    qv = np.array([3, 4, 5], np.int64)
    with pytest.raises(ValueError):
        P.peers_query(fake_factor, qu, qv, np.zeros(2))           # short output
    with pytest.raises(ValueError):
        P.peers_query(fake_factor, qu, qv[:2], np.zeros(3))       # qu and qv differ
    with pytest.raises(ValueError):
        P.peers_query(fake_factor, np.array([0, 2**31]), qv[:2], np.zeros(2))  # id beyond int32
    with pytest.raises(ValueError):
        P.peers_query(fake_factor, np.array([0.5, 1.0, 2.0]), qv, np.zeros(3))  # not integers
    with pytest.raises(ValueError):
        P.peers_query(fake_factor, torch.tensor([0, 1, 2]), torch.tensor([3, 4, 5]), np.zeros(3))  # int64 tensors
    with pytest.raises(ValueError):
        P.peers_query(fake_factor, qu, qv, np.zeros(3, np.float32))


def test_id_conversion_keeps_values():
    ptr, dev, keep, n = P._ids(np.array([5, 0, 2**31 - 1], np.int64), "qu")
    assert not dev and n == 3 and keep.dtype == np.int32 and keep.flags.c_contiguous
    assert keep.tolist() == [5, 0, 2**31 - 1]
    ptr, dev, keep, n = P._ids(np.arange(10, dtype=np.int32)[::3], "qu")
    assert keep.flags.c_contiguous and keep.tolist() == [0, 3, 6, 9]


def test_batch_and_server_checks(fake_factor):
    with pytest.raises(ValueError):
        P.peers_batch_query(C.c_void_p(0x2000), [fake_factor], [None], [None], [np.zeros(9)])
    with pytest.raises(ValueError):
        P.peers_batch_query(C.c_void_p(0x2000), [fake_factor], [np.arange(3)], [np.arange(3)], [np.zeros(4)])
    with pytest.raises(ValueError):
        P.peers_server_submit(C.c_void_p(0x3000), fake_factor, np.arange(3), np.arange(3), np.zeros(3, np.float32))
    with pytest.raises(ValueError):
        P.peers_server_submit(C.c_void_p(0x3000), fake_factor, np.arange(3), np.arange(2), np.zeros(3))


def test_unknown_factor_refused(monkeypatch):
    with pytest.raises(ValueError):
        P.peers_query_all_edges(C.c_void_p(0x7777), np.zeros(3))
