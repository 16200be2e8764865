"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each case swaps one oracle routine for a plausibly wrong variant and checks
that at least one of the closed-form or exact pins then fails. This shows the
pins constrain the oracle, rather than merely agreeing with it.
"""
import numpy as np
import pytest

import synth
from oracle import dense, laplacian, exact


def _pins_hold():
    """A compact subset of the pins in test_oracle_pins; True iff all hold."""
    ok = True
    g = synth.random_tree(30, seed=2, wlog=2.0, ground=4)
    R = dense.resistances(g, g.eu, g.ev)
    ok &= bool(np.max(np.abs(R * g.w - 1.0)) < 1e-12)
    g = synth.complete_graph(9, ground=8)
    R = dense.resistances(g, g.eu, g.ev)
    ok &= bool(np.max(np.abs(R - 2.0 / 9)) < 1e-12)
    g = synth.cycle_graph(11, ground=0)
    R = dense.resistances(g, np.zeros(11, np.int32), np.arange(11, dtype=np.int32))
    ok &= bool(np.max(np.abs(R - np.array([k * (11 - k) / 11 for k in range(11)]))) < 1e-12)
    g = synth.random_connected(9, extra=8, seed=3, dyadic=True, ground=5)
    qu, qv = np.array([0, 2, 7, 5]), np.array([3, 8, 1, 6])
    R = dense.resistances(g, qu, qv)
    ex = [exact.to_float(exact.resistance_cramer(g, int(a), int(b))) for a, b in zip(qu, qv)]
    ok &= bool(np.max(np.abs(R - ex) / np.array(ex)) < 1e-12)
    return ok


def test_unmutated_oracle_passes():
    assert _pins_hold()


def _bad_lap_sign(n, eu, ev, w, dtype=np.float64):
    L = np.zeros((n, n), dtype=dtype)
    for a, b, x in zip(eu.tolist(), ev.tolist(), w.tolist()):
        if a == b:
            continue
        L[a, a] += x
        L[b, b] += x
        L[a, b] += x      # wrong sign
        L[b, a] += x
    return L


def _bad_lap_one_endpoint(n, eu, ev, w, dtype=np.float64):
    L = np.zeros((n, n), dtype=dtype)
    for a, b, x in zip(eu.tolist(), ev.tolist(), w.tolist()):
        if a == b:
            continue
        L[a, a] += x      # dropped term: L[b, b] += x
        L[a, b] -= x
        L[b, a] -= x
    return L + np.eye(n) * 1e-3


def _bad_incidence_plus(n, g, qu, qv):
    r = laplacian.reduced_index(n, g)
    B = np.zeros((n - 1, len(qu)))
    for k, (a, b) in enumerate(zip(np.asarray(qu).tolist(), np.asarray(qv).tolist())):
        if a == b:
            continue
        if r[a] >= 0:
            B[r[a], k] += 1.0
        if r[b] >= 0:
            B[r[b], k] += 1.0  # e_u + e_v instead of e_u - e_v
    return B


def _bad_reduced_index(n, g):
    r = np.arange(n, dtype=np.int64)
    r[g] = -1                     # forgot to shift the ids above the ground down by one
    return np.minimum(r, n - 2)


def _bad_grounded_dense(L, g):
    keep = np.arange(1, L.shape[0])  # always drops node 0, whatever the ground
    return L[np.ix_(keep, keep)]


@pytest.mark.parametrize("target,attr,bad", [
    (dense, "laplacian_dense", _bad_lap_sign),
    (dense, "laplacian_dense", _bad_lap_one_endpoint),
    (dense, "incidence_columns", _bad_incidence_plus),
    (laplacian, "reduced_index", _bad_reduced_index),
    (dense, "grounded_dense", _bad_grounded_dense),
])
def test_planted_mistake_is_caught(monkeypatch, target, attr, bad):
    monkeypatch.setattr(target, attr, bad)
    try:
        held = _pins_hold()
    except Exception:
        held = False  # a crash also counts as caught
    assert not held
