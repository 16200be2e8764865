"""Pins for the oracle's spectral sparsifier (Section II-B, Algorithm 1).

* The counter-based generator is compared word for word with numpy's own
  Philox bit generator (numpy.random.Philox, the same 4x64, 10-round
  function): numpy increments its counter before each block, so its k-th
  block of four words is Philox at counter k + 1.
* The 128-bit product and the interval search are compared with Python's
  exact integers and a linear scan on small inputs.
* Closed form: when every edge has the same integer weight, draw i lands on
  edge floor(x_i m / 2^64) exactly.
* The draws follow p_e (a chi-square bound over many draws), the new weights
  are unbiased, and the sparsifier keeps the Laplacian quadratic form
  (the property Algorithm 1 exists for).
Planted mistakes in each step must fail one of these.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dense, sparsify


@pytest.mark.parametrize("key,start", [((0, 0), 0), ((5, 7), 0), ((2**64 - 1, 12345), 999), ((123456789, 0), 2**40)])
def test_philox_matches_numpy(key, start):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array([start, 0, 0, 0], dtype=np.uint64))
    raw = bg.random_raw(4 * 16).reshape(16, 4)
    for b in range(16):
        assert sparsify.philox4x64_10([start + b + 1, 0, 0, 0], key) == [int(x) for x in raw[b]]
    many = sparsify.philox4x64_10_many(np.arange(start + 1, start + 17, dtype=np.uint64), key)
    for w in range(4):
        assert np.array_equal(many[w], raw[:, w])


def test_mulhi_exact():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2**63, 1000, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 1000, dtype=np.uint64)
    b = rng.integers(1, 2**62, 1000, dtype=np.uint64)
    with np.errstate(over="ignore"):
        hi, lo = sparsify._mulhilo(a, b)
    for x, y, h, l in zip(a.tolist(), b.tolist(), hi.tolist(), lo.tolist()):
        assert h == (x * y) >> 64 and l == (x * y) & ((1 << 64) - 1)


def test_draws_linear_scan_small():
    rng = np.random.default_rng(2)
    # the last case has integer weights 1, 1, 2 (K = 4): draws land on
    # interval boundaries all the time
    tiny = (np.ones(3), np.ldexp(np.array([1.0, 1.0, 2.0]), -sparsify.scale_bits(3)))
    for m in (1, 2, 3, 7, "tiny"):
        if m == "tiny":
            w, R = tiny
            m = 3
        else:
            w = rng.uniform(0.5, 2, m)
            R = rng.uniform(0.05, 0.5, m) / w * rng.uniform(0.2, 1, m)
        k = sparsify.integer_weights(w, R)
        C = np.cumsum(k, dtype=np.uint64)
        K = int(C[-1])
        e = sparsify.draws(300, 77, K, C)
        for i in range(300):
            x = sparsify.philox4x64_10([i, 0, 0, 0], (77, 0))[0]
            t = (x * K) >> 64
            acc, pick = 0, None
            for j in range(m):
                acc += int(k[j])
                if t < acc:
                    pick = j
                    break
            assert e[i] == pick


def test_uniform_weights_closed_form():
    # w_e R_e = 1 exactly for every edge (powers of two): all k_e = 2^s
    m = 1000
    w = np.ldexp(1.0, np.arange(m) % 7 - 3)
    R = 1.0 / w
    k = sparsify.integer_weights(w, R)
    assert np.all(k == k[0]) and int(k[0]) == 1 << sparsify.scale_bits(m)
    C = np.cumsum(k, dtype=np.uint64)
    e = sparsify.draws(5000, 4242, int(C[-1]), C)
    for i in range(0, 5000, 97):
        x = sparsify.philox4x64_10([i, 0, 0, 0], (4242, 0))[0]
        assert e[i] == (x * m) >> 64


def _small_graph_with_R():
    g = synth.random_connected(60, extra=120, seed=8, wlog=1.0, ground=0)
    R = dense.resistances(g, g.eu, g.ev)
    return g, R


def test_draw_frequencies_follow_w_times_R():
    g, R = _small_graph_with_R()
    q = 200000
    counts, _ = sparsify.sparsify(g.w, R, q, 9)
    p = g.w * R / np.sum(g.w * R)
    expect = q * p
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    dof = g.m - 1
    # far beyond chance for a wrong distribution, comfortably met by the right one
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)
    assert counts.sum() == q


def test_new_weights_unbiased_and_exact_formula():
    g, R = _small_graph_with_R()
    q = 3000
    acc = np.zeros(g.m)
    for seed in range(40):
        counts, neww = sparsify.sparsify(g.w, R, q, seed)
        k = sparsify.integer_weights(g.w, R).astype(np.float64)
        K = float(np.sum(sparsify.integer_weights(g.w, R), dtype=np.uint64))
        want = counts * g.w * (K / (q * k))
        assert np.array_equal(neww[counts > 0], want[counts > 0]) and np.all(neww[counts == 0] == 0)
        acc += neww
    # E[new weight] = w_e: over 40 seeds the mean is within a few standard errors
    rel = np.abs(acc / 40 - g.w) / g.w
    assert np.median(rel) < 0.25


def test_sparsifier_keeps_quadratic_form():
    g = synth.random_connected(80, extra=800, seed=10, wlog=0.5, ground=0)
    R = dense.resistances(g, g.eu, g.ev)
    q = 8000
    counts, neww = sparsify.sparsify(g.w, R, q, 3)
    keep = counts > 0
    assert keep.sum() < g.m  # fewer edges than the graph
    rng = np.random.default_rng(4)
    for _ in range(20):
        x = rng.standard_normal(g.n)
        a = sparsify.laplacian_quadratic(g.n, g.eu, g.ev, g.w, x)
        b = sparsify.laplacian_quadratic(g.n, g.eu[keep], g.ev[keep], neww[keep], x)
        assert abs(b / a - 1) < 0.3


def test_invalid_inputs_refused():
    with pytest.raises(ValueError):
        sparsify.integer_weights(np.ones(3), np.array([0.5, -0.1, 0.2]))
    with pytest.raises(ValueError):
        sparsify.integer_weights(np.ones(3), np.array([0.5, np.nan, 0.2]))
    with pytest.raises(ValueError):
        sparsify.sparsify(np.ones(3), np.zeros(3), 10, 1)


# --------------------------------------------------------------- planted mistakes

def _philox_no_key_bump(counter, key):
    c = [int(x) for x in counter]
    k = [int(x) for x in key]
    M = sparsify.M64
    for r in range(10):
        p0 = sparsify.PHILOX_M0 * c[0]
        p1 = sparsify.PHILOX_M1 * c[2]
        c = [((p1 >> 64) ^ c[1] ^ k[0]) & M, p1 & M, ((p0 >> 64) ^ c[3] ^ k[1]) & M, p0 & M]
    return c


def _philox_swapped_multipliers(counter, key):
    c = [int(x) for x in counter]
    k = [int(x) for x in key]
    M = sparsify.M64
    for r in range(10):
        if r:
            k = [(k[0] + sparsify.PHILOX_W0) & M, (k[1] + sparsify.PHILOX_W1) & M]
        p0 = sparsify.PHILOX_M1 * c[0]
        p1 = sparsify.PHILOX_M0 * c[2]
        c = [((p1 >> 64) ^ c[1] ^ k[0]) & M, p1 & M, ((p0 >> 64) ^ c[3] ^ k[1]) & M, p0 & M]
    return c


def _draws_left(q, seed, K, C, chunk=1 << 20):
    x = sparsify.philox4x64_10_many(np.arange(q, dtype=np.uint64), (seed, 0))[0]
    with np.errstate(over="ignore"):
        t, _ = sparsify._mulhilo(x, np.uint64(K))
    return np.searchsorted(C, t, side="left")


def _weights_without_w(w, R):
    return sparsify.np.floor(np.ldexp(np.asarray(R, dtype=np.float64), sparsify.scale_bits(len(R)))).astype(np.uint64)


@pytest.mark.parametrize("attr,bad,test", [
    ("philox4x64_10", _philox_no_key_bump, test_philox_matches_numpy),
    ("philox4x64_10", _philox_swapped_multipliers, test_philox_matches_numpy),
    ("draws", _draws_left, test_draws_linear_scan_small),
    ("integer_weights", _weights_without_w, test_draw_frequencies_follow_w_times_R),
])
def test_planted_sparsifier_mistake_is_caught(monkeypatch, attr, bad, test):
    monkeypatch.setattr(sparsify, attr, bad)
    with pytest.raises(AssertionError):
        if test is test_philox_matches_numpy:
            test((5, 7), 0)
        else:
            test()
