"""Spectral sparsification by effective resistances (Section II-B, Algorithm 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 1 draws q edges, each independently with probability p_e
proportional to w_e R_e, and gives every drawn edge the weight w_e / (q p_e)
(an edge drawn c times gets c times that weight). Readings taken here, where
the paper leaves the procedure open:

* Probabilities are realized as integer weights, so that the cumulative
  distribution is exact whatever order a prefix sum runs in:
  k_e = floor(2^s * fl(w_e * R_e)) with s = 61 - ceil(log2 m). For a
  Laplacian 0 < w_e R_e <= 1 (Foster), so sum k_e < 2^62; inputs with
  w_e R_e outside [0, 2] or not finite are refused. p_e = k_e / K with
  K = sum k_e, which differs from w_e R_e / sum(w R) by at most 2^-s per edge.
* Draw i (i = 0 .. q-1) takes x, the first 64-bit output word of the
  counter-based generator Philox4x64-10 (Salmon, Moraes, Dror and Shaw,
  "Parallel random numbers: as easy as 1, 2, 3", SC 2011) at counter
  (i, 0, 0, 0) and key (seed, 0). It picks the edge e whose interval
  [C_{e-1}, C_e) of the inclusive prefix sums C of k holds t = floor(x K / 2^64).
* Outputs per edge: count_e (draws of e) and the new weight
  count_e * w_e * (K / (q k_e)) in FP64, evaluated in that order; 0 for an
  edge never drawn.
"""
from __future__ import annotations

import math

import numpy as np

M64 = (1 << 64) - 1
# Philox4x64 round multipliers and key increments (Salmon et al. 2011)
PHILOX_M0, PHILOX_M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
PHILOX_W0, PHILOX_W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B


def philox4x64_10(counter, key):
    """Four 64-bit output words for a 4-word counter and 2-word key (Python ints)."""
    c = [int(x) & M64 for x in counter]
    k = [int(x) & M64 for x in key]
    for r in range(10):
        if r:
            k = [(k[0] + PHILOX_W0) & M64, (k[1] + PHILOX_W1) & M64]
        p0 = PHILOX_M0 * c[0]
        p1 = PHILOX_M1 * c[2]
        c = [((p1 >> 64) ^ c[1] ^ k[0]) & M64, p1 & M64, ((p0 >> 64) ^ c[3] ^ k[1]) & M64, p0 & M64]
    return c


def _mulhilo(a, b):
    """High and low 64-bit words of a * b for uint64 arrays (b may be a scalar)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a0, a1 = a & m32, a >> s32
    b0, b1 = b & m32, b >> s32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> s32) + (p01 & m32) + (p10 & m32)
    hi = p11 + (p01 >> s32) + (p10 >> s32) + (mid >> s32)
    return hi, a * b


def philox4x64_10_many(c0, key):
    """Philox4x64-10 at counters (c0[i], 0, 0, 0): the four output words, as uint64 arrays."""
    with np.errstate(over="ignore"):
        c = [np.asarray(c0, dtype=np.uint64), np.zeros(len(c0), np.uint64), np.zeros(len(c0), np.uint64),
             np.zeros(len(c0), np.uint64)]
        k0, k1 = int(key[0]) & M64, int(key[1]) & M64
        for r in range(10):
            if r:
                k0, k1 = (k0 + PHILOX_W0) & M64, (k1 + PHILOX_W1) & M64
            h0, l0 = _mulhilo(c[0], PHILOX_M0)
            h1, l1 = _mulhilo(c[2], PHILOX_M1)
            c = [h1 ^ c[1] ^ np.uint64(k0), l1, h0 ^ c[3] ^ np.uint64(k1), l0]
    return c


def scale_bits(m: int) -> int:
    """s = 61 - ceil(log2 m): m edges of weight at most 2 * 2^s sum below 2^62."""
    return 61 - max(0, (int(m) - 1).bit_length())


def integer_weights(w, R) -> np.ndarray:
    w = np.asarray(w, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    x = w * R
    if not np.all(np.isfinite(x)) or np.any(x < 0) or np.any(x > 2):
        raise ValueError("w_e R_e must be finite and in [0, 2]")
    return np.floor(np.ldexp(x, scale_bits(len(x)))).astype(np.uint64)


def draws(q: int, seed: int, K: int, C: np.ndarray, chunk: int = 1 << 20) -> np.ndarray:
    """Edge index of every draw i = 0 .. q-1."""
    out = np.empty(q, dtype=np.int64)
    for s in range(0, q, chunk):
        e = min(q, s + chunk)
        x = philox4x64_10_many(np.arange(s, e, dtype=np.uint64), (seed, 0))[0]
        with np.errstate(over="ignore"):
            t, _ = _mulhilo(x, np.uint64(K))
        out[s:e] = np.searchsorted(C, t, side="right")
    return out


def sparsify(w, R, q: int, seed: int):
    """(counts int64[m], new weights float64[m]) of Algorithm 1 under the readings above."""
    k = integer_weights(w, R)
    C = np.cumsum(k, dtype=np.uint64)
    K = int(C[-1]) if len(C) else 0
    if K == 0:
        raise ValueError("no edge has a positive sampling weight")
    e = draws(int(q), int(seed), K, C)
    counts = np.bincount(e, minlength=len(k)).astype(np.int64)
    wf = np.asarray(w, dtype=np.float64)
    kf = k.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        neww = counts.astype(np.float64) * wf * (float(K) / (float(q) * kf))
    neww[counts == 0] = 0.0
    return counts, neww


def laplacian_quadratic(n, eu, ev, w, x) -> float:
    """x^T L x = sum over edges of w (x_u - x_v)^2 (eq 1), with math.fsum."""
    d = np.asarray(x)[np.asarray(eu)] - np.asarray(x)[np.asarray(ev)]
    return math.fsum((np.asarray(w) * d * d).tolist())
