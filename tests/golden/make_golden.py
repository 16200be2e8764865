"""Write oracle values for sampled edges and nodes of the full-size workloads.

Calls only ``oracle`` (and the seeded generators in ``synth``): the stored
expected values never come from the library under test. For each workload the
edge sample is: a seeded uniform sample of edges, and the highest- and
lowest-conductance edges. The node sample (node-to-ground resistances, eq 4
with t = g) is a seeded uniform sample of nodes.

    python tests/golden/make_golden.py C2 C3          # writes tests/golden/<cfg>_edges.json
    python tests/golden/make_golden.py ground C2 C3   # writes tests/golden/<cfg>_ground.json
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import sparse  # noqa: E402

WORKLOADS = {
    "C2": lambda: synth.pdn_two_layer(),
    "C3": lambda: synth.pdn_multilayer(),
}
SAMPLE = {"C2": 1000, "C3": 1000}
EXTREMES = 100

_ORACLE = None


def _init(cfg):
    global _ORACLE
    _ORACLE = sparse.SparseOracle(WORKLOADS[cfg](), ordering="nd")


def _solve(args):
    from threadpoolctl import threadpool_limits
    qu, qv = args
    with threadpool_limits(limits=1):  # one BLAS thread per worker process
        return _ORACLE.resistances(qu, qv)


def sample_edges(g, cfg):
    rng = synth.rng_for(7000 + int(cfg[1]))
    idx = set(rng.choice(g.m, size=SAMPLE[cfg], replace=False).tolist())
    order = np.argsort(g.w, kind="stable")
    idx.update(order[:EXTREMES].tolist())
    idx.update(order[-EXTREMES:].tolist())
    return np.array(sorted(idx), dtype=np.int64)


def make(cfg, workers=6):
    g = WORKLOADS[cfg]()
    edges = sample_edges(g, cfg)
    chunks = np.array_split(edges, workers * 4)
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=workers, initializer=_init, initargs=(cfg,)) as ex:
        parts = list(ex.map(_solve, [(g.eu[c], g.ev[c]) for c in chunks]))
    R = np.concatenate(parts)
    out = {
        "workload": cfg, "generator": g.name, "seed": g.meta.get("seed"), "n": g.n, "m": g.m,
        "oracle": "oracle.sparse.SparseOracle(ordering='nd'), 2 refinement steps, extended-precision residual",
        "seconds": round(time.time() - t0, 1), "edges": edges.tolist(), "R": [repr(float(x)) for x in R],
    }
    with open(os.path.join(HERE, f"{cfg}_edges.json"), "w") as f:
        json.dump(out, f)
    print(cfg, len(edges), "edges in", out["seconds"], "s")


GROUND_SAMPLE = 300


def make_ground(cfg, workers=6):
    g = WORKLOADS[cfg]()
    rng = synth.rng_for(7100 + int(cfg[1]))
    nodes = np.array(sorted(rng.choice(np.array([x for x in range(g.n) if x != g.ground]), size=GROUND_SAMPLE,
                                       replace=False).tolist()), dtype=np.int64)
    chunks = np.array_split(nodes, workers * 4)
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=workers, initializer=_init, initargs=(cfg,)) as ex:
        parts = list(ex.map(_solve, [(c, np.full(len(c), g.ground)) for c in chunks]))
    R = np.concatenate(parts)
    out = {
        "workload": cfg, "generator": g.name, "seed": g.meta.get("seed"), "n": g.n, "m": g.m, "ground": g.ground,
        "oracle": "oracle.sparse.SparseOracle(ordering='nd'), 2 refinement steps, extended-precision residual",
        "seconds": round(time.time() - t0, 1), "nodes": nodes.tolist(), "R": [repr(float(x)) for x in R],
    }
    with open(os.path.join(HERE, f"{cfg}_ground.json"), "w") as f:
        json.dump(out, f)
    print(cfg, len(nodes), "nodes in", out["seconds"], "s")


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "ground":
        for cfg in args[1:] or ["C2", "C3"]:
            make_ground(cfg)
    else:
        for cfg in args or ["C2", "C3"]:
            make(cfg)
