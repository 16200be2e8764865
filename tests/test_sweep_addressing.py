"""Every address one sweep forms, checked on the CPU at full size.

``tests/native/sweep_addressing.cpp`` runs the library's host preparation and
planner on a graph and replays the address arithmetic of every sweep kernel
in the integer widths the kernels use: the bottom sweep's 32-bit record,
query-record and top-store byte offsets, staging writes, partial-slot
indices (and that the ordered reduction reads only slots the sweep wrote),
the top-node and non-ancestor pair reads, the chain-level GEMM tiles'
gathered columns and output tiles, and the dense sums above bottom subtrees
(the B_S records each upload wave walks, every U_S column and B column read,
every dense sum written and read back). On graphs up to 20,000 nodes it also
checks the values of the dense form: the rows above a query's subtree from
B_S and w plus its sweep rows against the plain sum over every row. Each access is checked against the size of
its buffer. The program is built with AddressSanitizer and
UndefinedBehaviorSanitizer, so the host preparation (ingest, ordering,
symbolic and numeric factorization, plans) runs under them at the same time.
The 1M-node PDN case has a 1.75 GB top store, addressed with 32-bit offsets.
"""
import os
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "sweep_addressing.cpp")
HOST = os.path.join(ROOT, "paper_2606_31535_amd", "csrc", "host")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("addr") / "sweep_addressing")
    host = sorted(os.path.join(HOST, f) for f in os.listdir(HOST) if f.endswith(".cpp"))
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-pthread", "-I" + os.path.join(ROOT, "include"), SRC] + host + ["-o", out]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    return out


def _write(g, path):
    with open(path, "wb") as f:
        np.array([g.n, g.m], np.int64).tofile(f)
        np.array([g.ground, 1 if g.coords is not None else 0], np.int32).tofile(f)
        np.asarray(g.eu, np.int32).tofile(f)
        np.asarray(g.ev, np.int32).tofile(f)
        np.asarray(g.w, np.float64).tofile(f)
        if g.coords is not None:
            np.asarray(g.coords, np.float64).tofile(f)


def _run(checker, g, tmp_path, pairs, seed=5):
    path = str(tmp_path / "graph.bin")
    _write(g, path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([checker, path, str(pairs), str(seed)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, env=env, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-4000:]
    assert "ok:" in r.stdout


@pytest.mark.parametrize("name,gen,pairs", [
    ("mesh32", lambda: synth.mesh2d(), 5000),
    ("rgg", lambda: synth.rgg_knn(4000, seed=40011), 5000),
    ("tree", lambda: synth.random_tree(3000, seed=4, ground=7), 2000),
    ("pdn_small", lambda: synth.pdn_multilayer(side=48, layers=4, seed=12, long_frac=0.01), 20000),
])
def test_small_graphs(checker, tmp_path, name, gen, pairs):
    _run(checker, gen(), tmp_path, pairs)


def test_pdn_1m_nodes_full_size(checker, tmp_path):
    _run(checker, synth.pdn_multilayer(), tmp_path, 20000)
