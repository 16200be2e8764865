"""The device factorization's plan and steps, emulated on the CPU.

``tests/native/factor_emulation.cpp`` builds the sweep layout with
placeholders and the numeric plan the device factorization runs, performs
every step of that factorization on the CPU in the kernels' order with each
index checked against its buffer (and each front index against its column),
and compares the factor and the filled sweep layout with the host
factorization's (relative differences within 1e-11: both form each entry from
same-signed sums, so they differ only in summation order). Built with
AddressSanitizer and UndefinedBehaviorSanitizer.
"""
import os
import subprocess

import pytest

import synth
from test_sweep_addressing import _write

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "factor_emulation.cpp")
HOST = os.path.join(ROOT, "paper_2606_31535_amd", "csrc", "host")


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("fac") / "factor_emulation")
    host = sorted(os.path.join(HOST, f) for f in os.listdir(HOST) if f.endswith(".cpp"))
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-pthread", "-I" + os.path.join(ROOT, "include"), SRC] + host + ["-o", out]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    return out


def _run(emulator, g, tmp_path):
    path = str(tmp_path / "graph.bin")
    _write(g, path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([emulator, path], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env,
                       timeout=900)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-4000:]
    assert "ok:" in r.stdout


GRAPHS = {
    "mesh32": lambda: synth.mesh2d(),
    "random": lambda: synth.random_connected(1500, 3000, seed=2, wlog=2.0, multi=True, ground=5),
    "rgg": lambda: synth.rgg_knn(3000, seed=40021, ground=3),
    "pdn": lambda: synth.pdn_multilayer(side=24, layers=4, seed=5, long_frac=0.005),
    "tree": lambda: synth.random_tree(2000, seed=6, wlog=2.0, ground=9),
    "star": lambda: synth.star_graph(300, ground=0),
    "pdn_wide": lambda: synth.pdn_multilayer(side=60, layers=4, seed=7, long_frac=0.002),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_factor_emulation(emulator, tmp_path, name):
    _run(emulator, GRAPHS[name](), tmp_path)


def test_factor_emulation_two_layer_full_size(emulator, tmp_path):
    _run(emulator, synth.pdn_two_layer(), tmp_path)
