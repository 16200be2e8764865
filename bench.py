"""Benchmark: all-edge effective resistances per second on the 1M-node PDN mesh.

One "step" is one full pass of the hot path over the resident factor: every
edge's resistance (the query plan, the top-tree phase, the bottom subtree
sweep with fused accumulation, the ordered reduction) written to a device
buffer. Host preparation (ordering, symbolic, numeric L D L^T) and the upload
are timed separately and reported beside the result, as the paper reports
its factorization time separately from the query phase.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload C3|C2|C1|C4|C5]

Prints one JSON line. The default (the 1M-node PDN, C3) also carries the
metric's other half measured in the same run: a "batched" sub-object (256
random geometric graphs in one captured launch sequence, against the same
sweeps issued one graph at a time) and a "served" sub-object (8 resident PDN
factors under a Poisson request stream: saturation rate, p50/p99 latency at
25/50/90% load, against serving one request at a time). The CPU oracle leg
runs first, on a bounded edge sample over a forked process pool.
Only one GPU is used; --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402

METRIC = "all-edge resistances/s on 1M-node PDN (FP64, rel err<=1e-10); served p50/p99"
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector and FP64 matrix peak (dense)
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "C1": ("mesh32x32: 2D power-grid mesh 32x32, 4-neighbour, conductances log-uniform [0.1,10], ground 0, all edges",
           lambda: synth.mesh2d()),
    "C2": ("pdn2x512: 2-layer PDN mesh 512x512 per layer, H/V wires N(5,1) clipped at 0.1, 10% vias g=50, ground 0, all edges",
           lambda: synth.pdn_two_layer()),
    "C3": ("pdn4x500: 4-layer PDN mesh 500x500 per layer (1M nodes), alternating wire direction, layer conductances "
           "{1,2,4,8} x log-uniform [0.5,2], 5% vias g=100, 0.1% long edges g=0.01, ground 0, all edges",
           lambda: synth.pdn_multilayer()),
}


_ORACLE = None  # (oracle, eu, ev) inherited by the forked workers of cpu_baseline


def _oracle_chunk(idx):
    # one BLAS thread per worker process: the pool already uses every core
    from threadpoolctl import threadpool_limits
    so, eu, ev = _ORACLE
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        R = so.resistances(eu[idx], ev[idx])
        return R, time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_workers() -> int:
    """Worker processes for host-side pools: the cores this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(g, sample: int, seed: int = 11):
    """Time the CPU oracle (sparse per-pair solves, refined) on a bounded edge sample.

    The oracle factors the grounded Laplacian once (its own nested dissection
    and SuperLU), then a pool of forked worker processes, one per host core
    up to 16, solves disjoint slices of a seeded edge sample. Must run before
    this process touches the GPU (the workers are forked).
    """
    import multiprocessing
    from oracle import sparse
    global _ORACLE
    t0 = time.time()
    so = sparse.SparseOracle(g, ordering="nd")
    t_setup = time.time() - t0
    rng = synth.rng_for(seed)
    sel = rng.choice(g.m, size=min(sample, g.m), replace=False)
    workers = host_workers()
    chunks = [c for c in np.array_split(sel, workers * 4) if len(c)]
    _ORACLE = (so, np.asarray(g.eu), np.asarray(g.ev))
    t1 = time.perf_counter()
    with multiprocessing.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_oracle_chunk, chunks)
    t_solve = time.perf_counter() - t1
    _ORACLE = None
    R = np.concatenate([p[0] for p in parts])
    cpu_s = sum(p[1] for p in parts)
    return {
        "value": float(len(sel) / t_solve), "unit": "resistances/s", "cores": workers, "kind": "oracle",
        "cpu_model": cpu_model(), "nproc": os.cpu_count(),
        "sample": (f"{len(sel)} seeded edges of the same graph, per-pair sparse LU solves (oracle's own nested "
                   f"dissection + SuperLU) with 2 extended-precision refinement steps, {workers} forked worker "
                   f"processes; solve wall {t_solve:.1f} s ({cpu_s:.1f} core-s); the oracle's ordering and "
                   f"factorization ({t_setup:.1f} s, one core) are excluded"),
        "per_edge_core_s": round(cpu_s / len(sel), 4),
    }, sel, R


KERNEL_SOURCES = ("paper_2606_31535_amd/csrc/hip/sweep.hip", "paper_2606_31535_amd/csrc/hip/sweep_kernels.h",
                  "paper_2606_31535_amd/csrc/host/plan.cpp", "paper_2606_31535_amd/csrc/host/plan.h")


def kernel_source_hash() -> str:
    """sha256 over the sources that decide what the sweep kernels read and write."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, workload: str, key: str = "hbm_bytes_per_launch"):
    """HBM bytes (per launch, or the field `key`) from the committed rocprofv3 counter summary, or None.

    The summary (profiles/<kernel>_<workload>_traffic.txt) holds the
    FETCH_SIZE/WRITE_SIZE readings scaled by the copy-kernel calibration and
    the source hash they were taken at; a summary of other sources is ignored.
    """
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(fields[key].split()[0])
    except (KeyError, ValueError, IndexError):
        return None


def copy_calibration(nbytes: int, reps: int = 5) -> None:
    """Plain device-to-device copy of a known size (for scaling HBM byte counters)."""
    import torch
    n = nbytes // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps + 1,
                      "ms_per_copy": round(dt * 1e3, 4), "GB_per_s_read_plus_write": round(2 * n * 8 / dt / 1e9, 1)}))


def bench_batch(args, steps: int, warmup: int) -> dict:
    """Batched form: 256 random geometric graphs, all edges, one captured launch sequence per step.

    The step is the whole batch (every graph's all-edge sweep). The same graphs
    are also swept one factor at a time on the same stream (the plain form) and
    the two results are compared bit for bit.
    """
    import torch
    import paper_2606_31535_amd as P
    t0 = time.time()
    graphs = synth.rgg_batch(args.batch_count)
    t_gen = time.time() - t0
    t0 = time.time()
    hs = [P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords) for g in graphs]
    t_prep = time.time() - t0
    dev = P.peers_device_open(0)
    stream = torch.cuda.current_stream()
    t0 = time.time()
    fs = [P.peers_factor_upload(dev, h, stream) for h in hs]
    torch.cuda.synchronize()
    t_upload = time.time() - t0
    m_tot = sum(g.m for g in graphs)
    seq = [torch.empty(g.m, dtype=torch.float64, device="cuda") for g in graphs]
    bat = [torch.empty(g.m, dtype=torch.float64, device="cuda") for g in graphs]

    def run_seq():
        for f, o in zip(fs, seq):
            P.peers_query_all_edges(f, o, stream=stream)

    def run_bat():
        P.peers_batch_query(dev, fs, [None] * len(fs), [None] * len(fs), bat, stream=stream)

    for _ in range(warmup):
        run_seq()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run_seq()
    torch.cuda.synchronize()
    dt_seq = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    run_bat()  # builds, autotunes and captures
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    info = P.peers_batch_last_info(dev)
    for _ in range(warmup):
        run_bat()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run_bat()
    torch.cuda.synchronize()
    dt_bat = (time.perf_counter() - t0) / steps
    same = all(torch.equal(a.view(torch.int64), b.view(torch.int64)) for a, b in zip(seq, bat))
    foster = max(abs(math.fsum(g.w * o.cpu().numpy()) - (g.n - 1)) / (g.n - 1) for g, o in zip(graphs, bat))
    out = {
        "metric": "all-edge resistances/s, batch of 256 random geometric graphs (FP64), batched form",
        "value": round(m_tot / dt_bat, 1), "unit": "resistances/s", "steps": steps, "warmup": warmup,
        "ms_per_step": round(dt_bat * 1e3, 4), "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(graphs)} RGGs in the unit square, n ~ U[2000,50000], union of 6-NN, "
                               "w = 1/distance, ground 0, all edges",
                   "graphs": len(graphs), "sum_n": sum(g.n for g in graphs), "sum_m": m_tot},
        "plain_form": {"value": round(m_tot / dt_seq, 1), "ms_per_step": round(dt_seq * 1e3, 4),
                       "what": "the same sweeps issued one factor at a time on the same stream"},
        "speedup_vs_plain": round(dt_seq / dt_bat, 3),
        "bit_identical_to_plain": bool(same), "max_foster_rel_residual": foster,
        "autotuner": {"schedule": info["schedule_name"], "candidate_ms": info["candidate_ms"],
                      "stages": info["stages"], "bottom_items": info["bottom_items"],
                      "first_call_s": round(t_first, 3)},
        "t_gen_s": round(t_gen, 2), "t_prep_s": round(t_prep, 2), "t_upload_s": round(t_upload, 2),
    }
    for f in fs:
        P.peers_factor_release(f)
    P.peers_device_close(dev)
    for h in hs:
        P.peers_graph_destroy(h)
    return out


SERVED_SIDES = (128, 181, 222, 256, 320, 384, 448, 500)


def bench_served(args) -> dict:
    """Served form: 8 resident PDN factors, Poisson requests of 1..100k pairs.

    Saturation throughput is measured with the whole trace submitted at once;
    then the same kind of trace is replayed in real time at 25/50/90% of the
    saturation request rate. The baseline serves each request alone, one at a
    time (measured service times, first-come first-served over the same
    arrival times).
    """
    import threading
    import torch
    import paper_2606_31535_amd as P
    t0 = time.time()
    graphs = [synth.pdn_multilayer(side=sd, layers=4, seed=50000 + i) for i, sd in enumerate(SERVED_SIDES)]
    t_gen = time.time() - t0
    t0 = time.time()
    hs = [P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords) for g in graphs]
    t_prep = time.time() - t0
    dev = P.peers_device_open(0)
    t0 = time.time()
    fs = [P.peers_factor_upload(dev, h) for h in hs]
    torch.cuda.synchronize()
    t_upload = time.time() - t0
    used, budget = P.peers_device_usage(dev)
    nreq = args.served_requests

    def serve(trace, realtime):
        srv = P.peers_server_start(dev, max_batch_pairs=1 << 20, max_wait_us=500, streams=2)
        outs = [np.empty(len(r["qu"])) for r in trace]
        tickets = [None] * len(trace)
        keep = []
        start = time.perf_counter()

        def submitter():
            for i, r in enumerate(trace):
                if realtime:
                    delay = r["t"] - (time.perf_counter() - start)
                    if delay > 0:
                        time.sleep(delay)
                t, k = P.peers_server_submit(srv, fs[r["graph"]], r["qu"], r["qv"], outs[i])
                keep.append(k)
                tickets[i] = t

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        for t in tickets:
            st, res = P.peers_server_wait(srv, t, -1)
            assert st == 0 and res == 0, (st, res)
        wall = time.perf_counter() - start
        stats = P.peers_server_stats_get(srv)
        P.peers_server_stop(srv)
        return outs, wall, stats

    # warm the factors' workspaces and the server arenas
    serve(synth.served_trace(graphs, 16, qps=1e9, seed=7), False)
    sat_trace = synth.served_trace(graphs, nreq, qps=1e9, seed=synth.CONFIG_SEEDS["C5"])
    pairs = sum(len(r["qu"]) for r in sat_trace)
    outs, wall, st_sat = serve(sat_trace, False)
    sat_rps, sat_qps = pairs / wall, nreq / wall
    # one request at a time: service time of each request alone
    service = []
    same = True
    for r, o in zip(sat_trace, outs):
        R = np.empty(len(r["qu"]))
        t1 = time.perf_counter()
        P.peers_query(fs[r["graph"]], r["qu"], r["qv"], R)
        service.append(time.perf_counter() - t1)
        same = same and np.array_equal(R.view(np.int64), o.view(np.int64))
    alone_rps = pairs / sum(service)

    def fcfs(trace, svc):
        free, lat = 0.0, []
        for r, sv in zip(trace, svc):
            begin = max(free, r["t"])
            free = begin + sv
            lat.append(free - r["t"])
        return np.array(lat)

    levels = []
    for frac in (0.25, 0.5, 0.9):
        tr = synth.served_trace(graphs, nreq, qps=frac * sat_qps, seed=synth.CONFIG_SEEDS["C5"] + 1)
        _, wall, st = serve(tr, True)
        # the one-at-a-time baseline over the same arrivals: each request's
        # service time measured alone
        svc = []
        for r in tr:
            R = np.empty(len(r["qu"]))
            t1 = time.perf_counter()
            P.peers_query(fs[r["graph"]], r["qu"], r["qv"], R)
            svc.append(time.perf_counter() - t1)
        lat = fcfs(tr, svc) * 1e6
        npairs = sum(len(r["qu"]) for r in tr)
        levels.append({"load": frac, "qps": round(frac * sat_qps, 2), "requests": nreq,
                       "resistances_per_s": round(npairs / wall, 1),
                       "p50_us": round(st["p50_us"], 1), "p99_us": round(st["p99_us"], 1),
                       "max_us": round(st["max_us"], 1), "batches": st["batches"],
                       "memory_waits": st["memory_waits"],
                       "one_at_a_time": {"p50_us": round(float(np.percentile(lat, 50)), 1),
                                         "p99_us": round(float(np.percentile(lat, 99)), 1),
                                         "max_us": round(float(lat.max()), 1)}})
    ref = levels[-1]
    out = {
        "metric": "served: resistances/s and p50/p99 latency, 8 resident PDN factors (FP64)",
        "value": round(sat_rps, 1), "unit": "resistances/s", "requests": nreq,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "8 PDN meshes (4 layers, sides " + ",".join(map(str, SERVED_SIDES)) +
                               "), Poisson requests of 1..100000 pairs (log-uniform), 80% edges / 20% random pairs",
                   "factors": len(graphs), "nodes": [g.n for g in graphs], "requests": nreq, "pairs": pairs},
        "saturation": {"resistances_per_s": round(sat_rps, 1), "requests_per_s": round(sat_qps, 2),
                       "batches": st_sat["batches"], "p50_us": round(st_sat["p50_us"], 1),
                       "p99_us": round(st_sat["p99_us"], 1)},
        "one_at_a_time_resistances_per_s": round(alone_rps, 1),
        "speedup_vs_one_at_a_time": round(sat_rps / alone_rps, 3),
        "bit_identical_to_alone": bool(same),
        "load_levels": levels,
        "p50_us_at_90pct": ref["p50_us"], "p99_us_at_90pct": ref["p99_us"],
        "hbm_bytes": {"resident_factors_and_workspace": used, "budget": budget},
        "t_gen_s": round(t_gen, 2), "t_prep_s": round(t_prep, 2), "t_upload_s": round(t_upload, 2),
    }
    for f in fs:
        P.peers_factor_release(f)
    P.peers_device_close(dev)
    for h in hs:
        P.peers_graph_destroy(h)
    return out


def bench_plain(args, g, desc, cpu=None) -> dict:
    """The all-edge sweep of one resident factor (C1-C3); the headline line."""
    import torch
    import paper_2606_31535_amd as P

    t0 = time.time()
    h = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords)
    t_prep = time.time() - t0
    st = P.peers_graph_stats_get(h)
    dev = P.peers_device_open(0)
    stream = torch.cuda.current_stream()
    t0 = time.time()
    f = P.peers_factor_upload(dev, h, stream)
    torch.cuda.synchronize()
    t_upload = time.time() - t0
    resident, workspace = P.peers_factor_footprint(f)
    R = torch.empty(g.m, dtype=torch.float64, device="cuda")

    for _ in range(args.warmup):
        P.peers_query_all_edges(f, R, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P.peers_query_all_edges(f, R, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    Rh = R.cpu().numpy()

    # per-phase HIP-event times on the sweep's stream (separate profiled steps)
    phases = []
    for _ in range(max(1, min(3, args.steps))):
        P.peers_query_all_edges(f, R, flags=P.PEERS_PROFILE, stream=stream)
        phases.append(P.peers_factor_timings(f))
    torch.cuda.synchronize()
    ph = {k: float(np.mean([p[k] for p in phases])) for k in ("top_ms", "bottom_ms", "finish_ms", "total_ms")}
    tm = phases[-1]
    if ph["top_ms"] >= ph["bottom_ms"]:
        kname, ms, flops, nl = "gemm_level_kernel", ph["top_ms"], tm["top_flops"], tm["top_launches"]
        bound, fdef = "mfma", "2 * (sum over top-column entries L_ki of depth(k))"
    else:
        kname, ms, flops, nl = "bottom_kernel", ph["bottom_ms"], tm["bottom_flops"], tm["bottom_launches"]
        bound = "alu"
        fdef = ("2 * (sum over bottom-column entries L_ki of depth(k)) + 3 * (sum over edges whose lower "
                "endpoint is a bottom node of its depth)")
    achieved = flops / (ms * 1e-3) / 1e12
    roofline = {"bound": bound, "achieved": round(achieved, 4), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 5),
                "traffic": recorded_traffic(kname, args.workload), "source_hash": kernel_source_hash(),
                "kernel": kname, "launches_per_step": nl, "phase_ms": round(ms, 4),
                "algorithmic_flops": flops, "flops_definition": fdef}
    whole = tm["top_flops"] + tm["bottom_flops"] + tm["finish_flops"]
    # both sweep phases against the FP64 peak (the matrix cores and the vector
    # units have the same FP64 rate on this chip)
    phase_roofline = {
        name: {"phase_ms": round(ph[key], 4), "algorithmic_flops": tm[fk],
               "achieved": round(tm[fk] / (ph[key] * 1e-3) / 1e12, 4),
               "frac": round(tm[fk] / (ph[key] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 5), "launches": tm[lk]}
        for name, key, fk, lk in (("top", "top_ms", "top_flops", "top_launches"),
                                  ("bottom", "bottom_ms", "bottom_flops", "bottom_launches"))}
    phase_roofline["bottom"]["what"] = ("dense sums above bottom subtrees on the matrix cores (three side "
                                        "streams) beside the sweep of the rows from each subtree on")
    # HBM bytes of each phase from the committed counter summaries (null when
    # they were taken at other kernel sources): the chain levels' mean bytes per
    # launch times their launches, and the whole bottom phase
    lv_bytes = recorded_traffic("gemm_level_kernel", args.workload)
    hbm_phase = {"top": None if lv_bytes is None else lv_bytes * (tm["top_launches"] - 1),
                 "bottom": recorded_traffic("bottom_phase", args.workload, "hbm_bytes_per_sweep")}
    for name, b in hbm_phase.items():
        tbs = None if b is None else b / (phase_roofline[name]["phase_ms"] * 1e-3) / 1e12
        phase_roofline[name]["hbm"] = {"bytes": b, "TB_per_s": None if b is None else round(tbs, 3),
                                       "frac_of_hbm_peak": None if b is None else round(tbs * 1e3 / PEAK_HBM_GBS, 4)}
    phase_roofline["top"]["hbm"]["what"] = "gemm_level_kernel launches (the chain-rows launch not counted)"

    # accuracy on the stored oracle sample, and Foster's theorem on all edges
    acc = {"foster_rel_residual": float(abs(math.fsum(g.w * Rh) - (g.n - 1)) / (g.n - 1))}
    gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}_edges.json")
    if os.path.exists(gold):
        with open(gold) as fh:
            d = json.load(fh)
        gold_e = np.array(d["edges"])
        gold_R = np.array([float(x) for x in d["R"]])
        acc["max_rel_err_oracle_sample"] = float(np.max(np.abs(Rh[gold_e] - gold_R) / gold_R))
        acc["oracle_sample_edges"] = int(len(gold_e))

    # second workload on the same factor: every node's resistance to the
    # ground (eq 4, t = g), against the stored oracle sample
    Rg = torch.empty(g.n, dtype=torch.float64, device="cuda")
    P.peers_query_all_to_ground(f, Rg, stream=stream)  # builds and keeps its plan
    torch.cuda.synchronize()
    nsteps = max(1, min(args.steps, 10))
    t0 = time.perf_counter()
    for _ in range(nsteps):
        P.peers_query_all_to_ground(f, Rg, stream=stream)
    torch.cuda.synchronize()
    dtg = (time.perf_counter() - t0) / nsteps
    Rgh = Rg.cpu().numpy()
    ground = {"value": round(g.n / dtg, 1), "unit": "resistances/s", "ms_per_step": round(dtg * 1e3, 4),
              "sum_R_ug": math.fsum(Rgh), "what": "R between every node and the ground (resident plan)"}
    gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}_ground.json")
    if os.path.exists(gold):
        with open(gold) as fh:
            d = json.load(fh)
        gold_n = np.array(d["nodes"])
        gold_Rg = np.array([float(x) for x in d["R"]])
        ground["max_rel_err_oracle_sample"] = float(np.max(np.abs(Rgh[gold_n] - gold_Rg) / gold_Rg))
        ground["oracle_sample_nodes"] = int(len(gold_n))
    # Algorithm 1 on the device: sample 4n edges by w_e R_e from the sweep's
    # resistances (already in device memory)
    wd = torch.tensor(g.w, dtype=torch.float64, device="cuda")
    cd = torch.empty(g.m, dtype=torch.int32, device="cuda")
    nd = torch.empty(g.m, dtype=torch.float64, device="cuda")
    qs = 4 * g.n
    P.peers_sparsify(dev, wd, R, qs, 1, cd, nd, stream=stream)
    t0 = time.perf_counter()
    for k in range(nsteps):
        P.peers_sparsify(dev, wd, R, qs, 1 + k, cd, nd, stream=stream)
    torch.cuda.synchronize()
    dts = (time.perf_counter() - t0) / nsteps
    sparsifier = {"draws": qs, "ms_per_call": round(dts * 1e3, 4), "draws_per_s": round(qs / dts, 1),
                  "edges_kept": int((cd > 0).sum().item()), "edges": g.m,
                  "what": "Algorithm 1 on the all-edge resistances in device memory (synchronous call)"}
    del wd, cd, nd

    # Algorithm 8 step 1 on the device: a second handle of the same graph
    # whose factor is formed by its upload; HIP-event time of the
    # factorization, its factor against the host one, and its resistances
    t0 = time.time()
    hd = P.peers_graph_create(g.n, g.eu, g.ev, g.w, g.ground, coords=g.coords, numeric_on_device=True)
    t_create_d = time.time() - t0
    t0 = time.time()
    fd = P.peers_factor_upload(dev, hd, stream)
    torch.cuda.synchronize()
    t_upload_d = time.time() - t0
    std = P.peers_graph_stats_get(hd)
    Ld, Dd = P.peers_graph_export_factor(hd)
    Lh, Dh = P.peers_graph_export_factor(h)
    Rd = torch.empty(g.m, dtype=torch.float64, device="cuda")
    t0 = time.time()
    P.peers_query_all_edges(fd, Rd, stream=stream)
    torch.cuda.synchronize()
    t_first_sweep_d = time.time() - t0
    Rdh = Rd.cpu().numpy()
    nzR = Rh > 0
    device_factor = {
        "t_numeric_ms": round(std["t_numeric"] * 1e3, 3), "host_t_numeric_s": round(st["t_numeric"], 3),
        "speedup_vs_host_numeric": round(st["t_numeric"] / std["t_numeric"], 1),
        "upload_with_factorization_s": round(t_upload_d, 3),
        "one_shot_all_edges_s": round(t_create_d + t_upload_d + t_first_sweep_d, 3),
        "one_shot_what": "graph in to all-edge resistances in device memory: ingest, ordering and symbolic analysis "
                         "on the host, upload with the factorization on the device, first sweep",
        "max_rel_diff_L_vs_host": float(np.max(np.abs(Ld - Lh) / np.maximum(np.abs(Lh), 1e-300))) if len(Lh) else 0.0,
        "max_rel_diff_D_vs_host": float(np.max(np.abs(Dd - Dh) / Dh)),
        "max_rel_diff_R_vs_host_factor": float(np.max(np.abs(Rdh[nzR] - Rh[nzR]) / Rh[nzR])),
        "what": "cancellation-free L D L^T on the device (bottom subtrees per wavefront, chain pieces of <= 64 "
                "columns per level, L_U D L_U^T on the matrix cores); HIP-event time on the upload stream"}
    if "oracle_sample_edges" in acc:
        device_factor["max_rel_err_oracle_sample"] = float(np.max(np.abs(Rdh[gold_e] - gold_R) / gold_R))
    del Ld, Lh, Rd
    P.peers_factor_release(fd)
    P.peers_graph_destroy(hd)

    out = {
        "metric": METRIC, "value": round(g.m / dt, 1), "unit": "resistances/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "n": g.n, "m": g.m, "seed": g.meta.get("seed"), "nnz_l": st["nnz_l"],
                   "etree_height": st["height"], "f_sweep_fma": st["f_sweep"], "acc_terms": st["acc_terms"]},
        "roofline": roofline, "phase_roofline": phase_roofline, "phases_ms": {k: round(v, 4) for k, v in ph.items()},
        "whole_step": {"algorithmic_flops": whole, "TFLOP_per_s": round(whole / dt / 1e12, 3),
                       "frac_of_fp64_peak": round(whole / dt / 1e12 / PEAK_FP64_TFLOPS, 4)},
        "accuracy": acc,
        "t_prep_s": {"total": round(t_prep, 3), "ingest": round(st["t_ingest"], 3), "order": round(st["t_order"], 3),
                     "symbolic": round(st["t_symbolic"], 3), "numeric": round(st["t_numeric"], 3),
                     "upload": round(t_upload, 3), "upload_layout": round(tm["t_layout_s"], 3),
                     "upload_edge_plan": round(tm["t_edge_plan_s"], 3),
                     "upload_transfer": round(tm["t_transfer_s"], 3),
                     "upload_transform": round(tm["t_transform_s"], 3)},
        "t_query": {"plan_s": round(tm["t_edge_plan_s"], 4), "sweep_and_reduce_ms": round(dt * 1e3, 4),
                    "result_copy_ms": 0.0,
                    "resistances_per_s_including_plan": round(g.m / (tm["t_edge_plan_s"] + dt), 1),
                    "note": "all-edge plan built once at upload; results stay in device memory"},
        "hbm_bytes": {"resident": resident, "workspace": workspace},
        "node_to_ground": ground,
        "sparsifier": sparsifier,
        "device_factor": device_factor,
    }
    if cpu is not None:
        cb, sel, Rs = cpu
        cb["max_rel_diff_vs_gpu"] = float(np.max(np.abs(Rh[sel] - Rs) / Rs))
        out["cpu_baseline"] = cb
    if not args.no_cpu_scheme:
        # the paper's own parallel scheme (Algorithms 3-8) on this host's
        # cores, same factor and queries: the same-host context number
        Rc = np.full(g.m, np.nan)
        sc = P.peers_cpu_query(h, g.eu, g.ev, Rc, threads=host_workers())
        pc = {"value": round(g.m / sc["t_rows_s"], 1), "unit": "resistances/s", "cores": sc["threads"],
              "cpu_model": cpu_model(), "t_rows_s": round(sc["t_rows_s"], 3), "t_setup_s": round(sc["t_setup_s"], 3),
              "what": "Algorithms 3-8 (CAS row claims, incremental DFS with rollback, row-wise accumulation) in C++ "
                      "threads on the library's host factor, all edges",
              "max_rel_diff_vs_gpu": float(np.max(np.abs(Rc - Rh)[Rh > 0] / Rh[Rh > 0]))}
        if "oracle_sample_edges" in acc:
            pc["max_rel_err_oracle_sample"] = float(np.max(np.abs(Rc[gold_e] - gold_R) / gold_R))
        out["cpu_paper_scheme"] = pc
    P.peers_factor_release(f)
    P.peers_device_close(dev)
    P.peers_graph_destroy(h)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C3", choices=sorted(WORKLOADS) + ["C4", "C5"])
    ap.add_argument("--served-requests", type=int, default=200, help="requests per served trace (C5)")
    ap.add_argument("--batch-count", type=int, default=256, help="graphs in the C4 batch")
    ap.add_argument("--cpu-sample", type=int, default=768)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-scheme", action="store_true", help="leave out the paper's CPU scheme timing")
    ap.add_argument("--no-batched", action="store_true", help="leave the batched sub-object out of the C3 line")
    ap.add_argument("--no-served", action="store_true", help="leave the served sub-object out of the C3 line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the design notes describe how the "
              "sweep would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.workload == "C4":
        out = bench_batch(args, args.steps, args.warmup)
        out.update({"n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None})
        print(json.dumps(out))
        return
    if args.workload == "C5":
        out = bench_served(args)
        out.update({"n_gpus": 1, "steps": out["requests"], "warmup": 16, "higher_is_better": True,
                    "scaling": "weak", "vs_baseline": None})
        print(json.dumps(out))
        return

    desc, gen = WORKLOADS[args.workload]
    g = gen()
    # the oracle's CPU leg first: its worker processes are forked, before
    # anything here touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(g, args.cpu_sample)
    out = bench_plain(args, g, desc, cpu)
    print(json.dumps({"progress": "plain all-edge sweep done", "ms_per_step": out["ms_per_step"]}),
          file=sys.stderr, flush=True)
    if args.workload == "C3":
        # the metric's other half, on the same GPU in the same run: the batched
        # form (256 RGGs) and the served form (8 resident PDN factors)
        if not args.no_batched:
            out["batched"] = bench_batch(args, min(args.steps, 5), min(args.warmup, 2))
            print(json.dumps({"progress": "batched form done"}), file=sys.stderr, flush=True)
        if not args.no_served:
            out["served"] = bench_served(args)
            out["served_p50_us_at_90pct"] = out["served"]["p50_us_at_90pct"]
            out["served_p99_us_at_90pct"] = out["served"]["p99_us_at_90pct"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
