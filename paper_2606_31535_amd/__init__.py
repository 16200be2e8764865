"""Python binding of libpeers (exact effective resistances on MI355X).

Argument marshalling only: every computation happens in the native library
(host C++ preparation, HIP sweep kernels). The binding exposes the C ABI of
``include/peers.h`` under the same names and thin handle classes around them.
Device buffers and streams may be passed as torch tensors / streams; numpy
arrays are accepted for host data.

If the built library is missing this module raises on import of any entry
point: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libpeers.so")

PEERS_OK = 0
STATUS_NAMES = {
    0: "OK", -1: "E_INVALID_ARG", -2: "E_NODE_RANGE", -3: "E_WEIGHT", -4: "E_DISCONNECTED",
    -5: "E_NOT_SPD", -6: "E_HOST_OOM", -7: "E_OVER_BUDGET", -8: "E_HIP", -9: "E_BUSY",
    -10: "E_CANCELLED", -11: "E_TIMEOUT", -12: "E_UNSUPPORTED", -99: "E_INTERNAL",
}
PEERS_ORDER_AUTO, PEERS_ORDER_COORD, PEERS_ORDER_GRAPH, PEERS_ORDER_GIVEN = 0, 1, 2, 3
PEERS_OUT_DEVICE, PEERS_IN_DEVICE, PEERS_SYNC, PEERS_PROFILE = 1, 2, 4, 8


class PeersError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({msg})")
        self.status = status


class peers_graph_opts(C.Structure):
    _fields_ = [("ordering", C.c_int32), ("coords", C.POINTER(C.c_double)),
                ("given_order", C.POINTER(C.c_int32)), ("threads", C.c_int32), ("leaf_size", C.c_int32),
                ("store_offsets_64", C.c_int32), ("numeric_on_device", C.c_int32),
                ("sweep_only", C.c_int32)]


class peers_graph_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("N", C.c_int64), ("nnz_l", C.c_int64),
                ("height", C.c_int32), ("n_supernodes", C.c_int32), ("max_sn_width", C.c_int32),
                ("n_roots", C.c_int32), ("self_loops", C.c_int64), ("f_sweep", C.c_double),
                ("acc_terms", C.c_double), ("t_ingest", C.c_double), ("t_order", C.c_double),
                ("t_symbolic", C.c_double), ("t_numeric", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class peers_sweep_timings(C.Structure):
    _fields_ = [("top_ms", C.c_double), ("bottom_ms", C.c_double), ("finish_ms", C.c_double),
                ("total_ms", C.c_double), ("top_launches", C.c_int32), ("bottom_launches", C.c_int32),
                ("top_flops", C.c_double), ("bottom_flops", C.c_double), ("top_bytes", C.c_double),
                ("bottom_bytes", C.c_double), ("finish_flops", C.c_double), ("t_layout_s", C.c_double),
                ("t_edge_plan_s", C.c_double), ("t_transfer_s", C.c_double), ("t_transform_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class peers_batch_info(C.Structure):
    _fields_ = [("factors", C.c_int32), ("stages", C.c_int32), ("bottom_items", C.c_int64),
                ("schedule", C.c_int32), ("candidates", C.c_int32), ("candidate_ms", C.c_double * 8),
                ("schedule_name", C.c_char * 96), ("graph_reused", C.c_int32), ("last_ms", C.c_double),
                ("schedule_cached", C.c_int32), ("signature", C.c_uint64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["candidate_ms"] = list(self.candidate_ms)[: self.candidates]
        d["schedule_name"] = self.schedule_name.decode()
        return d


class peers_server_opts(C.Structure):
    _fields_ = [("max_batch_pairs", C.c_int32), ("max_wait_us", C.c_int32),
                ("queue_capacity", C.c_int32), ("streams", C.c_int32)]


class peers_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected", C.c_uint64),
                ("batches", C.c_uint64), ("p50_us", C.c_double), ("p99_us", C.c_double),
                ("max_us", C.c_double), ("resistances_per_s", C.c_double), ("memory_waits", C.c_uint64),
                ("arena_bytes", C.c_uint64), ("pending", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class peers_cpu_stats(C.Structure):
    _fields_ = [("threads", C.c_int32), ("rows", C.c_int64), ("t_setup_s", C.c_double), ("t_rows_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = C.c_void_p
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)

# name -> (restype, argtypes); every name is an exported symbol of include/peers.h
# or include/peers_cpu.h
SIGNATURES = {
    "peers_graph_create": (C.c_int, [C.c_int64, C.c_int64, _i32p, _i32p, _f64p, C.c_int32,
                                     C.POINTER(peers_graph_opts), C.POINTER(_vp)]),
    "peers_graph_stats_get": (C.c_int, [_vp, C.POINTER(peers_graph_stats)]),
    "peers_graph_export_symbolic": (C.c_int, [_vp, _i32p, _i32p, _i64p, _i32p, _i32p]),
    "peers_graph_export_factor": (C.c_int, [_vp, _f64p, _f64p]),
    "peers_graph_destroy": (None, [_vp]),
    "peers_device_open": (C.c_int, [C.c_int32, C.c_uint64, C.POINTER(_vp)]),
    "peers_device_close": (None, [_vp]),
    "peers_device_usage": (C.c_int, [_vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "peers_device_set_budget": (C.c_int, [_vp, C.c_uint64]),
    "peers_factor_upload": (C.c_int, [_vp, _vp, _vp, C.POINTER(_vp)]),
    "peers_factor_release": (None, [_vp]),
    "peers_factor_footprint": (C.c_int, [_vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "peers_factor_timings": (C.c_int, [_vp, C.POINTER(peers_sweep_timings)]),
    "peers_factor_export_columns": (C.c_int, [_vp, C.c_int64, _i32p, C.c_int64, _f64p, _vp]),
    "peers_query_all_edges": (C.c_int, [_vp, _vp, C.c_uint32, _vp]),
    "peers_query_all_to_ground": (C.c_int, [_vp, _vp, C.c_uint32, _vp]),
    "peers_query": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, C.c_uint32, _vp]),
    "peers_query_noalloc": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, C.c_uint32, _vp]),
    "peers_batch_query": (C.c_int, [_vp, C.c_int32, C.POINTER(_vp), _i64p, C.POINTER(_vp),
                                    C.POINTER(_vp), C.POINTER(_vp), C.c_uint32, _vp]),
    "peers_batch_last_info": (C.c_int, [_vp, C.POINTER(peers_batch_info)]),
    "peers_sparsify": (C.c_int, [_vp, C.c_int64, _vp, _vp, C.c_int64, C.c_uint64, _vp, _vp, C.c_uint32, _vp]),
    "peers_server_start": (C.c_int, [_vp, C.POINTER(peers_server_opts), C.POINTER(_vp)]),
    "peers_server_submit": (C.c_int, [_vp, _vp, C.c_int64, _i32p, _i32p, _f64p, C.POINTER(C.c_uint64)]),
    "peers_server_wait": (C.c_int, [_vp, C.c_uint64, C.c_int64, C.POINTER(C.c_int)]),
    "peers_server_cancel": (C.c_int, [_vp, C.c_uint64]),
    "peers_server_stats_get": (C.c_int, [_vp, C.POINTER(peers_server_stats)]),
    "peers_server_stop": (C.c_int, [_vp]),
    "peers_cpu_query": (C.c_int, [_vp, C.c_int64, _i32p, _i32p, C.c_int32, _f64p, C.POINTER(peers_cpu_stats)]),
    "peers_status_string": (C.c_char_p, [C.c_int]),
    "peers_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """Load libpeers.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libpeers.so not built at {LIB_PATH}; run paper_2606_31535_amd.build_lib")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status, where):
    if status != PEERS_OK:
        msg = lib().peers_last_error()
        raise PeersError(status, where, msg.decode() if msg else "")


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    h = getattr(stream, "cuda_stream", None)
    if h is not None:
        return int(h)
    raise TypeError("stream must be None, an int hipStream_t or a torch stream")


# edge count of every factor uploaded through this binding (all-edge outputs
# are checked against it); dropped on release
_FACTOR_EDGES = {}
_FACTOR_NODES = {}


def _is_tensor(x):
    return hasattr(x, "data_ptr") and hasattr(x, "is_contiguous") and not isinstance(x, np.ndarray)


def _ids(x, name):
    """(pointer, is_device, keep-alive object, length) of a 1-D node-id array.

    Host arrays of any integer type are converted to contiguous int32 (ids
    that do not fit raise); torch tensors are passed as they are and must be
    contiguous 1-D int32, since a device tensor cannot be converted here
    without a copy the caller would not see.
    """
    if _is_tensor(x):
        if x.dim() != 1 or not x.is_contiguous() or str(x.dtype) != "torch.int32":
            raise ValueError(f"{name}: a tensor of node ids must be contiguous 1-D torch.int32 "
                             f"(got {x.dtype}, shape {tuple(x.shape)})")
        return int(x.data_ptr()), bool(x.is_cuda), x, int(x.shape[0])
    a = np.asarray(x)
    if a.ndim != 1:
        raise ValueError(f"{name}: node ids must be a 1-D array")
    if a.dtype != np.int32:
        if a.size and not np.issubdtype(a.dtype, np.integer):
            raise ValueError(f"{name}: node ids must be integers (got {a.dtype})")
        b = a.astype(np.int32)
        if not np.array_equal(b, a):
            raise ValueError(f"{name}: node ids do not fit 32 bits")
        a = b
    a = np.ascontiguousarray(a)
    return a.ctypes.data, False, a, int(a.shape[0])


def _out(x, n, name):
    """(pointer, is_device) of a resistance output: contiguous 1-D float64 of length n."""
    if _is_tensor(x):
        if str(x.dtype) != "torch.float64" or x.dim() != 1 or not x.is_contiguous():
            raise ValueError(f"{name}: output tensor must be contiguous 1-D torch.float64 "
                             f"(got {x.dtype}, shape {tuple(x.shape)})")
        if int(x.shape[0]) != n:
            raise ValueError(f"{name}: output holds {int(x.shape[0])} values, the call writes {n}")
        return int(x.data_ptr()), bool(x.is_cuda)
    if isinstance(x, np.ndarray):
        if x.dtype != np.float64 or x.ndim != 1 or not x.flags.c_contiguous or not x.flags.writeable:
            raise ValueError(f"{name}: output array must be writeable contiguous 1-D float64 "
                             f"(got {x.dtype}, shape {x.shape})")
        if x.shape[0] != n:
            raise ValueError(f"{name}: output holds {x.shape[0]} values, the call writes {n}")
        return x.ctypes.data, False
    raise TypeError(f"{name}: expected a numpy array or a torch tensor")


def _factor_edges(f):
    key = f.value if isinstance(f, C.c_void_p) else int(f)
    if key not in _FACTOR_EDGES:
        raise ValueError("unknown factor handle (upload factors with peers_factor_upload)")
    return _FACTOR_EDGES[key]


# --------------------------------------------------------------------------- graph

def peers_graph_create(n, eu, ev, w, ground=0, coords=None, ordering=PEERS_ORDER_AUTO,
                       given_order=None, threads=0, leaf_size=0, store_offsets_64=False, numeric_on_device=False,
                       sweep_only=False):
    eu, ev, w = _i32(eu), _i32(ev), _f64(w)
    if not (eu.shape == ev.shape == w.shape):
        raise ValueError("eu, ev, w must have the same length")
    opts = peers_graph_opts()
    opts.ordering = ordering
    keep = []
    if coords is not None:
        c = _f64(coords).reshape(n, 3)
        keep.append(c)
        opts.coords = _ptr(c, C.c_double)
    if given_order is not None:
        go = _i32(given_order)
        keep.append(go)
        opts.given_order = _ptr(go, C.c_int32)
    opts.threads = threads
    opts.leaf_size = leaf_size
    opts.store_offsets_64 = 1 if store_offsets_64 else 0
    opts.numeric_on_device = 1 if numeric_on_device else 0
    opts.sweep_only = 1 if sweep_only else 0
    h = _vp()
    _check(lib().peers_graph_create(int(n), int(eu.shape[0]), _ptr(eu, C.c_int32), _ptr(ev, C.c_int32),
                                    _ptr(w, C.c_double), int(ground), C.byref(opts), C.byref(h)),
           "peers_graph_create")
    return h


def peers_graph_stats_get(g) -> dict:
    s = peers_graph_stats()
    _check(lib().peers_graph_stats_get(g, C.byref(s)), "peers_graph_stats_get")
    return s.as_dict()


def peers_graph_export_symbolic(g):
    st = peers_graph_stats_get(g)
    N, nnz, ns = st["N"], st["nnz_l"], st["n_supernodes"]
    perm = np.empty(N, np.int32)
    parent = np.empty(N, np.int32)
    colptr = np.empty(N + 1, np.int64)
    rowidx = np.empty(nnz, np.int32)
    snptr = np.empty(ns + 1, np.int32)
    _check(lib().peers_graph_export_symbolic(g, _ptr(perm, C.c_int32), _ptr(parent, C.c_int32),
                                             _ptr(colptr, C.c_int64), _ptr(rowidx, C.c_int32),
                                             _ptr(snptr, C.c_int32)), "peers_graph_export_symbolic")
    return {"perm": perm, "parent": parent, "colptr": colptr, "rowidx": rowidx, "snptr": snptr}


def peers_graph_export_factor(g):
    st = peers_graph_stats_get(g)
    Lx = np.empty(st["nnz_l"], np.float64)
    D = np.empty(st["N"], np.float64)
    _check(lib().peers_graph_export_factor(g, _ptr(Lx, C.c_double), _ptr(D, C.c_double)),
           "peers_graph_export_factor")
    return Lx, D


def peers_graph_destroy(g):
    if g:
        lib().peers_graph_destroy(g)


# --------------------------------------------------------------------------- device

def peers_device_open(ordinal=0, hbm_budget_bytes=0):
    h = _vp()
    _check(lib().peers_device_open(int(ordinal), int(hbm_budget_bytes), C.byref(h)), "peers_device_open")
    return h


def peers_device_close(d):
    if d:
        lib().peers_device_close(d)


def peers_device_usage(d):
    used, budget = C.c_uint64(), C.c_uint64()
    _check(lib().peers_device_usage(d, C.byref(used), C.byref(budget)), "peers_device_usage")
    return used.value, budget.value


def peers_device_set_budget(d, hbm_budget_bytes):
    _check(lib().peers_device_set_budget(d, int(hbm_budget_bytes)), "peers_device_set_budget")


def peers_factor_upload(d, g, stream=None):
    st = peers_graph_stats_get(g)
    h = _vp()
    _check(lib().peers_factor_upload(d, g, _stream_handle(stream), C.byref(h)), "peers_factor_upload")
    _FACTOR_EDGES[h.value] = int(st["m"])
    _FACTOR_NODES[h.value] = int(st["n"])
    return h


def peers_factor_release(f):
    if f:
        _FACTOR_EDGES.pop(f.value if isinstance(f, C.c_void_p) else int(f), None)
        _FACTOR_NODES.pop(f.value if isinstance(f, C.c_void_p) else int(f), None)
        lib().peers_factor_release(f)


def peers_factor_footprint(f):
    a, b = C.c_uint64(), C.c_uint64()
    _check(lib().peers_factor_footprint(f, C.byref(a), C.byref(b)), "peers_factor_footprint")
    return a.value, b.value


def peers_factor_timings(f) -> dict:
    o = peers_sweep_timings()
    _check(lib().peers_factor_timings(f, C.byref(o)), "peers_factor_timings")
    return o.as_dict()


def peers_factor_export_columns(f, nodes, ld, stream=None):
    """Columns of Z = D^{-1/2} L^{-1} as one sweep forms them, depth-indexed (k x ld)."""
    nodes = _i32(nodes)
    Z = np.empty((nodes.shape[0], int(ld)), np.float64)
    _check(lib().peers_factor_export_columns(f, int(nodes.shape[0]), _ptr(nodes, C.c_int32), int(ld),
                                             _ptr(Z, C.c_double), _stream_handle(stream)),
           "peers_factor_export_columns")
    return Z


def peers_query_all_edges(f, R_out, flags=0, stream=None):
    p, dev = _out(R_out, _factor_edges(f), "R_out")
    if dev:
        flags |= PEERS_OUT_DEVICE
    _check(lib().peers_query_all_edges(f, p, flags, _stream_handle(stream)), "peers_query_all_edges")
    return R_out


def peers_query_all_to_ground(f, R_out, flags=0, stream=None):
    """R_out[x] = resistance between node x and the ground, for every node (n values)."""
    key = f.value if isinstance(f, C.c_void_p) else int(f)
    if key not in _FACTOR_NODES:
        raise ValueError("unknown factor handle (upload factors with peers_factor_upload)")
    p, dev = _out(R_out, _FACTOR_NODES[key], "R_out")
    if dev:
        flags |= PEERS_OUT_DEVICE
    _check(lib().peers_query_all_to_ground(f, p, flags, _stream_handle(stream)), "peers_query_all_to_ground")
    return R_out


def peers_query(f, qu, qv, R_out, flags=0, stream=None):
    pu, du, ku, q = _ids(qu, "qu")
    pv, dv, kv, qv_len = _ids(qv, "qv")
    if q != qv_len:
        raise ValueError(f"qu has {q} ids and qv {qv_len}")
    pr, dr = _out(R_out, q, "R_out")
    if du != dv:
        raise ValueError("qu and qv must live on the same side")
    if du:
        flags |= PEERS_IN_DEVICE
    if dr:
        flags |= PEERS_OUT_DEVICE
    _check(lib().peers_query(f, q, pu, pv, pr, flags, _stream_handle(stream)), "peers_query")
    return R_out


def peers_query_noalloc(f, qu, qv, R_out, flags=0, stream=None):
    """peers_query without any device allocation (fixed per-GPU scratch array)."""
    pu, du, ku, q = _ids(qu, "qu")
    pv, dv, kv, qv_len = _ids(qv, "qv")
    if q != qv_len:
        raise ValueError(f"qu has {q} ids and qv {qv_len}")
    pr, dr = _out(R_out, q, "R_out")
    if du != dv:
        raise ValueError("qu and qv must live on the same side")
    if du:
        flags |= PEERS_IN_DEVICE
    if dr:
        flags |= PEERS_OUT_DEVICE
    _check(lib().peers_query_noalloc(f, q, pu, pv, pr, flags, _stream_handle(stream)), "peers_query_noalloc")
    return R_out


def peers_batch_query(d, factors, qus, qvs, R_outs, flags=0, stream=None):
    """Batched sweep of several factors; qus[i] None means all edges of factor i."""
    nb = len(factors)
    fa = (_vp * nb)(*factors)
    qa = (C.c_int64 * nb)()
    ua = (_vp * nb)()
    va = (_vp * nb)()
    ra = (_vp * nb)()
    devs = set()
    ins = set()
    keep = []
    for i in range(nb):
        if qus[i] is None:
            ua[i] = None
            va[i] = None
            qa[i] = 0
            n_out = _factor_edges(factors[i])
        else:
            pu, du, ku, q = _ids(qus[i], f"qus[{i}]")
            pv, dv, kv, q2 = _ids(qvs[i], f"qvs[{i}]")
            if q != q2:
                raise ValueError(f"qus[{i}] has {q} ids and qvs[{i}] {q2}")
            keep += [ku, kv]
            ins.update((du, dv))
            ua[i] = pu
            va[i] = pv
            qa[i] = q
            n_out = q
        p, dev = _out(R_outs[i], n_out, f"R_outs[{i}]")
        ra[i] = p
        devs.add(dev)
        if dev:
            flags |= PEERS_OUT_DEVICE
    if len(devs) > 1:
        raise ValueError("all outputs of a batch must be host arrays or all device tensors")
    if len(ins) > 1:
        raise ValueError("all pair lists of a batch must be host arrays or all device tensors")
    if True in ins:
        flags |= PEERS_IN_DEVICE
    _check(lib().peers_batch_query(d, nb, fa, qa, ua, va, ra, flags, _stream_handle(stream)), "peers_batch_query")
    return R_outs


def _vals(x, n, name):
    """(pointer, is_device, keep-alive) of a 1-D float64 input of length n."""
    if _is_tensor(x):
        if str(x.dtype) != "torch.float64" or x.dim() != 1 or not x.is_contiguous() or int(x.shape[0]) != n:
            raise ValueError(f"{name}: expected a contiguous 1-D torch.float64 tensor of length {n}")
        return int(x.data_ptr()), bool(x.is_cuda), x
    a = np.ascontiguousarray(x, dtype=np.float64)
    if a.ndim != 1 or a.shape[0] != n:
        raise ValueError(f"{name}: expected {n} values")
    return a.ctypes.data, False, a


def peers_sparsify(d, w, R, q, seed, count, w_new, flags=0, stream=None):
    """Algorithm 1: draw q edges with probability proportional to w_e R_e (see include/peers.h)."""
    m = int(len(w))
    pw, dw, kw = _vals(w, m, "w")
    pR, dR, kR = _vals(R, m, "R")
    if dw != dR:
        raise ValueError("w and R must live on the same side")
    if _is_tensor(count):
        ok = str(count.dtype) == "torch.int32" and count.dim() == 1 and count.is_contiguous() and count.shape[0] == m
        pc, dc = int(count.data_ptr()), bool(count.is_cuda)
    else:
        ok = isinstance(count, np.ndarray) and count.dtype == np.int32 and count.ndim == 1 and \
            count.flags.c_contiguous and count.shape[0] == m
        pc, dc = (count.ctypes.data if ok else 0), False
    if not ok:
        raise ValueError(f"count: expected a contiguous 1-D int32 array of length {m}")
    pn, dn = _out(w_new, m, "w_new")
    if dc != dn:
        raise ValueError("count and w_new must live on the same side")
    if dw:
        flags |= PEERS_IN_DEVICE
    if dn:
        flags |= PEERS_OUT_DEVICE
    _check(lib().peers_sparsify(d, m, pw, pR, int(q), int(seed), pc, pn, flags, _stream_handle(stream)),
           "peers_sparsify")
    return count, w_new


def peers_batch_last_info(d) -> dict:
    o = peers_batch_info()
    _check(lib().peers_batch_last_info(d, C.byref(o)), "peers_batch_last_info")
    return o.as_dict()


def peers_server_start(d, max_batch_pairs=0, max_wait_us=0, queue_capacity=0, streams=0):
    o = peers_server_opts(max_batch_pairs, max_wait_us, queue_capacity, streams)
    h = _vp()
    _check(lib().peers_server_start(d, C.byref(o), C.byref(h)), "peers_server_start")
    return h


def peers_server_submit(s, f, qu, qv, R_out):
    """Enqueue a request; R_out (host float64, length q) must stay alive until a
    peers_server_wait on the ticket returns PEERS_OK (or the server stops)."""
    pu, du, ku, q = _ids(qu, "qu")
    pv, dv, kv, q2 = _ids(qv, "qv")
    if du or dv:
        raise ValueError("server requests take host node ids")
    if q != q2:
        raise ValueError(f"qu has {q} ids and qv {q2}")
    pr, dr = _out(R_out, q, "R_out")
    if dr:
        raise ValueError("server results go to host memory")
    t = C.c_uint64()
    _check(lib().peers_server_submit(s, f, q, C.cast(pu, _i32p), C.cast(pv, _i32p), C.cast(pr, _f64p),
                                     C.byref(t)), "peers_server_submit")
    return t.value, (ku, kv, R_out)


def peers_server_wait(s, ticket, timeout_us=-1):
    r = C.c_int()
    st = lib().peers_server_wait(s, int(ticket), int(timeout_us), C.byref(r))
    return st, r.value


def peers_server_cancel(s, ticket):
    _check(lib().peers_server_cancel(s, int(ticket)), "peers_server_cancel")


def peers_server_stats_get(s) -> dict:
    o = peers_server_stats()
    _check(lib().peers_server_stats_get(s, C.byref(o)), "peers_server_stats_get")
    return o.as_dict()


def peers_server_stop(s):
    if s:
        _check(lib().peers_server_stop(s), "peers_server_stop")


def peers_cpu_query(g, qu, qv, R_out, threads=0):
    """The paper's CPU scheme (include/peers_cpu.h) on the graph's host factor; returns its statistics."""
    pu, du, ku, q = _ids(qu, "qu")
    pv, dv, kv, q2 = _ids(qv, "qv")
    if du or dv or q != q2:
        raise ValueError("host node ids of equal length expected")
    pr, dr = _out(R_out, q, "R_out")
    if dr:
        raise ValueError("the CPU scheme writes host memory")
    st = peers_cpu_stats()
    _check(lib().peers_cpu_query(g, q, C.cast(pu, _i32p), C.cast(pv, _i32p), int(threads), C.cast(pr, _f64p),
                                 C.byref(st)), "peers_cpu_query")
    return st.as_dict()


def peers_status_string(st) -> str:
    return lib().peers_status_string(int(st)).decode()


def peers_last_error() -> str:
    m = lib().peers_last_error()
    return m.decode() if m else ""
