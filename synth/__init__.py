"""Seeded synthetic workloads: graphs, ground nodes and query sets.

This module only builds inputs. It holds none of the effective-resistance
arithmetic, so both the product path and the CPU oracle may draw their inputs
from it. Every generator is deterministic in its seed (numpy ``PCG64``).

Workload shapes follow the paper's evaluation set (Section V-A): multi-layer
power-delivery-network meshes with alternating wire direction and vias stand in
for the IBM power-grid benchmarks, and random geometric graphs give many
graphs of uneven size for the batched form. The real matrices are not
available here; these are stand-ins of the same structure and scale.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

__all__ = [
    "Graph", "rng_for", "mesh2d", "pdn_two_layer", "pdn_multilayer", "rgg_knn",
    "rgg_batch", "served_trace", "path_graph", "star_graph", "cycle_graph",
    "complete_graph", "complete_bipartite", "torus2d", "torus3d", "hypercube",
    "grid_unit", "random_tree", "random_connected", "add_pendants",
    "random_pairs", "components", "CONFIG_SEEDS",
]

# numpy PCG64 seeds per workload (C1..C5); graph k of the batched set uses 40000+k
CONFIG_SEEDS = {"C1": 1000, "C2": 1001, "C3": 1002, "C4": 1003, "C5": 1004}


@dataclasses.dataclass
class Graph:
    """An undirected weighted multigraph given as an edge list.

    ``eu``/``ev`` are int32 endpoint ids in ``[0, n)``, ``w`` float64
    conductances (> 0). ``coords`` optionally holds float64 point coordinates
    of shape ``(n, 3)`` (mesh x, y, layer; or RGG x, y, 0). ``ground`` is the
    grounded node id.
    """
    n: int
    eu: np.ndarray
    ev: np.ndarray
    w: np.ndarray
    ground: int = 0
    coords: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.eu.shape[0])

    def scaled(self, factor: float) -> "Graph":
        return dataclasses.replace(self, w=self.w * factor, name=self.name + f"*{factor}")

    def relabeled(self, perm: np.ndarray) -> "Graph":
        """Return the same graph with node id x renamed to perm[x]."""
        perm = np.asarray(perm, dtype=np.int64)
        coords = None
        if self.coords is not None:
            coords = np.empty_like(self.coords)
            coords[perm] = self.coords
        return dataclasses.replace(
            self, eu=perm[self.eu].astype(np.int32), ev=perm[self.ev].astype(np.int32),
            ground=int(perm[self.ground]), coords=coords, name=self.name + "~relabel")


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _mk(n, eu, ev, w, ground=0, coords=None, name="", **meta) -> Graph:
    return Graph(n=int(n), eu=np.ascontiguousarray(eu, dtype=np.int32),
                 ev=np.ascontiguousarray(ev, dtype=np.int32),
                 w=np.ascontiguousarray(w, dtype=np.float64), ground=int(ground),
                 coords=None if coords is None else np.ascontiguousarray(coords, dtype=np.float64),
                 name=name, meta=dict(meta))


# ----------------------------------------------------------------------------
# connectivity helpers (graph structure only)

def components(n: int, eu: np.ndarray, ev: np.ndarray) -> np.ndarray:
    """Component label per node (union-find with path halving)."""
    parent = np.arange(n, dtype=np.int64)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    # vectorised label propagation is simpler for large graphs
    if n > 5000:
        import scipy.sparse as sp
        import scipy.sparse.csgraph as csg
        a = sp.coo_matrix((np.ones(len(eu)), (eu, ev)), shape=(n, n))
        _, lab = csg.connected_components(a, directed=False)
        return lab.astype(np.int64)
    for a, b in zip(eu.tolist(), ev.tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    return np.array([find(x) for x in range(n)], dtype=np.int64)


def _repair(n, eu, ev, w, coords, weight_fn: Callable[[float], float]):
    """Join every non-giant component to the largest one by one edge.

    The new edge links the closest pair of points (Euclidean, on ``coords``)
    between the component and the giant component; its conductance is
    ``weight_fn(distance)``. Returns the new arrays and the number of edges added.
    """
    lab = components(n, eu, ev)
    labels, counts = np.unique(lab, return_counts=True)
    if len(labels) == 1:
        return eu, ev, w, 0
    from scipy.spatial import cKDTree
    giant = labels[np.argmax(counts)]
    gidx = np.nonzero(lab == giant)[0]
    tree = cKDTree(coords[gidx])
    add_u, add_v, add_w = [], [], []
    for c in labels:
        if c == giant:
            continue
        cidx = np.nonzero(lab == c)[0]
        d, j = tree.query(coords[cidx], k=1)
        t = int(np.argmin(d))
        add_u.append(int(cidx[t]))
        add_v.append(int(gidx[j[t]]))
        add_w.append(weight_fn(float(d[t])))
    eu = np.concatenate([eu, np.array(add_u, dtype=np.int64)])
    ev = np.concatenate([ev, np.array(add_v, dtype=np.int64)])
    w = np.concatenate([w, np.array(add_w, dtype=np.float64)])
    return eu, ev, w, len(add_u)


# ----------------------------------------------------------------------------
# evaluation workloads

def mesh2d(nx: int = 32, ny: int = 32, seed: int = CONFIG_SEEDS["C1"], ground: int = 0) -> Graph:
    """4-neighbour nx-by-ny mesh, conductances 10**U(-1,1) (log-uniform in [0.1, 10])."""
    rng = rng_for(seed)
    idx = np.arange(nx * ny).reshape(ny, nx)
    hu, hv = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    vu, vv = idx[:-1, :].ravel(), idx[1:, :].ravel()
    eu = np.concatenate([hu, vu])
    ev = np.concatenate([hv, vv])
    w = 10.0 ** rng.uniform(-1.0, 1.0, size=eu.shape[0])
    yy, xx = np.divmod(np.arange(nx * ny), nx)
    coords = np.stack([xx, yy, np.zeros_like(xx)], axis=1).astype(np.float64)
    return _mk(nx * ny, eu, ev, w, ground, coords, name=f"mesh{nx}x{ny}", seed=seed)


def pdn_two_layer(side: int = 512, seed: int = CONFIG_SEEDS["C2"], via_frac: float = 0.10,
                  via_g: float = 50.0, ground: int = 0) -> Graph:
    """Two-layer power-grid mesh: horizontal wires on layer 1, vertical on layer 2.

    Wire conductance max(N(5,1), 0.1); vias (conductance ``via_g``) at a random
    ``via_frac`` of the grid points join the two layers.
    """
    rng = rng_for(seed)
    s2 = side * side
    idx = np.arange(s2).reshape(side, side)  # [y, x]
    hu, hv = idx[:, :-1].ravel(), idx[:, 1:].ravel()              # layer 1, along x
    vu, vv = s2 + idx[:-1, :].ravel(), s2 + idx[1:, :].ravel()    # layer 2, along y
    nw = hu.shape[0] + vu.shape[0]
    wires = np.maximum(rng.normal(5.0, 1.0, size=nw), 0.1)
    nvia = int(round(via_frac * s2))
    pts = np.sort(rng.choice(s2, size=nvia, replace=False))
    eu = np.concatenate([hu, vu, pts])
    ev = np.concatenate([hv, vv, pts + s2])
    w = np.concatenate([wires, np.full(nvia, via_g)])
    n = 2 * s2
    yy, xx = np.divmod(np.arange(s2), side)
    coords = np.concatenate([np.stack([xx, yy, np.zeros(s2)], 1), np.stack([xx, yy, np.ones(s2)], 1)])
    eu, ev, w, added = _repair(n, eu, ev, w, coords, lambda d: via_g)
    return _mk(n, eu, ev, w, ground, coords, name=f"pdn2x{side}", seed=seed, repaired=added)


def pdn_multilayer(side: int = 500, layers: int = 4, seed: int = CONFIG_SEEDS["C3"],
                   via_frac: float = 0.05, via_g: float = 100.0, long_frac: float = 0.001,
                   long_g: float = 0.01, ground: int = 0) -> Graph:
    """Multi-layer power-grid mesh with alternating wire direction.

    Layer l (1-based) runs along x when l is odd and along y when even; each
    wire segment has conductance 2**(l-1) * 2**U(-1,1) (log-uniform in
    [0.5, 2] times the layer multiplier 1, 2, 4, 8, ...). For every adjacent
    layer pair, vias of conductance ``via_g`` sit on a random ``via_frac`` of the
    (x, y) points. ``long_frac * n`` random long edges of conductance ``long_g``
    join uniformly drawn node pairs that are neither equal nor already adjacent.
    """
    rng = rng_for(seed)
    s2 = side * side
    idx = np.arange(s2).reshape(side, side)
    parts_u, parts_v, parts_w = [], [], []
    for l in range(layers):
        base = l * s2
        if l % 2 == 0:
            u, v = idx[:, :-1].ravel(), idx[:, 1:].ravel()
        else:
            u, v = idx[:-1, :].ravel(), idx[1:, :].ravel()
        g = (2.0 ** l) * 2.0 ** rng.uniform(-1.0, 1.0, size=u.shape[0])
        parts_u.append(base + u)
        parts_v.append(base + v)
        parts_w.append(g)
    nvia = int(round(via_frac * s2))
    for l in range(layers - 1):
        pts = np.sort(rng.choice(s2, size=nvia, replace=False))
        parts_u.append(l * s2 + pts)
        parts_v.append((l + 1) * s2 + pts)
        parts_w.append(np.full(nvia, via_g))
    eu = np.concatenate(parts_u).astype(np.int64)
    ev = np.concatenate(parts_v).astype(np.int64)
    w = np.concatenate(parts_w)
    n = layers * s2
    nlong = int(round(long_frac * n))
    if nlong:
        existing = set((np.minimum(eu, ev) * n + np.maximum(eu, ev)).tolist())
        lu, lv = [], []
        while len(lu) < nlong:
            a, b = (int(x) for x in rng.integers(0, n, size=2))
            if a == b:
                continue
            key = min(a, b) * n + max(a, b)
            if key in existing:
                continue
            existing.add(key)
            lu.append(a)
            lv.append(b)
        eu = np.concatenate([eu, np.array(lu, dtype=np.int64)])
        ev = np.concatenate([ev, np.array(lv, dtype=np.int64)])
        w = np.concatenate([w, np.full(nlong, long_g)])
    yy, xx = np.divmod(np.arange(s2), side)
    coords = np.concatenate([np.stack([xx, yy, np.full(s2, l)], 1) for l in range(layers)]).astype(np.float64)
    eu, ev, w, added = _repair(n, eu, ev, w, coords, lambda d: via_g)
    return _mk(n, eu, ev, w, ground, coords, name=f"pdn{layers}x{side}", seed=seed,
               repaired=added, long_edges=nlong)


def rgg_knn(n: int, k: int = 6, seed: int = 40000, ground: int = 0) -> Graph:
    """Random geometric graph: n uniform points in the unit square.

    Edge (a, b) exists when either point is among the other's k nearest
    neighbours; conductance 1/distance. Disconnected pieces are joined to the
    largest component by their closest pair of points (conductance 1/distance).
    """
    from scipy.spatial import cKDTree
    rng = rng_for(seed)
    pts = rng.uniform(0.0, 1.0, size=(n, 2))
    tree = cKDTree(pts)
    d, j = tree.query(pts, k=k + 1)
    a = np.repeat(np.arange(n), k)
    b = j[:, 1:].ravel()
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = np.unique(lo.astype(np.int64) * n + hi)
    eu, ev = np.divmod(key, n)
    dist = np.linalg.norm(pts[eu] - pts[ev], axis=1)
    w = 1.0 / dist
    coords = np.concatenate([pts, np.zeros((n, 1))], axis=1)
    eu, ev, w, added = _repair(n, eu, ev, w, coords, lambda dd: 1.0 / dd)
    return _mk(n, eu, ev, w, ground, coords, name=f"rgg{n}", seed=seed, repaired=added)


def rgg_batch(count: int = 256, base_seed: int = 40000, nmin: int = 2000, nmax: int = 50000,
              k: int = 6) -> list:
    """The batched workload: ``count`` RGGs, graph i seeded PCG64(base_seed + i), n ~ U{nmin..nmax}."""
    out = []
    for i in range(count):
        n = int(rng_for(base_seed + i).integers(nmin, nmax + 1))
        out.append(rgg_knn(n, k=k, seed=base_seed + i))
    return out


def served_trace(graphs: list, nreq: int, qps: float, seed: int = CONFIG_SEEDS["C5"],
                 max_pairs: int = 100000, edge_frac: float = 0.8):
    """Poisson request stream over resident graphs.

    Each request picks a graph uniformly, has size floor(exp(U(0, ln(max_pairs+1))))
    clipped to [1, max_pairs]; a fraction ``edge_frac`` of its pairs are uniformly
    sampled existing edges, the rest uniform node pairs u != v. Returns a list of
    dicts with arrival time (s), graph index and int32 endpoint arrays.
    """
    rng = rng_for(seed)
    t = 0.0
    reqs = []
    for r in range(nreq):
        t += rng.exponential(1.0 / qps)
        gi = int(rng.integers(0, len(graphs)))
        g = graphs[gi]
        size = int(math.floor(math.exp(rng.uniform(0.0, math.log(max_pairs + 1)))))
        size = max(1, min(max_pairs, size))
        ne = int(round(edge_frac * size))
        ei = rng.integers(0, g.m, size=ne)
        qu = [g.eu[ei]]
        qv = [g.ev[ei]]
        nr = size - ne
        if nr:
            a = rng.integers(0, g.n, size=nr)
            b = rng.integers(0, g.n - 1, size=nr)
            b = b + (b >= a)
            qu.append(a)
            qv.append(b)
        reqs.append({"t": t, "graph": gi, "qu": np.concatenate(qu).astype(np.int32),
                     "qv": np.concatenate(qv).astype(np.int32)})
    return reqs


def random_pairs(n: int, count: int, seed: int, distinct: bool = True):
    rng = rng_for(seed)
    a = rng.integers(0, n, size=count)
    if distinct:
        b = rng.integers(0, n - 1, size=count)
        b = b + (b >= a)
    else:
        b = rng.integers(0, n, size=count)
    return a.astype(np.int32), b.astype(np.int32)


# ----------------------------------------------------------------------------
# families with known answers (closed forms live in the tests, not here)

def path_graph(n: int, w=None, ground: int = 0) -> Graph:
    eu = np.arange(n - 1)
    ev = eu + 1
    w = np.ones(n - 1) if w is None else np.asarray(w, dtype=np.float64)
    return _mk(n, eu, ev, w, ground, name=f"path{n}")


def star_graph(n: int, w=None, center: int = 0, ground: int = 0) -> Graph:
    leaves = np.array([x for x in range(n) if x != center])
    eu = np.full(n - 1, center)
    w = np.ones(n - 1) if w is None else np.asarray(w, dtype=np.float64)
    return _mk(n, eu, leaves, w, ground, name=f"star{n}")


def cycle_graph(n: int, w: float = 1.0, ground: int = 0) -> Graph:
    eu = np.arange(n)
    ev = (eu + 1) % n
    return _mk(n, eu, ev, np.full(n, w), ground, name=f"cycle{n}")


def complete_graph(n: int, w: float = 1.0, ground: int = 0) -> Graph:
    a, b = np.triu_indices(n, 1)
    return _mk(n, a, b, np.full(a.shape[0], w), ground, name=f"K{n}")


def complete_bipartite(a: int, b: int, w: float = 1.0, ground: int = 0) -> Graph:
    u, v = np.meshgrid(np.arange(a), a + np.arange(b), indexing="ij")
    return _mk(a + b, u.ravel(), v.ravel(), np.full(a * b, w), ground, name=f"K{a},{b}")


def torus2d(k: int, w: float = 1.0, ground: int = 0) -> Graph:
    idx = np.arange(k * k).reshape(k, k)
    eu = np.concatenate([idx.ravel(), idx.ravel()])
    ev = np.concatenate([np.roll(idx, -1, axis=1).ravel(), np.roll(idx, -1, axis=0).ravel()])
    yy, xx = np.divmod(np.arange(k * k), k)
    coords = np.stack([xx, yy, np.zeros(k * k)], 1).astype(np.float64)
    return _mk(k * k, eu, ev, np.full(eu.shape[0], w), ground, coords, name=f"torus{k}x{k}")


def torus3d(k: int, w: float = 1.0, ground: int = 0) -> Graph:
    idx = np.arange(k ** 3).reshape(k, k, k)
    eu = np.concatenate([idx.ravel()] * 3)
    ev = np.concatenate([np.roll(idx, -1, axis=ax).ravel() for ax in range(3)])
    zz, rem = np.divmod(np.arange(k ** 3), k * k)
    yy, xx = np.divmod(rem, k)
    coords = np.stack([xx, yy, zz], 1).astype(np.float64)
    return _mk(k ** 3, eu, ev, np.full(eu.shape[0], w), ground, coords, name=f"torus3d{k}")


def hypercube(d: int, w: float = 1.0, ground: int = 0) -> Graph:
    n = 1 << d
    us, vs = [], []
    for bit in range(d):
        u = np.array([x for x in range(n) if not (x >> bit) & 1])
        us.append(u)
        vs.append(u | (1 << bit))
    return _mk(n, np.concatenate(us), np.concatenate(vs), np.full(d * n // 2, w), ground, name=f"Q{d}")


def grid_unit(a: int, b: int, ground: int = 0) -> Graph:
    """Unit-conductance a-by-b grid (path P_a times path P_b), node id = y*a + x."""
    idx = np.arange(a * b).reshape(b, a)
    eu = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    ev = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    yy, xx = np.divmod(np.arange(a * b), a)
    coords = np.stack([xx, yy, np.zeros(a * b)], 1).astype(np.float64)
    return _mk(a * b, eu, ev, np.ones(eu.shape[0]), ground, coords, name=f"grid{a}x{b}")


def random_tree(n: int, seed: int, wlog: float = 3.0, ground: int = 0) -> Graph:
    rng = rng_for(seed)
    parent = np.array([int(rng.integers(0, i)) for i in range(1, n)], dtype=np.int64)
    w = 10.0 ** rng.uniform(-wlog, wlog, size=n - 1)
    return _mk(n, np.arange(1, n), parent, w, ground, name=f"tree{n}")


def random_connected(n: int, extra: int, seed: int, wlog: float = 3.0, dyadic: bool = False,
                     ground: int = 0, multi: bool = False) -> Graph:
    """Random spanning tree plus ``extra`` random edges (parallel edges if ``multi``).

    Weights are log-uniform over 10**[-wlog, wlog], or with ``dyadic`` small
    powers of two times small odd integers (exactly representable).
    """
    rng = rng_for(seed)
    order = rng.permutation(n)
    eu = [int(order[i]) for i in range(1, n)]
    ev = [int(order[int(rng.integers(0, i))]) for i in range(1, n)]
    seen = set((min(a, b), max(a, b)) for a, b in zip(eu, ev))
    tries = 0
    while extra > 0 and tries < 100 * (extra + 1):
        tries += 1
        a, b = (int(x) for x in rng.integers(0, n, size=2))
        if a == b:
            continue
        key = (min(a, b), max(a, b))
        if key in seen and not multi:
            continue
        seen.add(key)
        eu.append(a)
        ev.append(b)
        extra -= 1
    m = len(eu)
    if dyadic:
        w = rng.integers(1, 8, size=m) * 2.0 ** rng.integers(-3, 4, size=m)
    else:
        w = 10.0 ** rng.uniform(-wlog, wlog, size=m)
    return _mk(n, eu, ev, w.astype(np.float64), ground, name=f"rand{n}+{extra}")


def add_pendants(g: Graph, count: int, seed: int, wlog: float = 1.0) -> tuple:
    """Attach ``count`` new degree-1 nodes to random existing nodes.

    Returns (new graph, int array of the indices of the added edges).
    """
    rng = rng_for(seed)
    hosts = rng.integers(0, g.n, size=count)
    new = g.n + np.arange(count)
    w = 10.0 ** rng.uniform(-wlog, wlog, size=count)
    eu = np.concatenate([g.eu.astype(np.int64), new])
    ev = np.concatenate([g.ev.astype(np.int64), hosts])
    ww = np.concatenate([g.w, w])
    coords = None
    if g.coords is not None:
        coords = np.concatenate([g.coords, g.coords[hosts] + np.array([0.25, 0.25, 0.0])])
    ng = _mk(g.n + count, eu, ev, ww, g.ground, coords, name=g.name + f"+{count}pend", **g.meta)
    return ng, g.m + np.arange(count)
