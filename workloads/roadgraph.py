"""Seeded synthetic road networks and vehicle origin/destination sets.

Stand-ins for the paper's North-West Delhi network (Section 5: 52 nodes,
128 roads, sensor-reported densities), which is not available.  Every array is
drawn from a ``numpy.random.Generator`` seeded by the caller, so the same call
always yields the same bytes.

This module only *draws inputs*: topology, lengths, speeds, signal timings,
sensed vehicle counts and OD pairs.  It contains none of the routing method's
arithmetic (travel times, waits, weights, pheromone) -- both the CPU oracle and
the GPU library consume what it produces.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, dijkstra, minimum_spanning_tree


@dataclass
class RoadGraph:
    """A directed road graph in CSR form (out-edges of node u are
    ``row_ptr[u] .. row_ptr[u+1]-1``, head node ``col[e]``)."""

    row_ptr: np.ndarray      # uint32 [n+1]
    col: np.ndarray          # uint32 [m]  head node of each directed road
    len_dm: np.ndarray       # uint32 [m]  length in decimetres (>= 1)
    speed_kmh: np.ndarray    # uint16 [m]  free-flow speed
    green_pm: np.ndarray     # uint16 [m]  green share (per mille) of approach e at its head node
    cycle_ms: np.ndarray     # uint32 [n]  signal cycle at node; 0 = no signal
    x_dm: np.ndarray         # int32  [n]
    y_dm: np.ndarray         # int32  [n]
    base_load: np.ndarray    # uint32 [m]  sensed vehicles on each road
    inst_node_off: Optional[np.ndarray] = None   # uint32 [k+1] node ranges of packed instances

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def tail(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.uint32), np.diff(self.row_ptr.astype(np.int64)))

    def out_degree(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def validate(self) -> None:
        n, m = self.n, self.m
        rp = self.row_ptr.astype(np.int64)
        assert rp[0] == 0 and rp[-1] == m and np.all(np.diff(rp) >= 0)
        assert np.all(self.col < n)
        assert not np.any(self.col == self.tail()), "self-loop"
        assert np.all(self.len_dm >= 1) and np.all(self.speed_kmh >= 1)
        assert np.all(self.green_pm <= 1000)
        for a in (self.row_ptr, self.col, self.len_dm, self.base_load, self.cycle_ms):
            assert a.dtype == np.uint32 and a.flags.c_contiguous
        for a in (self.speed_kmh, self.green_pm):
            assert a.dtype == np.uint16 and a.flags.c_contiguous
        for a in (self.x_dm, self.y_dm):
            assert a.dtype == np.int32 and a.flags.c_contiguous


@dataclass
class Vehicles:
    """Routing queries: vehicle ``i`` is at ``src[i]`` heading to ``dst[i]``.
    ``qid`` names the vehicle's random stream and never depends on its position
    in a batch."""

    qid: np.ndarray   # uint32 [V]
    src: np.ndarray   # uint32 [V]
    dst: np.ndarray   # uint32 [V]

    def __len__(self) -> int:
        return int(self.src.shape[0])


@dataclass
class Workload:
    name: str
    graph: RoadGraph
    vehicles: Vehicles
    params: dict = field(default_factory=dict)


# ---------------------------------------------------------------------------
# assembling CSR from a list of directed roads
# ---------------------------------------------------------------------------

def _to_csr(n, tails, heads, len_dm, speed, base_load, cycle, x, y, green_fn) -> RoadGraph:
    tails = np.asarray(tails, dtype=np.int64)
    heads = np.asarray(heads, dtype=np.int64)
    order = np.lexsort((heads, tails))           # by tail, then head
    tails, heads = tails[order], heads[order]
    len_dm = np.asarray(len_dm)[order]
    speed = np.asarray(speed)[order]
    base_load = np.asarray(base_load)[order]
    counts = np.bincount(tails, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    green = green_fn(tails, heads)
    g = RoadGraph(
        row_ptr=row_ptr.astype(np.uint32),
        col=heads.astype(np.uint32),
        len_dm=np.ascontiguousarray(len_dm, dtype=np.uint32),
        speed_kmh=np.ascontiguousarray(speed, dtype=np.uint16),
        green_pm=np.ascontiguousarray(green, dtype=np.uint16),
        cycle_ms=np.ascontiguousarray(cycle, dtype=np.uint32),
        x_dm=np.ascontiguousarray(x, dtype=np.int32),
        y_dm=np.ascontiguousarray(y, dtype=np.int32),
        base_load=np.ascontiguousarray(base_load, dtype=np.uint32),
    )
    g.validate()
    return g


def _strongly_connected(n, tails, heads) -> bool:
    a = sp.csr_matrix((np.ones(len(tails), dtype=np.int8), (tails, heads)), shape=(n, n))
    k, _ = connected_components(a, directed=True, connection="strong")
    return k == 1


# ---------------------------------------------------------------------------
# grid cities
# ---------------------------------------------------------------------------

def grid_graph(rows: int, cols: int, rng: np.random.Generator, *, spacing_dm: int = 1000,
               remove_frac: float = 0.0, speed_kmh: int = 50, load_mean: float = 3.0) -> RoadGraph:
    """rows x cols lattice of signalised intersections, two-way roads between
    4-neighbours.  Node id = r*cols + c, coordinates on a ``spacing_dm`` lattice.

    * each road (both directions) has length U{spacing .. 5*spacing} dm, so no
      road is shorter than the straight line between its ends;
    * every directed road carries Poisson(load_mean) sensed vehicles;
    * every node has a signal with cycle U{60000..120000} ms and split
      g ~ U{300..700} per mille: north/south approaches get g, east/west 1000-g;
    * ``remove_frac`` of the directed roads are deleted one at a time in random
      order, skipping any deletion that would break strong connectivity.
    """
    n = rows * cols
    idx = np.arange(n).reshape(rows, cols)
    ua = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])   # undirected roads
    ub = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    road_len = rng.integers(spacing_dm, 5 * spacing_dm + 1, size=ua.shape[0])
    tails = np.concatenate([ua, ub])
    heads = np.concatenate([ub, ua])
    lens = np.concatenate([road_len, road_len])
    m0 = tails.shape[0]
    keep = np.ones(m0, dtype=bool)
    n_remove = int(round(remove_frac * m0))
    if n_remove:
        removed = 0
        for e in rng.permutation(m0):
            keep[e] = False
            if _strongly_connected(n, tails[keep], heads[keep]):
                removed += 1
                if removed == n_remove:
                    break
            else:
                keep[e] = True
        assert removed == n_remove
    tails, heads, lens = tails[keep], heads[keep], lens[keep]
    m = tails.shape[0]
    base_load = rng.poisson(load_mean, size=m)
    cycle = rng.integers(60000, 120001, size=n)
    split = rng.integers(300, 701, size=n)
    x = (idx % cols).ravel() * spacing_dm
    y = (idx // cols).ravel() * spacing_dm

    def green_fn(t, h):
        vertical = (t // cols) != (h // cols)          # movement north/south
        g = split[h]
        return np.where(vertical, g, 1000 - g)

    return _to_csr(n, tails, heads, lens, np.full(m, speed_kmh), base_load, cycle, x, y, green_fn)


# ---------------------------------------------------------------------------
# planar road-like networks
# ---------------------------------------------------------------------------

def planar_graph(n: int, rng: np.random.Generator, *, spacing_dm: int = 1500, jitter_dm: int = 300,
                 mean_out_degree: float = 2.5, max_degree: int = 5, signal_frac: float = 0.6,
                 speeds=(30, 50, 70), len_median_dm: float = 2000.0, len_sigma: float = 0.5,
                 load_mean: float = 3.0) -> RoadGraph:
    """Random planar road network on a jittered lattice.

    Roads are two-way.  A random spanning tree of the lattice keeps the network
    connected; nodes left with one road get a second; further lattice links and
    single cell diagonals (never two in one cell, so no crossings) are added at
    random until the directed edge count reaches ``mean_out_degree * n``.  Every
    node ends with between 2 and ``max_degree`` roads.  Lengths are
    max(ceil(straight line), lognormal(median, sigma)); speeds are drawn from
    ``speeds``; ``signal_frac`` of the nodes are signalised with cycle
    U{60000..120000} ms and split g ~ U{300..700}: approaches sorted by source
    node alternate g, 1000-g.
    """
    cols = int(np.ceil(np.sqrt(n * 1.6)))
    rows = int(np.ceil(n / cols))
    assert rows >= 2 and cols >= 2
    N = rows * cols
    r = np.arange(N) // cols
    c = np.arange(N) % cols
    x = c * spacing_dm + rng.integers(-jitter_dm, jitter_dm + 1, size=N)
    y = r * spacing_dm + rng.integers(-jitter_dm, jitter_dm + 1, size=N)
    alive = np.arange(N) < n                      # last row may be partial
    idx = np.arange(N).reshape(rows, cols)
    la = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    lb = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    ok = alive[la] & alive[lb]
    la, lb = la[ok], lb[ok]
    # spanning tree: MST of random weights on the lattice
    w = rng.random(la.shape[0]) + 1.0
    A = sp.coo_matrix((w, (la, lb)), shape=(n, n)).tocsr()
    T = minimum_spanning_tree(A).tocoo()
    deg = np.zeros(n, dtype=np.int64)
    roads = set()

    def add(a, b):
        a, b = (a, b) if a < b else (b, a)
        if (a, b) in roads:
            return False
        roads.add((a, b))
        deg[a] += 1
        deg[b] += 1
        return True

    for a, b in zip(T.row.tolist(), T.col.tolist()):
        add(a, b)
    # candidate extras: unused lattice links and one random diagonal per cell
    cr = idx[:-1, :-1].ravel()
    diag_main = rng.random(cr.shape[0]) < 0.5
    da = np.where(diag_main, cr, cr + 1)
    db = np.where(diag_main, cr + cols + 1, cr + cols)
    okd = (da < n) & (db < n)
    da, db = da[okd], db[okd]
    cand_a = np.concatenate([la, da])
    cand_b = np.concatenate([lb, db])
    # neighbours list for the degree-1 fix
    nbrs = [[] for _ in range(n)]
    for a, b in zip(cand_a.tolist(), cand_b.tolist()):
        nbrs[a].append(b)
        nbrs[b].append(a)
    for v in rng.permutation(n).tolist():
        if deg[v] >= 2:
            continue
        opts = [u for u in nbrs[v] if deg[u] < max_degree and (min(u, v), max(u, v)) not in roads]
        if opts:
            add(v, opts[int(rng.integers(len(opts)))])
    target_roads = int(round(mean_out_degree * n / 2))
    for i in rng.permutation(cand_a.shape[0]).tolist():
        if len(roads) >= target_roads:
            break
        a, b = int(cand_a[i]), int(cand_b[i])
        if deg[a] < max_degree and deg[b] < max_degree:
            add(a, b)
    ra = np.array([p[0] for p in roads], dtype=np.int64)
    rb = np.array([p[1] for p in roads], dtype=np.int64)
    order = np.lexsort((rb, ra))
    ra, rb = ra[order], rb[order]
    x, y = x[:n], y[:n]
    euclid = np.ceil(np.hypot((x[ra] - x[rb]).astype(np.float64), (y[ra] - y[rb]).astype(np.float64)))
    drawn = np.rint(rng.lognormal(np.log(len_median_dm), len_sigma, size=ra.shape[0]))
    road_len = np.maximum(euclid, drawn).astype(np.int64)
    road_speed = rng.choice(np.asarray(speeds), size=ra.shape[0])
    tails = np.concatenate([ra, rb])
    heads = np.concatenate([rb, ra])
    lens = np.concatenate([road_len, road_len])
    spd = np.concatenate([road_speed, road_speed])
    m = tails.shape[0]
    base_load = rng.poisson(load_mean, size=m)
    signal = rng.random(n) < signal_frac
    cycle = np.where(signal, rng.integers(60000, 120001, size=n), 0)
    split = rng.integers(300, 701, size=n)

    def green_fn(t, h):
        # rank of each approach among the in-edges of its head, by source node
        order = np.lexsort((t, h))
        hs = h[order]
        start = np.searchsorted(hs, hs, side="left")
        rank = np.empty_like(order)
        rank[order] = np.arange(order.shape[0]) - start
        g = split[h]
        gm = np.where(rank % 2 == 0, g, 1000 - g)
        return np.where(cycle[h] > 0, gm, 1000)

    g = _to_csr(n, tails, heads, lens, spd, base_load, cycle, x, y, green_fn)
    deg_out = g.out_degree()
    assert deg_out.min() >= 1
    return g


def pack_graphs(graphs: List[RoadGraph]) -> RoadGraph:
    """Disjoint union of several graphs in one CSR; node and edge ids of
    instance i are offset by the node/edge counts of instances 0..i-1."""
    node_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    edge_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        node_off[i + 1] = node_off[i] + g.n
        edge_off[i + 1] = edge_off[i] + g.m
    row_ptr = np.concatenate([g.row_ptr[:-1].astype(np.int64) + edge_off[i] for i, g in enumerate(graphs)]
                             + [np.array([edge_off[-1]])])
    col = np.concatenate([g.col.astype(np.int64) + node_off[i] for i, g in enumerate(graphs)])
    cat = lambda name, dt: np.ascontiguousarray(np.concatenate([getattr(g, name) for g in graphs]), dtype=dt)
    out = RoadGraph(
        row_ptr=row_ptr.astype(np.uint32), col=col.astype(np.uint32),
        len_dm=cat("len_dm", np.uint32), speed_kmh=cat("speed_kmh", np.uint16),
        green_pm=cat("green_pm", np.uint16), cycle_ms=cat("cycle_ms", np.uint32),
        x_dm=cat("x_dm", np.int32), y_dm=cat("y_dm", np.int32),
        base_load=cat("base_load", np.uint32), inst_node_off=node_off.astype(np.uint32))
    out.validate()
    return out


# ---------------------------------------------------------------------------
# vehicles
# ---------------------------------------------------------------------------

def random_od(n: int, V: int, rng: np.random.Generator, *, node_lo: int = 0, qid0: int = 0) -> Vehicles:
    """V vehicles with independent uniform source/destination (src != dst)
    among nodes node_lo .. node_lo+n-1."""
    src = rng.integers(0, n, size=V)
    dst = rng.integers(0, n - 1, size=V)
    dst = np.where(dst >= src, dst + 1, dst)
    return Vehicles(qid=np.arange(qid0, qid0 + V, dtype=np.uint32),
                    src=(src + node_lo).astype(np.uint32), dst=(dst + node_lo).astype(np.uint32))


def shell_od(g: RoadGraph, V: int, rng: np.random.Generator, *, h_lo: int = 5, h_hi: int = 200,
             batch: int = 64) -> Vehicles:
    """V vehicles: uniform source, hop distance H ~ U{h_lo..h_hi} (breadth
    first, directed), destination uniform among nodes exactly H hops away.  A
    source without any node at distance H is redrawn."""
    n = g.n
    A = sp.csr_matrix((np.ones(g.m), g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(n, n))
    src_out, dst_out = [], []
    while len(src_out) < V:
        need = V - len(src_out)
        s_all = rng.integers(0, n, size=need)
        H_all = rng.integers(h_lo, h_hi + 1, size=need)
        order = np.argsort(H_all, kind="stable")      # similar depths share one search
        for b0 in range(0, need, batch):
            sel = order[b0:b0 + batch]
            s, H = s_all[sel], H_all[sel]
            d = dijkstra(A, unweighted=True, indices=s, limit=float(H.max()) + 0.5)
            for i in range(sel.shape[0]):
                shell = np.flatnonzero(d[i] == H[i])
                if shell.size and len(src_out) < V:
                    src_out.append(int(s[i]))
                    dst_out.append(int(shell[int(rng.integers(shell.size))]))
    V_ = len(src_out)
    return Vehicles(qid=np.arange(V_, dtype=np.uint32), src=np.array(src_out, dtype=np.uint32),
                    dst=np.array(dst_out, dtype=np.uint32))


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def default_params(**kw) -> dict:
    """Parameter set shared by the named workloads (alpha=1, beta=2,
    rho=0.5, tau0=1.0 in Q16.16; thresholds and deposit constant as chosen for
    this implementation)."""
    p = dict(ants=16, iterations=50, alpha=1, beta=2, max_steps=63,
             rho_q16=0x8000, tau0_q16=0x10000, tau_min_q16=1, tau_max_q16=1 << 24,
             q_deposit=65536 * 100000, theta=4, th_max=8, t_max_ms=20000, vmax_kmh=50,
             mode=0, flags=0, seed=1, iter_offset=0)
    p.update(kw)
    return p


def grid8(seed: int = 1) -> Workload:
    """8x8 grid, one vehicle corner to corner, 16 ants x 50 iterations."""
    rng = np.random.default_rng(seed)
    g = grid_graph(8, 8, rng)
    veh = Vehicles(qid=np.array([0], np.uint32), src=np.array([0], np.uint32), dst=np.array([63], np.uint32))
    return Workload("grid8x8_1veh_16ants_50it", g, veh,
                    default_params(ants=16, iterations=50, max_steps=g.n - 1, vmax_kmh=50))


def grid32(seed: int = 1, *, vehicles: int = 256, ants: int = 128, iterations: int = 100) -> Workload:
    """32x32 grid with 5% of directed roads removed (strongly connected), 256
    random OD vehicles, 128 ants x 100 iterations."""
    rng = np.random.default_rng(seed)
    g = grid_graph(32, 32, rng, remove_frac=0.05)
    veh = random_od(g.n, vehicles, rng)
    return Workload(f"grid32x32_{vehicles}veh_{ants}ants_{iterations}it", g, veh,
                    default_params(ants=ants, iterations=iterations, max_steps=min(g.n - 1, 1024), vmax_kmh=50))


def planar100k(seed: int = 1, *, n: int = 100000, vehicles: int = 4096, ants: int = 64,
               iterations: int = 50) -> Workload:
    """Planar road-like network (~2.5 roads out of each node), 4096 vehicles
    with hop distances U{5..200}, 64 ants x 50 iterations."""
    rng = np.random.default_rng(seed)
    g = planar_graph(n, rng)
    veh = shell_od(g, vehicles, rng)
    return Workload(f"planar{n // 1000}k_{vehicles}veh_{ants}ants_{iterations}it", g, veh,
                    default_params(ants=ants, iterations=iterations, max_steps=1024, vmax_kmh=70))


def multi_city(seed: int = 1, *, cities: int = 64, n_lo: int = 1000, n_hi: int = 50000,
               v_lo: int = 32, v_hi: int = 512, ants: int = 32, iterations: int = 30) -> Workload:
    """``cities`` independent planar networks with log-uniform sizes in
    [n_lo, n_hi] nodes and log-uniform [v_lo, v_hi] vehicles each, packed into
    one CSR with per-instance node offsets."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=cities)).astype(np.int64)
    nveh = np.exp(rng.uniform(np.log(v_lo), np.log(v_hi), size=cities)).astype(np.int64)
    graphs = [planar_graph(int(s), rng) for s in sizes]
    packed = pack_graphs(graphs)
    off = packed.inst_node_off.astype(np.int64)
    vs, qid0 = [], 0
    for i, g in enumerate(graphs):
        v = random_od(g.n, int(nveh[i]), rng, node_lo=int(off[i]), qid0=qid0)
        qid0 += len(v)
        vs.append(v)
    veh = Vehicles(qid=np.concatenate([v.qid for v in vs]), src=np.concatenate([v.src for v in vs]),
                   dst=np.concatenate([v.dst for v in vs]))
    return Workload(f"multicity{cities}_{len(veh)}veh_{ants}ants_{iterations}it", packed, veh,
                    default_params(ants=ants, iterations=iterations, max_steps=1024, vmax_kmh=70))


def from_edges(n: int, tails, heads, *, len_dm=1000, speed_kmh=50, green_pm=500, cycle_ms=0,
               x_dm=None, y_dm=None, base_load=0) -> RoadGraph:
    """Small hand-made graph from explicit directed roads (CSR order = sorted
    by tail, then head; per-road attributes follow the given road order).
    Scalars broadcast."""
    tails = np.asarray(tails, dtype=np.int64)
    heads = np.asarray(heads, dtype=np.int64)
    m = tails.shape[0]
    bc = lambda v, k: np.broadcast_to(np.asarray(v), (k,)).copy()
    x = bc(0 if x_dm is None else x_dm, n)
    y = bc(0 if y_dm is None else y_dm, n)
    gm = bc(green_pm, m)
    order = np.lexsort((heads, tails))
    gm_sorted = gm[order]

    def green_fn(t, h):
        return gm_sorted

    return _to_csr(n, tails, heads, bc(len_dm, m), bc(speed_kmh, m), bc(base_load, m),
                   bc(cycle_ms, n), x, y, green_fn)


def serving_city(seed: int = 1, *, n: int = 1_000_000, ants: int = 32, iterations: int = 20,
                 max_steps: int = 4096) -> Workload:
    """Planar road network of ~1M nodes / ~2.5M roads for routing queries
    (independent per-query pheromone, 32 ants x 20 iterations)."""
    rng = np.random.default_rng(seed)
    g = planar_graph(n, rng)
    return Workload(f"planar{n // 1000}k_serving_{ants}ants_{iterations}it", g,
                    random_od(g.n, 1, rng),
                    default_params(ants=ants, iterations=iterations, max_steps=max_steps, vmax_kmh=70, mode=1))


def query_stream(g: RoadGraph, count: int, rng: np.random.Generator, qid0: int = 0) -> np.ndarray:
    """count uniform random OD queries as uint32 [count, 3] (qid, src, dst)."""
    v = random_od(g.n, count, rng, qid0=qid0)
    return np.stack([v.qid, v.src, v.dst], axis=1).astype(np.uint32)
