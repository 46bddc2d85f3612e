"""Parity of the HIP path with the CPU oracle, through the C ABI.

Integer method: every comparison is exact (paths, costs, selection counts,
final pheromone and loads).  Each case prints its name before it runs."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_2010_14244_amd import gmacop
from workloads import (Vehicles, default_params, from_edges, grid8, grid32, grid_graph, pack_graphs,
                       planar_graph, random_od)

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    oracle.build(force=False)


def announce(name):
    print(f"\n[case] {name}", flush=True)


def run_gpu(g, veh, p):
    G = gmacop.gmacop_graph_create(g)
    try:
        r = gmacop.gmacop_route_batch(G, veh, p)
        if p["mode"] == gmacop.MODE_SHARED:
            r["tau"], r["load"] = gmacop.gmacop_state_get(G)
        return r
    finally:
        gmacop.gmacop_release(G)


def assert_same(got, want, S, state=True):
    assert got["steps_total"] == want["steps_total"], (got["steps_total"], want["steps_total"])
    assert got["path_len"].tolist() == want["path_len"].tolist()
    assert got["cost_ms"].tolist() == want["cost_ms"].tolist()
    for v in range(want["path_len"].shape[0]):
        L = int(want["path_len"][v])
        assert got["path_edges"][v, :L].tolist() == want["path_edges"][v, :L].tolist(), v
    if state:
        assert np.array_equal(got["tau"], want["tau"])
        assert np.array_equal(got["load"], want["load"])


def check(name, g, veh, p, state=True):
    announce(name)
    want = oracle.route(g, veh, p)
    got = run_gpu(g, veh, p)
    assert_same(got, want, p["max_steps"], state=state and p["mode"] == 0)
    return got, want


def test_grid8_workload():
    w = grid8()
    check(w.name, w.graph, w.vehicles, w.params)


# With few ants per vehicle a city that needs a whole CU's LDS would leave most
# of the CU idle, so the default plan sends it to the global walker; "lds"
# forces the LDS walkers for the same case.
PLAN_KINDS = pytest.mark.parametrize("kernel", ["", "lds"])


@PLAN_KINDS
def test_grid32_reduced(monkeypatch, kernel):
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    w = grid32(vehicles=48, ants=32, iterations=12)
    check(f"{w.name}_{kernel or 'plan'}", w.graph, w.vehicles, w.params)


@PLAN_KINDS
def test_grid32_frozen_loads(monkeypatch, kernel):
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    w = grid32(vehicles=32, ants=16, iterations=8)
    check(f"{w.name}_frozen_{kernel or 'plan'}", w.graph, w.vehicles, dict(w.params, flags=gmacop.NO_LOAD_UPDATE))


def test_planar_global_bitset_and_degree5():
    """More than 4096 nodes: visited bits in global memory; out-degree up to 5."""
    rng = np.random.default_rng(21)
    g = planar_graph(6000, rng)
    assert g.n > 4096 and g.out_degree().max() > 4
    V = random_od(g.n, 24, rng)
    p = default_params(ants=16, iterations=6, max_steps=400, vmax_kmh=70)
    check("planar6000", g, V, p)


@PLAN_KINDS
def test_planar_small_lds_degree5(monkeypatch, kernel):
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    rng = np.random.default_rng(22)
    g = planar_graph(3000, rng)
    V = random_od(g.n, 20, rng)
    p = default_params(ants=16, iterations=6, max_steps=300, vmax_kmh=70)
    check(f"planar3000_{kernel or 'plan'}", g, V, p)


def _hub_far_graph(rng, n=48, hub=32):
    """Node 0 has out-degree 32 and node n-1 in-degree 32 (the widest walker
    template); coordinates spread to the validated limit |x|, |y| < 2^30, with
    a few nodes clustered, so squared distances pass 2^44 and goal terms 2^32
    at low vmax; road lengths from 1 dm to 3e6 dm put eta at both clamps and
    give negative deltas (roads shorter than the straight line)."""
    tails = [0] * hub + list(range(1, hub + 1))
    heads = list(range(1, hub + 1)) + [n - 1] * hub
    seen = set(zip(tails, heads))
    for u in range(1, n):
        for h in rng.choice(n - 1, size=4, replace=False):
            h = int(h)
            if h != u and h != 0 and (u, h) not in seen:
                seen.add((u, h))
                tails.append(u)
                heads.append(h)
    m = len(tails)
    lim = 2 ** 30 - 1
    x = rng.integers(-lim, lim + 1, n)
    y = rng.integers(-lim, lim + 1, n)
    x[36:44] = rng.integers(-40, 40, 8)    # a cluster: short roads, eta at 65535
    y[36:44] = rng.integers(-40, 40, 8)
    x[:2] = [-lim, lim]
    y[:2] = [lim, -lim]
    ln = np.where(rng.random(m) < 0.25, rng.integers(1, 100, m), rng.integers(1000, 3_000_000, m))
    return from_edges(n, tails, heads, len_dm=ln, speed_kmh=rng.integers(5, 131, m),
                      green_pm=rng.integers(0, 1001, m), cycle_ms=rng.integers(0, 120_000, n),
                      x_dm=x, y_dm=y, base_load=rng.integers(0, 12, m))


@pytest.mark.parametrize("kernel,lanes,variant", [
    ("", 4, ""), ("lds", 1, ""), ("lds", 8, "node"), ("global", 4, ""), ("global", 1, ""), ("legacy", 1, "")])
def test_high_degree_and_far_coordinates(monkeypatch, kernel, lanes, variant):
    """Out- and in-degree 32, coordinates at the validated limit: the goal
    term's far-distance root, eta's clamps, and (at vmax 20) goal terms
    above 2^32, which send the city to the global walker; a packed pair of
    a near city and a far one mixes walkers in one iteration."""
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    monkeypatch.setenv("GMACOP_WALK_LANES", str(lanes))
    monkeypatch.setenv("GMACOP_GLB_LANES", str(lanes))
    monkeypatch.setenv("GMACOP_LDS_VARIANT", variant)
    rng = np.random.default_rng(31)
    g = _hub_far_graph(rng)
    assert g.out_degree().max() == 32
    V = Vehicles(qid=np.arange(40, dtype=np.uint32),
                 src=np.concatenate([np.zeros(8, np.uint32), rng.integers(0, g.n, 32).astype(np.uint32)]),
                 dst=np.concatenate([np.full(8, g.n - 1, np.uint32), rng.integers(0, g.n, 32).astype(np.uint32)]))
    V = Vehicles(qid=V.qid, src=V.src, dst=np.where(V.dst == V.src, (V.src + 1) % g.n, V.dst).astype(np.uint32))
    for vmax in (0, 400, 20):
        p = default_params(ants=16, iterations=4, max_steps=40, vmax_kmh=vmax)
        check(f"hub_far_{kernel or 'plan'}_L{lanes}{variant}_vmax{vmax}", g, V, p)
    near = grid_graph(4, 5, rng)
    packed = pack_graphs([near, g])
    off = int(packed.inst_node_off[1])
    vn = random_od(near.n, 10, rng)
    Vp = Vehicles(qid=np.arange(20, dtype=np.uint32), src=np.concatenate([vn.src, off + V.src[:10]]).astype(np.uint32),
                  dst=np.concatenate([vn.dst, off + V.dst[:10]]).astype(np.uint32))
    check(f"hub_far_packed_{kernel or 'plan'}_L{lanes}{variant}", packed, Vp,
          default_params(ants=16, iterations=3, max_steps=40, vmax_kmh=20))


@PLAN_KINDS
def test_parameter_variants(monkeypatch, kernel):
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    w = grid32(vehicles=16, ants=8, iterations=5)
    g, V = w.graph, w.vehicles
    for kw in (dict(alpha=0, beta=0), dict(alpha=2, beta=1, tau_max_q16=2 ** 20),
               dict(alpha=1, beta=3, tau0_q16=2 ** 12, tau_max_q16=2 ** 13 - 1),
               dict(rho_q16=0, q_deposit=0), dict(rho_q16=65536), dict(vmax_kmh=0, max_steps=200),
               dict(theta=1, th_max=0), dict(seed=0xDEADBEEF12345678, iter_offset=77), dict(max_steps=1),
               dict(ants=1), dict(t_max_ms=0)):
        check(f"grid32_{kernel or 'plan'}_{kw}", g, V, dict(w.params, **kw))


def test_edge_cases():
    w = grid8()
    g = w.graph
    # zero iterations, zero vehicles
    check("iterations0", g, w.vehicles, dict(w.params, iterations=0))
    check("no_vehicles", g, Vehicles(qid=np.zeros(0, np.uint32), src=np.zeros(0, np.uint32),
                                     dst=np.zeros(0, np.uint32)), w.params)
    # unreachable destination: one-way trap
    h = from_edges(4, [0, 0, 1, 2], [1, 2, 0, 3])      # 3 has no out-roads, 0 cannot reach... 0->2->3 ok; 3->x none
    Vt = Vehicles(qid=np.array([5, 6], np.uint32), src=np.array([3, 0], np.uint32), dst=np.array([0, 3], np.uint32))
    p = default_params(ants=8, iterations=4, max_steps=3, vmax_kmh=0)
    got, want = check("unreachable", h, Vt, p)
    assert want["path_len"][0] == 0 and want["cost_ms"][0] == 2 ** 32 - 1
    # several vehicles sharing qid and route
    Vd = Vehicles(qid=np.array([1, 1, 2], np.uint32), src=np.array([0, 0, 9], np.uint32),
                  dst=np.array([63, 63, 54], np.uint32))
    check("duplicate_qid", g, Vd, w.params)


def test_packed_instances():
    rng = np.random.default_rng(8)
    gs = [grid_graph(5, 6, rng), planar_graph(700, rng), grid_graph(3, 9, rng)]
    packed = pack_graphs(gs)
    off = packed.inst_node_off.astype(np.int64)
    vs = [random_od(gi.n, 6, rng, node_lo=int(off[i]), qid0=6 * i) for i, gi in enumerate(gs)]
    V = Vehicles(qid=np.concatenate([v.qid for v in vs]), src=np.concatenate([v.src for v in vs]),
                 dst=np.concatenate([v.dst for v in vs]))
    p = default_params(ants=12, iterations=6, max_steps=80, vmax_kmh=70)
    check("packed3", packed, V, p)


def test_device_pointer_mode_matches_host_mode():
    import torch
    w = grid32(vehicles=40, ants=16, iterations=6)
    announce("device_ptrs")
    G = gmacop.gmacop_graph_create(w.graph)
    try:
        host = gmacop.gmacop_route_batch(G, w.vehicles, w.params)
        b = gmacop.DeviceBatch(w.vehicles, w.params["max_steps"])
        gmacop.gmacop_route_batch_device(G, b, w.params)
        torch.cuda.synchronize()
        dev = b.result()
        assert_same(dev, host, w.params["max_steps"], state=False)
    finally:
        gmacop.gmacop_release(G)


def test_invalid_queries_match_oracle_codes():
    w = grid8()
    announce("error_codes")
    G = gmacop.gmacop_graph_create(w.graph)
    try:
        bad = [Vehicles(qid=np.array([0], np.uint32), src=np.array([3], np.uint32), dst=np.array([3], np.uint32)),
               Vehicles(qid=np.array([0], np.uint32), src=np.array([3], np.uint32), dst=np.array([64], np.uint32))]
        for V in bad:
            assert oracle.route_rc(w.graph, V, w.params) == oracle.E_INVAL
            with pytest.raises(gmacop.GmacopError) as ei:
                gmacop.gmacop_route_batch(G, V, w.params)
            assert ei.value.code == gmacop.E_INVAL
        for kw, code in ((dict(ants=0), gmacop.E_INVAL), (dict(rho_q16=70000), gmacop.E_INVAL),
                         (dict(beta=3), gmacop.E_RANGE), (dict(q_deposit=2 ** 62), gmacop.E_RANGE)):
            p = dict(w.params, **kw)
            assert oracle.route_rc(w.graph, w.vehicles, p) == code
            with pytest.raises(gmacop.GmacopError) as ei:
                gmacop.gmacop_route_batch(G, w.vehicles, p)
            assert ei.value.code == code
        # the handle still works after rejected calls
        ok = gmacop.gmacop_route_batch(G, w.vehicles, w.params)
        assert ok["steps_total"] == oracle.route(w.graph, w.vehicles, w.params)["steps_total"]
    finally:
        gmacop.gmacop_release(G)


def _digest_routes(path_edges, path_len):
    h = hashlib.sha256()
    for v in range(path_len.shape[0]):
        h.update(np.ascontiguousarray(path_edges[v, :int(path_len[v])], dtype=np.uint32).tobytes())
        h.update(b"|")
    return h.hexdigest()


def _full_workload(name):
    from workloads import Workload, multi_city, planar100k
    if name == "planar100k_indep256":
        w = planar100k(vehicles=256)
        return Workload(w.name, w.graph, w.vehicles, dict(w.params, mode=gmacop.MODE_INDEPENDENT))
    if name == "multicity_exact":
        w = multi_city()
        return Workload(w.name, w.graph, w.vehicles, dict(w.params, flags=gmacop.GOAL_EXACT))
    return {"grid32": grid32, "planar100k": planar100k, "multicity": multi_city}[name]()


@pytest.mark.parametrize("name", ["grid32", "planar100k", "multicity", "planar100k_indep256", "multicity_exact"])
def test_full_workload_against_stored_oracle_results(name):
    """Full-size workloads (32x32 grid: 256 vehicles x 128 ants x 100 it;
    100k-node planar city: 4096 x 64 x 50, and 256 vehicles in independent
    mode; 64 packed cities: 10466 x 32 x 30, also with the exact goal term)
    against the oracle's results stored by tests/golden/make_expected.py.
    Independent mode: every vehicle's final pheromone row, in vehicle order."""
    path = os.path.join(HERE, "golden", f"{name}_expected.json")
    with open(path) as f:
        want = json.load(f)
    w = _full_workload(name)
    assert w.name == want["workload"] and w.params == want["params"]
    announce(f"{name}: {w.name}")
    G = gmacop.gmacop_graph_create(w.graph)
    try:
        got = gmacop.gmacop_route_batch(G, w.vehicles, w.params)
        assert got["steps_total"] == want["steps_total"]
        assert got["cost_ms"].tolist() == want["cost_ms"]
        assert got["path_len"].tolist() == want["path_len"]
        assert _digest_routes(got["path_edges"], got["path_len"]) == want["routes_sha256"]
        if w.params["mode"] == gmacop.MODE_SHARED:
            tau, load = gmacop.gmacop_state_get(G)
            assert hashlib.sha256(tau.tobytes()).hexdigest() == want["tau_sha256"]
            assert hashlib.sha256(load.tobytes()).hexdigest() == want["load_sha256"]
        else:
            h = hashlib.sha256()
            for v in range(len(w.vehicles)):
                h.update(np.ascontiguousarray(gmacop.gmacop_vehicle_tau_get(G, v), np.uint32).tobytes())
            assert h.hexdigest() == want["tau_sha256"]
            assert hashlib.sha256(np.ascontiguousarray(w.graph.base_load, np.uint32).tobytes()).hexdigest() \
                == want["load_sha256"]        # loads stay frozen
    finally:
        gmacop.gmacop_release(G)

@pytest.mark.parametrize("kernel,lanes,bloom,variant", [
    ("legacy", 1, 11, ""), ("global", 1, 11, ""), ("global", 2, 11, ""), ("global", 4, 11, ""),
    ("global", 8, 11, ""), ("global", 4, 8, ""), ("lds", 1, 11, ""), ("lds", 2, 11, ""), ("lds", 4, 11, ""),
    ("lds", 8, 11, ""), ("lds", 1, 11, "node"), ("lds", 2, 11, "node"), ("lds", 4, 11, "node"),
    ("lds", 8, 11, "node")])
def test_walker_shapes_give_identical_results(monkeypatch, kernel, lanes, bloom, variant):
    """Every walker shape (first global-memory walker, global walker with
    1-8 lanes per ant and a small Bloom filter that sends most visited tests
    to the exact bitset, LDS-staged roads with 1-8 lanes and visited state
    per road (default) or per node) reproduces the oracle exactly."""
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    monkeypatch.setenv("GMACOP_WALK_LANES", str(lanes))
    monkeypatch.setenv("GMACOP_GLB_LANES", str(lanes))
    monkeypatch.setenv("GMACOP_BLOOM_LOG2", str(bloom))
    monkeypatch.setenv("GMACOP_LDS_VARIANT", variant)
    w = grid32(vehicles=24, ants=40, iterations=6)
    check(f"{w.name}_{kernel}_L{lanes}_b{bloom}{variant}", w.graph, w.vehicles, w.params)
    rng = np.random.default_rng(23)
    g = planar_graph(1500, rng)
    V = random_od(g.n, 12, rng)
    check(f"planar1500_{kernel}_L{lanes}_b{bloom}", g, V,
          default_params(ants=24, iterations=5, max_steps=300, vmax_kmh=70))


def test_mixed_walkers_in_one_iteration():
    """Packed cities where small ones are served from LDS and a large one by
    the global walker, all depositing on one shared pheromone vector."""
    rng = np.random.default_rng(41)
    gs = [grid_graph(4, 6, rng), planar_graph(12000, rng), planar_graph(900, rng), grid_graph(9, 9, rng)]
    packed = pack_graphs(gs)
    off = packed.inst_node_off.astype(np.int64)
    vs = [random_od(gi.n, 5, rng, node_lo=int(off[i]), qid0=5 * i) for i, gi in enumerate(gs)]
    V = Vehicles(qid=np.concatenate([v.qid for v in vs]), src=np.concatenate([v.src for v in vs]),
                 dst=np.concatenate([v.dst for v in vs]))
    p = default_params(ants=16, iterations=5, max_steps=500, vmax_kmh=70)
    check("mixed_cities", packed, V, p)
    check("mixed_cities_indep", packed, V, dict(p, mode=gmacop.MODE_INDEPENDENT), state=False)


def test_all_walker_kinds_in_one_iteration():
    """One launch sequence where a small grid uses the per-road-visited LDS
    walker, a 2000-node city whose per-road layout does not fit LDS at 128
    ants per block uses the per-node LDS walker, and a 12000-node city the
    global walker (on a second stream, beside the LDS walkers); all deposit on
    one shared pheromone vector.  Eager and HIP-graph launches."""
    rng = np.random.default_rng(43)
    gs = [grid_graph(8, 8, rng), planar_graph(2000, rng), planar_graph(12000, rng)]
    packed = pack_graphs(gs)
    off = packed.inst_node_off.astype(np.int64)
    vs = [random_od(gi.n, 3, rng, node_lo=int(off[i]), qid0=3 * i) for i, gi in enumerate(gs)]
    V = Vehicles(qid=np.concatenate([v.qid for v in vs]), src=np.concatenate([v.src for v in vs]),
                 dst=np.concatenate([v.dst for v in vs]))
    p = default_params(ants=128, iterations=3, max_steps=400, vmax_kmh=70)
    check("three_walker_kinds", packed, V, p)
    # the same call captured in a HIP graph (global walker forked onto a second stream), replayed twice
    import torch
    want = oracle.route(packed, V, p)
    G = gmacop.gmacop_graph_create(packed)
    stream = torch.cuda.Stream()
    try:
        b = gmacop.DeviceBatch(V, p["max_steps"])
        for rep in range(2):
            gmacop.gmacop_route_batch_device(G, b, dict(p, flags=gmacop.HIP_GRAPH), stream.cuda_stream)
            stream.synchronize()
            assert_same(b.result(), want, p["max_steps"], state=False)
            tau, load = gmacop.gmacop_state_get(G)
            assert np.array_equal(tau, want["tau"]) and np.array_equal(load, want["load"])
            assert_same(gmacop.gmacop_route_batch(G, V, p), want, p["max_steps"], state=False)
    finally:
        gmacop.gmacop_release(G)


def test_hip_graph_replays_match_eager():
    """The captured kernel sequence, replayed several times with eager calls
    and host synchronisations in between, gives the eager (and oracle) result
    every time; a changed argument recaptures."""
    import torch
    w = grid32(vehicles=32, ants=24, iterations=7)
    announce("hip_graph")
    want = oracle.route(w.graph, w.vehicles, w.params)
    G = gmacop.gmacop_graph_create(w.graph)
    stream = torch.cuda.Stream()
    try:
        b = gmacop.DeviceBatch(w.vehicles, w.params["max_steps"])
        pg = dict(w.params, flags=gmacop.HIP_GRAPH)
        for rep in range(4):
            gmacop.gmacop_route_batch_device(G, b, pg, stream.cuda_stream)
            stream.synchronize()
            assert_same(b.result(), want, w.params["max_steps"], state=False)
            tau, load = gmacop.gmacop_state_get(G)
            assert np.array_equal(tau, want["tau"]) and np.array_equal(load, want["load"])
            eager = gmacop.gmacop_route_batch(G, w.vehicles, w.params)       # eager work between replays
            assert_same(eager, want, w.params["max_steps"], state=False)
        p2 = dict(pg, seed=9)
        want2 = oracle.route(w.graph, w.vehicles, dict(w.params, seed=9))
        gmacop.gmacop_route_batch_device(G, b, p2, stream.cuda_stream)
        stream.synchronize()
        assert_same(b.result(), want2, w.params["max_steps"], state=False)
    finally:
        gmacop.gmacop_release(G)


def check_independent(name, g, veh, p):
    announce(name)
    want = oracle.route(g, veh, p)
    G = gmacop.gmacop_graph_create(g)
    try:
        got = gmacop.gmacop_route_batch(G, veh, p)
        assert_same(got, want, p["max_steps"], state=False)
        for v in range(len(veh)):
            assert np.array_equal(gmacop.gmacop_vehicle_tau_get(G, v), want["tau"][v]), v
    finally:
        gmacop.gmacop_release(G)
    return got, want


@pytest.mark.parametrize("kernel,lanes", [("lds", 4), ("lds", 1), ("global", 4), ("global", 1), ("legacy", 1)])
def test_independent_mode(monkeypatch, kernel, lanes):
    """Private pheromone per vehicle with frozen loads, both walkers, final
    pheromone of every vehicle included."""
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    monkeypatch.setenv("GMACOP_WALK_LANES", str(lanes))
    monkeypatch.setenv("GMACOP_GLB_LANES", str(lanes))
    w = grid32(vehicles=20, ants=24, iterations=9)
    check_independent(f"{w.name}_indep_{kernel}_L{lanes}", w.graph, w.vehicles,
                      dict(w.params, mode=gmacop.MODE_INDEPENDENT))
    rng = np.random.default_rng(31)
    g = planar_graph(5000, rng)
    V = random_od(g.n, 10, rng)
    check_independent(f"planar5000_indep_{kernel}_L{lanes}", g, V,
                      default_params(ants=16, iterations=6, max_steps=400, vmax_kmh=70, mode=gmacop.MODE_INDEPENDENT,
                                     rho_q16=0x3000))


def test_independent_alone_equals_in_mix():
    """A vehicle's independent-mode result is the same alone and in a batch,
    and over repeated calls on one handle (generations of lazy pheromone)."""
    w = grid32(vehicles=12, ants=16, iterations=6)
    p = dict(w.params, mode=gmacop.MODE_INDEPENDENT)
    announce("indep_alone_vs_mix")
    G = gmacop.gmacop_graph_create(w.graph)
    try:
        mix = gmacop.gmacop_route_batch(G, w.vehicles, p)
        for v in (0, 5, 11):
            one = Vehicles(qid=w.vehicles.qid[v:v + 1], src=w.vehicles.src[v:v + 1], dst=w.vehicles.dst[v:v + 1])
            alone = gmacop.gmacop_route_batch(G, one, p)
            L = int(mix["path_len"][v])
            assert alone["cost_ms"][0] == mix["cost_ms"][v] and alone["path_len"][0] == L
            assert alone["path_edges"][0, :L].tolist() == mix["path_edges"][v, :L].tolist()
        again = gmacop.gmacop_route_batch(G, w.vehicles, p)
        assert_same(again, mix, p["max_steps"], state=False)
    finally:
        gmacop.gmacop_release(G)


def test_router_results_equal_standalone_runs():
    """Queries served by the continuous-batching router, admitted over
    several steps while others are in flight and slots are reused, give the
    same routes as each query run alone (independent mode) and as the oracle."""
    from workloads import query_stream
    w = grid32(iterations=5)
    p = dict(w.params, ants=16, iterations=5, mode=gmacop.MODE_INDEPENDENT)
    rng = np.random.default_rng(5)
    od = query_stream(w.graph, 23, rng, qid0=100)
    announce("router")
    G = gmacop.gmacop_graph_create(w.graph)
    srv = gmacop.Server(G, p, max_slots=6)
    try:
        assert srv.slots == 6
        results, nxt, step = {}, 0, 0
        plan = [3, 0, 1, 4, 0, 2, 5, 0, 0, 3]          # arrivals per step, then drain
        while len(results) < od.shape[0]:
            k = plan[step] if step < len(plan) else od.shape[0]
            batch = od[nxt:nxt + k]
            adm, done = srv.step(batch)
            assert adm <= k
            nxt += adm
            for qid, path, cost in done:
                results[qid] = (path, cost)
            step += 1
            assert step < 200
        alone = {}
        for i in range(od.shape[0]):
            veh = Vehicles(qid=od[i:i + 1, 0], src=od[i:i + 1, 1], dst=od[i:i + 1, 2])
            r = gmacop.gmacop_route_batch(G, veh, p)
            L = int(r["path_len"][0])
            qid = int(od[i, 0])
            assert results[qid][1] == int(r["cost_ms"][0]), qid
            assert results[qid][0].tolist() == r["path_edges"][0, :L].tolist(), qid
            alone[qid] = r
        veh = Vehicles(qid=od[:6, 0], src=od[:6, 1], dst=od[:6, 2])
        want = oracle.route(w.graph, veh, p)
        for i in range(6):
            assert results[int(od[i, 0])][1] == int(want["cost_ms"][i])
    finally:
        srv.release()
        gmacop.gmacop_release(G)


def test_router_admission_limits():
    w = grid8()
    p = dict(w.params, ants=4, iterations=3)
    G = gmacop.gmacop_graph_create(w.graph)
    try:
        with pytest.raises(gmacop.GmacopError) as ei:
            gmacop.Server(G, p, max_slots=4, mem_budget_bytes=16)      # below one slot
        assert ei.value.code == gmacop.E_NOMEM
        srv = gmacop.Server(G, p, max_slots=2)
        od = np.array([[1, 0, 63], [2, 5, 60], [3, 9, 17]], np.uint32)
        adm, done = srv.step(od)
        assert adm == 2 and not done and srv.active() == 2
        adm, done = srv.step(od[2:])
        assert adm == 0
        adm, done = srv.step(od[2:])
        assert adm == 0 and len(done) == 2 and srv.active() == 0
        adm, done = srv.step(od[2:])
        assert adm == 1
        with pytest.raises(gmacop.GmacopError):
            srv.step(np.array([[4, 3, 3]], np.uint32))                 # src == dst
        srv.release()
    finally:
        gmacop.gmacop_release(G)
