"""Resume and sensed-load epochs on the GPU, through the C ABI: "run I1
iterations, save, restore, run the rest" equals a straight run and the
oracle; calls after gmacop_set_base_load, and router queries admitted after
gmacop_server_set_base_load, equal the oracle on the new loads.  Exact."""
import numpy as np
import pytest

import oracle
from paper_2010_14244_amd import gmacop
from workloads import Vehicles, default_params, grid32, planar_graph, random_od
from workloads.roadgraph import RoadGraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    oracle.build(force=False)


def announce(name):
    print(f"\n[case] {name}", flush=True)


def same_routes(a, b):
    assert a["path_len"].tolist() == b["path_len"].tolist()
    assert a["cost_ms"].tolist() == b["cost_ms"].tolist()
    for v in range(a["path_len"].shape[0]):
        L = int(a["path_len"][v])
        assert a["path_edges"][v, :L].tolist() == b["path_edges"][v, :L].tolist(), v


def with_base_load(g, load):
    d = dict(g.__dict__)
    d["base_load"] = np.ascontiguousarray(load, np.uint32)
    return RoadGraph(**d)


@pytest.mark.parametrize("kernel", ["", "lds", "global"])
def test_resume_equals_straight_run(monkeypatch, kernel):
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    announce(f"resume grid32 {kernel or 'plan'}")
    w = grid32(vehicles=40, ants=16, iterations=10)
    g, V, p = w.graph, w.vehicles, w.params
    I, I1 = p["iterations"], 4
    want = oracle.route(g, V, p)
    G = gmacop.gmacop_graph_create(g)
    H = gmacop.gmacop_graph_create(g)
    try:
        straight = gmacop.gmacop_route_batch(G, V, p)
        tau_s, load_s = gmacop.gmacop_state_get(G)
        same_routes(straight, want)
        assert np.array_equal(tau_s, want["tau"]) and np.array_equal(load_s, want["load"])
        # first part on G, then the rest on a fresh handle H from the saved state
        r1 = gmacop.gmacop_route_batch(G, V, dict(p, iterations=I1))
        tau1, load1 = gmacop.gmacop_state_get(G)
        gmacop.gmacop_state_set(H, tau1, load1)
        rest = dict(p, iterations=I - I1, iter_offset=I1, flags=p["flags"] | gmacop.RESUME)
        r2 = gmacop.gmacop_route_batch(H, V, rest, held=r1)
        same_routes(r2, want)
        tau2, load2 = gmacop.gmacop_state_get(H)
        assert np.array_equal(tau2, want["tau"]) and np.array_equal(load2, want["load"])
        assert r1["steps_total"] + r2["steps_total"] == want["steps_total"]
        # the same on G itself, whose state is still the saved one, replayed as a HIP graph
        import torch
        s = torch.cuda.Stream()
        b = gmacop.DeviceBatch(V, p["max_steps"])
        gmacop.gmacop_route_batch_device(G, b, dict(p, iterations=I1), s.cuda_stream)
        gmacop.gmacop_route_batch_device(G, b, dict(rest, flags=rest["flags"] | gmacop.HIP_GRAPH), s.cuda_stream)
        s.synchronize()
        r3 = b.result()
        same_routes(r3, want)
        tau3, load3 = gmacop.gmacop_state_get(G)
        assert np.array_equal(tau3, want["tau"]) and np.array_equal(load3, want["load"])
    finally:
        gmacop.gmacop_release(G)
        gmacop.gmacop_release(H)


def test_resume_checks():
    announce("resume checks")
    w = grid32(vehicles=8, ants=4, iterations=2)
    G = gmacop.gmacop_graph_create(w.graph)
    try:
        r = gmacop.gmacop_route_batch(G, w.vehicles, w.params)
        with pytest.raises(gmacop.GmacopError) as e:
            gmacop.gmacop_route_batch(G, w.vehicles, dict(w.params, mode=gmacop.MODE_INDEPENDENT,
                                                          flags=gmacop.RESUME), held=r)
        assert e.value.code == gmacop.E_UNSUPPORTED
        bad = {k: v.copy() if hasattr(v, "copy") else v for k, v in r.items()}
        bad["path_len"][0] = 3
        bad["path_edges"][0, :3] = [0, w.graph.m, 1]
        with pytest.raises(gmacop.GmacopError) as e:
            gmacop.gmacop_route_batch(G, w.vehicles, dict(w.params, flags=gmacop.RESUME), held=bad)
        assert e.value.code == gmacop.E_INVAL
        with pytest.raises(ValueError):
            gmacop.gmacop_state_set(G, np.zeros(3, np.uint32))
    finally:
        gmacop.gmacop_release(G)


@pytest.mark.parametrize("mode", [0, 1])
def test_base_load_epoch_matches_oracle(mode):
    announce(f"base load epoch mode{mode}")
    rng = np.random.default_rng(51)
    w = grid32(vehicles=32, ants=16, iterations=6)
    g, V = w.graph, w.vehicles
    p = dict(w.params, mode=mode)
    new_load = rng.poisson(6.0, size=g.m).astype(np.uint32)      # a busier epoch
    G = gmacop.gmacop_graph_create(g)
    try:
        before = gmacop.gmacop_route_batch(G, V, p)
        same_routes(before, oracle.route(g, V, p, want_state=False))
        gmacop.gmacop_set_base_load(G, new_load)
        after = gmacop.gmacop_route_batch(G, V, p)
        want = oracle.route(with_base_load(g, new_load), V, p)
        same_routes(after, want)
        assert after["steps_total"] == want["steps_total"]
        if mode == 0:
            tau, load = gmacop.gmacop_state_get(G)
            assert np.array_equal(tau, want["tau"]) and np.array_equal(load, want["load"])
    finally:
        gmacop.gmacop_release(G)


@pytest.mark.parametrize("kernel", ["", "global"])
def test_router_base_load_epoch(monkeypatch, kernel):
    """Queries admitted after gmacop_server_set_base_load are routed on the
    new loads (oracle, independent mode); queries in flight across the epoch
    still return simple connected routes."""
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    announce(f"router epoch {kernel or 'plan'}")
    rng = np.random.default_rng(52)
    g = planar_graph(2500, rng)
    p = default_params(ants=16, iterations=5, max_steps=300, vmax_kmh=70, mode=gmacop.MODE_INDEPENDENT)
    V1 = random_od(g.n, 12, rng, qid0=0)
    V2 = random_od(g.n, 12, rng, qid0=100)
    new_load = rng.poisson(7.0, size=g.m).astype(np.uint32)
    G = gmacop.gmacop_graph_create(g)
    try:
        srv = gmacop.Server(G, p, max_slots=16)
        od1 = np.stack([V1.qid, V1.src, V1.dst], axis=1).astype(np.uint32)
        od2 = np.stack([V2.qid, V2.src, V2.dst], axis=1).astype(np.uint32)
        results = {}
        na, done = srv.step(od1[:6])
        assert na == 6
        for _ in range(2):
            na, done = srv.step(od1[6:6])
            results.update({q: (pa, c) for q, pa, c in done})
        srv.set_base_load(new_load)                     # six queries in flight across the epoch
        pos = 0
        for _ in range(100):
            k = min(4, od2.shape[0] - pos)
            na, done = srv.step(od2[pos:pos + k])
            pos += na
            results.update({q: (pa, c) for q, pa, c in done})
            if pos == od2.shape[0] and srv.active() == 0:
                break
        srv.release()
    finally:
        gmacop.gmacop_release(G)
    want = oracle.route(with_base_load(g, new_load), V2, p, want_state=False)
    for v in range(len(V2)):
        path, cost = results[int(V2.qid[v])]
        L = int(want["path_len"][v])
        assert cost == int(want["cost_ms"][v]) and path.tolist() == want["path_edges"][v, :L].tolist(), v
    tails = g.tail()
    for v in range(6):                                   # across the epoch: valid routes
        path, cost = results[int(V1.qid[v])]
        if len(path):
            assert tails[path[0]] == V1.src[v] and g.col[path[-1]] == V1.dst[v]
            assert np.all(tails[path[1:]] == g.col[path[:-1]])
