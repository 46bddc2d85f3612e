"""Exact goal term (Calc_Dist as the shortest free-flow time to the
destination) on the GPU against the oracle, through the C ABI: the search's
rows element by element, the shortest-route baseline, and whole routing runs
with the exact term on every walker kind, both modes, packed cities and the
router.  Every comparison is exact."""
import numpy as np
import pytest

import oracle
from paper_2010_14244_amd import gmacop
from workloads import Vehicles, default_params, from_edges, grid32, grid_graph, pack_graphs, planar_graph, random_od

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


def one_way_graph(rng, n=300, m=1100):
    tails = rng.integers(0, n, size=m)
    heads = rng.integers(0, n - 1, size=m)
    heads = np.where(heads >= tails, heads + 1, heads)
    tails[:5] = n - 1
    return from_edges(n, tails, heads, len_dm=rng.integers(100, 9000, size=m),
                      speed_kmh=rng.choice([30, 50, 70], size=m), green_pm=rng.integers(200, 800, size=m),
                      cycle_ms=np.where(rng.random(n) < 0.5, 90000, 0))


def packed_cities(rng):
    gs = [grid_graph(5, 6, rng), planar_graph(700, rng), grid_graph(3, 9, rng), planar_graph(2500, rng)]
    return pack_graphs(gs), gs


@pytest.mark.parametrize("qcap", ["", "3"])
def test_goal_rows_match_oracle(monkeypatch, qcap):
    """Rows of the device search equal the oracle's Dijkstra rows, including
    nodes out of reach and other cities; qcap 3 forces frontier overflows,
    so most rounds scan the whole city."""
    monkeypatch.setenv("GMACOP_GOAL_QCAP", qcap)
    rng = np.random.default_rng(41)
    pk, _ = packed_cities(rng)
    sat = from_edges(7, [0, 1, 2, 3, 4], [1, 2, 3, 4, 5], len_dm=6_000_000, speed_kmh=1)
    for name, g in (("one_way", one_way_graph(rng)), ("planar4000", planar_graph(4000, rng)), ("packed", pk),
                    ("saturating_chain", sat)):
        announce(f"goal rows {name} qcap={qcap or 'default'}")
        dst = np.unique(np.concatenate([rng.integers(0, g.n, size=10), [g.n - 1, 0]])).astype(np.uint32)
        G = gmacop.gmacop_graph_create(g)
        try:
            got = gmacop.gmacop_goal_rows(G, dst)
        finally:
            gmacop.gmacop_release(G)
        p = default_params()
        for i, d in enumerate(dst.tolist()):
            want = oracle.goal_exact(g, p, d)
            assert got[i].tolist() == want.tolist(), (name, d)


def test_shortest_routes_match_oracle():
    rng = np.random.default_rng(42)
    pk, _ = packed_cities(rng)
    for name, g in (("planar3000", planar_graph(3000, rng)), ("one_way", one_way_graph(rng)), ("packed", pk)):
        announce(f"shortest routes {name}")
        if name == "packed":
            off = pk.inst_node_off.astype(np.int64)
            V = Vehicles(qid=np.arange(24, dtype=np.uint32),
                         src=np.concatenate([random_od(int(off[i + 1] - off[i]), 6, rng, node_lo=int(off[i])).src
                                             for i in range(4)]),
                         dst=np.zeros(24, np.uint32))
            dst = []
            for i in range(4):
                d = random_od(int(off[i + 1] - off[i]), 6, rng, node_lo=int(off[i])).dst
                dst.append(d)
            V = Vehicles(qid=V.qid, src=V.src, dst=np.concatenate(dst))
            keep = V.src != V.dst
            V = Vehicles(qid=V.qid[keep], src=V.src[keep], dst=V.dst[keep])
        else:
            V = random_od(g.n, 30, rng)
        S = 64 if name == "one_way" else 4096
        G = gmacop.gmacop_graph_create(g)
        try:
            got = gmacop.gmacop_shortest_routes(G, V, S)
        finally:
            gmacop.gmacop_release(G)
        p = default_params()
        t0, _ = oracle.edge_static(g, p)
        total = 0
        for v in range(len(V)):
            want = oracle.shortest_route(g, p, int(V.src[v]), int(V.dst[v]), S)
            L = int(got["path_len"][v])
            assert L == want.shape[0], (name, v)
            assert got["path_edges"][v, :L].tolist() == want.tolist(), (name, v)
            c = int(t0[want.astype(np.int64)].astype(np.int64).sum()) if L else 0xFFFFFFFF
            assert int(got["cost_ms"][v]) == c
            total += L
        assert got["steps_total"] == total


def run_both(g, V, p, name, state=True):
    announce(name)
    want = oracle.route(g, V, p)
    G = gmacop.gmacop_graph_create(g)
    try:
        got = gmacop.gmacop_route_batch(G, V, p)
        if p["mode"] == gmacop.MODE_SHARED and state:
            got["tau"], got["load"] = gmacop.gmacop_state_get(G)
    finally:
        gmacop.gmacop_release(G)
    assert got["steps_total"] == want["steps_total"], (got["steps_total"], want["steps_total"])
    assert got["path_len"].tolist() == want["path_len"].tolist()
    assert got["cost_ms"].tolist() == want["cost_ms"].tolist()
    for v in range(len(V)):
        L = int(want["path_len"][v])
        assert got["path_edges"][v, :L].tolist() == want["path_edges"][v, :L].tolist(), v
    if p["mode"] == gmacop.MODE_SHARED and state:
        assert np.array_equal(got["tau"], want["tau"]) and np.array_equal(got["load"], want["load"])
    return got, want


KINDS = pytest.mark.parametrize("kernel", ["", "lds", "global"])


@KINDS
@pytest.mark.parametrize("mode", [0, 1])
def test_exact_goal_grid32(monkeypatch, kernel, mode):
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    w = grid32(vehicles=40, ants=24, iterations=8)
    p = dict(w.params, mode=mode, flags=gmacop.GOAL_EXACT)
    run_both(w.graph, w.vehicles, p, f"exact grid32 {kernel or 'plan'} mode{mode}")


@KINDS
def test_exact_goal_planar_and_packed(monkeypatch, kernel):
    monkeypatch.setenv("GMACOP_WALK_KERNEL", kernel)
    rng = np.random.default_rng(43)
    g = planar_graph(3000, rng)
    V = random_od(g.n, 24, rng)
    p = default_params(ants=16, iterations=6, max_steps=400, flags=gmacop.GOAL_EXACT)
    got, want = run_both(g, V, p, f"exact planar3000 {kernel or 'plan'}")
    pk, gs = packed_cities(rng)
    off = pk.inst_node_off.astype(np.int64)
    vs = [random_od(gi.n, 5, rng, node_lo=int(off[i]), qid0=5 * i) for i, gi in enumerate(gs)]
    Vp = Vehicles(qid=np.concatenate([v.qid for v in vs]), src=np.concatenate([v.src for v in vs]),
                  dst=np.concatenate([v.dst for v in vs]))
    run_both(pk, Vp, dict(p, max_steps=300), f"exact packed {kernel or 'plan'}")


def test_exact_goal_raises_arrivals_on_planar():
    """Not a parity check: on a planar city the exact term lets far more
    ants arrive than the straight line does (the reason it exists)."""
    rng = np.random.default_rng(44)
    g = planar_graph(8000, rng)
    V = random_od(g.n, 64, rng)
    p = default_params(ants=16, iterations=4, max_steps=1024, vmax_kmh=70)
    G = gmacop.gmacop_graph_create(g)
    try:
        gmacop.gmacop_stats_get(G, reset=True)
        a = gmacop.gmacop_route_batch(G, V, p)
        s1 = gmacop.gmacop_stats_get(G, reset=True)
        b = gmacop.gmacop_route_batch(G, V, dict(p, flags=gmacop.GOAL_EXACT))
        s2 = gmacop.gmacop_stats_get(G, reset=True)
    finally:
        gmacop.gmacop_release(G)
    print(f"arrivals straight {s1['arrivals']} exact {s2['arrivals']}; routed {int((a['path_len'] > 0).sum())} vs "
          f"{int((b['path_len'] > 0).sum())} of {len(V)}", flush=True)
    assert s2["arrivals"] > s1["arrivals"] and (b["path_len"] > 0).sum() >= (a["path_len"] > 0).sum()


@pytest.mark.skip(reason="the router rejects GMACOP_GOAL_EXACT: a router run with it on the 1M-node city "
                         "faulted the GPU and the cause was not found (the search and the walkers pass their "
                         "batch tests)")
def test_exact_goal_router_matches_oracle():
    """Router with the exact term: every query's route equals an
    independent-mode oracle run of that query alone."""
    rng = np.random.default_rng(45)
    g = planar_graph(2500, rng)
    p = default_params(ants=16, iterations=5, max_steps=300, mode=gmacop.MODE_INDEPENDENT, flags=gmacop.GOAL_EXACT)
    V = random_od(g.n, 40, rng)
    announce("exact router planar2500")
    G = gmacop.gmacop_graph_create(g)
    try:
        srv = gmacop.Server(G, p, max_slots=16)
        od = np.stack([V.qid, V.src, V.dst], axis=1).astype(np.uint32)
        pos, results = 0, {}
        for step in range(200):
            k = min(3, od.shape[0] - pos)
            na, done = srv.step(od[pos:pos + k])
            pos += na
            for qid, path, cost in done:
                results[qid] = (path, cost)
            if len(results) == len(V):
                break
        srv.release()
    finally:
        gmacop.gmacop_release(G)
    assert len(results) == len(V)
    want = oracle.route(g, V, p, want_state=False)
    for v in range(len(V)):
        path, cost = results[int(V.qid[v])]
        L = int(want["path_len"][v])
        assert cost == int(want["cost_ms"][v]) and path.tolist() == want["path_edges"][v, :L].tolist(), v


def test_router_rejects_exact_goal():
    rng = np.random.default_rng(46)
    g = planar_graph(500, rng)
    p = default_params(ants=8, iterations=3, max_steps=100, mode=gmacop.MODE_INDEPENDENT, flags=gmacop.GOAL_EXACT)
    G = gmacop.gmacop_graph_create(g)
    try:
        with pytest.raises(gmacop.GmacopError) as e:
            gmacop.Server(G, p, max_slots=4)
        assert e.value.code == gmacop.E_UNSUPPORTED
    finally:
        gmacop.gmacop_release(G)
