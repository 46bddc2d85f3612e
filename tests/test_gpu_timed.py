"""Time-dependent signals (GMACOP_SIGNAL_TIMED) on the GPU against the
oracle, through the C ABI: routes, costs, selections, final pheromone and
loads, exactly, in both modes, with either goal term and on packed cities."""
import numpy as np
import pytest

import oracle
from paper_2010_14244_amd import gmacop
from workloads import Vehicles, default_params, grid32, grid_graph, pack_graphs, planar_graph, random_od

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    oracle.build(force=False)


def check(g, V, p, name):
    print(f"\n[case] {name}", flush=True)
    want = oracle.route(g, V, p)
    G = gmacop.gmacop_graph_create(g)
    try:
        got = gmacop.gmacop_route_batch(G, V, p)
        tau, load = gmacop.gmacop_state_get(G)
    finally:
        gmacop.gmacop_release(G)
    assert got["steps_total"] == want["steps_total"], (got["steps_total"], want["steps_total"])
    assert got["path_len"].tolist() == want["path_len"].tolist()
    assert got["cost_ms"].tolist() == want["cost_ms"].tolist()
    for v in range(len(V)):
        L = int(want["path_len"][v])
        assert got["path_edges"][v, :L].tolist() == want["path_edges"][v, :L].tolist(), v
    if p["mode"] == gmacop.MODE_SHARED:
        assert np.array_equal(tau, want["tau"]) and np.array_equal(load, want["load"])


@pytest.mark.parametrize("flags", [0, gmacop.NO_LOAD_UPDATE, gmacop.GOAL_EXACT])
def test_timed_grid32_shared(flags):
    w = grid32(vehicles=40, ants=16, iterations=8)
    check(w.graph, w.vehicles, dict(w.params, flags=flags | gmacop.SIGNAL_TIMED, t_max_ms=30000),
          f"timed grid32 flags={flags}")


def test_timed_independent_and_planar():
    w = grid32(vehicles=24, ants=16, iterations=6)
    check(w.graph, w.vehicles, dict(w.params, mode=gmacop.MODE_INDEPENDENT, flags=gmacop.SIGNAL_TIMED),
          "timed grid32 independent")
    rng = np.random.default_rng(71)
    g = planar_graph(3000, rng)
    V = random_od(g.n, 24, rng)
    check(g, V, default_params(ants=16, iterations=6, max_steps=400, vmax_kmh=70, flags=gmacop.SIGNAL_TIMED),
          "timed planar3000")
    check(g, V, default_params(ants=16, iterations=6, max_steps=400, flags=gmacop.SIGNAL_TIMED | gmacop.GOAL_EXACT,
                               t_max_ms=5000), "timed planar3000 exact goal")


def test_timed_packed():
    rng = np.random.default_rng(72)
    gs = [grid_graph(5, 6, rng), planar_graph(700, rng), grid_graph(3, 9, rng)]
    pk = pack_graphs(gs)
    off = pk.inst_node_off.astype(np.int64)
    vs = [random_od(gi.n, 6, rng, node_lo=int(off[i]), qid0=6 * i) for i, gi in enumerate(gs)]
    V = Vehicles(qid=np.concatenate([v.qid for v in vs]), src=np.concatenate([v.src for v in vs]),
                 dst=np.concatenate([v.dst for v in vs]))
    check(pk, V, default_params(ants=12, iterations=6, max_steps=80, vmax_kmh=70, flags=gmacop.SIGNAL_TIMED),
          "timed packed")


def test_timed_rejected_where_unsupported():
    w = grid32(vehicles=4, ants=4, iterations=2)
    G = gmacop.gmacop_graph_create(w.graph)
    try:
        with pytest.raises(gmacop.GmacopError) as e:
            gmacop.gmacop_route_batch(G, w.vehicles, dict(w.params, mode=gmacop.MODE_GREEDY, flags=gmacop.SIGNAL_TIMED))
        assert e.value.code == gmacop.E_UNSUPPORTED
        with pytest.raises(gmacop.GmacopError) as e:
            gmacop.Server(G, dict(w.params, flags=gmacop.SIGNAL_TIMED), max_slots=2)
        assert e.value.code == gmacop.E_UNSUPPORTED
    finally:
        gmacop.gmacop_release(G)


def test_timed_noalloc_and_hip_graph():
    import torch
    rng = np.random.default_rng(73)
    g = planar_graph(2000, rng)
    V = random_od(g.n, 20, rng)
    p = default_params(ants=16, iterations=5, max_steps=300, vmax_kmh=70, flags=gmacop.SIGNAL_TIMED)
    print("\n[case] timed noalloc and HIP graph", flush=True)
    want = oracle.route(g, V, p)
    G = gmacop.gmacop_graph_create(g)
    try:
        got = gmacop.gmacop_route_batch_noalloc(G, V, p)
        b = gmacop.DeviceBatch(V, p["max_steps"])
        gmacop.gmacop_route_batch_device(G, b, dict(p, flags=p["flags"] | gmacop.HIP_GRAPH),
                                         torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        r = b.result()
    finally:
        gmacop.gmacop_release(G)
    for x in (got, r):
        assert x["path_len"].tolist() == want["path_len"].tolist()
        assert x["cost_ms"].tolist() == want["cost_ms"].tolist()
        assert x["steps_total"] == want["steps_total"]
