"""The literal MACO-P vehicle loop (GMACOP_MODE_GREEDY) on the GPU against the
oracle, through the C ABI: every route, cost, move count and final marker,
exactly."""
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


def check(g, V, p, name, noalloc=False):
    announce(name)
    p = dict(p, mode=gmacop.MODE_GREEDY)
    want = oracle.greedy(g, V, p)
    G = gmacop.gmacop_graph_create(g)
    try:
        fn = gmacop.gmacop_route_batch_noalloc if noalloc else gmacop.gmacop_route_batch
        got = fn(G, V, p)
        marker, load = gmacop.gmacop_state_get(G)
    finally:
        gmacop.gmacop_release(G)
    assert got["steps_total"] == want["steps_total"], (got["steps_total"], want["steps_total"])
    assert got["path_len"].tolist() == want["path_len"].tolist()
    assert got["cost_ms"].tolist() == want["cost_ms"].tolist()
    for v in range(len(V)):
        L = int(want["path_len"][v])
        assert got["path_edges"][v, :L].tolist() == want["path_edges"][v, :L].tolist(), v
    assert marker.tolist() == want["marker"].tolist()
    assert load.tolist() == np.asarray(g.base_load).tolist()
    return got, want


def test_greedy_hand_example():
    g = from_edges(5, [0, 0, 1, 2, 3], [1, 2, 3, 3, 4], len_dm=1000, speed_kmh=50, base_load=[2, 1, 0, 0, 0])
    V = Vehicles(qid=np.arange(3, dtype=np.uint32), src=np.array([0, 0, 1], np.uint32),
                 dst=np.array([4, 4, 4], np.uint32))
    got, want = check(g, V, default_params(theta=2, max_steps=8), "greedy hand example")
    assert want["path_edges"][0, :3].tolist() == [0, 2, 4] and want["marker"].tolist() == [0, 0, 0, 0, 2]


@pytest.mark.parametrize("theta", [1, 25, 1000])
def test_greedy_planar(theta):
    rng = np.random.default_rng(61)
    g = planar_graph(3000, rng)
    V = random_od(g.n, 60, rng)
    check(g, V, default_params(theta=theta, max_steps=2048), f"greedy planar3000 theta={theta}")


def test_greedy_packed_and_crowded():
    """Four cities (one block each), and a grid with more vehicles than a
    block has threads; a short tick limit leaves some vehicles without a
    route."""
    rng = np.random.default_rng(62)
    gs = [grid_graph(5, 6, rng), planar_graph(700, rng), grid_graph(3, 9, rng), planar_graph(2500, rng)]
    pk = pack_graphs(gs)
    off = pk.inst_node_off.astype(np.int64)
    vs = [random_od(gi.n, 12, rng, node_lo=int(off[i]), qid0=12 * i) for i, gi in enumerate(gs)]
    V = Vehicles(qid=np.concatenate([v.qid for v in vs]), src=np.concatenate([v.src for v in vs]),
                 dst=np.concatenate([v.dst for v in vs]))
    check(pk, V, default_params(theta=5, max_steps=400), "greedy packed")
    w = grid32(vehicles=2500)
    check(w.graph, w.vehicles, default_params(theta=2000, max_steps=1023), "greedy grid32 2500 vehicles")
    got, want = check(w.graph, w.vehicles, default_params(theta=100, max_steps=12), "greedy grid32 12 ticks")
    assert (want["path_len"] == 0).any() and (want["path_len"] > 0).any()


def test_greedy_noalloc_and_device_buffers():
    import torch
    rng = np.random.default_rng(63)
    g = planar_graph(2000, rng)
    V = random_od(g.n, 30, rng)
    p = default_params(theta=10, max_steps=1024)
    got, want = check(g, V, p, "greedy noalloc", noalloc=True)
    G = gmacop.gmacop_graph_create(g)
    try:
        b = gmacop.DeviceBatch(V, p["max_steps"])
        gmacop.gmacop_route_batch_device(G, b, dict(p, mode=gmacop.MODE_GREEDY, flags=gmacop.HIP_GRAPH),
                                         torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        r = b.result()
    finally:
        gmacop.gmacop_release(G)
    assert r["path_len"].tolist() == want["path_len"].tolist() and r["cost_ms"].tolist() == want["cost_ms"].tolist()
    assert r["steps_total"] == want["steps_total"]
