"""gmacop_route_batch_noalloc (static per-GPU workspace, no device
allocation) against gmacop_route_batch, through the C ABI: identical paths,
costs, selection counts and final state, on two calls in a row, the second
with fewer vehicles, for each walker kind and both modes."""
import numpy as np
import pytest

from paper_2010_14244_amd import gmacop
from workloads import Vehicles, default_params, grid8, grid_graph, planar_graph, random_od

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def announce(name):
    print(f"\n[case] {name}", flush=True)


def head(veh, k):
    return Vehicles(qid=veh.qid[:k], src=veh.src[:k], dst=veh.dst[:k])


def same(a, b, S):
    assert a["steps_total"] == b["steps_total"], (a["steps_total"], b["steps_total"])
    assert a["path_len"].tolist() == b["path_len"].tolist()
    assert a["cost_ms"].tolist() == b["cost_ms"].tolist()
    for v in range(a["path_len"].shape[0]):
        L = int(a["path_len"][v])
        assert a["path_edges"][v, :L].tolist() == b["path_edges"][v, :L].tolist(), v


def twice(g, veh, p, small):
    """noalloc then the allocating entry point on the same graph handle, for
    the whole batch and then for its first `small` vehicles."""
    G = gmacop.gmacop_graph_create(g)
    try:
        for batch in (veh, head(veh, small)):
            got = gmacop.gmacop_route_batch_noalloc(G, batch, p)
            tau_a, load_a = gmacop.gmacop_state_get(G)
            want = gmacop.gmacop_route_batch(G, batch, p)
            tau_b, load_b = gmacop.gmacop_state_get(G)
            same(got, want, p["max_steps"])
            if p["mode"] == gmacop.MODE_SHARED:
                assert np.array_equal(tau_a, tau_b) and np.array_equal(load_a, load_b)
            assert got["steps_total"] > 0
    finally:
        gmacop.gmacop_release(G)


def test_noalloc_shared_lds_walker():
    announce("noalloc: grid8 shared, 12 then 5 vehicles, LDS walker")
    w = grid8()
    rng = np.random.default_rng(3)
    veh = random_od(w.graph.n, 12, rng)
    p = dict(w.params, iterations=10)
    twice(w.graph, veh, p, 5)


def test_noalloc_shared_global_walker(monkeypatch):
    announce("noalloc: planar 3000 nodes shared, 40 then 9 vehicles, global walker")
    monkeypatch.setenv("GMACOP_WALK_KERNEL", "global")
    rng = np.random.default_rng(11)
    g = planar_graph(3000, rng)
    veh = random_od(g.n, 40, rng)
    p = default_params(ants=16, iterations=6, max_steps=512, vmax_kmh=70)
    twice(g, veh, p, 9)


def test_noalloc_independent_both_walkers(monkeypatch):
    for kind in ("lds", "global"):
        announce(f"noalloc: grid 12x12 independent, 30 then 7 vehicles, walker {kind}")
        monkeypatch.setenv("GMACOP_WALK_KERNEL", kind)
        rng = np.random.default_rng(5)
        g = grid_graph(12, 12, rng)
        veh = random_od(g.n, 30, rng)
        p = default_params(ants=24, iterations=8, max_steps=143, mode=gmacop.MODE_INDEPENDENT)
        twice(g, veh, p, 7)


def test_noalloc_device_pointers():
    import torch
    announce("noalloc: device pointers, grid8 shared, 16 then 3 vehicles")
    w = grid8()
    rng = np.random.default_rng(8)
    veh = random_od(w.graph.n, 16, rng)
    p = dict(w.params, iterations=7)
    G = gmacop.gmacop_graph_create(w.graph)
    try:
        s = torch.cuda.Stream()
        for k in (16, 3):
            b = gmacop.DeviceBatch(head(veh, k), p["max_steps"])
            gmacop.gmacop_route_batch_device(G, b, p, s.cuda_stream, noalloc=True)
            s.synchronize()
            got = b.result()
            want = gmacop.gmacop_route_batch(G, head(veh, k), p)
            same(got, want, p["max_steps"])
    finally:
        gmacop.gmacop_release(G)


def test_noalloc_rejects_oversized_calls_and_flags():
    announce("noalloc: size limit and flags")
    w = grid8()
    G = gmacop.gmacop_graph_create(w.graph)
    try:
        rng = np.random.default_rng(9)
        veh = random_od(w.graph.n, 8, rng)
        # 8 vehicles x 2^20 ants x 63 steps of path entries exceed the workspace
        with pytest.raises(gmacop.GmacopError) as e:
            gmacop.gmacop_route_batch_noalloc(G, veh, dict(w.params, ants=1 << 20, iterations=1))
        assert e.value.code == gmacop.E_NOMEM
        for fl in (gmacop.HIP_GRAPH, gmacop.TIME_KERNELS):
            with pytest.raises(gmacop.GmacopError) as e:
                gmacop.gmacop_route_batch_noalloc(G, veh, dict(w.params, flags=fl))
            assert e.value.code == gmacop.E_INVAL
        # the workspace is still usable and the results still match
        a = gmacop.gmacop_route_batch_noalloc(G, veh, dict(w.params, iterations=3))
        b = gmacop.gmacop_route_batch(G, veh, dict(w.params, iterations=3))
        same(a, b, w.params["max_steps"])
    finally:
        gmacop.gmacop_release(G)
