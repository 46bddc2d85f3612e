"""Traffic simulation of trips along routes (gmacop_simulate) against the
oracle's orc_simulate, through the C ABI: every vehicle's arrival and wait
and every scenario's tick count, exactly; road counts in LDS and in global
memory; several scenarios in one call."""
import numpy as np
import pytest

import oracle
from paper_2010_14244_amd import gmacop
from workloads import default_params, from_edges, grid_graph, planar_graph, random_od
from workloads.roadgraph import Vehicles

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="k_simulate was written after GPU use closed for this repository and has never run "
                            "on a GPU; a CPU transliteration of it equals the oracle, the kernel itself is unchecked"),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    oracle.build(force=False)


def routes(g, V, S=64):
    p = default_params()
    path = np.zeros((len(V), S), np.uint32)
    plen = np.zeros(len(V), np.uint32)
    for i in range(len(V)):
        r = oracle.shortest_route(g, p, int(V.src[i]), int(V.dst[i]), S)
        path[i, :len(r)] = r
        plen[i] = len(r)
    return path, plen


def check(g, p, path, plen, spd, name, tick_ms=1000, max_ticks=20000, scen_off=None):
    print(f"\n[case] {name}", flush=True)
    G = gmacop.gmacop_graph_create(g)
    try:
        got = gmacop.gmacop_simulate(G, p, path, plen, spd, scen_off, tick_ms=tick_ms, max_ticks=max_ticks)
    finally:
        gmacop.gmacop_release(G)
    off = [0, len(plen)] if scen_off is None else list(scen_off)
    for b in range(len(off) - 1):
        lo, hi = off[b], off[b + 1]
        want = oracle.simulate(g, p, path[lo:hi], plen[lo:hi], spd[lo:hi], tick_ms=tick_ms, max_ticks=max_ticks)
        assert got["arrival_ms"][lo:hi].tolist() == want["arrival_ms"].tolist(), (name, b)
        assert got["wait_ms"][lo:hi].tolist() == want["wait_ms"].tolist(), (name, b)
        assert int(got["ticks"][b]) == want["ticks"], (name, b)
    return got


def test_hand_cases():
    merge = from_edges(4, [0, 1, 2], [2, 2, 3], len_dm=1000, speed_kmh=36, green_pm=[900, 100, 1000],
                       cycle_ms=[0, 0, 100000, 0])
    paths = np.array([[1, 2], [0, 2], [0, 2], [0, 2], [0, 2]], np.uint32)
    spd = np.array([36, 36, 33, 30, 28], np.uint32)
    for t_max in (3000, 20000):
        check(merge, default_params(theta=1000, t_max_ms=t_max), paths, np.full(5, 2, np.uint32), spd,
              f"T_max guard {t_max}")
    one = from_edges(2, [0], [1], len_dm=1000, speed_kmh=36)
    for theta in (1, 4, 5):
        check(one, default_params(theta=theta), np.zeros((5, 1), np.uint32), np.ones(5, np.uint32),
              np.full(5, 36, np.uint32), f"congestion theta={theta}")


@pytest.mark.parametrize("where", ["lds", "global"])
def test_random_and_converging_traffic(monkeypatch, where):
    monkeypatch.setenv("GMACOP_SIM_GLOBAL", "1" if where == "global" else "")
    rng = np.random.default_rng(95)
    for trial in range(4):
        g = grid_graph(6, 7, rng) if trial % 2 == 0 else planar_graph(300, rng)
        p = default_params(theta=int(rng.integers(2, 10)), th_max=int(rng.integers(1, 6)),
                           t_max_ms=int(rng.integers(2, 40)) * 1000)
        if trial < 2:
            V = random_od(g.n, 150, rng)
        else:   # every vehicle to one of two destinations: competing queues
            dsts = rng.choice(g.n, size=2, replace=False)
            src = rng.integers(0, g.n, size=300)
            dst = dsts[rng.integers(0, 2, size=300)]
            keep = src != dst
            V = Vehicles(qid=np.arange(keep.sum(), dtype=np.uint32), src=src[keep].astype(np.uint32),
                         dst=dst[keep].astype(np.uint32))
        path, plen = routes(g, V)
        spd = rng.integers(50, 81, size=len(V)).astype(np.uint32)
        check(g, p, path, plen, spd, f"{where} trial {trial}", tick_ms=int(rng.choice([500, 1000])))


def test_scenarios_in_one_call():
    """Runs of the same network with 30 to 900 vehicles, one workgroup each."""
    rng = np.random.default_rng(96)
    g = grid_graph(7, 7, rng)
    sizes = [30, 300, 900, 0, 120]
    paths, plens, spds = [], [], []
    for n in sizes:
        V = random_od(g.n, n, rng) if n else Vehicles(qid=np.zeros(0, np.uint32), src=np.zeros(0, np.uint32),
                                                         dst=np.zeros(0, np.uint32))
        pa, pl = routes(g, V)
        paths.append(pa)
        plens.append(pl)
        spds.append(rng.integers(50, 81, size=len(V)).astype(np.uint32))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    check(g, default_params(theta=4), np.concatenate(paths), np.concatenate(plens), np.concatenate(spds),
          "scenarios", scen_off=off)


def test_rejections():
    g = from_edges(3, [0, 1], [1, 2], len_dm=1000, speed_kmh=36)
    G = gmacop.gmacop_graph_create(g)
    try:
        for path, plen, spd in ((np.array([[1, 0]]), [2], [36]), (np.array([[0, 7]]), [2], [36]),
                                (np.array([[0, 1]]), [2], [0]), (np.array([[0, 1]]), [3], [36])):
            with pytest.raises(gmacop.GmacopError) as e:
                gmacop.gmacop_simulate(G, default_params(), path, plen, spd)
            assert e.value.code == gmacop.E_INVAL
        with pytest.raises(gmacop.GmacopError):
            gmacop.gmacop_simulate(G, default_params(), np.array([[0, 1]]), [2], [36], tick_ms=0)
    finally:
        gmacop.gmacop_release(G)
