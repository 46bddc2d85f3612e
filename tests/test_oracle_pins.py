"""Pins of the CPU oracle to facts fixed outside it: an independent Philox
implementation (rocRAND), Python's exact integer square root, hand-worked
examples, closed forms, exact roulette partition boundaries, chi-square
frequency tests, brute-force path enumeration, Dijkstra optimality bounds and
invariants.  No GPU needed."""
import json
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra
from scipy.stats import chisquare

from workloads import default_params, from_edges, grid_graph, grid8, grid32, pack_graphs, planar_graph, random_od
from workloads.roadgraph import Vehicles

HERE = os.path.dirname(os.path.abspath(__file__))


def veh(src, dst, qid=None):
    src = np.atleast_1d(np.asarray(src, np.uint32))
    dst = np.atleast_1d(np.asarray(dst, np.uint32))
    q = np.arange(src.shape[0], dtype=np.uint32) if qid is None else np.atleast_1d(np.asarray(qid, np.uint32))
    return Vehicles(qid=q, src=src, dst=dst)


# ---------------------------------------------------------------------------
# random numbers
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "philox_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_rocrand_ref.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return exe


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 0, 0, 0, 0, 0), (0, 0, 1, 0, 0, 0),
             (0x12345678, 0x9ABCDEF0, 3, 5, 49, 1023)]
    for _ in range(60):
        cases.append(tuple(int(v) for v in rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)))
    args = [hex(v) for c in cases for v in c]
    out = subprocess.check_output([rocrand_ref] + args, text=True).split("\n")
    for c, line in zip(cases, out):
        want = [int(w, 16) for w in line.split()]
        got = orc.philox4x32_10(c[2:], c[:2]).tolist()
        assert got == want, (c, got, want)


# ---------------------------------------------------------------------------
# integer square root
# ---------------------------------------------------------------------------

def test_isqrt_matches_python(orc):
    rng = np.random.default_rng(3)
    xs = [0, 1, 2, 3, 4, 2 ** 64 - 1, 2 ** 63, 2 ** 62 - 1]
    for b in range(1, 64):
        xs += [int(v) for v in rng.integers(0, 2 ** b, size=40, dtype=np.uint64)]
    roots = [int(v) for v in rng.integers(0, 2 ** 32, size=300, dtype=np.uint64)]
    for r in roots:
        for d in (-1, 0, 1):
            v = r * r + d
            if 0 <= v < 2 ** 64:
                xs.append(v)
    for x in xs:
        assert orc.isqrt(x) == math.isqrt(x), x


# ---------------------------------------------------------------------------
# hand-worked intersection
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def worked():
    with open(os.path.join(HERE, "golden", "intersection_worked_example.json")) as f:
        return json.load(f)


def worked_graph(w, load):
    gd = w["graph"]
    t = [a for a, b in gd["roads_tail_head"]]
    h = [b for a, b in gd["roads_tail_head"]]
    # roads are listed in CSR order already (sorted by tail)
    return from_edges(gd["n"], t, h, len_dm=gd["len_dm"], speed_kmh=gd["speed_kmh"], green_pm=gd["green_pm"],
                      cycle_ms=gd["cycle_ms"], x_dm=gd["x_dm"], y_dm=gd["y_dm"], base_load=load)


def test_worked_static(orc, worked):
    g = worked_graph(worked, 0)
    p = default_params(**worked["params"])
    t0, wf = orc.edge_static(g, p)
    assert t0.tolist() == worked["t0_ms"]["value"]
    assert wf.tolist() == worked["wf_ms"]["value"]


def test_worked_cost_and_preemption(orc, worked):
    p = default_params(**worked["params"])
    for sc in worked["scenarios"]:
        g = worked_graph(worked, sc["load"])
        cost, pre = orc.cost_table(g, p, np.asarray(sc["load"], np.uint32))
        assert pre.tolist() == sc["preempted"], sc["derivation"]
        assert cost.tolist() == sc["cost_ms"], sc["derivation"]


def test_worked_goal_and_eta(orc, worked):
    p = default_params(**worked["params"])
    sc = worked["scenarios"][0]
    g = worked_graph(worked, sc["load"])
    ge = worked["goal_and_eta"]
    assert (360 * 65536) // p["vmax_kmh"] == ge["k"]
    for node, h in ge["h_ms"].items():
        assert orc.goal(g, p, int(node), ge["dst"]) == h
    cost = sc["cost_ms"]
    h4 = ge["h_ms"]["4"]
    for road, eta in ge["eta_from_node_4_scenario_0"].items():
        head = worked["graph"]["roads_tail_head"][int(road)][1]
        delta = cost[int(road)] + ge["h_ms"][str(head)] - h4
        assert orc.eta(delta) == eta


# ---------------------------------------------------------------------------
# closed forms and special cases of single steps
# ---------------------------------------------------------------------------

def test_static_edge_cases(orc):
    g = from_edges(3, [0, 1, 1], [1, 0, 2], len_dm=[1, 10 ** 9, 1000], speed_kmh=[65535, 1, 36],
                   cycle_ms=[0, 0, 4 * 10 ** 9], green_pm=[500, 500, 0])
    p = default_params(t_max_ms=4 * 10 ** 9)
    t0, wf = orc.edge_static(g, p)
    assert t0[0] == 1                         # 360/65535 floors to 0 -> at least 1 ms
    assert t0[1] == 2 ** 31                   # 3.6e11 ms capped
    assert t0[2] == 10000                     # 1000*360/36
    assert wf[2] == (4 * 10 ** 9) ** 2 // (8 * 10 ** 9)   # all red: C/2
    assert wf[0] == 0 and wf[1] == 0          # heads 1, 0 unsignalised


def test_congestion_travel_threshold(orc):
    # one road 0->1, t0 = 7200; no signal.  travel = t0 while load <= theta
    g = from_edges(2, [0, 1], [1, 0], len_dm=1000)
    for theta in (1, 4, 7):
        p = default_params(theta=theta)
        for load in range(0, 30):
            cost, _ = orc.cost_table(g, p, np.array([load, 0], np.uint32))
            want = 7200 if load <= theta else (7200 * load) // theta
            assert cost[0] == want


def test_goal_is_lower_bound_of_travel_time(orc):
    """h(x) never exceeds the cheapest cost-table route from x to dst
    (straight line at the fastest speed is a lower bound)."""
    for w in (grid8(), grid32(iterations=1)):
        g, p = w.graph, w.params
        cost, _ = orc.cost_table(g, p, g.base_load)
        A = sp.csr_matrix((cost.astype(np.float64), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                          shape=(g.n, g.n))
        rng = np.random.default_rng(0)
        for dst in rng.integers(0, g.n, size=4):
            dist = dijkstra(A.T.tocsr(), indices=int(dst))     # to dst
            for x in rng.integers(0, g.n, size=40):
                assert orc.goal(g, p, int(x), int(dst)) <= dist[x] + 1e-9


def test_eta_closed_form(orc):
    two26 = 1 << 26
    cases = {two26: 1, two26 - 1: 1, two26 + 5: 1, 2 ** 40: 1, 1024: 65535, 1025: two26 // 1025,
             0: 65535, -5: 65535, -(2 ** 40): 65535, 1: 65535, 12343: 5436, 3000: two26 // 3000}
    for d, want in cases.items():
        assert orc.eta(d) == want, d


def _boundary(prefix_before, T):
    """Smallest 64-bit r with floor(r*T/2^64) >= prefix_before."""
    return -(-(prefix_before << 64) // T)


def test_roulette_partition_boundaries(orc):
    rng = np.random.default_rng(11)
    for trial in range(200):
        d = int(rng.integers(1, 9))
        w = [int(v) for v in rng.integers(0, 2 ** int(rng.integers(1, 60)), size=d, dtype=np.uint64)]
        if trial % 3 == 0:
            w[int(rng.integers(d))] = 0
        T = sum(w)
        if T == 0 or T >= 2 ** 64:
            continue
        P = 0
        for j, wj in enumerate(w):
            if wj == 0:
                continue
            lo = _boundary(P, T)                  # first r landing in bucket j
            hi = _boundary(P + wj, T) - 1         # last r landing in bucket j
            if lo <= hi:
                assert orc.roulette(w, lo) == j
                assert orc.roulette(w, hi) == j
                if lo > 0:
                    assert orc.roulette(w, lo - 1) != j
            P += wj
    # zero weights are never chosen; r at the extremes
    assert orc.roulette([0, 5, 0, 5], 0) == 1
    assert orc.roulette([0, 5, 0, 5], 2 ** 64 - 1) == 3
    assert orc.roulette([7], 2 ** 64 - 1) == 0


def test_roulette_frequencies_chi_square(orc):
    rng = np.random.default_rng(5)
    w = [1, 2, 3, 0, 10, 4]
    N = 60000
    counts = np.zeros(len(w))
    for r in rng.integers(0, 2 ** 64, size=N, dtype=np.uint64):
        counts[orc.roulette(w, int(r))] += 1
    assert counts[3] == 0
    nz = [j for j in range(len(w)) if w[j]]
    exp = np.array([w[j] for j in nz], float) / sum(w) * N
    assert chisquare(counts[nz], exp).pvalue > 1e-3


def test_evaporation_closed_form_half(orc):
    """rho = 1/2, no deposit: tau_t = max(tau_min, tau0 >> t) exactly."""
    p = default_params(rho_q16=0x8000, tau_min_q16=3)
    tau = 0x10000
    for t in range(1, 25):
        tau = orc.apply_tau(p, tau, 0, 0)
        assert tau == max(3, 0x10000 >> t)


def test_evaporation_error_bound_general_rho(orc):
    """tau0 (1-rho)^t - tau_t lies in [0, 1/rho) raw units while unclamped."""
    for rho in (1, 0x1000, 0x4000, 0x5555, 0xC000, 0xFFFF):
        p = default_params(rho_q16=rho, tau_min_q16=1, tau_max_q16=1 << 24)
        a = (65536 - rho) / 65536
        tau, exact = 1 << 24, float(1 << 24)
        for t in range(1, 60):
            tau = orc.apply_tau(p, tau, 0, 0)
            exact *= a
            if tau == 1:
                break
            err = exact - tau
            assert -1e-6 <= err < 65536 / rho + 1e-6


def test_apply_penalty_and_clamp(orc):
    p = default_params(rho_q16=0, theta=4, tau_min_q16=1, tau_max_q16=1 << 24)
    assert orc.apply_tau(p, 100, 1000, 4) == 1100            # load <= theta: full deposit
    assert orc.apply_tau(p, 100, 1000, 8) == 600             # 1000*4/8
    assert orc.apply_tau(p, 100, 7, 6) == 104                # floor(28/6) = 4
    assert orc.apply_tau(p, 100, 2 ** 62 + 3, 2 ** 32 - 1) == 1 << 24   # clamp high
    p2 = default_params(rho_q16=65536, tau_min_q16=9)
    assert orc.apply_tau(p2, 1000, 0, 0) == 9                # full evaporation -> tau_min
    # exact penalty on large deposits: floor(D*theta/load) by big-int arithmetic
    rng = np.random.default_rng(1)
    for _ in range(300):
        D = int(rng.integers(0, 2 ** 62, dtype=np.uint64))
        L = int(rng.integers(5, 2 ** 32, dtype=np.uint64))
        want = min(1 << 24, max(1, D * 4 // L))
        assert orc.apply_tau(p, 0, D, L) == want


# ---------------------------------------------------------------------------
# walks
# ---------------------------------------------------------------------------

def test_walk_chain_is_unique(orc):
    n = 7
    t = list(range(n - 1)) + list(range(1, n))
    h = list(range(1, n)) + list(range(n - 1))
    g = from_edges(n, t, h, len_dm=[1000 + 10 * i for i in range(2 * (n - 1))])
    p = default_params(max_steps=n - 1, vmax_kmh=0)
    cost, _ = orc.cost_table(g, p, g.base_load)
    tau = np.full(g.m, 0x10000, np.uint32)
    for ant in range(20):
        ok, path, cs, sel = orc.walk(g, p, tau, cost, 3, 0, n - 1, ant, 0)
        assert ok and sel == n - 1
        heads = g.col[path].tolist()
        assert heads == list(range(1, n))
        assert cs == int(cost[path].astype(np.int64).sum())


def test_walk_max_steps_and_dead_end(orc):
    # 0 -> 1 -> 2 (dead end: 2 only leads back to 1), 0 -> 3 -> 4
    g = from_edges(5, [0, 0, 1, 2, 3], [1, 3, 2, 1, 4])
    p = default_params(max_steps=10, vmax_kmh=0)
    cost, _ = orc.cost_table(g, p, g.base_load)
    tau = np.full(g.m, 0x10000, np.uint32)
    outcomes = set()
    for ant in range(200):
        ok, path, cs, sel = orc.walk(g, p, tau, cost, 0, 0, 4, ant, 0)
        outcomes.add((ok, tuple(g.col[path].tolist())))
    assert outcomes == {(True, (3, 4)), (False, (1, 2))}
    p1 = default_params(max_steps=1, vmax_kmh=0)
    ok, path, cs, sel = orc.walk(g, p1, tau, cost, 0, 0, 4, 0, 0)
    assert not ok and len(path) == 1 and sel == 1


def star_graph():
    """Node 0 with roads to 1, 2, 3 of free-flow time 2^20, 2^21, 2^22 ms
    (len 2^17, 2^18, 2^19 dm at 45 km/h: len*360/45 = 8*len), no signals,
    empty roads; each leads on to 4."""
    return from_edges(5, [0, 0, 0, 1, 2, 3], [1, 2, 3, 4, 4, 4],
                      len_dm=[2 ** 17, 2 ** 18, 2 ** 19, 1000, 1000, 1000], speed_kmh=45)


def test_first_step_frequencies_chi_square(orc):
    """eta = 2^26 / cost = 64, 32, 16 -> weights (beta=2) 4096 : 1024 : 256."""
    g = star_graph()
    p = default_params(max_steps=4, vmax_kmh=0, alpha=1, beta=2)
    cost, _ = orc.cost_table(g, p, g.base_load)
    assert cost[:3].tolist() == [2 ** 20, 2 ** 21, 2 ** 22]
    tau = np.full(g.m, 0x10000, np.uint32)
    N = 12000
    counts = np.zeros(3)
    for q in range(N):
        ok, path, cs, sel = orc.walk(g, p, tau, cost, q, 0, 4, 0, 0)
        assert ok
        counts[int(path[0])] += 1
    exp = np.array([16, 4, 1]) / 21 * N
    assert chisquare(counts, exp).pvalue > 1e-3


def test_uniform_walk_when_alpha_beta_zero(orc):
    g = star_graph()
    p = default_params(max_steps=4, vmax_kmh=0, alpha=0, beta=0)
    cost, _ = orc.cost_table(g, p, g.base_load)
    tau = np.arange(g.m, dtype=np.uint32) + 5
    N = 9000
    counts = np.zeros(3)
    for q in range(N):
        counts[int(orc.walk(g, p, tau, cost, q, 0, 4, 1, 2)[1][0])] += 1
    assert chisquare(counts, np.full(3, N / 3)).pvalue > 1e-3


def _enumerate_outcomes(g, cost, tau, src, dst, alpha, beta, max_steps):
    """All walk outcomes with their exact probabilities (goal term off):
    weight tau^alpha * eta^beta with eta = clamp(2^26 // cost, 1, 65535)."""
    out = {}

    def rec(u, visited, path, prob):
        if len(path) == max_steps:
            out[(False, tuple(path))] = out.get((False, tuple(path)), 0) + prob
            return
        rs, re = int(g.row_ptr[u]), int(g.row_ptr[u + 1])
        ws = []
        for e in range(rs, re):
            x = int(g.col[e])
            if x in visited:
                ws.append(0)
            else:
                eta = min(65535, max(1, (1 << 26) // max(1, int(cost[e]))))
                ws.append(int(tau[e]) ** alpha * eta ** beta)
        T = sum(ws)
        if T == 0:
            out[(False, tuple(path))] = out.get((False, tuple(path)), 0) + prob
            return
        for j, wj in enumerate(ws):
            if wj == 0:
                continue
            e = rs + j
            x = int(g.col[e])
            if x == dst:
                key = (True, tuple(path + [e]))
                out[key] = out.get(key, 0) + prob * wj / T
            else:
                rec(x, visited | {x}, path + [e], prob * wj / T)

    rec(src, {src}, [], 1.0)
    return out


def test_whole_path_distribution_3x3(orc):
    """Frequencies of complete walks on a 3x3 grid against exact path
    probabilities from brute-force enumeration of all self-avoiding walks."""
    rng = np.random.default_rng(2)
    g = grid_graph(3, 3, rng)
    p = default_params(max_steps=6, vmax_kmh=0)
    cost, _ = orc.cost_table(g, p, g.base_load)
    tau = rng.integers(1, 4, size=g.m).astype(np.uint32) * 0x4000
    probs = _enumerate_outcomes(g, cost, tau, 0, 8, 1, 2, p["max_steps"])
    assert abs(sum(probs.values()) - 1) < 1e-9
    N = 30000
    counts = {}
    for q in range(N):
        ok, path, cs, sel = orc.walk(g, p, tau, cost, q, 0, 8, 0, 0)
        key = (ok, tuple(int(e) for e in path))
        assert key in probs
        counts[key] = counts.get(key, 0) + 1
    keys = sorted(probs, key=lambda k: -probs[k])
    big = [k for k in keys if probs[k] * N >= 10]
    obs = [counts.get(k, 0) for k in big] + [N - sum(counts.get(k, 0) for k in big)]
    exp = [probs[k] * N for k in big] + [N * (1 - sum(probs[k] for k in big))]
    if exp[-1] < 5:
        obs[-2] += obs.pop()
        exp[-2] += exp.pop()
    exp = np.asarray(exp) * (sum(obs) / sum(exp))
    assert len(obs) > 5
    assert chisquare(obs, exp).pvalue > 1e-3


# ---------------------------------------------------------------------------
# whole runs
# ---------------------------------------------------------------------------

def _check_paths(g, veh_, res, max_steps):
    for v in range(len(veh_)):
        L = int(res["path_len"][v])
        if L == 0:
            assert res["cost_ms"][v] == 2 ** 32 - 1
            continue
        assert L <= max_steps
        path = res["path_edges"][v, :L].astype(np.int64)
        tails = g.tail()[path]
        heads = g.col[path]
        assert tails[0] == veh_.src[v] and heads[-1] == veh_.dst[v]
        assert np.all(tails[1:] == heads[:-1])                         # connected
        nodes = np.concatenate([[veh_.src[v]], heads])
        assert np.unique(nodes).shape[0] == nodes.shape[0]             # simple


def test_route_invariants_frozen_load(orc):
    """Loads frozen: every reported cost is the cost-table sum of its path,
    it is never below the Dijkstra optimum, best-so-far never increases, and
    pheromone stays within [tau_min, tau_max]."""
    w = grid32(vehicles=24, ants=16, iterations=8)
    g, V = w.graph, w.vehicles
    p = dict(w.params, flags=orc.FLAG_NO_LOAD_UPDATE)
    res = orc.route(g, V, p, want_hist=True)
    _check_paths(g, V, res, p["max_steps"])
    cost, _ = orc.cost_table(g, p, g.base_load)
    A = sp.csr_matrix((cost.astype(np.float64), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                      shape=(g.n, g.n))
    opt = dijkstra(A, indices=V.src.astype(np.int64))
    for v in range(len(V)):
        L = int(res["path_len"][v])
        assert L > 0
        pc = int(cost[res["path_edges"][v, :L].astype(np.int64)].astype(np.int64).sum())
        assert res["cost_ms"][v] == pc
        assert pc >= opt[v, V.dst[v]] - 1e-6
    hist = res["best_hist"].astype(np.int64)
    assert np.all(np.diff(hist, axis=0) <= 0)
    assert np.all(res["tau"] >= p["tau_min_q16"]) and np.all(res["tau"] <= p["tau_max_q16"])
    assert res["load"].tolist() == g.base_load.tolist()


def test_route_finds_optimum_on_tiny_graph(orc):
    rng = np.random.default_rng(4)
    g = grid_graph(3, 4, rng)
    V = veh([0, 11, 3], [11, 0, 8])
    p = default_params(ants=64, iterations=20, max_steps=11, flags=orc.FLAG_NO_LOAD_UPDATE, vmax_kmh=50)
    res = orc.route(g, V, p)
    cost, _ = orc.cost_table(g, p, g.base_load)
    A = sp.csr_matrix((cost.astype(np.float64), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                      shape=(g.n, g.n))
    opt = dijkstra(A, indices=V.src.astype(np.int64))
    for v in range(3):
        assert res["cost_ms"][v] == int(opt[v, V.dst[v]])


def test_shared_load_is_base_plus_best_route_count(orc):
    w = grid32(vehicles=40, ants=8, iterations=6)
    g, V, p = w.graph, w.vehicles, w.params
    res = orc.route(g, V, p, want_hist=True)
    _check_paths(g, V, res, p["max_steps"])
    cnt = np.zeros(g.m, np.int64)
    for v in range(len(V)):
        L = int(res["path_len"][v])
        np.add.at(cnt, res["path_edges"][v, :L].astype(np.int64), 1)
    assert (res["load"].astype(np.int64) - g.base_load.astype(np.int64)).tolist() == cnt.tolist()
    assert np.all(np.diff(res["best_hist"].astype(np.int64), axis=0) <= 0)


def test_tau_constant_without_evaporation_or_deposit(orc):
    w = grid8()
    p = dict(w.params, rho_q16=0, q_deposit=0, iterations=5)
    res = orc.route(w.graph, w.vehicles, p)
    assert np.all(res["tau"] == p["tau0_q16"])


def test_independent_vehicle_equals_alone(orc):
    """Independent mode: a vehicle's result does not depend on the others,
    and equals a shared-mode run of that vehicle alone with frozen loads."""
    w = grid32(vehicles=5, ants=8, iterations=5)
    g, V = w.graph, w.vehicles
    p = dict(w.params, mode=orc.MODE_INDEPENDENT)
    res = orc.route(g, V, p)
    for v in range(len(V)):
        one = Vehicles(qid=V.qid[v:v + 1], src=V.src[v:v + 1], dst=V.dst[v:v + 1])
        alone = orc.route(g, one, dict(w.params, flags=orc.FLAG_NO_LOAD_UPDATE))
        assert alone["cost_ms"][0] == res["cost_ms"][v]
        L = int(alone["path_len"][0])
        assert L == res["path_len"][v]
        assert alone["path_edges"][0, :L].tolist() == res["path_edges"][v, :L].tolist()
        assert alone["tau"].tolist() == res["tau"][v].tolist()


def test_packed_instances_equal_separate_runs(orc):
    rng = np.random.default_rng(9)
    gs = [grid_graph(4, 5, rng), planar_graph(300, rng), grid_graph(6, 3, rng)]
    packed = pack_graphs(gs)
    off = packed.inst_node_off.astype(np.int64)
    eoff = np.concatenate([[0], np.cumsum([x.m for x in gs])])
    vs, q0 = [], 0
    for i, gi in enumerate(gs):
        vs.append(random_od(gi.n, 4, rng, qid0=q0))
        q0 += 4
    p = default_params(ants=8, iterations=6, max_steps=40, vmax_kmh=70)
    allv = Vehicles(qid=np.concatenate([v.qid for v in vs]),
                    src=np.concatenate([v.src + off[i] for i, v in enumerate(vs)]).astype(np.uint32),
                    dst=np.concatenate([v.dst + off[i] for i, v in enumerate(vs)]).astype(np.uint32))
    res = orc.route(packed, allv, p)
    tot = 0
    for i, gi in enumerate(gs):
        r = orc.route(gi, vs[i], p)
        tot += r["steps_total"]
        sl = slice(4 * i, 4 * i + 4)
        assert r["cost_ms"].tolist() == res["cost_ms"][sl].tolist()
        assert r["path_len"].tolist() == res["path_len"][sl].tolist()
        for v in range(4):
            L = int(r["path_len"][v])
            assert (r["path_edges"][v, :L].astype(np.int64) + eoff[i]).tolist() == \
                res["path_edges"][4 * i + v, :L].tolist()
        assert r["tau"].tolist() == res["tau"][eoff[i]:eoff[i + 1]].tolist()
        assert r["load"].tolist() == res["load"][eoff[i]:eoff[i + 1]].tolist()
    assert tot == res["steps_total"]


def test_seed_and_iteration_offset_change_the_stream(orc):
    w = grid32(vehicles=8, ants=8, iterations=3)
    a = orc.route(w.graph, w.vehicles, w.params)
    b = orc.route(w.graph, w.vehicles, dict(w.params, seed=2))
    c = orc.route(w.graph, w.vehicles, dict(w.params, iter_offset=7))
    assert a["steps_total"] != b["steps_total"] or a["path_edges"].tolist() != b["path_edges"].tolist()
    assert a["steps_total"] != c["steps_total"] or a["path_edges"].tolist() != c["path_edges"].tolist()


def test_parameter_checks(orc):
    w = grid8()
    g, V, p = w.graph, w.vehicles, w.params
    assert orc.route_rc(g, V, p) == 0
    for bad in (dict(ants=0), dict(max_steps=0), dict(theta=0), dict(rho_q16=65537), dict(tau_min_q16=0),
                dict(tau0_q16=0x10, tau_min_q16=0x20), dict(tau0_q16=1 << 25), dict(mode=2)):
        assert orc.route_rc(g, V, dict(p, **bad)) == orc.E_INVAL, bad
    assert orc.route_rc(g, veh([5], [5]), p) == orc.E_INVAL
    assert orc.route_rc(g, veh([5], [64]), p) == orc.E_INVAL
    # bit budget: alpha*bits(tau_max) + 16*beta + ceil(log2(max degree)) <= 64
    assert orc.route_rc(g, V, dict(p, beta=2, alpha=1, tau_max_q16=2 ** 30)) == orc.E_RANGE  # 31+32+2 = 65
    assert orc.route_rc(g, V, dict(p, beta=2, alpha=1, tau_max_q16=2 ** 30 - 1)) == 0       # 30+32+2 = 64
    assert orc.route_rc(g, V, dict(p, beta=3, alpha=1, tau_max_q16=2 ** 24)) == orc.E_RANGE  # 25+48+2 = 75
    assert orc.route_rc(g, V, dict(p, q_deposit=2 ** 62)) == orc.E_RANGE


def test_deposit_closed_form_on_a_chain(orc):
    """Chain 0 -> 1 -> 2 (with the reverse roads): every ant takes the only
    route, cost C = 2 * 7200 ms.  With 3 ants each deposits floor(q / C) =
    455111 per road, so after iteration 1: tau = 65536/2 + 3*455111 =
    1398101; after iteration 2: floor(1398101/2) + 1365333 = 2064383.  The
    reverse roads only evaporate: 65536 >> 2 = 16384."""
    g = from_edges(3, [0, 1, 1, 2], [1, 0, 2, 1], len_dm=1000)
    V = veh([0], [2], qid=[4])
    p = default_params(ants=3, iterations=2, max_steps=2, vmax_kmh=0, rho_q16=0x8000, q_deposit=65536 * 100000)
    res = orc.route(g, V, p)
    assert res["cost_ms"][0] == 14400 and res["path_len"][0] == 2
    fwd = [0, 2]          # CSR order: (0,1), (1,0), (1,2), (2,1)
    back = [1, 3]
    assert [int(res["tau"][e]) for e in fwd] == [2064383, 2064383]
    assert [int(res["tau"][e]) for e in back] == [16384, 16384]
    assert res["load"].tolist() == [1, 0, 1, 0]


def _draw_top_bit(orc, seed, qid, ant, it, step):
    x = orc.philox4x32_10([qid, ant, it, step], [seed & 0xFFFFFFFF, seed >> 32])
    return int(x[1]) >> 31            # r = x1 * 2^32 + x0; r >= 2^63 iff top bit of x1


def test_equal_cost_route_found_later_does_not_replace_best(orc):
    """Diamond 0 -> {1, 2} -> 3, both routes cost the same, pheromone frozen
    (rho = 0, q = 0).  Every ant arrives with the same cost, so each
    iteration's best ant is ant 0, which takes road 0->1 iff its first draw
    is below 2^63.  The vehicle's best route must stay the one found in
    iteration 0 even when iteration 1's best ant takes the other branch."""
    g = from_edges(4, [0, 0, 1, 2], [1, 2, 3, 3], len_dm=1000)
    p = default_params(ants=2, iterations=2, max_steps=3, vmax_kmh=0, rho_q16=0, q_deposit=0)
    qid = next(q for q in range(1000) if _draw_top_bit(orc, p["seed"], q, 0, 0, 0) !=
               _draw_top_bit(orc, p["seed"], q, 0, 1, 0))
    res = orc.route(g, veh([0], [3], qid=[qid]), p)
    first_edge = 0 if _draw_top_bit(orc, p["seed"], qid, 0, 0, 0) == 0 else 1
    assert res["path_edges"][0, :2].tolist() == [first_edge, 2 + first_edge]
    assert res["cost_ms"][0] == 14400


# ---------------------------------------------------------------------------
# the random-number reading: counter layout and output word order
# ---------------------------------------------------------------------------

def _star_chain(stages):
    """Hubs 0, 4, 8, ..., 4*stages.  Hub 4k has three roads, to 4k+1, 4k+2
    and 4k+3, of free-flow time 2^20, 2^21 and 2^22 ms (lengths 2^17, 2^18,
    2^19 dm at 45 km/h); each of those nodes has one road on to hub 4k+4.
    No signals, empty roads."""
    tails, heads, lens = [], [], []
    for k in range(stages):
        h = 4 * k
        for b, ln in zip((1, 2, 3), (2 ** 17, 2 ** 18, 2 ** 19)):
            tails.append(h)
            heads.append(h + b)
            lens.append(ln)
        for b in (1, 2, 3):
            tails.append(h + b)
            heads.append(h + 4)
            lens.append(1000)
    return from_edges(4 * stages + 1, tails, heads, len_dm=lens, speed_kmh=45)


def test_walk_draws_follow_the_documented_counter_and_word_order(orc, rocrand_ref):
    """Known answers for the walk's choices.  At hub 4k (step s = 2k) the
    weights are tau * eta^2 with eta = 2^26 / cost = 64, 32, 16.  The draw of
    step s of ant `ant` of vehicle `qid` in iteration `it` is Philox4x32-10
    with key (seed low word, seed high word) and counter (qid, ant,
    iter_offset + it, s), read as r = x1 * 2^32 + x0; the road taken is the
    first whose inclusive prefix of weights exceeds floor(r * T / 2^64).  The
    draws come from rocRAND's engine, the bucket from exact integer
    arithmetic here, so a different counter layout or word order fails."""
    stages = 6
    g = _star_chain(stages)
    seed = 0x0123456789ABCDEF
    tau = np.full(g.m, 0x10000, np.uint32)
    w = [0x10000 * 64 ** 2, 0x10000 * 32 ** 2, 0x10000 * 16 ** 2]
    T = sum(w)
    cases = [(7, 3, 0, 0), (3, 7, 0, 0), (1000, 1, 5, 0), (12, 40, 2, 9), (0, 0, 0, 0), (0xFFFFFFFE, 63, 1, 4000),
             (99, 99, 11, 1), (2 ** 20 + 5, 5, 0, 123)]
    args, keys = [], []
    for qid, ant, it, off in cases:
        for k in range(stages):
            args += [hex(seed & 0xFFFFFFFF), hex(seed >> 32), hex(qid), hex(ant), hex(off + it), hex(2 * k)]
            keys.append((qid, ant, it, off, k))
    out = subprocess.check_output([rocrand_ref] + args, text=True).split("\n")
    expect = {}
    for key, line in zip(keys, out):
        x = [int(v, 16) for v in line.split()]
        r = (x[1] << 32) | x[0]
        target = (r * T) >> 64
        prefix, j = 0, None
        for jj, wj in enumerate(w):
            prefix += wj
            if prefix > target:
                j = jj
                break
        expect[key] = j
    chosen = {0: 0, 1: 0, 2: 0}
    for qid, ant, it, off in cases:
        p = default_params(max_steps=2 * stages, vmax_kmh=0, seed=seed, iter_offset=off)
        cost, _ = orc.cost_table(g, p, g.base_load)
        assert cost[:3].tolist() == [2 ** 20, 2 ** 21, 2 ** 22]
        ok, path, cs, sel = orc.walk(g, p, tau, cost, qid, 0, 4 * stages, ant, it)
        assert ok and sel == 2 * stages
        heads = g.col[path].tolist()
        for k in range(stages):
            j = heads[2 * k] - 4 * k - 1
            assert j == expect[(qid, ant, it, off, k)], (qid, ant, it, off, k)
            chosen[j] += 1
    assert min(chosen.values()) > 0         # every bucket was exercised


# ---------------------------------------------------------------------------
# step order of an iteration: apply the pheromone before the load update
# ---------------------------------------------------------------------------

def test_pheromone_is_penalised_by_the_load_the_ants_saw(orc):
    """Chain 0 -> 1 -> 2 with reverse roads (roads in CSR order: (0,1),
    (1,0), (1,2), (2,1)), free-flow 7200 ms each, no signals, sensed load 4
    on road (0,1), theta = 4, three ants, rho = 1/2, q = 65536 * 10^5, loads
    updated from the best routes.

    Iteration 0: loads (4,0,0,0), all roads cost 7200, the only route costs
    14400, each ant deposits floor(q / 14400) = 455111, D = 1365333 on roads
    0 and 2.  The apply uses the loads the ants saw: road 0 has load 4 <=
    theta, so tau = 32768 + 1365333 = 1398101 on both roads.  Then the load
    becomes (5,0,1,0).
    Iteration 1: road 0 costs floor(7200 * 5 / 4) = 9000, the route 16200,
    each ant deposits floor(q / 16200) = 404543, D = 1213629.  Road 0 is
    congested: D' = floor(1213629 * 4 / 5) = 970903, tau = floor(1398101 / 2)
    + 970903 = 1669953; road 2: 699050 + 1213629 = 1912679; reverse roads
    16384.  16200 is not cheaper than 14400, so the best route keeps cost
    14400 and the loads stay (5,0,1,0).  Applying after the load update would
    penalise iteration 0's deposit on road 0 (1125034 instead of 1398101)."""
    g = from_edges(3, [0, 1, 1, 2], [1, 0, 2, 1], len_dm=1000, base_load=[4, 0, 0, 0])
    p = default_params(ants=3, iterations=1, max_steps=2, vmax_kmh=0, rho_q16=0x8000, q_deposit=65536 * 100000,
                       theta=4)
    one = orc.route(g, veh([0], [2], qid=[4]), p)
    assert one["cost_ms"][0] == 14400
    assert one["tau"].tolist() == [1398101, 32768, 1398101, 32768]
    assert one["load"].tolist() == [5, 0, 1, 0]
    two = orc.route(g, veh([0], [2], qid=[4]), dict(p, iterations=2))
    assert two["cost_ms"][0] == 14400 and two["path_len"][0] == 2
    assert two["tau"].tolist() == [1669953, 16384, 1912679, 16384]
    assert two["load"].tolist() == [5, 0, 1, 0]


# ---------------------------------------------------------------------------
# exact goal term (Calc_Dist as the shortest free-flow time to the destination)
# ---------------------------------------------------------------------------

def _reverse_dijkstra(g, t0, dst):
    """Shortest free-flow time from every node to dst by scipy, as the
    oracle reports it: min(d, 2^32 - 2), and 2^32 - 1 where dst is out of reach."""
    tails = g.tail().astype(np.int64)
    heads = g.col.astype(np.int64)
    best = {}
    for u, x, w in zip(tails.tolist(), heads.tolist(), t0.tolist()):   # parallel roads: the faster one
        best[(u, x)] = min(w, best.get((u, x), w))
    keys = np.array(list(best.keys()), dtype=np.int64).reshape(-1, 2)
    A = sp.csr_matrix((np.array(list(best.values()), dtype=np.float64), (keys[:, 0], keys[:, 1])),
                      shape=(g.n, g.n))
    d = dijkstra(A.T.tocsr(), indices=int(dst))
    out = np.full(g.n, 0xFFFFFFFF, np.uint64)
    fin = np.isfinite(d)
    out[fin] = np.minimum(d[fin], 0xFFFFFFFE).astype(np.uint64)
    return out.astype(np.uint32)


def _one_way_graph(rng, n=70, m=260):
    """Random directed roads (some one-way, some parallel), with nodes that
    cannot reach others; signals on half the nodes."""
    tails = rng.integers(0, n, size=m)
    heads = rng.integers(0, n - 1, size=m)
    heads = np.where(heads >= tails, heads + 1, heads)
    tails[:5] = n - 1                # node n-1 only leaves: nothing reaches it
    return from_edges(n, tails, heads, len_dm=rng.integers(100, 9000, size=m),
                      speed_kmh=rng.choice([30, 50, 70], size=m), green_pm=rng.integers(200, 800, size=m),
                      cycle_ms=np.where(rng.random(n) < 0.5, 90000, 0))


def test_exact_goal_matches_scipy_dijkstra(orc):
    rng = np.random.default_rng(21)
    p = default_params(flags=orc.FLAG_GOAL_EXACT)
    cases = [(_one_way_graph(rng), None), (planar_graph(900, rng), None)]
    for g, _ in cases:
        t0, _ = orc.edge_static(g, p)
        for dst in rng.integers(0, g.n, size=8).tolist() + [g.n - 1]:
            want = _reverse_dijkstra(g, t0, dst)
            got = orc.goal_exact(g, p, dst)
            assert got.tolist() == want.tolist(), dst
            assert got[dst] == 0
    # the one-way graph has nodes that cannot reach some destinations
    g = cases[0][0]
    assert np.any(orc.goal_exact(g, p, g.n - 1) == 0xFFFFFFFF)


def test_exact_goal_saturates_and_marks_unreachable(orc):
    """Chain 0 -> 1 -> ... -> 5 of roads whose free-flow time is capped at
    2^31 ms (6e6 dm at 1 km/h); node 6 is isolated.  By hand: h(5) = 0,
    h(4) = 2^31, h(3..0) = 2^32 - 2 (saturated), h(6) = 2^32 - 1."""
    g = from_edges(7, [0, 1, 2, 3, 4], [1, 2, 3, 4, 5], len_dm=6_000_000, speed_kmh=1)
    p = default_params(flags=orc.FLAG_GOAL_EXACT)
    t0, _ = orc.edge_static(g, p)
    assert t0.tolist() == [2 ** 31] * 5
    assert orc.goal_exact(g, p, 5).tolist() == [0xFFFFFFFE] * 4 + [2 ** 31, 0, 0xFFFFFFFF]


def test_exact_goal_is_consistent_and_tight(orc):
    """Bellman's equations of shortest distances: along every road the term
    drops by at most the road's free-flow time, and from every node that
    reaches dst some road drops it by exactly that."""
    rng = np.random.default_rng(22)
    g = planar_graph(1500, rng)
    p = default_params(flags=orc.FLAG_GOAL_EXACT)
    t0, _ = orc.edge_static(g, p)
    tails = g.tail()
    for dst in rng.integers(0, g.n, size=4).tolist():
        h = orc.goal_exact(g, p, dst).astype(np.int64)
        assert np.all(h < 0xFFFFFFFE)                       # strongly connected, short distances
        slack = t0.astype(np.int64) + h[g.col] - h[tails]
        assert slack.min() >= 0
        tight = np.zeros(g.n, bool)
        tight[tails[slack == 0]] = True
        tight[dst] = True
        assert tight.all()


def diamond_with_signals():
    """0 -> 1 -> 3 and 0 -> 2 -> 3, every road 65536 ms of free flow (8192 dm
    at 45 km/h).  Node 1 and node 2 have 100 s signals; the approach 0 -> 1
    has 500 per mille green (wait 50000^2 / 200000 = 12500 ms), 0 -> 2 none
    (wait 100000^2 / 200000 = 50000, capped at T_max = 20000 ms); no loads."""
    return from_edges(4, [0, 0, 1, 2], [1, 2, 3, 3], len_dm=8192, speed_kmh=45,
                      green_pm=[500, 0, 1000, 1000], cycle_ms=[0, 100000, 100000, 0])


def test_exact_goal_first_step_frequencies(orc):
    """With the exact term h = (131072, 65536, 65536, 0) the reduced costs
    of the two first roads are their signal waits alone, 12500 and 20000 ms,
    so eta = floor(2^26 / delta) = 5368 and 3355 and (beta = 2) the first
    road is taken with probability 5368^2 / (5368^2 + 3355^2).  The
    straight-line term is 0 here (all coordinates equal), which would give
    eta = 859 and 784 instead."""
    g = diamond_with_signals()
    p = default_params(max_steps=3, vmax_kmh=0, alpha=1, beta=2, flags=orc.FLAG_GOAL_EXACT)
    cost, pre = orc.cost_table(g, p, g.base_load)
    assert cost.tolist() == [65536 + 12500, 65536 + 20000, 65536, 65536] and not pre.any()
    assert orc.goal_exact(g, p, 3).tolist() == [131072, 65536, 65536, 0]
    tau = np.full(g.m, 0x10000, np.uint32)
    N = 12000
    first = np.zeros(2)
    for q in range(N):
        ok, path, cs, sel = orc.walk(g, p, tau, cost, q, 0, 3, 0, 0)
        assert ok and len(path) == 2
        first[int(path[0])] += 1
    p1 = 5368 ** 2 / (5368 ** 2 + 3355 ** 2)
    assert chisquare(first, np.array([p1, 1 - p1]) * N).pvalue > 1e-3


@pytest.mark.parametrize("mode", [0, 1])
def test_exact_goal_routes_are_valid_and_bounded(orc, mode):
    """Whole runs with the exact term: simple connected routes whose cost is
    the cost-table sum of the path and never below the optimum; the tiny
    grid's optimum is reached."""
    w = grid32(vehicles=16, ants=16, iterations=6)
    g, V = w.graph, w.vehicles
    p = dict(w.params, mode=mode, flags=orc.FLAG_NO_LOAD_UPDATE | orc.FLAG_GOAL_EXACT)
    res = orc.route(g, V, p)
    _check_paths(g, V, res, p["max_steps"])
    cost, _ = orc.cost_table(g, p, g.base_load)
    A = sp.csr_matrix((cost.astype(np.float64), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                      shape=(g.n, g.n))
    opt = dijkstra(A, indices=V.src.astype(np.int64))
    for v in range(len(V)):
        L = int(res["path_len"][v])
        assert L > 0
        assert res["cost_ms"][v] == int(cost[res["path_edges"][v, :L].astype(np.int64)].astype(np.int64).sum())
        assert res["cost_ms"][v] >= opt[v, V.dst[v]] - 1e-6
    rng = np.random.default_rng(4)
    gt = grid_graph(3, 4, rng)
    Vt = veh([0, 11, 3], [11, 0, 8])
    pt = default_params(ants=64, iterations=20, max_steps=11, mode=mode,
                        flags=orc.FLAG_NO_LOAD_UPDATE | orc.FLAG_GOAL_EXACT)
    rt = orc.route(gt, Vt, pt)
    ct, _ = orc.cost_table(gt, pt, gt.base_load)
    At = sp.csr_matrix((ct.astype(np.float64), gt.col.astype(np.int64), gt.row_ptr.astype(np.int64)),
                       shape=(gt.n, gt.n))
    ot = dijkstra(At, indices=Vt.src.astype(np.int64))
    for v in range(3):
        assert rt["cost_ms"][v] == int(ot[v, Vt.dst[v]])


def test_shortest_route_is_a_shortest_path(orc):
    """The Dijkstra baseline: a simple connected src -> dst route whose
    free-flow time equals scipy's shortest distance, every road tight."""
    rng = np.random.default_rng(23)
    g = planar_graph(1200, rng)
    p = default_params()
    t0, _ = orc.edge_static(g, p)
    A = sp.csr_matrix((t0.astype(np.float64), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                      shape=(g.n, g.n))
    V = random_od(g.n, 12, rng)
    d = dijkstra(A, indices=V.src.astype(np.int64))
    tails = g.tail()
    for v in range(len(V)):
        path = orc.shortest_route(g, p, int(V.src[v]), int(V.dst[v]), 4096)
        assert path.shape[0] > 0
        assert tails[path[0]] == V.src[v] and g.col[path[-1]] == V.dst[v]
        assert np.all(tails[path[1:]] == g.col[path[:-1]])
        nodes = np.concatenate([[V.src[v]], g.col[path]])
        assert np.unique(nodes).shape[0] == nodes.shape[0]
        assert int(t0[path.astype(np.int64)].astype(np.int64).sum()) == int(d[v, V.dst[v]])


def test_shortest_route_ties_and_limits(orc):
    """Two equal routes 0 -> 1 -> 3 and 0 -> 2 -> 3: the first road in road
    order (0 -> 1, road 0) is taken.  Out of reach, or longer than the
    limit: empty."""
    g = from_edges(5, [0, 0, 1, 2], [1, 2, 3, 3], len_dm=1000, speed_kmh=50)
    p = default_params()
    assert orc.shortest_route(g, p, 0, 3, 8).tolist() == [0, 2]
    assert orc.shortest_route(g, p, 0, 4, 8).tolist() == []
    assert orc.shortest_route(g, p, 0, 3, 1).tolist() == []
    assert orc.shortest_route(g, p, 0, 1, 1).tolist() == [0]


# ---------------------------------------------------------------------------
# literal MACO-P vehicle loop (Fig. 3) in synchronous ticks
# ---------------------------------------------------------------------------

def greedy_diamond(base):
    """0 -> 1 -> 3 -> 4 and 0 -> 2 -> 3 -> 4, equal roads (exact terms 3T, 2T, 2T, T, 0);
    roads in id order: (0,1), (0,2), (1,3), (2,3), (3,4); `base` = initial markers."""
    return from_edges(5, [0, 0, 1, 2, 3], [1, 2, 3, 3, 4], len_dm=1000, speed_kmh=50, base_load=base)


def test_greedy_hand_derived_ticks(orc):
    """Vehicles A, B at 0 and C at 1, all to 4; markers (2, 1, 0, 0, 0); theta 2.
    Tick 0: N = 3 > 2, so A and B take the second least of (e1: 1, e0: 2), e0; C takes e2.
      M = 3: e0 -> 2 + 2 - 1 = 3, e1 -> max(0, 1 - 3) = 0, e2 -> max(0, 1 - 2) = 0, e3, e4 -> 0.
    Tick 1: N = 3: A, B take e2 (the only candidate), C takes e4 and arrives.
      M = 3: e0 -> 0, e2 -> 0 + 2 - 1 = 1, e4 -> max(0, 1 - 2) = 0.
    Tick 2: N = 2, not above 2: A and B take e4 and arrive.  M = 2: e4 -> 2, e2 -> 0.
    Routes A, B = (e0, e2, e4), C = (e2, e4); 8 moves; final markers (0, 0, 0, 0, 2)."""
    g = greedy_diamond([2, 1, 0, 0, 0])
    p = default_params(theta=2, max_steps=8)
    r = orc.greedy(g, veh([0, 0, 1], [4, 4, 4]), p)
    assert r["path_len"].tolist() == [3, 3, 2]
    assert r["path_edges"][0, :3].tolist() == [0, 2, 4] and r["path_edges"][1, :3].tolist() == [0, 2, 4]
    assert r["path_edges"][2, :2].tolist() == [2, 4]
    assert r["steps_total"] == 8
    assert r["marker"].tolist() == [0, 0, 0, 0, 2]
    cost, _ = orc.cost_table(g, p, g.base_load)
    assert r["cost_ms"].tolist() == [int(cost[[0, 2, 4]].sum())] * 2 + [int(cost[[2, 4]].sum())]
    # N = 3 is not above theta 3: the least marker, e1, for A and B
    r3 = orc.greedy(g, veh([0, 0, 1], [4, 4, 4]), dict(p, theta=3))
    assert r3["path_edges"][0, :3].tolist() == [1, 3, 4] and r3["path_edges"][1, :3].tolist() == [1, 3, 4]
    # equal markers: the lower road id
    re = orc.greedy(greedy_diamond([1, 1, 0, 0, 0]), veh([0], [4]), dict(p, theta=5))
    assert re["path_edges"][0, :3].tolist() == [0, 2, 4]
    # a tie for second place: 0 -> {1, 2, 3} -> 4 with markers (0, 1, 1): least e0, then e1 and e2 tied at 1;
    # two vehicles (N = 2 above theta 1) take the second least, the lower id e1, then e4
    fan = from_edges(5, [0, 0, 0, 1, 2, 3], [1, 2, 3, 4, 4, 4], len_dm=1000, speed_kmh=50,
                     base_load=[0, 1, 1, 0, 0, 0])
    rt = orc.greedy(fan, veh([0, 0], [4, 4]), dict(p, theta=1))
    assert rt["path_edges"][0, :2].tolist() == [1, 4] and rt["path_edges"][1, :2].tolist() == [1, 4]
    # one vehicle, one tick: the chosen road gains one, the others lose one (floored at zero)
    r1 = orc.greedy(greedy_diamond([4, 4, 4, 4, 4]), veh([0], [1]), dict(p, theta=5))
    assert r1["path_edges"][0, :1].tolist() == [0] and r1["marker"].tolist() == [5, 3, 3, 3, 3]


def test_greedy_routes_descend_to_the_destination(orc):
    """Every route: simple, connected, the exact term strictly decreasing
    along it, ending at the destination; cost = cost-table sum; moves =
    total length; vehicles whose destination is out of reach get none."""
    rng = np.random.default_rng(24)
    g = planar_graph(1500, rng)
    V = random_od(g.n, 40, rng)
    p = default_params(theta=20, max_steps=4096)
    r = orc.greedy(g, V, p)
    cost, _ = orc.cost_table(g, p, g.base_load)
    _check_paths(g, V, r, p["max_steps"])
    for v in range(len(V)):
        L = int(r["path_len"][v])
        assert L > 0
        h = orc.goal_exact(g, p, int(V.dst[v])).astype(np.int64)
        nodes = np.concatenate([[V.src[v]], g.col[r["path_edges"][v, :L]]]).astype(np.int64)
        assert np.all(np.diff(h[nodes]) < 0)
        assert r["cost_ms"][v] == int(cost[r["path_edges"][v, :L].astype(np.int64)].astype(np.int64).sum())
    assert r["steps_total"] == int(r["path_len"].sum())
    one_way = from_edges(4, [0, 1, 2], [1, 2, 1])            # 3 cannot be reached from 0
    ru = orc.greedy(one_way, veh([0], [3]), p)
    assert ru["path_len"].tolist() == [0] and ru["cost_ms"].tolist() == [0xFFFFFFFF]


# ---------------------------------------------------------------------------
# time-dependent signals (green windows, the ant's clock, the T_max guard)
# ---------------------------------------------------------------------------

def signal_star():
    """Roads 0->3, 1->3, 2->3 into a 100 s signal (greens 500, 300, 200 per
    mille), 3->4 and 4->5 into a 90 s signal at 5 (greens 700 then 600, which
    overrun the cycle), 5->6 unsignalised; every road 10 s of free flow
    (len 1000 dm at 36 km/h)."""
    return from_edges(7, [0, 1, 2, 3, 4, 3, 5], [3, 3, 3, 4, 5, 5, 6], len_dm=1000, speed_kmh=36,
                      green_pm=[500, 300, 200, 1000, 700, 600, 1000], cycle_ms=[0, 0, 0, 100000, 0, 90000, 0])


def test_signal_windows_by_hand(orc):
    """Node 3: windows [0, 50 s), [50, 80 s), [80, 100 s).  Node 5 (C = 90 s):
    roads 3->5 (600) and 4->5 (700) in road order: 3->5 is road 4, so
    [0, 54 s), then 4->5 from 54 s for 63 s (wrapping)."""
    g = signal_star()
    s, w = orc.signal_windows(g)
    order = list(zip(g.tail().tolist(), g.col.tolist()))
    got = {order[e]: (int(s[e]), int(w[e])) for e in range(g.m)}
    assert got[(0, 3)] == (0, 50000) and got[(1, 3)] == (50000, 30000) and got[(2, 3)] == (80000, 20000)
    assert got[(3, 5)] == (0, 54000) and got[(4, 5)] == (54000, 63000)
    assert got[(3, 4)] == (0, 0) and got[(5, 6)] == (0, 0)


def test_timed_wait_by_hand(orc):
    """Road 1->3 (window [50, 80 s) of 100 s, 10 s of travel): entered at
    35 s it reaches the signal at 45 s and waits 5 s; entered at 45 s it
    arrives in the green; entered at 80 s it would wait 60 s and is given the
    green after T_max = 20 s.  With the approach preempted (the longest
    queue) it never waits."""
    g = signal_star()
    p = default_params(t_max_ms=20000)
    e = [i for i, (a, b) in enumerate(zip(g.tail().tolist(), g.col.tolist())) if (a, b) == (1, 3)][0]
    assert orc.timed_cost(g, p, e, 35000) == 15000
    assert orc.timed_cost(g, p, e, 45000) == 10000
    assert orc.timed_cost(g, p, e, 80000) == 30000
    assert orc.timed_cost(g, p, e, 35000 + 3 * 100000) == 15000
    gl = from_edges(7, [0, 1, 2, 3, 4, 3, 5], [3, 3, 3, 4, 5, 5, 6], len_dm=1000, speed_kmh=36,
                    green_pm=[500, 300, 200, 1000, 700, 600, 1000], cycle_ms=[0, 0, 0, 100000, 0, 90000, 0],
                    base_load=[0, 3, 0, 0, 0, 0, 0])
    assert orc.timed_cost(gl, p, e, 35000) == 10000 and orc.timed_cost(gl, p, e, 80000) == 10000


def test_timed_waits_average_to_the_fixed_wait(orc):
    """Over one cycle of integer arrival times the waits of an approach with
    red time r sum to r(r+1)/2 (the uniform-arrival expectation behind the
    fixed-time wait floor(r^2 / 2C), up to the half-step)."""
    C, green = 2000, 300
    g = from_edges(3, [0, 1], [1, 2], len_dm=[1000, 1000], speed_kmh=36, green_pm=[green, 1000],
                   cycle_ms=[0, C, 0])
    p = default_params(t_max_ms=10 ** 6)
    travel = 10000
    total = sum(orc.timed_cost(g, p, 0, clock) - travel for clock in range(C))
    r = C - C * green // 1000
    assert total == r * (r + 1) // 2


def test_timed_route_costs_follow_the_clock(orc):
    """Whole runs with time-dependent signals and frozen loads: each reported
    route cost equals its roads' costs re-evaluated along the route with the
    clock (the cost so far) as entry time; the optimum of a tiny grid is
    reached under the timed costs too."""
    w = grid32(vehicles=12, ants=16, iterations=5)
    g, V = w.graph, w.vehicles
    p = dict(w.params, flags=orc.FLAG_NO_LOAD_UPDATE | orc.FLAG_SIGNAL_TIMED)
    res = orc.route(g, V, p)
    _check_paths(g, V, res, p["max_steps"])
    for v in range(len(V)):
        L = int(res["path_len"][v])
        assert L > 0
        clock = 0
        for e in res["path_edges"][v, :L].tolist():
            clock += orc.timed_cost(g, p, e, clock)
        assert res["cost_ms"][v] == clock


# ---------------------------------------------------------------------------
# traffic simulation of the trips (Section 5: routes driven through the
# preemptive signals; overall travel time)
# ---------------------------------------------------------------------------

def merge_graph(green_e0, green_e1, cycle=100000, speed=36):
    """Roads e0 = 0->2, e1 = 1->2, e2 = 2->3 (road ids in that order), 1000 dm
    each; node 2 signalised with the given greens (per mille) of a 100 s cycle,
    so e0's window is [0, C*g0/1000) and e1's follows it."""
    return from_edges(4, [0, 1, 2], [2, 2, 3], len_dm=1000, speed_kmh=speed,
                      green_pm=[green_e0, green_e1, 1000], cycle_ms=[0, 0, cycle, 0])


def test_sim_one_road_by_hand(orc):
    """1000 dm at 36 km/h: 360000 units of 1/360 dm, 36000 a tick: 10 ticks;
    at 30 km/h (the vehicle slower than the road) 12; 1001 dm at 36 km/h 11."""
    g = from_edges(2, [0], [1], len_dm=[1000], speed_kmh=36)
    p = default_params()
    assert orc.simulate(g, p, np.array([[0]]), [1], [36])["arrival_ms"].tolist() == [10000]
    assert orc.simulate(g, p, np.array([[0]]), [1], [30])["arrival_ms"].tolist() == [12000]
    assert orc.simulate(g, p, np.array([[0]]), [1], [90])["arrival_ms"].tolist() == [10000]   # the road's limit
    g1 = from_edges(2, [0], [1], len_dm=[1001], speed_kmh=36)
    r = orc.simulate(g1, p, np.array([[0]]), [1], [36])
    assert r["arrival_ms"].tolist() == [11000] and r["ticks"] == 11 and r["last_ms"] == 11000


def test_sim_unsignalised_crossing_takes_a_tick(orc):
    g = from_edges(3, [0, 1], [1, 2], len_dm=1000, speed_kmh=36)
    r = orc.simulate(g, default_params(), np.array([[0, 1]]), [2], [36])
    assert r["arrival_ms"].tolist() == [21000] and r["wait_ms"].tolist() == [0]


def test_sim_longest_queue_and_window(orc):
    """A on e0 and B1, B2 on e1 reach the stop line together (tick 10).
    e0's window [0, 10 s) has closed and B's queue (2) is the longest, so A
    waits one tick, then holds the only queue and passes: 22 s against 21 s.
    With Th_max = 0, A's queue of 1 exceeds it: green at once.  With the
    windows swapped (e0 [0, 90 s)), A passes in its window although B's queue
    is longer."""
    paths = np.array([[0, 2], [1, 2], [1, 2]])
    p = default_params()
    r = orc.simulate(merge_graph(100, 900), p, paths, [2, 2, 2], [36, 36, 36])
    assert r["arrival_ms"].tolist() == [22000, 21000, 21000] and r["wait_ms"].tolist() == [1000, 0, 0]
    r = orc.simulate(merge_graph(100, 900), dict(p, th_max=0), paths, [2, 2, 2], [36, 36, 36])
    assert r["arrival_ms"].tolist() == [21000, 21000, 21000]
    r = orc.simulate(merge_graph(900, 100), p, paths, [2, 2, 2], [36, 36, 36])
    assert r["arrival_ms"].tolist() == [21000, 21000, 21000] and r["mean_ms"] == 21000.0


def test_sim_t_max_guard(orc):
    """B1..B4 on e0 reach the stop line at ticks 10, 11, 12, 13 (36, 33, 30,
    28 km/h: 10, 11, 12, 13 ticks of travel), A on e1 at tick 10.  Every
    tick both queues hold one vehicle and the tie goes to e0, the lower road
    id; A's window [90, 100 s) is closed.  T_max = 3 s: A has waited 3 s at
    tick 13 and goes: 24 s.  T_max = 20 s: A goes at tick 14, once e0 is
    empty: 25 s.  The B's pass as they arrive and drive e2 at their own
    speeds too (10, 11, 12, 13 ticks): 21, 23, 25, 27 s."""
    g = merge_graph(900, 100)
    paths = np.array([[1, 2], [0, 2], [0, 2], [0, 2], [0, 2]])
    spd = [36, 36, 33, 30, 28]
    p = default_params(theta=1000)
    r = orc.simulate(g, dict(p, t_max_ms=3000), paths, [2] * 5, spd)
    assert r["arrival_ms"].tolist() == [24000, 21000, 23000, 25000, 27000]
    assert r["wait_ms"].tolist() == [3000, 0, 0, 0, 0]
    r = orc.simulate(g, dict(p, t_max_ms=20000), paths, [2] * 5, spd)
    assert r["arrival_ms"].tolist() == [25000, 21000, 23000, 25000, 27000] and r["wait_ms"][0] == 4000
    assert r["last_ms"] == 27000


def test_sim_congestion(orc):
    """Five vehicles on one road: above theta = 4 each covers
    floor(36 * 4 / 5) = 28 km/h, so ceil(360000 / 28000) = 13 ticks; at
    theta = 5 the road is not congested: 10 ticks."""
    g = from_edges(2, [0], [1], len_dm=1000, speed_kmh=36)
    paths = np.zeros((5, 1), np.uint32)
    assert orc.simulate(g, default_params(theta=4), paths, [1] * 5, [36] * 5)["arrival_ms"].tolist() == [13000] * 5
    assert orc.simulate(g, default_params(theta=5), paths, [1] * 5, [36] * 5)["arrival_ms"].tolist() == [10000] * 5
    r = orc.simulate(g, default_params(theta=1), paths, [1] * 5, [36] * 5)   # floor(36/5) = 7: 52 ticks
    assert r["arrival_ms"].tolist() == [52000] * 5


def test_sim_free_flow_closed_form(orc):
    """No signals, no congestion: a vehicle's trip is, road by road, the
    ticks its speed needs to cover the road, plus one tick per crossing."""
    rng = np.random.default_rng(91)
    g = grid_graph(6, 6, rng)
    g.cycle_ms[:] = 0
    p = default_params(theta=10**6)
    V = random_od(g.n, 40, rng)
    S = 64
    paths = np.zeros((len(V), S), np.uint32)
    plen = np.zeros(len(V), np.uint32)
    for i in range(len(V)):
        r = orc.shortest_route(g, p, int(V.src[i]), int(V.dst[i]), S)
        paths[i, :len(r)] = r
        plen[i] = len(r)
    spd = rng.integers(50, 81, size=len(V)).astype(np.uint32)
    tick = 700
    res = orc.simulate(g, p, paths, plen, spd, tick_ms=tick)
    for i in range(len(V)):
        if plen[i] == 0:
            assert res["arrival_ms"][i] == 0xFFFFFFFF
            continue
        ticks = int(plen[i]) - 1
        for e in paths[i, :plen[i]]:
            v = min(int(spd[i]), int(g.speed_kmh[e]))
            ticks += -(-int(g.len_dm[e]) * 360 // (v * tick))
        assert int(res["arrival_ms"][i]) == ticks * tick, i
    assert res["wait_ms"].sum() == 0


def test_sim_no_route_limit_and_rejections(orc):
    g = from_edges(3, [0, 1], [1, 2], len_dm=1000, speed_kmh=36)
    p = default_params()
    paths = np.array([[0, 1], [0, 0], [1, 0]])
    r = orc.simulate(g, p, paths, [2, 0, 1], [36, 36, 36])
    assert r["arrival_ms"].tolist() == [21000, 0xFFFFFFFF, 10000] and r["arrived"] == 2
    r = orc.simulate(g, p, paths[:1], [2], [36], max_ticks=15)          # cut before the end
    assert r["arrival_ms"].tolist() == [0xFFFFFFFF] and r["ticks"] == 15 and r["mean_ms"] is None
    for bad_paths, bad_len, bad_spd in ((np.array([[1, 0]]), [2], [36]),      # not connected
                                        (np.array([[0, 7]]), [2], [36]),      # road out of range
                                        (np.array([[0, 1]]), [2], [0]),       # no speed
                                        (np.array([[0, 1]]), [3], [36])):     # longer than its row
        with pytest.raises(ValueError):
            orc.simulate(g, p, bad_paths, bad_len, bad_spd)
