"""CPU oracle for the GMACO-P routing hot path -- TEST INFRASTRUCTURE ONLY.

A plain single-threaded C implementation (``gmacop_oracle.c``) of every step
the GPU library computes, loaded with ctypes.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg use it; the GPU library never calls
it and shares no code with it.

Paper: Jindal & Bedi, "GMACO-P: GPU assisted Preemptive MACO algorithm for
enabling Smart Transportation", arXiv 2010.14244 (Section 4.1 Fig. 3 MACO-P
vehicle loop; Section 4.2 Alg. 1 host driver and Alg. 2 kernel steps).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmacop_oracle.c")
_LIB = os.path.join(_HERE, "libgmacop_oracle.so")

MODE_SHARED = 0
MODE_INDEPENDENT = 1
FLAG_NO_LOAD_UPDATE = 1
FLAG_GOAL_EXACT = 16
FLAG_SIGNAL_TIMED = 64

E_INVAL = -1
E_RANGE = -2


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/libgmacop_oracle.so`` (gcc, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Graph(C.Structure):
    _fields_ = [("n", C.c_uint32), ("m", C.c_uint32),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("len_dm", C.c_void_p),
                ("speed_kmh", C.c_void_p), ("green_pm", C.c_void_p), ("cycle_ms", C.c_void_p),
                ("x_dm", C.c_void_p), ("y_dm", C.c_void_p), ("base_load", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("ants", C.c_uint32), ("iterations", C.c_uint32), ("alpha", C.c_uint32),
                ("beta", C.c_uint32), ("max_steps", C.c_uint32),
                ("rho_q16", C.c_uint32), ("tau0_q16", C.c_uint32), ("tau_min_q16", C.c_uint32),
                ("tau_max_q16", C.c_uint32), ("q_deposit", C.c_uint64),
                ("theta", C.c_uint32), ("th_max", C.c_uint32), ("t_max_ms", C.c_uint32),
                ("vmax_kmh", C.c_uint32), ("mode", C.c_uint32), ("flags", C.c_uint32),
                ("seed", C.c_uint64), ("iter_offset", C.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        alt = os.environ.get("GMACOP_ORACLE_LIB")     # a test build of the oracle (mutation tests)
        if alt:
            L = C.CDLL(alt)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB)
        vp, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_isqrt.argtypes = [u64]
        L.orc_isqrt.restype = u64
        L.orc_edge_static.argtypes = [vp, vp, vp, vp]
        L.orc_cost_table.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.orc_goal.argtypes = [vp, vp, u32, u32]
        L.orc_goal.restype = u64
        L.orc_goal_exact.argtypes = [vp, vp, u32, vp]
        L.orc_signal_windows.argtypes = [vp, vp, vp]
        L.orc_timed_cost.argtypes = [vp, vp, u32, u64]
        L.orc_timed_cost.restype = u32
        L.orc_greedy.argtypes = [vp, vp, vp, u32, vp, vp, vp, vp, vp, vp, vp]
        L.orc_greedy.restype = C.c_int
        L.orc_shortest_route.argtypes = [vp, vp, u32, u32, u32, vp]
        L.orc_shortest_route.restype = u32
        L.orc_eta.argtypes = [C.c_int64]
        L.orc_eta.restype = u32
        L.orc_roulette.argtypes = [vp, u32, u64]
        L.orc_roulette.restype = u32
        L.orc_apply_tau.argtypes = [vp, u32, u64, u32]
        L.orc_apply_tau.restype = u32
        L.orc_walk.argtypes = [vp, vp, vp, vp, u32, u32, u32, u32, u32, vp, vp, vp, vp]
        L.orc_walk.restype = C.c_int
        L.orc_route.argtypes = [vp, vp, vp, vp, u32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_route.restype = C.c_int
        L.orc_simulate.argtypes = [vp, vp, vp, u32, vp, vp, u32, u32, u32, vp, vp, vp]
        L.orc_simulate.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class _GraphRef:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, g):
        self.arrays = dict(row_ptr=np.ascontiguousarray(g.row_ptr, np.uint32),
                           col=np.ascontiguousarray(g.col, np.uint32),
                           len_dm=np.ascontiguousarray(g.len_dm, np.uint32),
                           speed_kmh=np.ascontiguousarray(g.speed_kmh, np.uint16),
                           green_pm=np.ascontiguousarray(g.green_pm, np.uint16),
                           cycle_ms=np.ascontiguousarray(g.cycle_ms, np.uint32),
                           x_dm=np.ascontiguousarray(g.x_dm, np.int32),
                           y_dm=np.ascontiguousarray(g.y_dm, np.int32),
                           base_load=np.ascontiguousarray(g.base_load, np.uint32))
        a = self.arrays
        self.n = a["row_ptr"].shape[0] - 1
        self.m = a["col"].shape[0]
        self.s = _Graph(self.n, self.m, *[_ptr(a[k]) for k in
                                          ("row_ptr", "col", "len_dm", "speed_kmh", "green_pm", "cycle_ms",
                                           "x_dm", "y_dm", "base_load")])


def _params(p: dict) -> _Params:
    return _Params(*[int(p[name]) for name, _ in _Params._fields_])


# ---------------------------------------------------------------------------
# step-level entry points (used by the pinning tests)
# ---------------------------------------------------------------------------

def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def isqrt(x: int) -> int:
    return int(lib().orc_isqrt(int(x)))


def edge_static(g, p: dict):
    gr, pp = _GraphRef(g), _params(p)
    t0 = np.zeros(gr.m, np.uint32)
    wf = np.zeros(gr.m, np.uint32)
    lib().orc_edge_static(C.byref(gr.s), C.byref(pp), _ptr(t0), _ptr(wf))
    return t0, wf


def cost_table(g, p: dict, load: np.ndarray):
    gr, pp = _GraphRef(g), _params(p)
    t0, wf = edge_static(g, p)
    load = np.ascontiguousarray(load, np.uint32)
    cost = np.zeros(gr.m, np.uint32)
    pre = np.zeros(gr.m, np.uint8)
    lib().orc_cost_table(C.byref(gr.s), C.byref(pp), _ptr(load), _ptr(t0), _ptr(wf), _ptr(cost), _ptr(pre))
    return cost, pre.astype(bool)


def goal(g, p: dict, node: int, dst: int) -> int:
    gr, pp = _GraphRef(g), _params(p)
    return int(lib().orc_goal(C.byref(gr.s), C.byref(pp), node, dst))


def goal_exact(g, p: dict, dst: int) -> np.ndarray:
    """Exact goal row for destination dst: uint32 [n] shortest free-flow
    time to dst (0xFFFFFFFF where dst cannot be reached)."""
    gr, pp = _GraphRef(g), _params(p)
    h = np.zeros(gr.n, np.uint32)
    lib().orc_goal_exact(C.byref(gr.s), C.byref(pp), int(dst), _ptr(h))
    return h


def shortest_route(g, p: dict, src: int, dst: int, max_len: int) -> np.ndarray:
    """Shortest free-flow route (road ids) from src to dst; empty when dst is
    out of reach, the time is capped, or the route exceeds max_len roads."""
    gr, pp = _GraphRef(g), _params(p)
    path = np.zeros(max(1, max_len), np.uint32)
    n = lib().orc_shortest_route(C.byref(gr.s), C.byref(pp), int(src), int(dst), int(max_len), _ptr(path))
    return path[:n].copy()


def signal_windows(g):
    """Per road: start (ms, modulo the head's cycle) and length of its approach's green."""
    gr = _GraphRef(g)
    s = np.zeros(gr.m, np.uint32)
    w = np.zeros(gr.m, np.uint32)
    lib().orc_signal_windows(C.byref(gr.s), _ptr(s), _ptr(w))
    return s, w


def timed_cost(g, p: dict, e: int, clock: int) -> int:
    """Cost of road e entered at time `clock` with time-dependent signals (sensed loads)."""
    gr, pp = _GraphRef(g), _params(p)
    return int(lib().orc_timed_cost(C.byref(gr.s), C.byref(pp), int(e), int(clock)))


def eta(delta: int) -> int:
    return int(lib().orc_eta(int(delta)))


def roulette(w, r: int) -> int:
    w = np.ascontiguousarray(w, dtype=np.uint64)
    return int(lib().orc_roulette(_ptr(w), w.shape[0], int(r)))


def apply_tau(p: dict, tau: int, deposit: int, load: int) -> int:
    pp = _params(p)
    return int(lib().orc_apply_tau(C.byref(pp), int(tau), int(deposit), int(load)))


def walk(g, p: dict, tau, cost, qid: int, src: int, dst: int, ant: int, it: int):
    """One ant walk; returns (arrived, path edges, cost sum, selections)."""
    gr, pp = _GraphRef(g), _params(p)
    tau = np.ascontiguousarray(tau, np.uint32)
    cost = np.ascontiguousarray(cost, np.uint32)
    path = np.zeros(max(1, p["max_steps"]), np.uint32)
    ln, cs, sel = C.c_uint32(0), C.c_uint32(0), C.c_uint64(0)
    ok = lib().orc_walk(C.byref(gr.s), C.byref(pp), _ptr(tau), _ptr(cost), qid, src, dst, ant, it,
                        _ptr(path), C.byref(ln), C.byref(cs), C.byref(sel))
    return bool(ok), path[:ln.value].copy(), int(cs.value), int(sel.value)


# ---------------------------------------------------------------------------
# whole run
# ---------------------------------------------------------------------------

def route(g, veh, p: dict, *, want_state: bool = True, want_hist: bool = False) -> dict:
    """Run the whole method on the CPU.  Returns dict with path_edges
    [V, max_steps], path_len [V], cost_ms [V], steps_total, and optionally
    tau/load (final state) and best_hist [iterations, V].  Raises on an
    invalid-parameter return code (the code is in ``err.args[1]``)."""
    gr, pp = _GraphRef(g), _params(p)
    qid = np.ascontiguousarray(veh.qid, np.uint32)
    src = np.ascontiguousarray(veh.src, np.uint32)
    dst = np.ascontiguousarray(veh.dst, np.uint32)
    V, S = src.shape[0], int(p["max_steps"])
    path = np.zeros((V, max(S, 1)), np.uint32)
    plen = np.zeros(V, np.uint32)
    cost = np.zeros(V, np.uint32)
    steps = C.c_uint64(0)
    n_tau = 1 if p["mode"] == MODE_SHARED else V
    tau = np.zeros(n_tau * gr.m, np.uint32) if want_state else None
    load = np.zeros(gr.m, np.uint32) if want_state else None
    hist = np.zeros((p["iterations"], V), np.uint32) if want_hist else None
    rc = lib().orc_route(C.byref(gr.s), _ptr(qid), _ptr(src), _ptr(dst), V, C.byref(pp),
                         _ptr(path), _ptr(plen), _ptr(cost), C.byref(steps), _ptr(tau), _ptr(load), _ptr(hist))
    if rc != 0:
        raise ValueError("oracle rejected input", rc)
    out = dict(path_edges=path, path_len=plen, cost_ms=cost, steps_total=int(steps.value))
    if want_state:
        out["tau"] = tau.reshape(n_tau, gr.m) if n_tau > 1 else tau
        out["load"] = load
    if want_hist:
        out["best_hist"] = hist
    return out


def route_rc(g, veh, p: dict) -> int:
    """Return code only (0, E_INVAL, E_RANGE)."""
    try:
        route(g, veh, p, want_state=False)
        return 0
    except ValueError as e:
        return e.args[1]


def greedy(g, veh, p: dict) -> dict:
    """Literal MACO-P vehicle loop (Fig. 3) in synchronous ticks: path_edges
    [V, max_steps], path_len, cost_ms, steps_total and the final markers."""
    gr, pp = _GraphRef(g), _params(p)
    src = np.ascontiguousarray(veh.src, np.uint32)
    dst = np.ascontiguousarray(veh.dst, np.uint32)
    V, S = src.shape[0], int(p["max_steps"])
    off = getattr(g, "inst_node_off", None)
    city = None
    if off is not None:
        city = np.repeat(np.arange(len(off) - 1, dtype=np.uint32), np.diff(np.asarray(off, np.int64))).astype(np.uint32)
    path = np.zeros((V, max(S, 1)), np.uint32)
    plen = np.zeros(V, np.uint32)
    cost = np.zeros(V, np.uint32)
    mark = np.zeros(gr.m, np.uint32)
    steps = C.c_uint64(0)
    rc = lib().orc_greedy(C.byref(gr.s), _ptr(src), _ptr(dst), V, C.byref(pp), _ptr(city), _ptr(path), _ptr(plen),
                          _ptr(cost), C.byref(steps), _ptr(mark))
    if rc != 0:
        raise ValueError("oracle rejected input", rc)
    return dict(path_edges=path, path_len=plen, cost_ms=cost, steps_total=int(steps.value), marker=mark)



def simulate(g, p: dict, path_edges, path_len, speed_kmh, *, tick_ms: int = 1000, max_ticks: int = 100000) -> dict:
    """Traffic simulation of the vehicles' trips along their routes (Section
    5; orc_simulate): arrival_ms and wait_ms per vehicle (arrival 2^32-1: no
    route or not arrived), ticks run, and over the vehicles that arrived the
    mean and the last arrival time (the overall travel time, ms)."""
    gr, pp = _GraphRef(g), _params(p)
    path = np.ascontiguousarray(path_edges, np.uint32)
    if path.ndim != 2:
        raise ValueError("path_edges must be [vehicles, stride]")
    V, S = path.shape
    plen = np.ascontiguousarray(path_len, np.uint32)
    spd = np.ascontiguousarray(speed_kmh, np.uint32)
    if plen.shape != (V,) or spd.shape != (V,):
        raise ValueError("path_len and speed_kmh need one entry per vehicle")
    arr = np.zeros(V, np.uint32)
    wait = np.zeros(V, np.uint32)
    ticks = C.c_uint32(0)
    rc = lib().orc_simulate(C.byref(gr.s), C.byref(pp), _ptr(path), S, _ptr(plen), _ptr(spd), V, int(tick_ms),
                            int(max_ticks), _ptr(arr), _ptr(wait), C.byref(ticks))
    if rc != 0:
        raise ValueError("oracle rejected input", rc)
    done = arr != 0xFFFFFFFF
    return dict(arrival_ms=arr, wait_ms=wait, ticks=int(ticks.value), arrived=int(done.sum()),
                mean_ms=float(arr[done].astype(np.float64).mean()) if done.any() else None,
                last_ms=int(arr[done].max()) if done.any() else None)
