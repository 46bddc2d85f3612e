"""Python binding of the GMACO-P C ABI (``include/gmacop.h``).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libgmacop.so``.  The functions carry the C names.  Importing this module
does not load the library; the first call does, and raises ``GmacopError`` if
the library has not been built -- there is no other implementation to fall
back to.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgmacop.so")

OK = 0
E_INVAL = -1
E_RANGE = -2
E_NOMEM = -3
E_DEVICE = -4
E_UNSUPPORTED = -5

MODE_SHARED = 0
MODE_INDEPENDENT = 1
MODE_GREEDY = 2
NO_LOAD_UPDATE = 1
DEVICE_PTRS = 2

TIME_KERNELS = 4
HIP_GRAPH = 8
GOAL_EXACT = 16
RESUME = 32
SIGNAL_TIMED = 64

EXPORTED = ("gmacop_graph_create", "gmacop_route_batch", "gmacop_route_batch_noalloc", "gmacop_state_get", "gmacop_state_set",
            "gmacop_set_base_load", "gmacop_server_set_base_load", "gmacop_vehicle_tau_get",
            "gmacop_goal_rows", "gmacop_shortest_routes", "gmacop_simulate", "gmacop_stats_get", "gmacop_server_create", "gmacop_server_info", "gmacop_server_step",
            "gmacop_server_release", "gmacop_release", "gmacop_last_error")
KERNELS = ("walk", "best", "edge", "cost", "walk_lds", "walk_glb", "goal")
WALKERS = ("lds", "glb", "first")


class GmacopError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gmacop error {code}: {msg}")
        self.code = code


class _Desc(C.Structure):
    _fields_ = [("n_nodes", C.c_uint32), ("n_edges", C.c_uint32),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("len_dm", C.c_void_p),
                ("speed_kmh", C.c_void_p), ("green_pm", C.c_void_p), ("cycle_ms", C.c_void_p),
                ("x_dm", C.c_void_p), ("y_dm", C.c_void_p), ("base_load", C.c_void_p),
                ("n_instances", C.c_uint32), ("inst_node_off", C.c_void_p)]


class _OD(C.Structure):
    _fields_ = [("qid", C.c_uint32), ("src", C.c_uint32), ("dst", C.c_uint32)]


class _Params(C.Structure):
    _fields_ = [("ants", C.c_uint32), ("iterations", C.c_uint32), ("alpha", C.c_uint32), ("beta", C.c_uint32),
                ("max_steps", C.c_uint32), ("rho_q16", C.c_uint32), ("tau0_q16", C.c_uint32),
                ("tau_min_q16", C.c_uint32), ("tau_max_q16", C.c_uint32), ("q_deposit", C.c_uint64),
                ("theta", C.c_uint32), ("th_max", C.c_uint32), ("t_max_ms", C.c_uint32), ("vmax_kmh", C.c_uint32),
                ("mode", C.c_uint32), ("flags", C.c_uint32), ("seed", C.c_uint64), ("iter_offset", C.c_uint32)]


class _Result(C.Structure):
    _fields_ = [("path_edges", C.c_void_p), ("path_len", C.c_void_p), ("cost_ms", C.c_void_p),
                ("steps_total", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("launches", C.c_uint64 * 7), ("ms", C.c_double * 7), ("selections", C.c_uint64),
                ("candidates", C.c_uint64), ("arrivals", C.c_uint64), ("deposit_roads", C.c_uint64),
                ("longest_walks", C.c_uint64), ("walker_selections", C.c_uint64 * 3),
                ("walker_candidates", C.c_uint64 * 3), ("walker_arrivals", C.c_uint64 * 3),
                ("walker_deposit_roads", C.c_uint64 * 3)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libgmacop.so (raises GmacopError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise GmacopError(E_UNSUPPORTED, f"HIP library not built: {_LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(_LIB_PATH)
        vp = C.c_void_p
        L.gmacop_graph_create.argtypes = [C.POINTER(_Desc), C.POINTER(vp)]
        L.gmacop_graph_create.restype = C.c_int
        L.gmacop_route_batch.argtypes = [vp, vp, C.c_uint32, C.POINTER(_Params), C.POINTER(_Result), vp]
        L.gmacop_route_batch.restype = C.c_int
        L.gmacop_route_batch_noalloc.argtypes = [vp, vp, C.c_uint32, C.POINTER(_Params), C.POINTER(_Result), vp]
        L.gmacop_route_batch_noalloc.restype = C.c_int
        L.gmacop_state_get.argtypes = [vp, vp, vp, vp]
        L.gmacop_state_get.restype = C.c_int
        L.gmacop_state_set.argtypes = [vp, vp, vp, vp]
        L.gmacop_state_set.restype = C.c_int
        L.gmacop_set_base_load.argtypes = [vp, vp, vp]
        L.gmacop_set_base_load.restype = C.c_int
        L.gmacop_server_set_base_load.argtypes = [vp, vp, vp]
        L.gmacop_server_set_base_load.restype = C.c_int
        L.gmacop_vehicle_tau_get.argtypes = [vp, C.c_uint32, vp, vp]
        L.gmacop_vehicle_tau_get.restype = C.c_int
        L.gmacop_goal_rows.argtypes = [vp, vp, C.c_uint32, vp, vp]
        L.gmacop_goal_rows.restype = C.c_int
        L.gmacop_shortest_routes.argtypes = [vp, vp, C.c_uint32, C.c_uint32, C.POINTER(_Result), vp]
        L.gmacop_shortest_routes.restype = C.c_int
        L.gmacop_simulate.argtypes = [vp, C.POINTER(_Params), vp, C.c_uint32, vp, vp, vp, C.c_uint32, C.c_uint32,
                                      C.c_uint32, vp, vp, vp, vp]
        L.gmacop_simulate.restype = C.c_int
        L.gmacop_stats_get.argtypes = [vp, C.POINTER(_Stats), C.c_int, vp]
        L.gmacop_stats_get.restype = C.c_int
        u32p = C.POINTER(C.c_uint32)
        L.gmacop_server_create.argtypes = [vp, C.POINTER(_Params), C.c_uint32, C.c_uint64, C.POINTER(vp)]
        L.gmacop_server_create.restype = C.c_int
        L.gmacop_server_info.argtypes = [vp, u32p, u32p, C.POINTER(C.c_uint64)]
        L.gmacop_server_info.restype = C.c_int
        L.gmacop_server_step.argtypes = [vp, vp, u32p, vp, vp, vp, vp, C.c_uint32, u32p, vp]
        L.gmacop_server_step.restype = C.c_int
        L.gmacop_server_release.argtypes = [vp]
        L.gmacop_server_release.restype = None
        L.gmacop_release.argtypes = [vp]
        L.gmacop_release.restype = None
        L.gmacop_last_error.argtypes = []
        L.gmacop_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise GmacopError(rc, lib().gmacop_last_error().decode())


def _params(p: dict) -> _Params:
    return _Params(*[int(p[name]) for name, _ in _Params._fields_])


class Graph:
    """Owner of a device-resident graph handle."""

    def __init__(self, handle: int, n: int, m: int):
        self.handle = handle
        self.n, self.m = n, m

    def __del__(self):
        try:
            gmacop_release(self)
        except Exception:
            pass


def gmacop_graph_create(g) -> Graph:
    """Upload a ``workloads.RoadGraph``-like object (CSR arrays) to the GPU."""
    arrays = dict(row_ptr=np.ascontiguousarray(g.row_ptr, np.uint32), col=np.ascontiguousarray(g.col, np.uint32),
                  len_dm=np.ascontiguousarray(g.len_dm, np.uint32),
                  speed_kmh=np.ascontiguousarray(g.speed_kmh, np.uint16),
                  green_pm=np.ascontiguousarray(g.green_pm, np.uint16),
                  cycle_ms=np.ascontiguousarray(g.cycle_ms, np.uint32),
                  x_dm=np.ascontiguousarray(g.x_dm, np.int32), y_dm=np.ascontiguousarray(g.y_dm, np.int32),
                  base_load=np.ascontiguousarray(g.base_load, np.uint32))
    off = getattr(g, "inst_node_off", None)
    off = None if off is None else np.ascontiguousarray(off, np.uint32)
    n = arrays["row_ptr"].shape[0] - 1
    m = arrays["col"].shape[0]
    d = _Desc(n, m, *[arrays[k].ctypes.data for k in ("row_ptr", "col", "len_dm", "speed_kmh", "green_pm",
                                                       "cycle_ms", "x_dm", "y_dm", "base_load")],
              1 if off is None else off.shape[0] - 1, None if off is None else off.ctypes.data)
    h = C.c_void_p()
    _check(lib().gmacop_graph_create(C.byref(d), C.byref(h)))
    return Graph(h.value, n, m)


def _od_array(veh) -> np.ndarray:
    od = np.empty((len(veh), 3), dtype=np.uint32)
    od[:, 0] = veh.qid
    od[:, 1] = veh.src
    od[:, 2] = veh.dst
    return od


def gmacop_route_batch(g: Graph, veh, p: dict, stream: Optional[int] = None, held: Optional[dict] = None) -> dict:
    """Route the vehicles with host buffers (synchronous).  Returns dict with
    path_edges [V, max_steps], path_len [V], cost_ms [V], steps_total.  With
    the RESUME flag, `held` is the previous call's result dict."""
    return _route_host(lib().gmacop_route_batch, g, veh, p, stream, held)


def gmacop_route_batch_noalloc(g: Graph, veh, p: dict, stream: Optional[int] = None) -> dict:
    """gmacop_route_batch on the library's static per-GPU workspace (no
    device allocation); host buffers, synchronous."""
    return _route_host(lib().gmacop_route_batch_noalloc, g, veh, p, stream)


def _route_host(fn, g: Graph, veh, p: dict, stream: Optional[int], held: Optional[dict] = None) -> dict:
    od = _od_array(veh)
    V, S = od.shape[0], int(p["max_steps"])
    path = np.zeros((V, max(S, 1)), np.uint32)
    plen = np.zeros(V, np.uint32)
    cost = np.zeros(V, np.uint32)
    if held is not None:   # GMACOP_RESUME: the previous call's results are read back as the best routes held
        path[:] = held["path_edges"][:, :max(S, 1)]
        plen[:] = held["path_len"]
        cost[:] = held["cost_ms"]
    steps = np.zeros(1, np.uint64)
    res = _Result(path.ctypes.data, plen.ctypes.data, cost.ctypes.data, steps.ctypes.data)
    pp = _params(dict(p, flags=int(p.get("flags", 0)) & ~DEVICE_PTRS))
    _check(fn(g.handle, od.ctypes.data if V else None, V, C.byref(pp), C.byref(res), stream))
    return dict(path_edges=path, path_len=plen, cost_ms=cost, steps_total=int(steps[0]))


class DeviceBatch:
    """Device-resident queries and result buffers (torch tensors on the GPU),
    for calls that enqueue without synchronising (GMACOP_DEVICE_PTRS)."""

    def __init__(self, veh, max_steps: int, device="cuda"):
        import torch
        od = _od_array(veh).view(np.int32)
        V = od.shape[0]
        self.V, self.S = V, int(max_steps)
        self.od = torch.from_numpy(od.copy()).to(device)
        self.path = torch.zeros((V, max(self.S, 1)), dtype=torch.int32, device=device)
        self.path_len = torch.zeros(V, dtype=torch.int32, device=device)
        self.cost = torch.zeros(V, dtype=torch.int32, device=device)
        self.steps = torch.zeros(1, dtype=torch.int64, device=device)

    def result(self) -> dict:
        """Copy results to host numpy arrays (synchronises)."""
        return dict(path_edges=self.path.cpu().numpy().view(np.uint32), path_len=self.path_len.cpu().numpy().view(np.uint32),
                    cost_ms=self.cost.cpu().numpy().view(np.uint32), steps_total=int(self.steps.cpu().item()))


def gmacop_route_batch_device(g: Graph, b: DeviceBatch, p: dict, stream: Optional[int] = None,
                              noalloc: bool = False) -> None:
    """Enqueue a routing call on ``stream`` with device buffers (no sync);
    ``noalloc`` calls gmacop_route_batch_noalloc."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    res = _Result(b.path.data_ptr(), b.path_len.data_ptr(), b.cost.data_ptr(), b.steps.data_ptr())
    pp = _params(dict(p, flags=int(p.get("flags", 0)) | DEVICE_PTRS))
    fn = lib().gmacop_route_batch_noalloc if noalloc else lib().gmacop_route_batch
    _check(fn(g.handle, b.od.data_ptr() if b.V else None, b.V, C.byref(pp), C.byref(res), stream))


def gmacop_state_get(g: Graph, stream: Optional[int] = None):
    """(tau_q16 [m], load [m]) after the last shared-mode call."""
    tau = np.zeros(g.m, np.uint32)
    load = np.zeros(g.m, np.uint32)
    _check(lib().gmacop_state_get(g.handle, tau.ctypes.data, load.ctypes.data, stream))
    return tau, load


def gmacop_state_set(g: Graph, tau=None, load=None, stream: Optional[int] = None) -> None:
    """Replace the shared-mode pheromone and/or current loads the graph holds."""
    t = None if tau is None else np.ascontiguousarray(tau, np.uint32)
    l = None if load is None else np.ascontiguousarray(load, np.uint32)
    for a in (t, l):
        if a is not None and a.shape != (g.m,):
            raise ValueError("state arrays need one entry per road")
    _check(lib().gmacop_state_set(g.handle, None if t is None else t.ctypes.data,
                                  None if l is None else l.ctypes.data, stream))


def gmacop_set_base_load(g: Graph, base_load, stream: Optional[int] = None) -> None:
    """A new epoch of sensed loads for later calls on the graph."""
    b = np.ascontiguousarray(base_load, np.uint32)
    if b.shape != (g.m,):
        raise ValueError("base_load needs one entry per road")
    _check(lib().gmacop_set_base_load(g.handle, b.ctypes.data, stream))


def gmacop_vehicle_tau_get(g: Graph, vehicle: int, stream: Optional[int] = None) -> np.ndarray:
    """Independent mode: pheromone [m] of the vehicle at batch position
    ``vehicle`` after the last call's final iteration."""
    tau = np.zeros(g.m, np.uint32)
    _check(lib().gmacop_vehicle_tau_get(g.handle, int(vehicle), tau.ctypes.data, stream))
    return tau


def gmacop_goal_rows(g: Graph, dst, stream: Optional[int] = None) -> np.ndarray:
    """Exact goal term rows: uint32 [len(dst), n], shortest free-flow time of
    every node to each destination (0xFFFFFFFF: out of reach)."""
    d = np.ascontiguousarray(dst, np.uint32).reshape(-1)
    h = np.zeros((d.shape[0], g.n), np.uint32)
    _check(lib().gmacop_goal_rows(g.handle, d.ctypes.data if d.shape[0] else None, d.shape[0],
                                  h.ctypes.data if d.shape[0] else None, stream))
    return h


def gmacop_shortest_routes(g: Graph, veh, max_steps: int, stream: Optional[int] = None) -> dict:
    """Shortest free-flow route per vehicle (road ids), as gmacop_route_batch's result dict."""
    od = _od_array(veh)
    V, S = od.shape[0], int(max_steps)
    path = np.zeros((V, max(S, 1)), np.uint32)
    plen = np.zeros(V, np.uint32)
    cost = np.zeros(V, np.uint32)
    steps = np.zeros(1, np.uint64)
    res = _Result(path.ctypes.data, plen.ctypes.data, cost.ctypes.data, steps.ctypes.data)
    _check(lib().gmacop_shortest_routes(g.handle, od.ctypes.data if V else None, V, S, C.byref(res), stream))
    return dict(path_edges=path, path_len=plen, cost_ms=cost, steps_total=int(steps[0]))


def gmacop_simulate(g: Graph, p: dict, path_edges, path_len, speed_kmh, scen_off=None, *, tick_ms: int = 1000,
                    max_ticks: int = 100000, stream: Optional[int] = None) -> dict:
    """Traffic simulation of trips along given routes (gmacop_simulate).
    path_edges [V, stride] roads, path_len [V], speed_kmh [V]; scen_off
    [S + 1] splits the vehicles into scenarios simulated on their own (one
    scenario when None).  Returns arrival_ms and wait_ms per vehicle and
    ticks per scenario."""
    path = np.ascontiguousarray(path_edges, np.uint32)
    if path.ndim != 2:
        raise ValueError("path_edges must be [vehicles, stride]")
    V, S = path.shape
    plen = np.ascontiguousarray(path_len, np.uint32)
    spd = np.ascontiguousarray(speed_kmh, np.uint32)
    if plen.shape != (V,) or spd.shape != (V,):
        raise ValueError("path_len and speed_kmh need one entry per vehicle")
    off = np.ascontiguousarray([0, V] if scen_off is None else scen_off, np.uint32)
    if off.ndim != 1 or off.shape[0] < 2 or int(off[-1]) != V:
        raise ValueError("scen_off must run from 0 to the vehicle count")
    nscen = off.shape[0] - 1
    arr = np.zeros(max(V, 1), np.uint32)
    wait = np.zeros(max(V, 1), np.uint32)
    ticks = np.zeros(nscen, np.uint32)
    pp = _params(p)
    _check(lib().gmacop_simulate(g.handle, C.byref(pp), path.ctypes.data, S, plen.ctypes.data, spd.ctypes.data,
                                 off.ctypes.data, nscen, int(tick_ms), int(max_ticks), arr.ctypes.data,
                                 wait.ctypes.data, ticks.ctypes.data, stream))
    return dict(arrival_ms=arr[:V], wait_ms=wait[:V], ticks=ticks)


def gmacop_stats_get(g: Graph, reset: bool = False, stream: Optional[int] = None) -> dict:
    """Work counters and per-kernel launch counts / summed event times."""
    st = _Stats()
    _check(lib().gmacop_stats_get(g.handle, C.byref(st), 1 if reset else 0, stream))
    return dict(launches={k: int(st.launches[i]) for i, k in enumerate(KERNELS)},
                ms={k: float(st.ms[i]) for i, k in enumerate(KERNELS)},
                selections=int(st.selections), candidates=int(st.candidates), arrivals=int(st.arrivals),
                deposit_roads=int(st.deposit_roads), longest_walks=int(st.longest_walks),
                walkers={w: dict(selections=int(st.walker_selections[i]), candidates=int(st.walker_candidates[i]),
                                 arrivals=int(st.walker_arrivals[i]), deposit_roads=int(st.walker_deposit_roads[i]))
                         for i, w in enumerate(WALKERS)})


def gmacop_release(g: Graph) -> None:
    if g is not None and g.handle:
        lib().gmacop_release(g.handle)
        g.handle = None


class Server:
    """Continuous-batching router (gmacop_server_*): independent-mode queries
    admitted while others are in flight, one iteration per step."""

    def __init__(self, g: Graph, p: dict, max_slots: int = 0, mem_budget_bytes: int = 0):
        h = C.c_void_p()
        pp = _params(dict(p, mode=MODE_INDEPENDENT))
        _check(lib().gmacop_server_create(g.handle, C.byref(pp), int(max_slots), int(mem_budget_bytes), C.byref(h)))
        self.handle = h.value
        self.graph = g                      # keeps the graph alive
        self.max_steps = int(p["max_steps"])
        self.iterations = int(p["iterations"])
        sl, act, bps = C.c_uint32(), C.c_uint32(), C.c_uint64()
        _check(lib().gmacop_server_info(self.handle, C.byref(sl), C.byref(act), C.byref(bps)))
        self.slots, self.bytes_per_slot = int(sl.value), int(bps.value)
        self._qid = np.zeros(self.slots, np.uint32)
        self._len = np.zeros(self.slots, np.uint32)
        self._cost = np.zeros(self.slots, np.uint32)
        self._paths = np.zeros((self.slots, max(self.max_steps, 1)), np.uint32)

    def active(self) -> int:
        act = C.c_uint32()
        _check(lib().gmacop_server_info(self.handle, None, C.byref(act), None))
        return int(act.value)

    def step(self, od: np.ndarray, stream: Optional[int] = None):
        """od: uint32 [k, 3] (qid, src, dst) to admit.  Returns (admitted count,
        list of (qid, path edges, cost)) for the queries that completed."""
        od = np.ascontiguousarray(od, np.uint32).reshape(-1, 3)
        na, nd = C.c_uint32(od.shape[0]), C.c_uint32(0)
        _check(lib().gmacop_server_step(self.handle, od.ctypes.data if od.shape[0] else None, C.byref(na),
                                        self._qid.ctypes.data, self._len.ctypes.data, self._cost.ctypes.data,
                                        self._paths.ctypes.data, self.slots, C.byref(nd), stream))
        done = [(int(self._qid[i]), self._paths[i, :int(self._len[i])].copy(), int(self._cost[i]))
                for i in range(nd.value)]
        return int(na.value), done

    def set_base_load(self, base_load, stream: Optional[int] = None) -> None:
        """A new epoch of sensed loads for this router, from its next step on."""
        b = np.ascontiguousarray(base_load, np.uint32)
        if b.shape != (self.graph.m,):
            raise ValueError("base_load needs one entry per road")
        _check(lib().gmacop_server_set_base_load(self.handle, b.ctypes.data, stream))

    def release(self):
        if self.handle:
            lib().gmacop_server_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
