#!/usr/bin/env python3
"""Throughput of the GMACO-P routing hot path on one MI355X.

One step = one gmacop_route_batch call over the whole workload: every
iteration's cost table, ant walks, best-route reduction, deposit,
evaporation and load update.  Default workload: 64 packed planar cities
(843,944 intersections, 2,124,622 roads), 10,466 vehicles x 32 ants x 30
iterations, shared pheromone and loads per city.  Queries and result
buffers are resident in device memory before the timed region starts.

Prints one JSON line: ant edge-selections per second (every roulette choice
an ant makes), the dominant walk kernel's position against HBM bandwidth,
the routed fraction, the plain per-query form against the batched one, the
continuous-batching router on the 1M-node city (p50/p99 latency and
sustained queries/s at several offered rates), and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of a walk kernel (what one lane must read or write):
#   per selection: row_ptr[u], row_ptr[u+1] (8 B) + path entry written (4 B)
#   per candidate road examined: col, tau, cost (12 B) + head x, y (8 B)
#   per road an arriving ant deposits on: path entry re-read (4 B) + 64-bit atomic add (8 B)
BYTES_PER_SELECTION = 12
BYTES_PER_CANDIDATE = 20
BYTES_PER_DEPOSIT_ROAD = 12

KERNEL_LIBRARY = os.path.join(ROOT, "paper_2010_14244_amd", "libgmacop.so")
LLVM_BIN = "/opt/rocm/llvm/bin"
# walker kinds of the library's statistics: (stats kernel key, stats walker key, kernel names)
WALKER_KINDS = {"lds": ("walk_lds", "lds", "k_walk_ldsr / k_walk_lds"), "glb": ("walk_glb", "glb", "k_walk_glb")}


def kernel_isa_hash(lib_path, symbol_re):
    """SHA-256 prefix of one kernel's gfx950 machine code in a built library:
    the code object is taken from the library's offload bundle, disassembled
    with llvm-objdump, and the instructions of the first symbol matching
    `symbol_re` are hashed as text, with the offsets of the loads from the
    kernel-argument block masked (adding an argument moves them; what the
    kernel does is unchanged).  None when the tools or the kernel are missing."""
    import re
    import struct
    import subprocess
    import tempfile
    try:
        sec = subprocess.run([os.path.join(LLVM_BIN, "llvm-readelf"), "-S", "-W", lib_path],
                             capture_output=True, text=True, check=True).stdout
        off = size = None
        for line in sec.splitlines():
            f = line.replace("[ ", "[").split()
            if ".hip_fatbin" in f:
                i = f.index(".hip_fatbin")
                off, size = int(f[i + 3], 16), int(f[i + 4], 16)
        if off is None:
            return None
        with open(lib_path, "rb") as fh:
            fh.seek(off)
            b = fh.read(size)
        if b[:24] != b"__CLANG_OFFLOAD_BUNDLE__":
            return None
        code, p = None, 32
        for _ in range(struct.unpack_from("<Q", b, 24)[0]):
            o, n, tl = struct.unpack_from("<QQQ", b, p)
            if "gfx950" in b[p + 24:p + 24 + tl].decode():
                code = b[o:o + n]
            p += 24 + tl
        if code is None:
            return None
        with tempfile.NamedTemporaryFile(suffix=".co") as tf:
            tf.write(code)
            tf.flush()
            dis = subprocess.run([os.path.join(LLVM_BIN, "llvm-objdump"), "-d", tf.name],
                                 capture_output=True, text=True, check=True).stdout
    except (OSError, subprocess.CalledProcessError, ValueError, struct.error, UnicodeDecodeError):
        return None
    sym, body = re.compile(symbol_re), None
    kernarg = re.compile(r"^(s_load_\w+\s+[^,]+,\s*s\[0:1\],\s*)0x[0-9a-f]+$")
    for line in dis.splitlines():
        if line.endswith(">:"):
            if body is not None:
                break
            if sym.search(line):
                body = []
            continue
        if body is not None:
            t = line.split("//")[0].strip()
            if t:
                body.append(kernarg.sub(r"\1OFF", t))
    if not body:
        return None
    return hashlib.sha256("\n".join(body).encode()).hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed PMC
    profile (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel
    calibration), or None when there is none or the kernel's machine code in
    the built library differs from the one the counters were taken on."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    try:
        vals = {}
        with open(path) as f:
            for line in f:
                if ":" in line and line.split(":")[0].strip().startswith(("pmc_", "kernel_isa", "kernel_symbol")):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
        if kernel_isa_hash(KERNEL_LIBRARY, vals["kernel_symbol_re"]) != vals["kernel_isa_sha256_prefix"]:
            return None
        return (float(vals["pmc_walk_fetch_kib"]) * float(vals["pmc_fetch_scale"]) +
                float(vals["pmc_walk_write_kib"]) * float(vals["pmc_write_scale"])) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def make_workload(name):
    import workloads
    table = {"grid8": workloads.grid8, "grid32": workloads.grid32, "planar100k": workloads.planar100k,
             "multicity": workloads.multi_city}
    return table[name]()


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def cpu_baseline(w, vehicles):
    """The oracle, as is, on the same graph and parameters for the first
    `vehicles` vehicles and all iterations, one thread."""
    import oracle
    from workloads import Vehicles
    oracle.build(force=False)
    V = w.vehicles
    k = min(vehicles, len(V))
    sub = Vehicles(qid=V.qid[:k], src=V.src[:k], dst=V.dst[:k])
    t = time.perf_counter()
    r = oracle.route(w.graph, sub, w.params, want_state=False)
    dt = time.perf_counter() - t
    model, ncpu, avail = host_cpu()
    return {"value": r["steps_total"] / dt, "unit": "edge-selections/s", "cores": 1, "kind": "oracle",
            "host_cores": ncpu, "host_cores_available": avail, "cpu_model": model,
            "sample": f"{w.name}: first {k} of {len(V)} vehicles, all {w.params['iterations']} iterations "
                      f"({r['steps_total']} selections in {dt:.1f} s, single thread)"}


def cpu_serving_baseline(w, od, count):
    """The oracle on the router's own query stream, one query at a time
    (independent mode: each query's result depends on it alone): its
    sequential query rate, one thread."""
    import oracle
    from workloads import Vehicles
    oracle.build(force=False)
    k = min(count, od.shape[0])
    t = time.perf_counter()
    sel = 0
    for i in range(k):
        one = Vehicles(qid=od[i:i + 1, 0].copy(), src=od[i:i + 1, 1].copy(), dst=od[i:i + 1, 2].copy())
        sel += oracle.route(w.graph, one, w.params, want_state=False)["steps_total"]
    dt = time.perf_counter() - t
    return {"qps": k / dt, "edge_selections_per_s": sel / dt, "cores": 1, "kind": "oracle",
            "sample": f"{w.name}: the first {k} queries of the router's stream, one at a time ({dt:.1f} s)"}


def measure_forms(gmacop, G, w, stream_obj, max_vehicles):
    """Independent-mode routing of the first `max_vehicles` vehicles, two
    ways: the plain per-query form (one gmacop_route_batch per vehicle,
    kernels launched one by one) and the batched form (one call for all of
    them, replayed as a HIP graph).  Per-vehicle results are identical;
    reports edge-selections/s of both and their ratio."""
    V = w.vehicles
    nv = min(len(V), max_vehicles)
    p = dict(w.params, mode=gmacop.MODE_INDEPENDENT)
    stream = stream_obj.cuda_stream
    sub = type(V)(qid=V.qid[:nv], src=V.src[:nv], dst=V.dst[:nv])
    batch = gmacop.DeviceBatch(sub, p["max_steps"])
    pb = dict(p, flags=p["flags"] | gmacop.HIP_GRAPH)
    gmacop.gmacop_route_batch_device(G, batch, pb, stream)       # warm-up + capture
    stream_obj.synchronize()
    t = time.perf_counter()
    gmacop.gmacop_route_batch_device(G, batch, pb, stream)
    stream_obj.synchronize()
    t_batched = time.perf_counter() - t
    rb = batch.result()
    singles = [gmacop.DeviceBatch(type(V)(qid=V.qid[i:i + 1], src=V.src[i:i + 1], dst=V.dst[i:i + 1]), p["max_steps"])
               for i in range(nv)]
    gmacop.gmacop_route_batch_device(G, singles[0], p, stream)   # warm-up
    stream_obj.synchronize()
    t = time.perf_counter()
    for b in singles:
        gmacop.gmacop_route_batch_device(G, b, p, stream)
    stream_obj.synchronize()
    t_plain = time.perf_counter() - t
    sel_plain = 0
    for i, b in enumerate(singles):
        r = b.result()
        sel_plain += r["steps_total"]
        assert r["cost_ms"][0] == rb["cost_ms"][i] and r["path_len"][0] == rb["path_len"][i], i
    assert sel_plain == rb["steps_total"], (sel_plain, rb["steps_total"])
    return {"mode": "independent", "vehicles": nv,
            "plain_per_query": {"value": sel_plain / t_plain, "ms": t_plain * 1e3, "launch": "eager, one call per vehicle"},
            "batched": {"value": rb["steps_total"] / t_batched, "ms": t_batched * 1e3, "launch": "hip_graph, one call"},
            "batched_over_plain": t_plain / t_batched,
            "routed_fraction": float((rb["path_len"] > 0).mean()) if nv else None}


def measure_goal_exact(gmacop, G, w, b, stream_obj, steps, log):
    """The same batched workload with the exact goal term (the shortest
    free-flow time to each vehicle's destination, searched on the device once
    per call): selections/s over `steps` whole calls, routed fraction, ant
    arrival rate, and the search's and walks' event-timed share of a call."""
    p = dict(w.params, flags=w.params["flags"] | gmacop.GOAL_EXACT)
    stream = stream_obj.cuda_stream
    pg = dict(p, flags=p["flags"] | gmacop.HIP_GRAPH)
    gmacop.gmacop_route_batch_device(G, b, pg, stream)          # warm-up + capture
    stream_obj.synchronize()
    gmacop.gmacop_stats_get(G, reset=True)
    t = time.perf_counter()
    for _ in range(steps):
        gmacop.gmacop_route_batch_device(G, b, pg, stream)
    stream_obj.synchronize()
    dt = time.perf_counter() - t
    st = gmacop.gmacop_stats_get(G, reset=True)
    res = b.result()
    gmacop.gmacop_route_batch_device(G, b, dict(p, flags=p["flags"] | gmacop.TIME_KERNELS), stream)
    stream_obj.synchronize()
    kt = gmacop.gmacop_stats_get(G, reset=True)
    V = len(w.vehicles)
    out = {"value": st["selections"] / dt, "unit": "edge-selections/s", "ms_per_step": dt / steps * 1e3,
           "steps": steps, "routed_fraction": float((res["path_len"] > 0).mean()) if V else None,
           "ant_arrival_rate": st["arrivals"] / max(1, steps * V * p["ants"] * p["iterations"]),
           "goal_search_ms": kt["ms"]["goal"], "walk_phase_ms": kt["ms"]["walk"],
           "selections_per_step": st["selections"] // max(1, steps)}
    log(f"[bench] exact goal: {out['value'] / 1e9:.2f} G selections/s, {out['ms_per_step']:.1f} ms/call "
        f"(search {out['goal_search_ms']:.2f} ms), routed {out['routed_fraction']:.3f}, "
        f"arrivals {out['ant_arrival_rate']:.3f}")
    return out


def run_serving(args, log):
    """Continuous-batching router on the 1M-node city: Poisson arrivals at
    each rate in --rates, 32 ants x 20 iterations per query.  Latency is
    arrival to result, queueing for a slot included."""
    import numpy as np
    import workloads
    from paper_2010_14244_amd import gmacop, serve
    import torch

    log("[bench] generating the serving city")
    w = workloads.serving_city(n=args.serve_nodes)
    g, p = w.graph, dict(w.params)
    G = gmacop.gmacop_graph_create(g)
    srv = gmacop.Server(G, p, max_slots=args.serve_slots)
    stream_obj = torch.cuda.Stream()
    stream = stream_obj.cuda_stream
    log(f"[bench] {w.name}: n={g.n} m={g.m} slots={srv.slots} ({srv.bytes_per_slot / 2**20:.1f} MiB each)")
    rng = np.random.default_rng(7)
    qid0, runs, first_od = 0, [], None
    for rate in [float(r) for r in args.rates.split(",")]:
        n = max(int(rate * args.serve_seconds), args.serve_min_queries + args.serve_warmup)
        od = workloads.query_stream(g, n, rng, qid0=qid0)
        if first_od is None:
            first_od = od
        qid0 += n
        arr = serve.poisson_arrivals(n, rate, rng)
        gmacop.gmacop_stats_get(G, reset=True)
        r = serve.serve(srv, od, arr, warmup=args.serve_warmup, stream=stream, log=log)
        st = gmacop.gmacop_stats_get(G)
        lat = r["latency_s"][args.serve_warmup:]
        routed = np.array([len(r["results"][int(q)][0]) > 0 for q in od[args.serve_warmup:, 0]])
        lat_routed = lat[routed]
        run = {"offered_qps": rate, "queries": n, "measured_queries": int(lat.shape[0]),
               "sustained_qps": r["sustained_qps"], "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
               "routed_fraction": float(routed.mean()),
               "routed_qps": r["sustained_qps"] * float(routed.mean()),
               "routed_p50_ms": float(np.percentile(lat_routed, 50) * 1e3) if lat_routed.size else None,
               "routed_p99_ms": float(np.percentile(lat_routed, 99) * 1e3) if lat_routed.size else None,
               "ant_arrival_rate": st["arrivals"] / max(1, n * p["ants"] * p["iterations"]),
               "steps": r["steps"], "edge_selections_per_s": st["selections"] / r["wall_s"]}
        runs.append(run)
        log(f"[bench] serve {rate:.0f}/s: sustained {r['sustained_qps']:.0f}/s p50 {r['p50_ms']:.1f} ms "
            f"p99 {r['p99_ms']:.1f} ms routed {run['routed_fraction']:.3f}, {r['steps']} steps")
    srv.release()
    gmacop.gmacop_release(G)
    out = {"workload": w.name, "nodes": g.n, "roads": g.m, "ants": p["ants"], "iterations": p["iterations"],
           "max_steps": p["max_steps"], "slots": srv.slots, "mode": "independent",
           "goal": "straight line at the top speed", "runs": runs}
    return out, (w, first_od)


def walker_roofline(st, kernel_ms_key, walker_key, workload, names):
    """Effective bandwidth of one walker kind from its event times and
    counters (algorithmic bytes / average launch time)."""
    nl = st["launches"][kernel_ms_key]
    if not nl or st["ms"][kernel_ms_key] <= 0:
        return None
    ms = st["ms"][kernel_ms_key] / nl
    c = st["walkers"][walker_key]
    byts = (BYTES_PER_SELECTION * c["selections"] + BYTES_PER_CANDIDATE * c["candidates"] +
            BYTES_PER_DEPOSIT_ROAD * c["deposit_roads"]) / nl
    gbs = byts / (ms * 1e-3) / 1e9
    return {"kernel": names, "launches_timed": nl, "avg_launch_ms": round(ms, 5),
            "algorithmic_bytes_per_launch": int(byts), "achieved": round(gbs, 2),
            "selections_per_launch": c["selections"] / nl,
            "mean_candidates_per_selection": c["candidates"] / max(1, c["selections"])}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="multicity", choices=["grid8", "grid32", "planar100k", "multicity"])
    ap.add_argument("--no-serve", action="store_true", help="skip the continuous-batching router runs")
    ap.add_argument("--rates", default="2000,5000,10000,20000", help="router: offered query rates")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="router: seconds of arrivals per rate")
    ap.add_argument("--serve-min-queries", type=int, default=10000, help="router: measured queries per rate")
    ap.add_argument("--serve-warmup", type=int, default=200, help="router: queries excluded from latency stats")
    ap.add_argument("--serve-slots", type=int, default=4096, help="router: slot limit (memory may allow fewer)")
    ap.add_argument("--serve-nodes", type=int, default=1_000_000, help="router: city size")
    ap.add_argument("--no-exact", action="store_true", help="skip the exact-goal-term runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-vehicles", type=int, default=1280,
                    help="CPU oracle: the first this many vehicles (about 14 s of one core on the 64 cities)")
    ap.add_argument("--cpu-serve-queries", type=int, default=16,
                    help="CPU oracle: router queries timed one at a time (0: none)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="skip the event-timed pass (roofline becomes null)")
    ap.add_argument("--eager", action="store_true", help="launch kernel by kernel instead of replaying a HIP graph")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the timed steps, run 4 device-to-device copies of this many MiB (a known-size "
                         "reference for hardware byte counters)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the plain-per-query vs batched comparison (independent mode)")
    ap.add_argument("--forms-vehicles", type=int, default=512, help="plain vs batched: the first this many vehicles")
    ap.add_argument("--kernel-isa-hash", nargs=2, metavar=("LIBRARY", "SYMBOL_RE"),
                    help="print the machine-code hash of a kernel in a built library (as the profiles record it) "
                         "and exit")
    args = ap.parse_args()
    if args.kernel_isa_hash:
        print(kernel_isa_hash(*args.kernel_isa_hash))
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is designed but not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2010_14244_amd import gmacop

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log(f"[bench] generating workload {args.workload}")
    w = make_workload(args.workload)
    g, V, p = w.graph, w.vehicles, dict(w.params)
    G = gmacop.gmacop_graph_create(g)
    b = gmacop.DeviceBatch(V, p["max_steps"])
    stream_obj = torch.cuda.Stream()          # default priority
    stream = stream_obj.cuda_stream
    p_run = dict(p, flags=p["flags"] | (0 if args.eager else gmacop.HIP_GRAPH))

    log(f"[bench] {w.name}: n={g.n} m={g.m} vehicles={len(V)} warmup={args.warmup}")
    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib << 18, dtype=torch.int32, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        gmacop.gmacop_route_batch_device(G, b, p_run, stream)
    stream_obj.synchronize()
    gmacop.gmacop_stats_get(G, reset=True)

    # timed region: K whole routing calls, inputs and outputs resident on the device
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        gmacop.gmacop_route_batch_device(G, b, p_run, stream)
        stream_obj.synchronize()
        lat.append(time.perf_counter() - t0)
        log(f"[bench] step {i}: {lat[-1] * 1e3:.2f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    st = gmacop.gmacop_stats_get(G, reset=True)
    res = b.result()
    sel = st["selections"]
    assert sel == res["steps_total"] * args.steps, (sel, res["steps_total"])
    routed = float((res["path_len"] > 0).mean()) if len(V) else None
    arrival_rate = st["arrivals"] / max(1, args.steps * len(V) * p["ants"] * p["iterations"])

    roofline, walkers = None, {}
    if not args.no_kernel_timing:
        # second timed pass: the same calls launched kernel by kernel, each
        # bracketed by HIP events on the stream it runs on
        for i in range(args.steps):
            gmacop.gmacop_route_batch_device(G, b, dict(p, flags=p["flags"] | gmacop.TIME_KERNELS), stream)
        stream_obj.synchronize()
        kt = gmacop.gmacop_stats_get(G)
        for kind, (mkey, wkey, names) in WALKER_KINDS.items():
            r = walker_roofline(kt, mkey, wkey, w.name, names)
            if r:
                walkers[kind] = r
        if walkers:
            dom = max(walkers, key=lambda k: walkers[k]["avg_launch_ms"] * walkers[k]["launches_timed"])
            d = walkers[dom]
            kernel = "k_walk_glb" if dom == "glb" else "k_walk_ldsr"
            traffic = measured_traffic(kernel, w.name)
            roofline = {"bound": "hbm", "kernel": d["kernel"], "achieved": d["achieved"], "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(d["achieved"] / HBM_PEAK_GBS, 5),
                        "traffic": None if traffic is None else round(traffic),
                        "achieved_kind": "effective: algorithmic bytes / average launch time",
                        "measured_frac": None if traffic is None else
                        round(traffic / (d["avg_launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                        "limiter": "dependent chain of the longest walks (latency), not bandwidth",
                        "avg_launch_ms": d["avg_launch_ms"], "launches_timed": d["launches_timed"],
                        "algorithmic_bytes_per_launch": d["algorithmic_bytes_per_launch"],
                        "selections_per_launch": d["selections_per_launch"],
                        "mean_candidates_per_selection": d["mean_candidates_per_selection"],
                        "longest_walk_per_iteration": kt["longest_walks"] / max(1, kt["launches"]["walk"])}
        n_it = max(1, kt["launches"]["walk"])
        log("[bench] event-timed pass, per call: " + ", ".join(
            f"{k} {kt['ms'][k] / args.steps:.3f} ms ({kt['launches'][k] // args.steps}x)" for k in kt["ms"]) +
            f"; walk phase {kt['ms']['walk'] / n_it:.3f} ms per iteration")

    out = {
        "metric": "ant edge-selections/sec",
        "value": sel / elapsed,
        "unit": "edge-selections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w.name, "nodes": g.n, "roads": g.m,
                   "cities": 1 if g.inst_node_off is None else int(g.inst_node_off.shape[0] - 1),
                   "vehicles": len(V), "ants": p["ants"], "iterations": p["iterations"], "mode": "shared",
                   "launch": "eager" if args.eager else "hip_graph", "selections_per_step": sel // args.steps},
        "routing": {"routed_fraction": routed, "ant_arrival_rate": arrival_rate},
        "call_latency_ms": {"p50": percentile(lat, 0.5) * 1e3, "p99": percentile(lat, 0.99) * 1e3},
        "roofline": roofline,
        "walkers": walkers,
    }
    if not args.no_exact:
        out["goal_exact"] = measure_goal_exact(gmacop, G, w, b, stream_obj, args.steps, log)
    if not args.no_forms:
        log("[bench] plain per-query vs batched (independent mode)")
        out["forms"] = measure_forms(gmacop, G, w, stream_obj, args.forms_vehicles)
        f = out["forms"]
        log(f"[bench] forms: plain {f['plain_per_query']['ms']:.1f} ms, batched {f['batched']['ms']:.1f} ms, "
            f"ratio {f['batched_over_plain']:.1f}")
    gmacop.gmacop_release(G)
    del b
    torch.cuda.empty_cache()
    served = None
    if not args.no_serve:
        out["serving"], served = run_serving(args, log)
    if not args.no_cpu:
        log(f"[bench] timing the CPU oracle on the first {args.cpu_vehicles} vehicles")
        cb = cpu_baseline(w, args.cpu_vehicles)
        cb["extrapolated_full_call_s"] = out["config"]["selections_per_step"] / cb["value"]
        if served is not None and served[1] is not None and args.cpu_serve_queries:
            log(f"[bench] timing the CPU oracle on {args.cpu_serve_queries} router queries")
            cb["serving"] = cpu_serving_baseline(served[0], served[1], args.cpu_serve_queries)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
