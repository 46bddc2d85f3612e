"""Write the oracle's expected results for the full-size workloads that are
too slow to run inside a test.  Calls only the CPU oracle and the seeded
workload generators; the GPU library is never involved.

    python tests/golden/make_expected.py grid32

Stores, per workload: selections, per-vehicle best cost and length, and
SHA-256 digests of the best routes (each row truncated to its length), the
final pheromone (independent mode: every vehicle's row, in vehicle order)
and the final loads.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402


def digest_routes(path_edges, path_len) -> str:
    h = hashlib.sha256()
    for v in range(path_len.shape[0]):
        h.update(np.ascontiguousarray(path_edges[v, :int(path_len[v])], dtype=np.uint32).tobytes())
        h.update(b"|")
    return h.hexdigest()


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint32).tobytes()).hexdigest()


def with_params(w, **kw):
    return workloads.Workload(w.name, w.graph, w.vehicles, dict(w.params, **kw))


WORKLOADS = {   # name: (generator call as stored, workload)
    "grid32": ("workloads.grid32()", lambda: workloads.grid32()),
    "planar100k": ("workloads.planar100k()", lambda: workloads.planar100k()),
    "multicity": ("workloads.multi_city()", lambda: workloads.multi_city()),
    # independent mode (private pheromone per vehicle, frozen loads), 256 vehicles
    "planar100k_indep256": ("workloads.planar100k(vehicles=256), mode=1",
                            lambda: with_params(workloads.planar100k(vehicles=256), mode=1)),
    # the exact goal term (flag 16) on the 64 packed cities
    "multicity_exact": ("workloads.multi_city(), flags=16",
                        lambda: with_params(workloads.multi_city(), flags=oracle.FLAG_GOAL_EXACT)),
}


def main(names):
    for name in names:
        gen, make = WORKLOADS[name]
        w = make()
        t = time.time()
        r = oracle.route(w.graph, w.vehicles, w.params)
        dt = time.time() - t
        out = dict(workload=w.name, generator=gen, params=w.params,
                   steps_total=r["steps_total"], cost_ms=r["cost_ms"].tolist(), path_len=r["path_len"].tolist(),
                   routes_sha256=digest_routes(r["path_edges"], r["path_len"]),
                   tau_sha256=digest(r["tau"]), load_sha256=digest(r["load"]),
                   oracle_seconds=round(dt, 1))
        with open(os.path.join(HERE, f"{name}_expected.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, r["steps_total"], f"{dt:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
