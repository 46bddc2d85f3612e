"""Write the oracle's expected results for the full-size workloads that are
too slow to run inside a test.  Calls only the CPU oracle and the seeded
workload generators; the GPU library is never involved.

    python tests/golden/make_expected.py grid32

Stores, per workload: selections, per-vehicle best cost and length, and
SHA-256 digests of the best routes (each row truncated to its length), the
final pheromone and the final loads.
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


WORKLOADS = {
    "grid32": lambda: workloads.grid32(),
    "planar100k": lambda: workloads.planar100k(),
    "multicity": lambda: workloads.multi_city(),
}


def main(names):
    for name in names:
        w = WORKLOADS[name]()
        t = time.time()
        r = oracle.route(w.graph, w.vehicles, w.params)
        dt = time.time() - t
        out = dict(workload=w.name, generator=f"workloads.{name}()", params=w.params,
                   steps_total=r["steps_total"], cost_ms=r["cost_ms"].tolist(), path_len=r["path_len"].tolist(),
                   routes_sha256=digest_routes(r["path_edges"], r["path_len"]),
                   tau_sha256=digest(r["tau"]), load_sha256=digest(r["load"]),
                   oracle_seconds=round(dt, 1))
        with open(os.path.join(HERE, f"{name}_expected.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, r["steps_total"], f"{dt:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
