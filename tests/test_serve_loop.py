"""Host logic of the continuous-batching loop (paper_2010_14244_amd/serve.py)
against a stand-in server: first-come-first-served admission, no batch
larger than the free slots, every query completed once, latency counted
from arrival; and bench.py's one-GPU contract.  No GPU."""
import numpy as np

from paper_2010_14244_amd import serve


class FakeServer:
    """`slots` slots; a query completes `iters` steps after its admission
    (its 'path' is [qid], its 'cost' qid).  Records what each step offered."""

    def __init__(self, slots, iters):
        self.slots, self.iters = slots, iters
        self.flight = []     # [qid, steps left]
        self.offered = []    # (queries handed in, free slots) per step
        self.order = []      # qids in admission order

    def step(self, od, stream=None):
        free = self.slots - len(self.flight)
        self.offered.append((len(od), free))
        take = min(len(od), free)
        for q in od[:take]:
            self.flight.append([int(q[0]), self.iters])
            self.order.append(int(q[0]))
        for f in self.flight:
            f[1] -= 1
        done = [(f[0], np.array([f[0]], np.uint32), f[0]) for f in self.flight if f[1] == 0]
        self.flight = [f for f in self.flight if f[1] > 0]
        return take, done

    def active(self):
        return len(self.flight)


def _od(n):
    q = np.arange(100, 100 + n, dtype=np.uint32)
    return np.stack([q, q % 7, q % 7 + 1], axis=1).astype(np.uint32)


def test_burst_is_admitted_in_order_and_bounded_by_free_slots():
    n, slots, iters = 2000, 48, 5
    srv = FakeServer(slots, iters)
    od = _od(n)
    r = serve.serve(srv, od, np.zeros(n), warmup=0)
    assert srv.order == od[:, 0].tolist()                      # FIFO
    assert all(k <= free for k, free in srv.offered)           # never more than the free slots
    assert max(k for k, _ in srv.offered) <= slots
    assert sorted(r["results"]) == od[:, 0].tolist()           # each query once
    assert all(path.tolist() == [q] and cost == q for q, (path, cost) in r["results"].items())
    lat = r["latency_s"]
    assert np.all(lat >= 0) and np.all(np.diff(lat) >= -1e-9)  # same arrival, FIFO: non-decreasing
    # steps: the queue drains slots at a time, each batch needing `iters` steps
    assert r["steps"] == iters * ((n + slots - 1) // slots)


def test_spread_arrivals_idle_waits_and_latency_from_arrival():
    n, slots, iters = 300, 16, 3
    rng = np.random.default_rng(5)
    arr = serve.poisson_arrivals(n, 20000.0, rng)
    assert np.all(np.diff(arr) > 0)
    srv = FakeServer(slots, iters)
    r = serve.serve(srv, _od(n), arr, warmup=20)
    assert srv.order == _od(n)[:, 0].tolist()
    assert all(k <= free for k, free in srv.offered)
    assert np.all(r["latency_s"] >= 0)
    assert len(r["results"]) == n and r["sustained_qps"] > 0


def test_poisson_arrivals_rate():
    arr = serve.poisson_arrivals(200000, 5000.0, np.random.default_rng(1))
    gaps = np.diff(arr)
    assert abs(gaps.mean() * 5000.0 - 1.0) < 0.01
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.02             # exponential: cv = 1


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asking for more exits with a message
    before anything touches a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
