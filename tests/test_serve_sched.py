"""The request scheduler of the serving loop (host logic, CPU): FIFO
admission by memory budget and free slots, continuous batching (requests
that arrive while a batch runs start on another slot before it ends),
max-batch, rejections, and queueing under load.  The scheduler is the
library's own header, compiled with a simulated device on a virtual clock
(tests/serve_sim.cpp)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2508_05797_amd", "csrc")

DONE, REJ_INVALID, REJ_BUDGET = 1, 2, 3


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("serve") / "libserve_sim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC,
                    os.path.join(HERE, "serve_sim.cpp"), "-o", so], check=True)
    L = ctypes.CDLL(so)
    L.sim_run.restype = ctypes.c_int
    return L


def run(sim, arrival, cost, budget, max_batch, slots, base, per_byte,
        valid=None):
    n = len(arrival)
    arrival = np.ascontiguousarray(arrival, np.float64)
    cost = np.ascontiguousarray(cost, np.uint64)
    valid = np.ones(n, np.uint8) if valid is None else np.ascontiguousarray(valid, np.uint8)
    out = dict(latency=np.zeros(n), outcome=np.zeros(n, np.int8),
               launch=np.zeros(n), slot=np.zeros(n, np.int32),
               batch=np.zeros(n, np.int32), done=np.zeros(n))
    stats = np.zeros(5, np.uint64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = sim.sim_run(ctypes.c_uint32(n), p(arrival), p(cost), p(valid),
                     ctypes.c_uint64(budget), ctypes.c_uint32(max_batch),
                     ctypes.c_uint32(slots), ctypes.c_double(base),
                     ctypes.c_double(per_byte), p(out["latency"]),
                     p(out["outcome"]), p(out["launch"]), p(out["slot"]),
                     p(out["batch"]), p(out["done"]), p(stats))
    assert rc == 0, "launch on a busy slot or executor error"
    out["stats"] = dict(zip(["launches", "rejected", "max_queue",
                             "max_inflight", "max_bytes"], stats.tolist()))
    out["arrival"], out["cost"] = arrival, cost
    return out


def poisson(n, rate, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def check_invariants(o, budget, max_batch, slots):
    ok = o["outcome"] == DONE
    # each admitted request starts no earlier than it arrives, ends after it
    # starts, and its latency is completion minus arrival
    assert np.all(o["launch"][ok] >= o["arrival"][ok])
    assert np.all(o["done"][ok] > o["launch"][ok])
    assert np.allclose(o["latency"][ok], o["done"][ok] - o["arrival"][ok])
    # FIFO: launch order follows arrival order
    idx = np.nonzero(ok)[0]
    assert np.all(np.diff(o["launch"][idx]) >= 0)
    assert np.all(np.diff(o["batch"][idx]) >= 0)
    # batch sizes
    _, counts = np.unique(o["batch"][idx], return_counts=True)
    assert counts.max() <= max_batch
    # budget: bytes in flight at every launch instant (intervals [launch, done))
    for t in np.unique(o["launch"][idx]):
        live = ok & (o["launch"] <= t) & (o["done"] > t)
        assert int(o["cost"][live].sum()) <= budget
    # slots: batches on one slot do not overlap
    for s in range(slots):
        m = ok & (o["slot"] == s)
        b = sorted({(o["launch"][i], o["done"][i]) for i in np.nonzero(m)[0]})
        for (l0, d0), (l1, _d1) in zip(b, b[1:]):
            assert l1 >= d0
    assert o["stats"]["max_inflight"] <= slots
    assert o["stats"]["max_bytes"] <= budget


def test_all_complete_invariants(sim):
    rng = np.random.default_rng(1)
    n = 3000
    arr = poisson(n, 1000.0, 2)
    cost = rng.integers(1, 10_000, n)
    o = run(sim, arr, cost, budget=60_000, max_batch=16, slots=4, base=2e-3,
            per_byte=1e-7)
    assert np.all(o["outcome"] == DONE)
    check_invariants(o, 60_000, 16, 4)


def test_overlap(sim):
    """A request arriving while a batch runs starts on a free slot at once
    and finishes before the earlier batch; with one slot it waits."""
    o = run(sim, [0.0, 0.1, 0.2], [10, 10, 10], budget=1000, max_batch=8,
            slots=2, base=1.0, per_byte=0.0)
    assert o["launch"].tolist() == [0.0, 0.1, 1.0]   # third waits for a slot
    assert o["slot"][0] != o["slot"][1]
    assert o["done"][1] < o["done"][0] + 0.5
    assert o["stats"]["max_inflight"] == 2
    # one slot: the second request waits for the first batch
    o1 = run(sim, [0.0, 0.1], [10, 10], budget=1000, max_batch=8, slots=1,
             base=1.0, per_byte=0.0)
    assert o1["launch"].tolist() == [0.0, 1.0]


def test_arrivals_join_the_next_batch(sim):
    """Requests that arrive while every slot is busy are batched together
    when a slot frees up."""
    arr = [0.0] + [0.1 + 0.01 * i for i in range(10)]
    o = run(sim, arr, [1] * 11, budget=1000, max_batch=64, slots=1, base=1.0,
            per_byte=0.0)
    assert o["batch"].tolist() == [0] + [1] * 10
    assert np.all(o["launch"][1:] == 1.0)


def test_memory_admission_head_of_line(sim):
    """The FIFO head waits until its bytes fit; later small requests do not
    overtake it."""
    o = run(sim, [0.0, 0.01, 0.02], [80, 50, 10], budget=100, max_batch=8,
            slots=4, base=1.0, per_byte=0.0)
    assert o["launch"][0] == 0.0
    assert o["launch"][1] == pytest.approx(o["done"][0])
    assert o["launch"][2] >= o["launch"][1]
    check_invariants(o, 100, 8, 4)


def test_max_batch(sim):
    o = run(sim, np.zeros(10), np.ones(10), budget=1000, max_batch=4, slots=1,
            base=1.0, per_byte=0.0)
    assert o["batch"].tolist() == [0] * 4 + [1] * 4 + [2] * 2


def test_rejections(sim):
    o = run(sim, [0.0, 0.1, 0.2, 0.3], [10, 500, 10, 10], budget=100,
            max_batch=8, slots=2, base=0.5, per_byte=0.0,
            valid=[1, 1, 0, 1])
    assert o["outcome"].tolist() == [DONE, REJ_BUDGET, REJ_INVALID, DONE]
    assert o["latency"][1] == -1 and o["latency"][2] == -1
    assert o["stats"]["rejected"] == 2


def test_latency_under_load(sim):
    """Below capacity the latency stays near the service time; above it the
    queue grows without bound (open loop: arrivals do not wait)."""
    n, size, base, per_byte, slots = 4000, 1000, 1e-3, 1e-6, 2
    # capacity with full batches of 32: slots * 32 * size / (base + 32 * size * per_byte)
    cap_bytes = slots * 32 * size / (base + 32 * size * per_byte)
    for load, bounded in ((0.25, True), (0.5, True), (2.0, False)):
        rate = load * cap_bytes / size
        o = run(sim, poisson(n, rate, 7), np.full(n, size), budget=10**9,
                max_batch=32, slots=slots, base=base, per_byte=per_byte)
        lat = o["latency"]
        p99 = np.percentile(lat, 99)
        if bounded:
            assert p99 < 10 * (base + 32 * size * per_byte), (load, p99)
        else:
            assert lat[-100:].mean() > 20 * lat[:100].mean()
            assert o["stats"]["max_queue"] > 500
        check_invariants(o, 10**9, 32, slots)
