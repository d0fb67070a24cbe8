"""The serving loop on the GPU: requests arriving open-loop are admitted by
memory and slots, batched continuously with overlapping batches, and every
request's offsets are identical to the same request chunked alone and to
the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_05797_amd import binding, datagen

pytestmark = pytest.mark.gpu

WIN = {"ram": 4096, "ae": 4096, "maxp": 2048, "ae_min": 4096}


def say(*a):
    print(*a, flush=True)


def make_requests(n_req, seed, pool_bytes, rate, small_windows=False):
    rng = np.random.default_rng(seed)
    sizes = datagen.lognormal_sizes(n_req, seed, median=16384, sigma=1.5,
                                    lo=0, hi=4 << 20)
    sizes[:2] = [0, 1]
    offs = rng.integers(0, pool_bytes - sizes + 1)
    algos = [["ram", "ae", "maxp", "ae_min"][i] for i in rng.integers(0, 4, n_req)]
    if small_windows:
        windows = rng.choice([64, 300, 1024, 4096], n_req)
    else:
        windows = [WIN[a] for a in algos]
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    arrivals[:64] = 0.0          # a burst: several slots fill at once
    return offs, sizes, algos, np.asarray(windows), arrivals


def check_served(host, pool, reqs, cuts, n_cuts, st, check_oracle=True):
    nc = n_cuts.cpu().numpy()
    cu = cuts.cpu().numpy()
    for i, q in enumerate(reqs):
        assert st[i] == 0, (i, st[i])
        algo = ["ram", "ae", "maxp", "ae_min"][int(q["algo"])]
        o, n = int(q["offset"]), int(q["n"])
        got = cu[int(q["cut_base"]):int(q["cut_base"]) + int(nc[i])]
        alone = binding.chunk(pool[o:o + n], algo, int(q["window"]),
                              int(q["max_chunk"])).cpu().numpy()
        assert np.array_equal(got, alone), (i, algo, n)
        if check_oracle:
            exp = oracle.chunk(algo, host[o:o + n], int(q["window"]),
                               int(q["max_chunk"]))
            assert np.array_equal(got.astype(np.uint64), exp), (i, algo, n)


def test_serve_mixed_equals_alone():
    host, _ = datagen.mixed_stream(512, 41)            # 32 MiB pool
    pool = torch.from_numpy(host).cuda()
    offs, sizes, algos, windows, arr = make_requests(1500, 42, host.size, 20000.0)
    reqs, total = binding.requests(offs, sizes, algos, windows, 65536, arr)
    say("case serve mixed", len(reqs), int(sizes.sum()))
    cuts, n_cuts, lat, st, stats = binding.serve(pool, reqs, total,
                                                 budget_bytes=256 << 20,
                                                 max_batch=32, slots=4)
    say("stats", stats)
    assert stats["launches"] > 10
    assert stats["max_inflight"] >= 2          # batches overlapped
    assert np.all(lat >= 0)
    assert stats["bytes_done"] == int(sizes.sum())
    check_served(host, pool, reqs, cuts, n_cuts, st)
    assert binding.device_errors() == 0


def test_serve_small_budget_and_windows():
    """A budget of a few MiB makes admission wait for memory; windows vary
    per request."""
    host = datagen.uniform(16 << 20, 51)
    host[1 << 20:(1 << 20) + 300000] = 9
    pool = torch.from_numpy(host).cuda()
    offs, sizes, algos, windows, arr = make_requests(600, 52, host.size, 50000.0,
                                                     small_windows=True)
    reqs, total = binding.requests(offs, sizes, algos, windows, 8192, arr)
    budget = int(sizes.max()) * 2 + (1 << 20)
    say("case serve small budget", budget)
    cuts, n_cuts, lat, st, stats = binding.serve(pool, reqs, total,
                                                 budget_bytes=budget,
                                                 max_batch=64, slots=3)
    say("stats", stats)
    assert stats["rejected"] == 0
    check_served(host, pool, reqs, cuts, n_cuts, st)


def test_serve_rejections():
    host = datagen.uniform(4 << 20, 61)
    pool = torch.from_numpy(host).cuda()
    offs = np.array([0, 100, 5000, 0, 7])
    sizes = np.array([70000, 2 << 20, 30000, 50000, 12345])
    algos = ["ram", "ae", "maxp", "ram", "ae"]
    windows = np.array([4096, 4096, 2048, 100, 4096])   # request 3: below min
    reqs, total = binding.requests(offs, sizes, algos, windows, 65536,
                                   [0.0, 0.0, 0.001, 0.001, 0.002])
    say("case serve rejections")
    cuts, n_cuts, lat, st, stats = binding.serve(
        pool, reqs, total, budget_bytes=1 << 20, max_batch=8, slots=2,
        min_window=2048, max_chunk=65536)
    assert st.tolist() == [0, -2, 0, -1, 0]      # too big for the budget; invalid
    assert lat[1] == -1 and lat[3] == -1
    assert stats["rejected"] == 2
    keep = [0, 2, 4]
    nc = n_cuts.cpu().numpy()
    cu = cuts.cpu().numpy()
    for i in keep:
        q = reqs[i]
        o, n = int(q["offset"]), int(q["n"])
        exp = oracle.chunk(algos[i], host[o:o + n], int(q["window"]), 65536)
        got = cu[int(q["cut_base"]):int(q["cut_base"]) + int(nc[i])]
        assert np.array_equal(got.astype(np.uint64), exp)


def test_serve_small_min_window_with_maxp():
    """min_window below 15 (no MAXP block summaries for that window) with
    MAXP requests of larger windows among the requests: the reservation
    still covers their block summaries, and every request equals the
    oracle."""
    host, _ = datagen.mixed_stream(128, 71)            # 8 MiB pool
    pool = torch.from_numpy(host).cuda()
    rng = np.random.default_rng(72)
    k = 400
    sizes = datagen.lognormal_sizes(k, 73, median=16384, sigma=1.5, lo=1,
                                    hi=1 << 20)
    offs = rng.integers(0, host.size - sizes + 1)
    algos = [["ram", "maxp", "ae"][i] for i in rng.integers(0, 3, k)]
    windows = np.array([{"ram": 5, "maxp": 2048, "ae": 300}[a] for a in algos])
    arr = np.cumsum(rng.exponential(1.0 / 30000.0, k))
    reqs, total = binding.requests(offs, sizes, algos, windows, 65536, arr)
    say("case serve min window 5 with maxp")
    cuts, n_cuts, lat, st, stats = binding.serve(pool, reqs, total,
                                                 budget_bytes=64 << 20,
                                                 max_batch=64, slots=3,
                                                 min_window=5)
    assert stats["rejected"] == 0
    check_served(host, pool, reqs, cuts, n_cuts, st)
