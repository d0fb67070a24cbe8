"""The batched many-file path (GPU): every job's offsets equal the oracle's
on that buffer alone, rejected jobs do not disturb the others, the plain
one-call-per-job path agrees, and a batch captured into a HIP graph gives
the same result on every replay."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2508_05797_amd import binding, datagen

pytestmark = pytest.mark.gpu

ALGO_W = {"ram": 4096, "ae": 4096, "maxp": 2048, "ae_min": 4096}


def say(*a):
    print(*a, flush=True)


def make_files(n_files, seed, max_len=3 << 20):
    """Log-normal sizes (median 16 KiB here), uniform bytes, each file at an
    unaligned offset inside one device buffer."""
    rng = np.random.default_rng(seed)
    sizes = datagen.lognormal_sizes(n_files, seed, median=16384, sigma=1.5,
                                    lo=0, hi=max_len)
    sizes[:3] = [0, 1, 4097]
    gaps = rng.integers(0, 16, n_files)
    offs = np.zeros(n_files, np.int64)
    pos = 0
    for i, (s, g) in enumerate(zip(sizes, gaps)):
        pos += int(g)
        offs[i] = pos
        pos += int(s)
    host = datagen.uniform(pos + 64, seed + 1)
    # a few constant runs so the chains have lockstep stretches
    host[1000:70000] = 7
    return host, offs, sizes


def check_batch(b, host, offs, sizes, algos, windows, maxc):
    torch.cuda.synchronize()
    nc = b.n_cuts.cpu().numpy()
    cuts = b.cuts.cpu().numpy()
    st = b.statuses()
    for j in range(len(sizes)):
        assert st[j] == 0, (j, st[j])
        x = host[offs[j]:offs[j] + sizes[j]]
        exp = oracle.chunk(algos[j], x, windows[j], maxc[j])
        got = cuts[int(b.cut_base[j]):int(b.cut_base[j]) + int(nc[j])]
        assert got.size == exp.size and np.array_equal(got.astype(np.uint64), exp), \
            (j, algos[j], sizes[j])


def test_batch_mixed_algorithms():
    host, offs, sizes = make_files(300, 3)
    rng = np.random.default_rng(5)
    algos = [["ram", "ae", "maxp", "ae_min"][i] for i in rng.integers(0, 4, 300)]
    windows = [ALGO_W[a] for a in algos]
    d = torch.from_numpy(host).cuda()
    b = binding.Batch(d, offs, sizes, algos, windows, 65536)
    say("case batch mixed", b.n_jobs, b.total_bytes)
    b.run()
    check_batch(b, host, offs, sizes, algos, windows, [65536] * 300)
    assert binding.device_errors() == 0


def test_batch_constant_blocks():
    """Several long RAM jobs of constant 64 KiB blocks (chains that never
    meet; segment entries from the gate pass, which first checks each job
    with one wave) beside mixed and small jobs, at aligned and unaligned
    offsets."""
    blocks = datagen.constant_blocks(160, 21)                    # 10 MiB
    mixed, _ = datagen.mixed_stream(96, 22)                      # 6 MiB
    host = np.concatenate([blocks, mixed, blocks[:4 << 20], np.zeros(64, np.uint8)])
    b0, m0, c0 = 0, blocks.size, blocks.size + mixed.size
    offs = np.array([b0, b0 + 7, b0 + (1 << 20), m0, c0, b0 + 65536, m0 + 5,
                     b0 + 100, c0 + 3, 0], np.int64)
    sizes = np.array([blocks.size, blocks.size - 7, 8 << 20, mixed.size, 4 << 20,
                      6 << 20, 1 << 20, 5000, (4 << 20) - 3, 123], np.int64)
    algos = ["ram", "ram", "ram", "ram", "ram", "ram", "ae", "ram", "ram", "maxp"]
    windows = [ALGO_W[a] for a in algos]
    d = torch.from_numpy(host).cuda()
    binding.set_tuning(524288, 0)
    try:
        b = binding.Batch(d, offs, sizes, algos, windows, 65536)
        say("case batch constant blocks", b.n_jobs, b.total_bytes)
        b.run()
        check_batch(b, host, offs, sizes, algos, windows, [65536] * len(sizes))
    finally:
        binding.set_tuning(0, 0)
    assert binding.device_errors() == 0


@pytest.mark.parametrize("algo", ["ram", "ae", "maxp", "ae_min"])
def test_batch_equals_plain(algo):
    host, offs, sizes = make_files(120, 11)
    d = torch.from_numpy(host).cuda()
    w = ALGO_W[algo]
    b1 = binding.Batch(d, offs, sizes, algo, w, 65536)
    b2 = binding.Batch(d, offs, sizes, algo, w, 65536)
    say("case batch vs plain", algo)
    b1.run()
    b2.run_each()
    torch.cuda.synchronize()
    assert torch.equal(b1.n_cuts, b2.n_cuts)
    for j in range(len(sizes)):
        assert torch.equal(b1.result(j), b2.result(j)), j
    check_batch(b1, host, offs, sizes, [algo] * 120, [w] * 120, [65536] * 120)


def test_batches_on_two_streams():
    """Two batches enqueued at once on two caller streams (each stream has
    its own workspace and side streams) both give the oracle's offsets."""
    host, offs, sizes = make_files(200, 21)
    rng = np.random.default_rng(22)
    algos = [["ram", "ae", "maxp", "ae_min"][i] for i in rng.integers(0, 4, 200)]
    windows = [ALGO_W[a] for a in algos]
    d = torch.from_numpy(host).cuda()
    ba = binding.Batch(d, offs, sizes, algos, windows, 65536)
    bb = binding.Batch(d, offs[::-1].copy(), sizes[::-1].copy(), algos[::-1],
                       windows[::-1], 65536)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    say("case two streams", ba.n_jobs, ba.total_bytes)
    torch.cuda.synchronize()
    for _ in range(2):                   # the first run makes the side streams
        ba.run(stream=sa)
        bb.run(stream=sb)
    torch.cuda.synchronize()
    check_batch(ba, host, offs, sizes, algos, windows, [65536] * 200)
    check_batch(bb, host, offs[::-1], sizes[::-1], algos[::-1], windows[::-1],
                [65536] * 200)
    assert binding.device_errors(sa) == 0 and binding.device_errors(sb) == 0


def test_batch_many_jobs():
    """More jobs than one planning block holds (2,600, so three blocks), the
    four algorithms interleaved, and invalid jobs among them: every valid
    job equals the oracle and each algorithm's items stay its own."""
    host, offs, sizes = make_files(2600, 41, max_len=256 << 10)
    rng = np.random.default_rng(43)
    algos = [["ram", "ae", "maxp", "ae_min"][i] for i in rng.integers(0, 4, 2600)]
    windows = np.array([ALGO_W[a] for a in algos], np.uint32)
    bad = rng.choice(np.arange(3, 2600), 25, replace=False)
    windows[bad] = 0                     # rejected by the planner
    d = torch.from_numpy(host).cuda()
    b = binding.Batch(d, offs, sizes, algos, windows, 65536)
    say("case batch many jobs", b.n_jobs, b.total_bytes)
    b.run()
    torch.cuda.synchronize()
    nc = b.n_cuts.cpu().numpy()
    cuts = b.cuts.cpu().numpy()
    st = b.statuses()
    bad_set = set(int(j) for j in bad)
    for j in range(2600):
        if j in bad_set:
            assert st[j] == -1 and nc[j] == 0, (j, st[j], nc[j])   # CDC_EINVAL
            continue
        assert st[j] == 0, (j, st[j])
        x = host[offs[j]:offs[j] + sizes[j]]
        exp = oracle.chunk(algos[j], x, int(windows[j]), 65536)
        got = cuts[int(b.cut_base[j]):int(b.cut_base[j]) + int(nc[j])]
        assert np.array_equal(got.astype(np.uint64), exp), (j, algos[j], sizes[j])
    assert binding.device_errors() == 0


def test_batch_many_short_chain_jobs():
    """9,000 RAM / AE / AE-Min jobs, more chain items than a batch runs AE
    with successor words for (8,192), so AE and AE-Min take their leaner
    walkers here, some of them over several segments: every job equals the
    oracle."""
    n = 9000
    host, offs, sizes = make_files(n, 47, max_len=1 << 20)
    rng = np.random.default_rng(48)
    algos = [["ram", "ae", "ae_min"][i] for i in rng.integers(0, 3, n)]
    windows = [ALGO_W[a] for a in algos]
    assert sum(1 for j in range(n) if algos[j] != "ram" and sizes[j] > 512 << 10) > 0
    d = torch.from_numpy(host).cuda()
    b = binding.Batch(d, offs, sizes, algos, windows, 65536)
    say("case batch many short chain jobs", b.n_jobs, b.total_bytes)
    b.run()
    check_batch(b, host, offs, sizes, algos, windows, [65536] * n)
    assert binding.device_errors() == 0


def test_batch_rejects_invalid_jobs():
    host, offs, sizes = make_files(40, 21)
    d = torch.from_numpy(host).cuda()
    windows = np.full(40, 300, np.uint32)
    maxc = np.full(40, 4000, np.uint32)
    windows[5] = 0          # invalid window
    maxc[9] = 300           # max chunk not above the window
    b = binding.Batch(d, offs, sizes, "ram", windows, maxc)
    b.host_jobs["cut_offsets"][13] = 0
    b.jobs = torch.from_numpy(b.host_jobs.view(np.uint8).copy()).cuda()
    if sizes[13] == 0:
        pytest.skip("job 13 is empty")
    say("case batch invalid")
    b.run()
    torch.cuda.synchronize()
    st = b.statuses()
    nc = b.n_cuts.cpu().numpy()
    for j in range(40):
        if j in (5, 9, 13):
            assert st[j] == -1 and nc[j] == 0, (j, st[j], nc[j])
        else:
            assert st[j] == 0
            x = host[offs[j]:offs[j] + sizes[j]]
            exp = oracle.chunk("ram", x, 300, 4000)
            assert np.array_equal(b.result(j).cpu().numpy().astype(np.uint64), exp)


@pytest.mark.parametrize("eager_first", [False, True])
def test_batch_graph_replay(eager_first):
    """Capture one batched call per algorithm into a HIP graph after a
    reservation, replay it several times with eager work in between, and
    check every replay; then change the descriptors' data and replay.  With
    an eager call first, the batch's side streams exist when the capture
    starts, so the graph holds the algorithms as parallel branches (forked
    and joined by events); without, the capture runs them in order."""
    host, offs, sizes = make_files(200, 31)
    d = torch.from_numpy(host).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        binding.reserve(int(sizes.sum()) + (1 << 20), 256, 2048, 65536, stream=s)
        bs = [binding.Batch(d, offs, sizes, a, ALGO_W[a], 65536)
              for a in ("ram", "ae", "maxp")]
        if eager_first:
            for b in bs:
                b.run(stream=s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            for b in bs:
                b.run(stream=s)
    for rep in range(3):
        for b in bs:
            b.n_cuts.zero_()
            b.cuts.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say("case graph replay", rep)
        for b, a in zip(bs, ("ram", "ae", "maxp")):
            check_batch(b, host, offs, sizes, [a] * 200, [ALGO_W[a]] * 200,
                        [65536] * 200)
        _ = (d.float().sum()).item()      # unrelated eager work
    # new bytes under the same descriptors
    host2 = datagen.uniform(host.size, 99)
    d.copy_(torch.from_numpy(host2).cuda())
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for b, a in zip(bs, ("ram", "ae", "maxp")):
        check_batch(b, host2, offs, sizes, [a] * 200, [ALGO_W[a]] * 200,
                    [65536] * 200)


def test_autotune_then_capture():
    """The autotuner picks a tuning from its grid, reserves the workspace,
    and the batch under that tuning (eager and captured) still equals the
    oracle; tuning the same shape again reuses the choice."""
    host, offs, sizes = make_files(150, 71)
    d = torch.from_numpy(host).cuda()
    algos = ["ram", "ae", "maxp"] * 50
    windows = [ALGO_W[a] for a in algos]
    s = torch.cuda.Stream()
    try:
        with torch.cuda.stream(s):
            b = binding.Batch(d, offs, sizes, algos, windows, 65536)
            torch.cuda.synchronize()
            say("case autotune")
            t1 = binding.autotune(b, reps=1, stream=s)
            assert t1["chain_segment"] in (256 << 10, 512 << 10, 1 << 20, 2 << 20, 4 << 20)
            assert t1["maxp_segment"] in (16 << 10, 32 << 10, 64 << 10, 128 << 10,
                                          256 << 10, 512 << 10, 1 << 20)
            assert t1["waves_per_block"] in (1, 2, 4)
            assert binding.get_tuning() == t1
            assert binding.autotune(b, reps=1, stream=s) == t1
            b.cuts.fill_(-1)
            b.run(stream=s)
            torch.cuda.synchronize()
            check_batch(b, host, offs, sizes, algos, windows, [65536] * 150)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                b.run(stream=s)
        for _ in range(2):
            b.cuts.fill_(-1)
            b.n_cuts.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            check_batch(b, host, offs, sizes, algos, windows, [65536] * 150)
    finally:
        binding.set_tuning()


def test_capture_needs_reservation():
    """Under stream capture a batch that no reservation covers is refused
    with CDC_ENOMEM before anything is enqueued (nothing may allocate)."""
    host, offs, sizes = make_files(20, 31)
    d = torch.from_numpy(host).cuda()
    b = binding.Batch(d, offs, sizes, "ram", 4096, 65536)
    s = torch.cuda.Stream()              # a stream without a workspace yet
    torch.cuda.synchronize()
    say("case capture without reservation")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rc = binding.lib().cdc_chunk_batch(ctypes.c_void_p(b.jobs.data_ptr()),
                                           b.n_jobs, ctypes.c_void_p(s.cuda_stream))
    assert rc == -2                      # CDC_ENOMEM
    assert "cdc_reserve" in binding.lib().cdc_last_error().decode()


def test_small_window_with_maxp_blocks():
    """A batch whose smallest window is below 15 (no MAXP block summaries for
    it) beside MAXP jobs with large windows (which need them): sized without
    a reservation, every job equals the oracle; also many small misaligned
    MAXP jobs, each needing up to two partial tiles."""
    host, offs, sizes = make_files(160, 91, max_len=1 << 20)
    d = torch.from_numpy(host).cuda()
    algos = ["ram", "maxp"] * 80
    windows = [8, 2048] * 80
    b = binding.Batch(d, offs, sizes, algos, windows, 65536)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        say("case small window + maxp blocks", b.n_jobs)
        b.run(stream=s)
    check_batch(b, host, offs, sizes, algos, windows, [65536] * 160)
    # many small MAXP jobs at odd addresses: 1,500 jobs of 1..2,000 bytes
    rng = np.random.default_rng(92)
    k = 1500
    ln = rng.integers(1, 2000, k)
    of = np.cumsum(ln + rng.integers(1, 16, k)) - ln
    assert int(of[-1] + ln[-1]) <= host.size
    al = ["maxp"] * (k - 1) + ["ram"]
    wi = [15] * (k - 1) + [3]
    b2 = binding.Batch(d, of, ln, al, wi, 4000)
    with torch.cuda.stream(s):
        say("case many small maxp jobs", b2.n_jobs)
        b2.run(stream=s)
    check_batch(b2, host, of, ln, al, wi, [4000] * k)
    assert binding.device_errors(s) == 0


def test_autotune_small_window_mix():
    """The autotuner on a batch that mixes a window below 15 with MAXP jobs
    returns a tuning whose batch equals the oracle (its trials used to fail
    for want of block summaries and were timed anyway)."""
    host, offs, sizes = make_files(60, 93)
    d = torch.from_numpy(host).cuda()
    algos = ["ae", "maxp", "ram"] * 20
    windows = [5, 2048, 4096] * 20
    s = torch.cuda.Stream()
    try:
        with torch.cuda.stream(s):
            b = binding.Batch(d, offs, sizes, algos, windows, 65536)
            torch.cuda.synchronize()
            say("case autotune small window")
            binding.autotune(b, reps=1, stream=s)
            b.cuts.fill_(-1)
            b.run(stream=s)
        check_batch(b, host, offs, sizes, algos, windows, [65536] * 60)
    finally:
        binding.set_tuning()


def test_graph_replay_after_workspace_growth():
    """A batch captured after a reservation, then a much larger call on the
    same stream (the workspace grows and is replaced): replaying the graph
    still gives the oracle's offsets, since the buffer the graph was
    captured with stays allocated."""
    host, offs, sizes = make_files(100, 95)
    d = torch.from_numpy(host).cuda()
    algos = ["ram", "ae", "maxp", "ae_min"] * 25
    windows = [ALGO_W[a] for a in algos]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        binding.reserve(int(sizes.sum()) + 4096, 128, 2048, 65536, stream=s)
        b = binding.Batch(d, offs, sizes, algos, windows, 65536)
        b.run(stream=s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            b.run(stream=s)
    big = torch.from_numpy(datagen.uniform(96 << 20, 96)).cuda()
    with torch.cuda.stream(s):
        say("case growth after capture")
        c = binding.chunk(big, "ram", 1, 2, stream=s)   # a large workspace
        assert int(c[-1].item()) == big.numel()
    for rep in range(2):
        b.cuts.fill_(-1)
        b.n_cuts.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say("case replay after growth", rep)
        check_batch(b, host, offs, sizes, algos, windows, [65536] * 100)
    del big
