"""Parity of the HIP path with the oracle, element by element (GPU).

Cut offsets are integers, so the bar is bit-exact equality with the oracle
on the same seeded bytes.  Inputs: the 8 MiB uniform RAM workload, an
adversarial suite (constant runs, ramps, sawtooth near the window length,
two-valued and spike data, Zipf text), ragged lengths around the window,
the maximum chunk and the 1 KiB tile, every base-pointer misalignment, and
segment lengths from far below to far above the window (the result may not
depend on how the stream is split).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_05797_amd import binding, datagen

pytestmark = pytest.mark.gpu

ALGOS = ["ram", "ae", "maxp", "ae_min"]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available()
    binding.lib()
    yield
    binding.set_tuning(0, 0)
    assert binding.device_errors() == 0


def gpu_cuts(x, algo, w, M, offset=0):
    """Chunk x on the device; offset > 0 places it at an unaligned address."""
    buf = torch.zeros(x.size + offset + 64, dtype=torch.uint8, device="cuda")
    if x.size:
        buf[offset:offset + x.size] = torch.from_numpy(x).cuda()
    view = buf[offset:offset + x.size]
    return binding.chunk(view, algo, w, M).cpu().numpy().astype(np.uint64)


def check(x, algo, w, M, offset=0, tag=""):
    say("case", tag, algo, "n=%d w=%d M=%d off=%d" % (x.size, w, M, offset))
    got = gpu_cuts(x, algo, w, M, offset)
    exp = oracle.chunk(algo, x, w, M)
    if got.size != exp.size or not np.array_equal(got, exp):
        k = 0
        while k < min(got.size, exp.size) and got[k] == exp[k]:
            k += 1
        raise AssertionError(
            "%s %s n=%d w=%d M=%d off=%d: %d vs %d cuts, first diff at %d: "
            "gpu %s oracle %s" % (tag, algo, x.size, w, M, offset, got.size,
                                  exp.size, k, got[k:k + 3], exp[k:k + 3]))


def test_ram_8mib_uniform():
    x = datagen.uniform(8 << 20, 1)
    check(x, "ram", 4096, 65536, tag="C1")


@pytest.mark.parametrize("algo", ALGOS)
def test_mixed_16mib(algo):
    x, _ = datagen.mixed_stream(256, 2)
    w = 2048 if algo == "maxp" else 4096
    check(x, algo, w, 65536, tag="mix")


def adversarial(n, w, rng):
    yield "zeros", np.zeros(n, np.uint8)
    yield "ff", np.full(n, 255, np.uint8)
    yield "const7f", np.full(n, 0x7F, np.uint8)
    yield "ramp_up", (np.arange(n) % 256).astype(np.uint8)
    yield "ramp_down", (255 - np.arange(n) % 256).astype(np.uint8)
    for p in (w - 1, w, w + 1, w + 2):
        yield "saw%d" % p, (np.arange(n) % max(p, 1) * 255 // max(p, 1)).astype(np.uint8)
    yield "two_val", rng.choice(np.array([0x7F, 0x80], np.uint8), n)
    yield "signed_trap", rng.choice(np.array([0, 0x7F, 0x80, 0xFF], np.uint8), n)
    sp = np.zeros(n, np.uint8)
    sp[rng.integers(0, n, max(1, n // (3 * w + 1)))] = 255
    yield "spikes", sp
    yield "zipf", datagen.zipf_table(datagen.PRINTABLE)[rng.integers(0, 1 << 20, n)]
    yield "uniform", rng.integers(0, 256, n).astype(np.uint8)
    runs = np.repeat(rng.integers(0, 256, n // 700 + 1).astype(np.uint8), 700)[:n]
    yield "runs", runs


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("w,M", [(1, 2), (3, 7), (15, 16), (64, 1000),
                                 (600, 4000), (4096, 65536), (9000, 30000),
                                 (20000, 70000)])
def test_adversarial(algo, w, M):
    rng = np.random.default_rng(w * 7 + M)
    n = max(3 * M + 333, 20000)
    for name, x in adversarial(n, w, rng):
        check(x, algo, w, M, tag=name)


@pytest.mark.parametrize("algo", ALGOS)
def test_ragged_lengths(algo):
    rng = np.random.default_rng(4)
    w, M = 100, 700
    base = rng.integers(0, 256, 40000).astype(np.uint8)
    lens = [0, 1, 2, 15, 16, 17, w - 1, w, w + 1, w + 2, 2 * w + 1, M - 1, M,
            M + 1, 1023, 1024, 1025, 16383, 16385, 39999]
    for n in lens:
        check(base[:n], algo, w, M, tag="len")
        check(np.zeros(n, np.uint8), algo, w, M, tag="len0")


@pytest.mark.parametrize("algo", ALGOS)
def test_base_alignment(algo):
    rng = np.random.default_rng(5)
    x = rng.integers(0, 256, 30011).astype(np.uint8)
    x[10000:14000] = 3
    for off in range(16):
        check(x, algo, 200, 3000, offset=off, tag="align")


@pytest.mark.parametrize("algo", ALGOS)
def test_segment_invariance(algo):
    """The split into segments is a tuning choice; offsets must not move."""
    x, _ = datagen.mixed_stream(24, 9, block=4096)
    x = np.concatenate([x, np.full(50000, 9, np.uint8), x[:7777]])
    w = 300 if algo != "maxp" else 100
    exp = oracle.chunk(algo, x, w, 5000)
    try:
        for seg in [16, 100, 1000, 1024, 4099, 5000, 65536, 1 << 20]:
            binding.set_tuning(seg, 0)
            say("case seg", algo, seg)
            got = gpu_cuts(x, algo, w, 5000)
            assert np.array_equal(got, exp), (algo, seg)
    finally:
        binding.set_tuning(0, 0)


@pytest.mark.parametrize("algo", ["ram", "ae", "ae_min"])
@pytest.mark.parametrize("seg", [2048, 8192, 65536, 300000])
def test_resolution_rounds(algo, seg):
    """Short segments and long constant runs: many fix-up chains do not meet
    the speculative ones within their segment (chains with different phases
    never meet inside a constant run), so the parallel rounds and the ordered
    pass both have work; offsets must not move."""
    x, _ = datagen.mixed_stream(48, 12)
    rng = np.random.default_rng(seg)
    runs = [np.full(int(rng.integers(20000, 90000)), int(rng.integers(0, 256)),
                    np.uint8) for _ in range(6)]
    x = np.concatenate([x[:700000], runs[0], runs[1], x[700000:1500000],
                        runs[2], runs[3], runs[4], x[1500000:], runs[5]])
    exp = oracle.chunk(algo, x, 1500, 9000)
    try:
        binding.set_tuning(seg, 0)
        say("case rounds", algo, seg)
        got = gpu_cuts(x, algo, 1500, 9000)
        assert np.array_equal(got, exp), (algo, seg)
    finally:
        binding.set_tuning(0, 0)


@pytest.mark.parametrize("seg", [0, 65536, 300000, 1 << 21])
def test_constant_blocks(seg):
    """Blocks of one value each, the value changing from block to block: RAM
    chains keep their distance across every border (each border moves every
    chain by w + 1 or by max_chunk), so no speculative list is landed on and
    segment entries come from the runs of one value of at least max_chunk
    bytes.  Also: the blocks off the tile grid (an unaligned base; blocks
    of 4,133 bytes, whose value changes fall at every offset inside tiles);
    blocks shorter than max_chunk (65,000 bytes: no gates, the ordered pass
    settles the job); max_chunk longer than a block; a small window over
    4 KiB blocks; such blocks between mixed data; AE and AE-Min."""
    x = datagen.constant_blocks(1024, 5)                     # 64 MiB
    try:
        binding.set_tuning(seg, 0)
        check(x, "ram", 4096, 65536, tag="blocks seg=%d" % seg)
        if seg == 0:
            check(x, "ram", 4096, 65536, offset=5, tag="blocks unaligned")
            check(x[:16 << 20], "ram", 4096, 131072, tag="blocks M>block")
            check(datagen.constant_blocks(256, 6, block=65000), "ram", 4096,
                  65536, tag="blocks 65000")
            check(datagen.constant_blocks(4096, 7, block=4096), "ram", 100,
                  1000, tag="blocks 4k")
            # value changes at every offset inside tiles (tiles of two values)
            check(datagen.constant_blocks(3000, 8, block=4133), "ram", 100,
                  1000, tag="blocks 4133")
            check(datagen.constant_blocks(3000, 8, block=4133), "ram", 100,
                  1000, offset=11, tag="blocks 4133 unaligned")
            # extreme windows: w = 1, w = max_chunk - 1 (every chunk w + 1
            # long), w close to max_chunk, and a small max_chunk
            small = x[:8 << 20]
            for w_, M_ in ((1, 65536), (4096, 4097), (60000, 65536), (100, 101),
                           (2000, 2048)):
                check(small, "ram", w_, M_, tag="blocks w=%d M=%d" % (w_, M_))
            m, _ = datagen.mixed_stream(256, 3)
            y = np.concatenate([m[:5 << 20], x[:8 << 20], m[5 << 20:11 << 20],
                                x[8 << 20:12 << 20], m[11 << 20:]])
            check(y, "ram", 4096, 65536, tag="blocks in mixed")
            check(y[3:], "ram", 4096, 65536, tag="blocks in mixed, shifted")
            for algo in ("ae", "ae_min"):
                check(x, algo, 4096, 65536, tag="blocks")
    finally:
        binding.set_tuning(0, 0)


def dense_max(n, rate, rng, hi=255, lo_cap=255):
    """Bytes below lo_cap with the value hi planted at the given rate: how
    many of a tile's maxima there are (and whether its summary lists them
    all) is set by the rate."""
    x = rng.integers(0, lo_cap, n, dtype=np.uint8)
    x[rng.random(n) < rate] = hi
    return x


@pytest.mark.parametrize("algo", ["ram", "ae", "ae_min"])
@pytest.mark.parametrize("w,M", [(1024, 65536), (3000, 3001), (4096, 8192),
                                 (4096, 65536), (5000, 131072), (2047, 60000)])
def test_tile_maxima_density(algo, w, M):
    # chains stepping from one summarised maximum to the next: tiles with
    # one, a few, exactly seven and many maxima; maxima spaced near the
    # window; text whose largest symbol is rare or common
    rng = np.random.default_rng(w * 7 + M)
    n = (3 << 20) + 777
    for rate in (1 / 20000, 1 / 4096, 1 / 1024, 1 / 146, 1 / 64, 1 / 8):
        check(dense_max(n, rate, rng), algo, w, M, tag="dense%g" % rate)
    check(dense_max(n, 1 / 300, rng, hi=122, lo_cap=122), algo, w, M, tag="text_hi")
    spaced = rng.integers(0, 200, n, dtype=np.uint8)
    spaced[::w + 1] = 255
    spaced[w // 2::3 * w] = 255
    check(spaced, algo, w, M, tag="spaced")


@pytest.mark.parametrize("w,M", [(1500, 9000), (4096, 65536), (1500, 1501),
                                 (4096, 4097)])
def test_constant_segments(w, M):
    """RAM over runs that cover whole segments (resolved arithmetically:
    every chunk inside such a run is w + 1 long), runs of different values
    back to back, runs at the stream's ends, and max_chunk = w + 1 (fixed
    size chunks whatever the bytes)."""
    rng = np.random.default_rng(w + M)
    x, _ = datagen.mixed_stream(16, 5)
    parts = [np.full(300000, 0, np.uint8), x[:200000],
             np.full(250000, 255, np.uint8), np.full(180000, 7, np.uint8),
             x[200000:700000], np.full(400000, int(rng.integers(0, 256)), np.uint8),
             x[700000:], np.full(123457, 3, np.uint8)]
    x = np.concatenate(parts)
    exp = oracle.chunk("ram", x, w, M)
    try:
        for seg, off in ((16384, 0), (65536, 5)):
            binding.set_tuning(seg, 0)
            say("case constant segments", w, M, seg, off)
            got = gpu_cuts(x, "ram", w, M, off)
            assert np.array_equal(got, exp), (w, M, seg, off)
    finally:
        binding.set_tuning(0, 0)


@pytest.mark.slow
@pytest.mark.parametrize("algo", ["ram", "ae", "maxp"])
def test_mixed_1gib(algo):
    """The 1 GiB mixed stream at full size, whole cut list vs the oracle."""
    x, _ = datagen.mixed_stream(16384, 2024)
    w = 2048 if algo == "maxp" else 4096
    check(x, algo, w, 65536, tag="C2")


@pytest.mark.slow
def test_past_4gib():
    """A buffer longer than 2^32 bytes (ragged length), zero except for
    random stretches across 2^31 and 2^32 and at its end and a constant run
    of another value: every algorithm's single call, and a batch whose
    second job starts past 2^32, equal the oracle (positions are 64-bit from
    the job start to the output)."""
    n = (1 << 32) + (96 << 20) + 12345
    x = np.zeros(n, np.uint8)
    rnd = datagen.uniform(28 << 20, 41)
    x[(1 << 31) - (2 << 20):(1 << 31) + (2 << 20)] = rnd[:4 << 20]
    x[(1 << 32) - (8 << 20):(1 << 32) + (8 << 20)] = rnd[4 << 20:20 << 20]
    x[(1 << 32) + (40 << 20):(1 << 32) + (41 << 20)] = 201
    x[n - (8 << 20):] = rnd[20 << 20:]
    d = torch.from_numpy(x).cuda()
    win = {"ram": 4096, "ae": 4096, "maxp": 2048, "ae_min": 4096}
    for algo in ALGOS:
        say("case past 4 GiB", algo, "n=%d" % n)
        got = binding.chunk(d, algo, win[algo], 65536).cpu().numpy().astype(np.uint64)
        exp = oracle.chunk(algo, x, win[algo], 65536)
        assert got.size == exp.size and np.array_equal(got, exp), algo
        assert int(got[-1]) == n
    # a batch: a small job, then one from 3 MiB below 2^32 to the end
    lo = (1 << 32) - (3 << 20) + 7
    offs = np.array([1000, lo], np.int64)
    sizes = np.array([5 << 20, n - lo], np.int64)
    for algo in ["ram", "maxp"]:
        say("case past 4 GiB batch", algo)
        b = binding.Batch(d, offs, sizes, algo, win[algo], 65536)
        b.run()
        torch.cuda.synchronize()
        assert (b.statuses() == 0).all()
        for j in range(2):
            exp = oracle.chunk(algo, x[offs[j]:offs[j] + sizes[j]], win[algo], 65536)
            got = b.result(j).cpu().numpy().astype(np.uint64)
            assert got.size == exp.size and np.array_equal(got, exp), (algo, j)
    del d
    torch.cuda.empty_cache()


@pytest.mark.slow
@pytest.mark.parametrize("w", [4096, 1 << 20])
def test_max_chunk_limit(w):
    """The largest max_chunk (2^28) and a window of 1 MiB: zeros with two
    255 bytes (after each, RAM scans the zeros up to the forced cut at
    s + 2^28) and a random stretch, about 640 MiB in all."""
    M = 1 << 28
    n = (640 << 20) + 77
    x = np.zeros(n, np.uint8)
    x[0] = 255
    x[300 << 20] = 255
    x[500 << 20:501 << 20] = datagen.uniform(1 << 20, 43)
    d = torch.from_numpy(x).cuda()
    for algo in ALGOS:
        wa = min(w, 4096) if algo == "maxp" else w
        say("case max chunk", algo, "w=%d M=%d n=%d" % (wa, M, n))
        got = binding.chunk(d, algo, wa, M).cpu().numpy().astype(np.uint64)
        exp = oracle.chunk(algo, x, wa, M)
        assert got.size == exp.size and np.array_equal(got, exp), algo
        if algo in ("ram", "maxp"):
            assert M in np.diff(np.concatenate([[0], exp.astype(np.int64)]))
    del d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("algo", ["ram", "ae", "ae_min"])
def test_walk_stats_account_for_every_chunk(algo):
    # cdc_walk_stats: the speculation walk of each segment takes every chunk
    # from the segment's start to the first cut past its end.  On uniform
    # bytes a speculative chain meets the true one within a few chunks, so
    # the step kinds add up to the cuts within a few per segment, and no
    # step is a run of one value; MAXP reports none
    x = datagen.uniform(16 << 20, 31)
    d = torch.from_numpy(x).cuda()
    binding.set_tuning(1 << 20, 0)
    cuts = binding.chunk(d, algo, 4096, 65536)
    st = binding.walk_stats()
    binding.set_tuning(0, 0)
    exp = oracle.chunk(algo, x, 4096, 65536)
    assert np.array_equal(cuts.cpu().numpy().astype(np.uint64), exp)
    assert st["segments"] == 16
    steps = st["steps_successor"] + st["steps_fast"] + st["steps_run"] + st["steps_exact"]
    assert abs(steps - exp.size) <= 16 * 4, (steps, exp.size)
    assert st["steps_run"] == 0
    assert st["steps_successor"] > 0
    binding.chunk(d, "maxp", 2048, 65536)
    assert binding.walk_stats()["segments"] == 0
