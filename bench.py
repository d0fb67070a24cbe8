"""Benchmark of the chunk-boundary path on one MI355X.

Legs, all on seeded synthetic data resident in HBM before timing:

  stream  (the headline ``value``) one step chunks a 1 GiB stream of 64 KiB
          blocks (50% uniform random, 30% Zipf(1.1) text over 64 symbols,
          20% constant runs) with RAM (w=4096), AE-Max (w=4096) and MAXP
          (w=2048 each side), max chunk 64 KiB: three passes of the whole hot
          path over the same bytes, as one cdc_chunk_batch of three jobs
          (its segment lengths chosen by cdc_autotune before timing).
          value = bytes chunked per second over the timed steps (GB = 1e9
          B), the median of five timed runs of K steps.  The same chunkings
          as single cdc_chunk calls give each algorithm's whole-call rate
          and fraction of the HBM peak, and the kernel times of the
          roofline.
  snap    backup snapshots: a 512 MiB uniform base and 8 versions (each
          edits 1% of its 4 KiB regions), every version chunked, every chunk
          fingerprinted (SHA-256) and counted in a device table of distinct
          chunks, per algorithm (windows for ~8 KiB chunks); the dedup ratio
          must equal the one from the oracle's cuts hashed on the host.
  batch   20,000 files of log-normal sizes (median 64 KiB, sigma 2.0,
          clipped to 1 KiB .. 256 MiB; uniform random bytes), every file
          under every algorithm as one cdc_chunk_batch of 60,000 jobs, tuned
          by cdc_autotune and captured in a HIP graph, against one cdc_chunk
          call per file and algorithm (the plain path).
  serve   open-loop Poisson arrivals of requests (sizes as the batch leg,
          algorithm uniform over RAM / AE / MAXP, bytes at random places of
          the resident batch buffer) at 25 / 50 / 90 % of the measured
          batched peak, at least 10^6 requests per level, served by
          cdc_serve (admission by an HBM budget, continuous batching on a
          stream pool): p50 / p99 latency and sustained GB/s; one more level
          at 50 % with a budget small enough that admission waits for memory.

Also reported: the roofline of the stream leg's dominant kernel (its
algorithmic bytes, the stream read once, over its average duration from HIP
events on the launch stream, against the 8 TB/s HBM peak; traffic from
rocprofv3 FETCH_SIZE / WRITE_SIZE when they were taken on the current kernel
source) and each algorithm's whole-call fraction of the peak; RAM on 256 MiB
of constant 64 KiB blocks whose value changes (the hardest input for its
resolution); the bytes each pattern handles per algorithm (oracle); and the
oracle timed on this host (cpu_baseline: one core on a sample of the stream;
all cores on the many-file set), whose cuts also check the GPU's.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--legs stream,snap,batch,serve] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("GB/s chunked, bit-exact cuts, batched vs plain, % HBM peak; "
          "serve p99 ms")
HBM_PEAK_GBS = 8000.0
STREAM_BLOCKS = 16384          # 16384 x 64 KiB = 1 GiB
STREAM_SEED = 2024
ALGOS = [("ram", 4096), ("ae", 4096), ("maxp", 2048)]
WINDOW = dict(ALGOS)
MAX_CHUNK = 65536
MAX_CHUNK_LIMIT = 1 << 28
REPEATS = 5
N_FILES = 20000
FILES_SEED = 7
SNAP_BASE = 512 << 20
SNAP_VERSIONS = 8
SNAP_SEED = 2025
WIN8K = {"ram": 7936, "ae": 7936, "maxp": 444}   # ~8 KiB mean chunks
SERVE_SEED = 11
SERVE_LOADS = (0.25, 0.5, 0.9)
SERVE_SECONDS = 0.5            # arrivals per load level (at least)
SERVE_MIN_REQUESTS = 1000000
SERVE_BUDGET = 32 << 30        # HBM for requests in flight
SERVE_SMALL_BUDGET = 256 << 20
SERVE_SLOTS = 4
SERVE_MAX_BATCH = 16384
CONST_BLOCKS = 4096            # 256 MiB of constant 64 KiB blocks
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_2508_05797_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    """Digest of every device source (kernels and the headers they use)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def load_traffic():
    """Counter-based HBM bytes per launch, valid only for the kernel source
    they were measured on."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_sha():
        return None
    return t


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
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def events():
    import torch
    return (torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True))


def spread(xs):
    return {"median": round(statistics.median(xs), 4), "min": round(min(xs), 4),
            "max": round(max(xs), 4),
            "stdev": round(statistics.stdev(xs), 4) if len(xs) > 1 else 0.0,
            "runs": [round(x, 4) for x in xs]}


def timed(fn, steps, torch):
    """Milliseconds per call of fn over `steps` calls (events on the current
    stream)."""
    e0, e1 = events()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


# ----------------------------------------------------------------- stream leg
def stream_leg(args, binding, datagen, torch, np):
    log("stream: generating the 1 GiB mixed stream ...")
    x, _ = datagen.mixed_stream(STREAM_BLOCKS, STREAM_SEED)
    n = x.size
    dev = torch.device("cuda:0")
    d = torch.from_numpy(x).to(dev)
    bufs = {a: (torch.empty(binding.max_cuts(n, w), dtype=torch.int64, device=dev),
                torch.empty(1, dtype=torch.int64, device=dev)) for a, w in ALGOS}
    # the step: the stream under the three algorithms as one batched call
    # (three jobs on the same bytes; the library runs the algorithms side by
    # side)
    b3 = binding.Batch(d, [0] * len(ALGOS), [n] * len(ALGOS),
                       [a for a, _w in ALGOS], [w for _a, w in ALGOS], MAX_CHUNK)
    step_tuning = binding.autotune(b3, reps=3)
    binding.set_tuning(0, 0, 0)

    def step():
        b3.run()

    def single(only=None):
        for algo, w in ALGOS:
            if only and algo != only:
                continue
            cuts, nc = bufs[algo]
            binding.chunk_into(d, algo, w, MAX_CHUNK, cuts, nc)

    for _ in range(args.warmup):
        step()
        single()
    torch.cuda.synchronize()
    # timed region: K steps, REPEATS times
    step_ms = [timed(step, args.steps, torch) for _ in range(REPEATS)]
    ms_step = statistics.median(step_ms)
    # the same chunkings as single calls: per-algorithm whole-call rates
    per_algo, per_algo_ms, breakdown, walk = {}, {}, {}, {}
    for algo, _w in ALGOS:
        ms = [timed(lambda: single(algo), args.steps, torch) for _ in range(REPEATS)]
        per_algo_ms[algo] = spread(ms)
        per_algo[algo] = round(n / (statistics.median(ms) * 1e-3) / 1e9, 2)
        binding.set_profiling(2)
        binding.kernel_times()
        single(algo)
        breakdown[algo] = {k: round(v[1] / max(v[0], 1), 4)
                           for k, v in binding.kernel_times().items()}
        binding.set_profiling(0)
        if algo != "maxp":
            walk[algo] = binding.walk_stats()
    # HIP events around each call's main kernels on the launch stream
    binding.set_profiling(1)
    binding.kernel_times()
    for _ in range(args.steps):
        single()
    ktimes = binding.kernel_times()
    binding.set_profiling(0)
    seq_ms = timed(single, args.steps, torch)

    per_kernel = {k: tot / max(c, 1) for k, (c, tot) in ktimes.items()}
    dom = max(per_kernel, key=per_kernel.get)
    avg_ms = per_kernel[dom]
    achieved = n / (avg_ms * 1e-3) / 1e9
    traffic = load_traffic()
    torch.cuda.synchronize()
    assert (b3.statuses() == 0).all(), "batched step failed"
    gpu_cuts = {}
    for j, (a, _w) in enumerate(ALGOS):
        got = b3.result(j)
        assert torch.equal(got, bufs[a][0][:int(bufs[a][1].item())]), \
            "batched and single call differ: " + a
        gpu_cuts[a] = got.cpu().numpy().astype(np.uint64)
    assert binding.device_errors() == 0
    whole = {}
    for a, _w in ALGOS:
        t = statistics.median(per_algo_ms[a]["runs"]) * 1e-3
        gbs = (n + 8 * gpu_cuts[a].size) / t / 1e9
        whole[a] = {"gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "ms": round(t * 1e3, 4)}
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_bytes_per_launch": n,
            "traffic": (traffic or {}).get("bytes_per_launch", {}).get(dom),
            "whole_call": whole,
            "whole_call_note": "per algorithm: (n + 8 x cuts) / median call "
                               "time / 8 TB/s, over every kernel of the call"}
    value = len(ALGOS) * n / (ms_step * 1e-3) / 1e9
    seq = len(ALGOS) * n / (seq_ms * 1e-3) / 1e9
    del d, bufs, b3
    torch.cuda.empty_cache()
    return dict(x=x, value=value, ms_step=ms_step, seq_gbs=seq, roof=roof,
                step_tuning=step_tuning, step_spread=spread(step_ms),
                per_algo=per_algo, per_algo_ms=per_algo_ms, breakdown=breakdown,
                walk=walk,
                kernel_avg_ms={k: round(v, 4) for k, v in per_kernel.items()},
                gpu_cuts=gpu_cuts)


def constant_blocks_leg(args, binding, datagen, torch, np, check):
    """RAM over 256 MiB of constant 64 KiB blocks whose value changes."""
    x = datagen.constant_blocks(CONST_BLOCKS, 5)
    d = torch.from_numpy(x).cuda()
    cuts = torch.empty(binding.max_cuts(x.size, 4096), dtype=torch.int64, device="cuda")
    nc = torch.empty(1, dtype=torch.int64, device="cuda")
    run = lambda: binding.chunk_into(d, "ram", 4096, MAX_CHUNK, cuts, nc)
    run()
    torch.cuda.synchronize()
    ms = [timed(run, 5, torch) for _ in range(REPEATS)]
    binding.set_profiling(2)
    binding.kernel_times()
    run()
    breakdown = {k: round(v[1] / max(v[0], 1), 4)
                 for k, v in binding.kernel_times().items()}
    binding.set_profiling(0)
    out = {"workload": "RAM w=4096 over 256 MiB of constant 64 KiB blocks, "
                       "value changing per block",
           "gbs": round(x.size / (statistics.median(ms) * 1e-3) / 1e9, 2),
           "ms": spread(ms), "kernel_breakdown_ms": breakdown}
    if check:
        import oracle
        exp = oracle.chunk("ram", x, 4096, MAX_CHUNK)
        got = cuts[:int(nc.item())].cpu().numpy().astype(np.uint64)
        out["bit_exact_vs_oracle"] = bool(np.array_equal(got, exp))

    def variant(data_dev, host):
        """The same call timed on other bytes or another address."""
        c = torch.empty(binding.max_cuts(host.size, 4096), dtype=torch.int64, device="cuda")
        k = torch.empty(1, dtype=torch.int64, device="cuda")
        f = lambda: binding.chunk_into(data_dev, "ram", 4096, MAX_CHUNK, c, k)
        f()
        torch.cuda.synchronize()
        vm = [timed(f, 2, torch) for _ in range(3)]
        r = {"gbs": round(host.size / (statistics.median(vm) * 1e-3) / 1e9, 2),
             "ms": spread(vm)}
        if check:
            import oracle
            r["bit_exact_vs_oracle"] = bool(np.array_equal(
                c[:int(k.item())].cpu().numpy().astype(np.uint64),
                oracle.chunk("ram", host, 4096, MAX_CHUNK)))
        return r
    # the same blocks 5 bytes off the 1 KiB tile grid of the address
    buf = torch.zeros(x.size + 64, dtype=torch.uint8, device="cuda")
    buf[5:5 + x.size] = d
    out["offset_5_bytes"] = variant(buf[5:5 + x.size], x)
    del buf
    # blocks shorter than max_chunk (no run is a gate: settled in order)
    y = datagen.constant_blocks(CONST_BLOCKS * 65536 // 65000, 6, block=65000)
    dy = torch.from_numpy(y).cuda()
    out["blocks_65000_bytes"] = variant(dy, y)
    del d, dy
    return out


# -------------------------------------------------------------- snapshot leg
def snapshot_leg(args, binding, datagen, torch, np, check):
    log("snap: generating the base and %d versions ..." % SNAP_VERSIONS)
    versions = list(datagen.snapshot_versions(SNAP_BASE, SNAP_VERSIONS, SNAP_SEED))
    total = sum(v.size for v in versions)
    out = {"versions": len(versions), "bytes": total, "windows": WIN8K,
           "algorithms": {}}
    devs = [torch.from_numpy(v).cuda() for v in versions]
    streams = [torch.cuda.Stream() for _ in versions]
    torch.cuda.synchronize()
    for a, w in WIN8K.items():
        room = [binding.max_cuts(v.size, w) for v in versions]
        cuts = [torch.empty(r, dtype=torch.int64, device="cuda") for r in room]
        ncs = [torch.empty(1, dtype=torch.int64, device="cuda") for _ in versions]
        dgs = [torch.empty((r, 32), dtype=torch.uint8, device="cuda") for r in room]
        table = binding.Dedup(sum(room))

        # the versions are independent: one stream each, forked from and
        # joined back into the current stream (a version alone holds too
        # few chunks to fill the device with one hash per lane)
        def on_streams(work):
            cur = torch.cuda.current_stream()
            fork = torch.cuda.Event()
            fork.record(cur)
            for st, args_ in zip(streams, work):
                st.wait_event(fork)
                yield st, args_
            for st in streams:
                j = torch.cuda.Event()
                j.record(st)
                cur.wait_event(j)

        def chunk_all():
            for st, (d, c, k) in on_streams(zip(devs, cuts, ncs)):
                binding.chunk_into(d, a, w, MAX_CHUNK, c, k, stream=st)

        def fp_all():
            for st, (d, c, k, g) in on_streams(zip(devs, cuts, ncs, dgs)):
                binding.fingerprint_into(d, c, k, g, stream=st)

        chunk_all()
        fp_all()
        torch.cuda.synchronize()
        t_chunk = [timed(chunk_all, 1, torch) for _ in range(REPEATS)]
        t_fp = [timed(fp_all, 1, torch) for _ in range(REPEATS)]
        e0, e1 = events()
        e0.record()
        for g, c, k in zip(dgs, cuts, ncs):
            table.add(g, c, k)
        e1.record()
        torch.cuda.synchronize()
        st = table.stats()
        table.close()
        rec = {"chunk_gbs": round(total / (statistics.median(t_chunk) * 1e-3) / 1e9, 1),
               "fingerprint_gbs": round(total / (statistics.median(t_fp) * 1e-3) / 1e9, 1),
               "dedup_count_ms": round(e0.elapsed_time(e1), 3),
               "chunks": st["chunks"], "unique_chunks": st["unique_chunks"],
               "dedup_ratio": round(st["total_bytes"] / st["unique_bytes"], 6),
               "collisions": st["collisions"]}
        if check:
            rec.update(snapshot_oracle(a, w, versions, cuts, ncs, st, np))
        log("snap:", a, rec)
        out["algorithms"][a] = rec
        del cuts, ncs, dgs
    del devs
    torch.cuda.empty_cache()
    return out


def snapshot_oracle(a, w, versions, cuts, ncs, st, np):
    """The oracle's cuts of every version (all host cores), equal to the
    GPU's, hashed on the host: the dedup ratio they give."""
    import oracle
    _m, cores = host_cpu()
    with ThreadPoolExecutor(max(1, cores)) as pool:
        exp = list(pool.map(lambda v: oracle.chunk(a, v, w, MAX_CHUNK), versions))
    same = all(np.array_equal(c[:int(k.item())].cpu().numpy().astype(np.uint64), e)
               for c, k, e in zip(cuts, ncs, exp))

    def digests(args_):
        v, e = args_
        mv = memoryview(v)
        out, s = [], 0
        for c in e.tolist():
            out.append((hashlib.sha256(mv[s:c]).digest(), c - s))
            s = c
        return out

    with ThreadPoolExecutor(max(1, cores)) as pool:
        parts = list(pool.map(digests, zip(versions, exp)))
    seen, tot = {}, 0
    for part in parts:
        for key, ln in part:
            seen.setdefault(key, ln)
            tot += ln
    ratio = tot / sum(seen.values())
    return {"cuts_bit_exact_vs_oracle": bool(same),
            "oracle_dedup_ratio": round(ratio, 6),
            "dedup_ratio_equals_oracle": bool(
                st["total_bytes"] == tot and st["unique_bytes"] == sum(seen.values()))}


# ------------------------------------------------------------------ batch leg
def batch_leg(binding, datagen, torch, np):
    log("batch: generating %d files ..." % N_FILES)
    sizes = datagen.lognormal_sizes(N_FILES, FILES_SEED)
    host, offs = datagen.many_files(sizes, FILES_SEED)
    total = int(sizes.sum())
    d = torch.from_numpy(host).cuda()
    stream = torch.cuda.Stream()
    out = {"files": N_FILES, "bytes": total}
    # every file under every algorithm: one job table of 3 x 20,000 jobs, so
    # one batched call runs the three algorithms side by side
    k = len(ALGOS)
    job_offs = np.tile(offs[:-1], k)
    job_sizes = np.tile(sizes, k)
    job_algos = [a for a, _w in ALGOS for _ in range(N_FILES)]
    job_wins = np.repeat([w for _a, w in ALGOS], N_FILES)
    with torch.cuda.stream(stream):
        b = binding.Batch(d, job_offs, job_sizes, job_algos, job_wins, MAX_CHUNK)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out["tuning"] = binding.autotune(b, reps=2, stream=stream)
        log("batch: autotune -> %s (%.1f s)" % (out["tuning"], time.perf_counter() - t0))
        # reserve for the batch, then capture one batched call
        binding.reserve(k * total, k * N_FILES, min(w for _, w in ALGOS),
                        MAX_CHUNK, stream=stream)
        b.cuts.fill_(-1)
        b.n_cuts.fill_(-1)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            b.run(stream=stream)
        g.replay()
        torch.cuda.synchronize()
        reps = 5
        ms = []
        for _ in range(REPEATS):
            e0, e1 = events()
            e0.record(stream)
            for _ in range(reps):
                g.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1) / reps)
    ms_batched = statistics.median(ms)
    assert (b.statuses() == 0).all(), "batch job failed"
    batched_nc = b.n_cuts.clone()
    batched_cuts = b.cuts.clone()

    # plain: one cdc_chunk per file and algorithm, on one stream
    with torch.cuda.stream(stream):
        b.cuts.fill_(-1)
        b.n_cuts.fill_(-1)
        b.run_each(stream=stream)             # warm-up
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record(stream)
        b.run_each(stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1)
    same = torch.equal(batched_nc, b.n_cuts) and torch.equal(batched_cuts, b.cuts)
    steps_bytes = len(ALGOS) * total
    out.update({
        "batched_gbs": round(steps_bytes / (ms_batched * 1e-3) / 1e9, 2),
        "plain_gbs": round(steps_bytes / (ms_plain * 1e-3) / 1e9, 2),
        "batched_ms": spread(ms), "plain_ms": round(ms_plain, 3),
        "batched_identical_to_plain": bool(same),
        "n_cuts": {a: int(batched_nc[i * N_FILES:(i + 1) * N_FILES].sum().item())
                   for i, (a, _w) in enumerate(ALGOS)},
    })
    out["speedup"] = round(out["batched_gbs"] / out["plain_gbs"], 2)
    log("batch:", out)
    del g, b
    return d, host, offs, sizes, out


def many_files_oracle(host, offs, sizes, np):
    """The oracle over every file under every algorithm, on all host cores."""
    import oracle
    model, cores = host_cpu()
    jobs = [(a, w, int(o), int(s)) for a, w in ALGOS for o, s in zip(offs[:-1], sizes)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max(1, cores)) as pool:
        list(pool.map(lambda j: oracle.chunk(j[0], host[j[2]:j[2] + j[3]], j[1],
                                             MAX_CHUNK), jobs))
    t = time.perf_counter() - t0
    total = len(ALGOS) * int(sizes.sum())
    return {"value": round(total / t / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "oracle", "cpu_model": model,
            "sample": "every file of the many-file set under RAM, AE and MAXP "
                      "(%d jobs, %.2f GB), a thread per core" % (len(jobs), total / 1e9)}


# ------------------------------------------------------------------ serve leg
def serve_leg(pool, binding, datagen, torch, np):
    rng = np.random.default_rng(SERVE_SEED)
    pool_n = pool.numel()

    def draw(k, seed):
        sizes = datagen.lognormal_sizes(k, seed)
        sizes = np.minimum(sizes, pool_n)
        offs = (rng.random(k) * (pool_n - sizes + 1)).astype(np.int64)
        algos = [ALGOS[i][0] for i in rng.integers(0, 3, k)]
        wins = np.array([WINDOW[a] for a in algos])
        return offs, sizes, algos, wins

    # batched peak on the serving mix: one batch of 20,000 requests
    offs, sizes, algos, wins = draw(N_FILES, SERVE_SEED)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = binding.Batch(pool, offs, sizes, algos, wins, MAX_CHUNK)
        torch.cuda.synchronize()
        binding.autotune(b, reps=2, stream=stream)
        e0, e1 = events()
        e0.record(stream)
        for _ in range(3):
            b.run(stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
    peak = int(sizes.sum()) / (e0.elapsed_time(e1) / 3 * 1e-3)
    mean_size = float(datagen.lognormal_sizes(200000, SERVE_SEED + 1).mean())
    del b
    out = {"batched_peak_gbs": round(peak / 1e9, 2), "budget_bytes": SERVE_BUDGET,
           "slots": SERVE_SLOTS, "max_batch": SERVE_MAX_BATCH, "loads": []}
    # untimed warm-up of the serving path, as the other legs' warm-up steps
    rate = SERVE_LOADS[0] * peak / mean_size
    kw = max(100, int(rate * 0.2))
    offs, sizes, algos, wins = draw(kw, SERVE_SEED + 9)
    reqs, total = binding.requests(offs, sizes, algos, wins, MAX_CHUNK,
                                   np.cumsum(rng.exponential(1.0 / rate, kw)))
    binding.serve(pool, reqs, total, budget_bytes=SERVE_BUDGET,
                  max_batch=SERVE_MAX_BATCH, slots=SERVE_SLOTS)
    del reqs
    # the last level: a budget small enough that admission by memory binds
    # (one batch in flight), at a load below what that budget sustains
    levels = [(l, SERVE_BUDGET) for l in SERVE_LOADS] + [(0.1, SERVE_SMALL_BUDGET)]
    for i, (load, budget) in enumerate(levels):
        rate = load * peak / mean_size
        k = max(SERVE_MIN_REQUESTS, int(rate * SERVE_SECONDS))
        offs, sizes, algos, wins = draw(k, SERVE_SEED + 10 + i)
        arr = np.cumsum(rng.exponential(1.0 / rate, k))
        reqs, total = binding.requests(offs, sizes, algos, wins, MAX_CHUNK, arr)
        log("serve: load %.2f budget %d MiB, %d requests, %.2f GB offered over %.2f s"
            % (load, budget >> 20, k, sizes.sum() / 1e9, arr[-1]))
        cuts, n_cuts, lat, st, stats = binding.serve(
            pool, reqs, total, budget_bytes=budget,
            max_batch=SERVE_MAX_BATCH, slots=SERVE_SLOTS)
        ok = st == 0
        # a sample of requests: served result == the same request alone
        nc = n_cuts.cpu().numpy()
        same = True
        for j in rng.choice(k, min(k, 64), replace=False):
            q = reqs[j]
            o, n = int(q["offset"]), int(q["n"])
            alone = binding.chunk(pool[o:o + n], algos[j], int(q["window"]),
                                  MAX_CHUNK)
            cb = int(q["cut_base"])
            same = same and torch.equal(cuts[cb:cb + int(nc[j])], alone)
        lat_ms = lat[ok] * 1e3
        rec = {"load": load, "budget_bytes": budget, "requests": k,
               "offered_gbs": round(sizes.sum() / arr[-1] / 1e9, 2),
               "sustained_gbs": round(stats["bytes_done"] / stats["elapsed"] / 1e9, 2),
               "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
               "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
               "failed": int((~ok).sum()),
               "larger_than_budget": int((sizes + 8 * ((sizes - 1) // (wins + 1) + 1) > budget).sum()),
               "launches": stats["launches"],
               "max_inflight": stats["max_inflight"],
               "max_queue": stats["max_queue"],
               "sample_identical_to_alone": bool(same)}
        log("serve:", rec)
        out["loads"].append(rec)
        del cuts, n_cuts
    return out


# ------------------------------------------------------------------- oracle
def cpu_baseline(x, gpu_cuts, np):
    """The oracle, one core, on a bounded sample of the stream (its first
    256 MiB under each algorithm), and a check of the GPU's cuts over the
    whole stream."""
    import oracle
    model, cores = host_cpu()
    sample = x[:256 << 20]
    total_t = 0.0
    for algo, w in ALGOS:
        t0 = time.perf_counter()
        oracle.chunk(algo, sample, w, MAX_CHUNK)
        total_t += time.perf_counter() - t0
    gbs = len(ALGOS) * sample.size / total_t / 1e9
    exact = True
    with ThreadPoolExecutor(len(ALGOS)) as pool:
        exp = dict(zip([a for a, _ in ALGOS],
                       pool.map(lambda aw: oracle.chunk(aw[0], x, aw[1], MAX_CHUNK), ALGOS)))
    for algo, _w in ALGOS:
        same = np.array_equal(gpu_cuts[algo], exp[algo])
        log("oracle %s: %d cuts, gpu %d cuts, identical=%s"
            % (algo, exp[algo].size, gpu_cuts[algo].size, same))
        exact = exact and same
    shares = {}
    for algo, w in ALGOS:
        e, r = oracle.pattern_bytes(algo, sample, w, MAX_CHUNK)
        shares[algo] = {"ebs_bytes": e, "rs_bytes": r,
                        "ebs_share": round(e / max(e + r, 1), 4)}
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_cores": cores,
            "sample": "the first 256 MiB of the stream leg's bytes, each of RAM, "
                      "AE, MAXP once, single-threaded scalar C (gcc -O2)"}, exact, shares


def copy_calibration():
    """A plain elementwise copy (reads 1 GiB, writes 1 GiB per launch): what
    the FETCH_SIZE / WRITE_SIZE counters report for it scales theirs for
    the chunking kernels."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(7)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(a, 1, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n,
                      "launches": 3}), flush=True)


def profile_calls(args):
    """The stream leg's single calls alone, without tuning or timing."""
    import numpy as np
    import torch
    from paper_2508_05797_amd import binding, datagen
    binding.lib()
    binding.set_tuning()
    x, _ = datagen.mixed_stream(STREAM_BLOCKS, STREAM_SEED)
    d = torch.from_numpy(x).to("cuda:0")
    for algo, w in ALGOS:
        for _ in range(args.steps):
            cuts = binding.chunk(d, algo, w, MAX_CHUNK)
        torch.cuda.synchronize()
        print(json.dumps({"algorithm": algo, "calls": args.steps,
                          "cuts": int(cuts.numel())}), flush=True)


def profile_constant_blocks(args):
    """RAM single calls on the constant-block input alone (for profilers)."""
    import torch
    from paper_2508_05797_amd import binding, datagen
    binding.lib()
    binding.set_tuning()
    x = datagen.constant_blocks(CONST_BLOCKS, 5)
    d = torch.from_numpy(x).to("cuda:0")
    for _ in range(args.steps):
        cuts = binding.chunk(d, "ram", 4096, MAX_CHUNK)
    torch.cuda.synchronize()
    print(json.dumps({"algorithm": "ram", "input": "constant blocks",
                      "calls": args.steps, "cuts": int(cuts.numel())}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--legs", default="stream,snap,batch,serve")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle (no cpu_baseline, no checks)")
    ap.add_argument("--profile-calls", action="store_true",
                    help="only chunk the 1 GiB stream with single calls of "
                         "each algorithm, --steps times (a short command for "
                         "profilers; prints one line per algorithm)")
    ap.add_argument("--profile-constant-blocks", action="store_true",
                    help="only chunk the 256 MiB constant-block input with RAM "
                         "single calls, --steps times (for profilers)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy kernel three "
                         "times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library runs on a single MI355X "
              "and has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))
    if args.copy_calibration:
        copy_calibration()
        return
    if args.profile_calls:
        profile_calls(args)
        return
    if args.profile_constant_blocks:
        profile_constant_blocks(args)
        return

    import numpy as np
    import torch
    from paper_2508_05797_amd import binding, datagen

    binding.lib()                 # raises if the library is not built
    binding.set_tuning()
    check = not args.no_cpu

    out = {"metric": METRIC, "value": None, "unit": "GB/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u8", "data": "synthetic",
           "config": {"workload": "1 GiB stream of 64 KiB blocks: 50% uniform, "
                                  "30% Zipf(1.1) text over 64 symbols, 20% "
                                  "constant runs; RAM w=4096, AE w=4096, MAXP "
                                  "w=2048, max chunk 64 KiB",
                      "bytes": STREAM_BLOCKS * 65536,
                      "algorithms": [a for a, _ in ALGOS],
                      "max_chunk_limit": MAX_CHUNK_LIMIT,
                      "parallelism": "single GPU"},
           "roofline": None, "cpu_baseline": None}
    s = None
    if "stream" in legs:
        s = stream_leg(args, binding, datagen, torch, np)
        out["value"] = round(s["value"], 2)
        out["ms_per_step"] = round(s["ms_step"], 4)
        out["roofline"] = s["roof"]
        out["step"] = ("one cdc_chunk_batch over the three (stream, algorithm) "
                       "jobs; value from the median of %d timed runs of K steps; "
                       "roofline and per-algorithm rates from the same "
                       "chunkings as single cdc_chunk calls" % REPEATS)
        out["step_ms"] = s["step_spread"]
        out["step_tuning"] = s["step_tuning"]
        out["sequential_gbs"] = round(s["seq_gbs"], 2)
        out["per_algorithm_gbs"] = s["per_algo"]
        out["per_algorithm_ms"] = s["per_algo_ms"]
        out["kernel_avg_ms"] = s["kernel_avg_ms"]
        out["kernel_breakdown_ms"] = s["breakdown"]
        out["walk_steps"] = s["walk"]
        out["walk_steps_note"] = ("RAM / AE speculation chunks by how each was "
                                  "decided (successor word, fast step from the "
                                  "tile summaries, run of one value, exact "
                                  "patterns) and tiles whose bytes the extreme "
                                  "byte search / range scan read, all passes")
        out["n_cuts"] = {a: int(c.size) for a, c in s["gpu_cuts"].items()}
        out["constant_blocks"] = constant_blocks_leg(args, binding, datagen, torch,
                                                     np, check)
    if "snap" in legs:
        out["snapshots"] = snapshot_leg(args, binding, datagen, torch, np, check)
    pool = None
    if "batch" in legs or "serve" in legs:
        binding.set_tuning()
        pool, host, offs, sizes, b = batch_leg(binding, datagen, torch, np)
        if "batch" in legs:
            out["batch"] = b
            if check:
                out["cpu_baseline_many_files"] = many_files_oracle(host, offs, sizes, np)
        del host
    if "serve" in legs:
        binding.set_tuning()
        out["serve"] = serve_leg(pool, binding, datagen, torch, np)
    if s is not None and check:
        log("oracle leg ...")
        out["cpu_baseline"], out["bit_exact_vs_oracle"], out["pattern_bytes"] = \
            cpu_baseline(s["x"], s["gpu_cuts"], np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
