"""Benchmark: chunk-boundary finding on the 1 GiB mixed stream (MI355X).

One step chunks the 1 GiB stream of 64 KiB blocks (50% uniform random, 30%
Zipf text, 20% constant runs) with RAM (w=4096), AE-Max (w=4096) and MAXP
(w=2048 each side), max chunk 64 KiB: the whole hot path, three times over
the same resident bytes.  ``value`` is bytes chunked per second over the
timed steps (GB = 1e9 B); the inputs are in HBM before timing starts.

Also reported:
  * roofline: the dominant kernel's algorithmic bytes (the stream, read once)
    over its average duration from HIP events on the launch stream, against
    the 8 TB/s HBM peak; traffic from rocprofv3 FETCH_SIZE / WRITE_SIZE
    counters when they were taken on the current kernel source;
  * cpu_baseline: the scalar oracle on this host, single thread, on the same
    stream (whose cuts also check the GPU's, bit for bit);
  * per-algorithm GB/s.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("GB/s chunked, bit-exact cuts, batched vs plain, % HBM peak; "
          "serve p99 ms")
HBM_PEAK_GBS = 8000.0
STREAM_BLOCKS = 16384          # 16384 x 64 KiB = 1 GiB
STREAM_SEED = 2024
ALGOS = [("ram", 4096), ("ae", 4096), ("maxp", 2048)]
MAX_CHUNK = 65536
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2508_05797_amd", "csrc",
                          "chain_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


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


def cpu_baseline(x, gpu_cuts):
    import numpy as np
    import oracle
    total_t, exact = 0.0, True
    for algo, w in ALGOS:
        t0 = time.perf_counter()
        c = oracle.chunk(algo, x, w, MAX_CHUNK)
        total_t += time.perf_counter() - t0
        g = gpu_cuts[algo]
        same = (g.size == c.size) and bool(np.array_equal(g, c))
        log("oracle %s: %d cuts, gpu %d cuts, identical=%s"
            % (algo, c.size, g.size, same))
        exact = exact and same
    gbs = len(ALGOS) * x.size / total_t / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": "the full 1 GiB stream, each of RAM, AE, MAXP once, "
                      "single-threaded scalar C (gcc -O2)"}, exact


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seg", type=int, default=0,
                    help="segment length in bytes (0: the library's choice)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle leg (no cpu_baseline, no check)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build runs on a single MI355X "
              "and has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2508_05797_amd import binding, datagen
    from paper_2508_05797_amd import build as cdc_build

    if not os.path.exists(binding.LIB_PATH):
        cdc_build.build()
    binding.lib()
    binding.set_tuning(args.seg, 0)

    log("generating the 1 GiB mixed stream ...")
    x, _ = datagen.mixed_stream(STREAM_BLOCKS, STREAM_SEED)
    n = x.size
    dev = torch.device("cuda:0")
    d = torch.from_numpy(x).to(dev)
    stream = torch.cuda.current_stream()
    bufs = {}
    for algo, w in ALGOS:
        bufs[algo] = (torch.empty(binding.max_cuts(n, w), dtype=torch.int64,
                                  device=dev),
                      torch.empty(1, dtype=torch.int64, device=dev))

    def step(only=None):
        for algo, w in ALGOS:
            if only and algo != only:
                continue
            cuts, nc = bufs[algo]
            binding.chunk_into(d, algo, w, MAX_CHUNK, cuts, nc)

    log("warmup ...")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Timed region: K steps; HIP events around each call's main kernel.
    binding.set_profiling(1)
    binding.kernel_times()                      # clear earlier records
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    ms_total = t0.elapsed_time(t1)
    ktimes = binding.kernel_times()
    binding.set_profiling(0)
    ms_step = ms_total / args.steps
    value = len(ALGOS) * n / (ms_step * 1e-3) / 1e9

    # Per-algorithm throughput (separate short runs of each algorithm), then
    # one traced run per algorithm for the per-kernel breakdown.
    per_algo, breakdown = {}, {}
    for algo, _w in ALGOS:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            step(algo)
        e1.record()
        torch.cuda.synchronize()
        per_algo[algo] = round(n / (e0.elapsed_time(e1) / args.steps * 1e-3)
                               / 1e9, 2)
        binding.set_profiling(2)
        step(algo)
        breakdown[algo] = {k: round(v[1] / max(v[0], 1), 4)
                           for k, v in binding.kernel_times().items()}
        binding.set_profiling(0)

    # Roofline of the dominant kernel: the stream's bytes per launch over
    # the launch's average duration.
    per_kernel = {k: tot / max(c, 1) for k, (c, tot) in ktimes.items()}
    dom = max(per_kernel, key=per_kernel.get)
    avg_ms = per_kernel[dom]
    achieved = n / (avg_ms * 1e-3) / 1e9
    traffic = load_traffic()
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_bytes_per_launch": n,
            "traffic": (traffic or {}).get("bytes_per_launch", {}).get(dom)}

    gpu_cuts = {}
    for algo, _w in ALGOS:
        cuts, nc = bufs[algo]
        gpu_cuts[algo] = cuts[:int(nc.item())].cpu().numpy().astype(np.uint64)
    assert binding.device_errors() == 0

    cpu, exact = (None, None)
    if not args.no_cpu:
        log("oracle leg ...")
        cpu, exact = cpu_baseline(x, gpu_cuts)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "1 GiB stream of 64 KiB blocks: 50% uniform, "
                               "30% Zipf(1.1) text over 64 symbols, 20% "
                               "constant runs; RAM w=4096, AE w=4096, MAXP "
                               "w=2048, max chunk 64 KiB",
                   "bytes": n, "algorithms": [a for a, _ in ALGOS],
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "bit_exact_vs_oracle": exact,
        "per_algorithm_gbs": per_algo,
        "kernel_avg_ms": {k: round(v, 4) for k, v in per_kernel.items()},
        "kernel_breakdown_ms": breakdown,
        "n_cuts": {a: int(c.size) for a, c in gpu_cuts.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
