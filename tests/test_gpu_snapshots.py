"""Backup-snapshot workload (GPU): a uniform random base and 8 successive
versions, each editing 1% of its 4 KiB regions by an insert, delete or
overwrite of 1..512 random bytes.  Every version is chunked on the GPU and
by the oracle with windows that give about 8 KiB average chunks; the cuts
are identical, and so is the dedup ratio (total bytes over the bytes of
distinct chunk contents) over all versions."""
import hashlib
import threading

import numpy as np
import pytest
import torch

import oracle
from paper_2508_05797_amd import binding, datagen

pytestmark = pytest.mark.gpu

# windows that give ~8 KiB average chunks on uniform random bytes
WIN8K = {"ram": 7936, "ae": 7936, "maxp": 444, "ae_min": 7936}
MAX_CHUNK = 65536


def say(*a):
    print(*a, flush=True)


class Dedup:
    """Distinct chunk contents, keyed by a 128-bit BLAKE2b digest."""

    def __init__(self):
        self.seen = set()
        self.total = 0
        self.unique = 0

    def add(self, data, cuts):
        mv = memoryview(data)
        start = 0
        for c in cuts.tolist():
            key = hashlib.blake2b(mv[start:c], digest_size=16).digest()
            if key not in self.seen:
                self.seen.add(key)
                self.unique += c - start
            self.total += c - start
            start = c

    @property
    def ratio(self):
        return self.total / max(self.unique, 1)


def run_snapshots(base_size, algos, seed):
    gpu = {a: Dedup() for a in algos}
    cpu = {a: Dedup() for a in algos}
    for v, x in enumerate(datagen.snapshot_versions(base_size, 8, seed)):
        d = torch.from_numpy(x).cuda()
        got = {a: binding.chunk(d, a, WIN8K[a], MAX_CHUNK).cpu().numpy().astype(np.uint64)
               for a in algos}
        exp = {}

        def work(a):
            exp[a] = oracle.chunk(a, x, WIN8K[a], MAX_CHUNK)
        th = [threading.Thread(target=work, args=(a,)) for a in algos]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for a in algos:
            assert np.array_equal(got[a], exp[a]), (v, a)
            gpu[a].add(x, got[a])
            cpu[a].add(x, exp[a])
        say("version", v, x.size, {a: got[a].size for a in algos})
        del d
    for a in algos:
        assert gpu[a].ratio == cpu[a].ratio
        assert gpu[a].total == cpu[a].total
    return {a: gpu[a].ratio for a in algos}


def test_snapshots_small():
    ratios = run_snapshots(16 << 20, ["ram", "ae", "maxp", "ae_min"], 81)
    say("dedup", ratios)
    for a, r in ratios.items():
        # 9 versions differing in ~1% of regions: many chunks repeat (RAM
        # and AE resynchronise slowly after a shift on uniform bytes)
        assert 2.0 < r < 9.0, (a, r)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_snapshots_512mib():
    ratios = run_snapshots(512 << 20, ["ram", "ae", "maxp"], 2025)
    say("dedup", ratios)
    for a, r in ratios.items():
        assert 2.0 < r < 9.0, (a, r)
