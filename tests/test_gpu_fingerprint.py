"""Chunk fingerprints and the distinct-chunk count on the device (GPU).

Every digest equals hashlib's SHA-256 of the same bytes, for chunks of every
length around the 64-byte block and its padding boundaries, at every base
alignment; over the backup-snapshot workload (a uniform base and 8 edited
versions) the device's distinct-chunk count and bytes equal those of the
oracle's cuts hashed on the host, for RAM, AE and MAXP.
"""
import hashlib

import numpy as np
import pytest
import torch

import oracle
from paper_2508_05797_amd import binding, datagen

pytestmark = pytest.mark.gpu

WIN8K = {"ram": 7936, "ae": 7936, "maxp": 444}
MAX_CHUNK = 65536


def say(*a):
    print(*a, flush=True)


def host_digests(x, cuts):
    out, start = [], 0
    mv = memoryview(x)
    for c in cuts.tolist():
        out.append(hashlib.sha256(mv[start:c]).digest())
        start = c
    return out


def test_digests_every_length_and_alignment():
    rng = np.random.default_rng(3)
    lens = list(range(0, 130)) + [183, 191, 192, 255, 256, 257, 1000, 4095,
                                  4096, 4097, 65535, 65536, 65537, 200001]
    for off in range(16):
        k = len(lens)
        seq = np.array(lens)[rng.permutation(k)]
        seq = seq[seq > 0]
        x = rng.integers(0, 256, int(seq.sum()) + off + 32).astype(np.uint8)
        d = torch.from_numpy(x).cuda()[off:off + int(seq.sum())]
        host = x[off:off + int(seq.sum())]
        cuts = np.cumsum(seq)
        say("case digests off=%d chunks=%d" % (off, cuts.size))
        got = binding.fingerprint(d, torch.from_numpy(cuts.astype(np.int64)).cuda())
        got = got.cpu().numpy()
        exp = host_digests(host, cuts)
        for i, e in enumerate(exp):
            assert bytes(got[i]) == e, (off, i, int(seq[i]))
    # all-0xFF bytes, with chunks ending at the padding boundaries
    x = np.full(300, 255, np.uint8)
    d = torch.from_numpy(x).cuda()
    got = binding.fingerprint(d, torch.tensor([1, 56, 120, 300], dtype=torch.int64,
                                              device="cuda")).cpu().numpy()
    assert [bytes(r) for r in got] == host_digests(x, np.array([1, 56, 120, 300]))


def run_versions(base_size, seed, algos):
    dd = {a: binding.Dedup(4 * base_size // 4096 + 1000) for a in algos}
    host_seen = {a: {} for a in algos}
    host_tot = {a: 0 for a in algos}
    for v, x in enumerate(datagen.snapshot_versions(base_size, 8, seed)):
        d = torch.from_numpy(x).cuda()
        for a in algos:
            w = WIN8K[a]
            cuts = torch.empty(binding.max_cuts(x.size, w), dtype=torch.int64,
                               device="cuda")
            nc = torch.empty(1, dtype=torch.int64, device="cuda")
            binding.chunk_into(d, a, w, MAX_CHUNK, cuts, nc)
            dg = torch.empty((cuts.numel(), 32), dtype=torch.uint8, device="cuda")
            binding.fingerprint_into(d, cuts, nc, dg)
            dd[a].add(dg, cuts, nc)
            k = int(nc.item())
            exp_cuts = oracle.chunk(a, x, w, MAX_CHUNK)
            assert np.array_equal(cuts[:k].cpu().numpy().astype(np.uint64), exp_cuts)
            exp = host_digests(x, exp_cuts)
            got = dg[:k].cpu().numpy()
            for i, e in enumerate(exp):
                assert bytes(got[i]) == e, (v, a, i)
            start = 0
            for c, e in zip(exp_cuts.tolist(), exp):
                host_seen[a].setdefault((e, c - start), c - start)
                host_tot[a] += c - start
                start = c
        say("version", v, x.size)
        del d
    out = {}
    for a in algos:
        st = dd[a].stats()
        uniq = sum(host_seen[a].values())
        assert st["flags"] == 0 and st["collisions"] == 0, st
        assert st["total_bytes"] == host_tot[a], (a, st)
        assert st["unique_chunks"] == len(host_seen[a]), (a, st)
        assert st["unique_bytes"] == uniq, (a, st, uniq)
        out[a] = st["total_bytes"] / st["unique_bytes"]
        dd[a].close()
    return out


def test_snapshot_dedup_16mib():
    ratios = run_versions(16 << 20, 81, ["ram", "ae", "maxp"])
    say("dedup ratios", ratios)
    for a, r in ratios.items():
        assert 2.0 < r < 9.0, (a, r)


def test_dedup_table_counts_repeats_within_and_across_lists():
    """The same list added twice, and a list with repeated chunks: every
    chunk after its first copy is a duplicate; reset empties the table."""
    x = np.concatenate([np.full(5000, 7, np.uint8)] * 3 +
                       [np.arange(256, dtype=np.uint8)] * 4)
    d = torch.from_numpy(x).cuda()
    cuts = torch.tensor([5000, 10000, 15000, 15256, 15512, 15768, 16024],
                        dtype=torch.int64, device="cuda")
    nc = torch.tensor([7], dtype=torch.int64, device="cuda")
    dg = torch.empty((7, 32), dtype=torch.uint8, device="cuda")
    binding.fingerprint_into(d, cuts, nc, dg)
    t = binding.Dedup(100)
    t.add(dg, cuts, nc)
    st = t.stats()
    assert st["unique_chunks"] == 2 and st["unique_bytes"] == 5256
    assert st["chunks"] == 7 and st["total_bytes"] == 16024
    t.add(dg, cuts, nc)
    st = t.stats()
    assert st["unique_chunks"] == 2 and st["total_bytes"] == 2 * 16024
    t.reset()
    t.add(dg[:1], cuts[:1], torch.tensor([1], dtype=torch.int64, device="cuda"))
    assert t.stats()["unique_bytes"] == 5000
    t.close()
