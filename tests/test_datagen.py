"""The seeded input generators: determinism and the recipe's statistics."""
import hashlib

import numpy as np

from paper_2508_05797_amd import datagen


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_deterministic():
    assert _sha(datagen.uniform(1 << 16, 1)) == _sha(datagen.uniform(1 << 16, 1))
    assert _sha(datagen.uniform(1 << 16, 1)) != _sha(datagen.uniform(1 << 16, 2))
    a, ka = datagen.mixed_stream(64, 9)
    b, kb = datagen.mixed_stream(64, 9)
    assert _sha(a) == _sha(b) and (ka == kb).all()


def test_mixed_stream_composition():
    n_blocks = 16384
    rng = np.random.Generator(np.random.PCG64(0))
    kinds = datagen.mixed_block_kinds(n_blocks, rng)
    assert (kinds == 0).sum() == 8192
    assert (kinds == 1).sum() == 4915
    assert (kinds == 2).sum() == 3277


def test_mixed_stream_blocks():
    data, kinds = datagen.mixed_stream(40, 3)
    blocks = data.reshape(40, datagen.BLOCK)
    for b, k in zip(blocks, kinds):
        if k == 2:
            assert (b == b[0]).all()
        elif k == 1:
            assert np.isin(b, datagen.PRINTABLE).all()
        else:
            assert np.unique(b).size > 200


def test_zipf_frequencies():
    rng = np.random.Generator(np.random.PCG64(1))
    table = datagen.zipf_table(np.arange(64, dtype=np.uint8))
    draws = table[rng.integers(0, table.size, 2_000_000)]
    freq = np.bincount(draws, minlength=64) / draws.size
    p = datagen.zipf_probs()
    assert abs(p[0] - 0.2505) < 1e-3 and abs(p[-1] - 0.00258) < 1e-4
    assert np.allclose(freq, p, atol=4e-3 * np.sqrt(p) + 2e-4)


def test_lognormal_sizes():
    s = datagen.lognormal_sizes(20000, 5)
    assert s.min() >= 1024 and s.max() <= 256 << 20
    assert abs(np.median(s) / 65536 - 1) < 0.1
    assert 0.01 < (s == 1024).mean() < 0.03


def test_edit_version():
    rng = np.random.Generator(np.random.PCG64(2))
    base = np.frombuffer(rng.bytes(4096 * 500), np.uint8).copy()
    v = datagen.edit_version(base, rng)
    assert abs(v.size - base.size) <= 5 * 512
    # 1% of 500 regions = 5 edited regions; everything else is unchanged, so
    # the common prefix reaches at least the first edited region.
    same = np.flatnonzero(base[:min(v.size, base.size)] != v[:min(v.size, base.size)])
    assert same.size > 0 and v.size != base.size or same.size > 0
    versions = list(datagen.snapshot_versions(4096 * 300, 3, 4))
    assert len(versions) == 4


def test_constant_blocks():
    x = datagen.constant_blocks(40, 3, block=1000)
    assert x.size == 40000
    b = x.reshape(40, 1000)
    assert (b == b[:, :1]).all()
    assert len(set(b[:, 0].tolist())) > 20
    assert np.array_equal(x, datagen.constant_blocks(40, 3, block=1000))
