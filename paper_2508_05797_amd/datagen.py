"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws bytes and sizes; it holds no chunking arithmetic, and
both the oracle-side tests and the GPU path consume exactly what it returns.
All generators use numpy's PCG64 with an explicit seed, so a given
(recipe, seed) always yields the same bytes.

Recipes (the paper's datasets are not available; these stand in for them):

* ``uniform(n, seed)``: i.i.d. uniform bytes (compressed payloads).
* ``mixed_stream(n_blocks, seed)``: 64 KiB blocks, exactly 50% uniform random,
  30% Zipf(s=1.1) over 64 printable symbols (text / source code), 20%
  constant-byte runs (zero-filled VM and database regions), in a seeded
  shuffled order.  The rank-to-byte map of the Zipf symbols is a seeded
  permutation of space, newline, 0-9, A-Z, a-z.
* ``snapshot_versions(...)``: a uniform random base plus successive versions,
  each editing 1% of its 4 KiB regions by insert / delete / overwrite of 1-512
  random bytes (nightly backups, web and database snapshots).
* ``lognormal_sizes(...)``: file sizes for many-file sets (source trees).
* ``constant_blocks(n_blocks, seed)``: 64 KiB blocks each of one byte value,
  the value changing from block to block (zero-filled and padded regions of
  VM images and databases back to back; RAM chains never meet inside such
  runs, the hardest case for the segment-parallel resolution).
"""
import numpy as np

BLOCK = 65536
ZIPF_S = 1.1
ZIPF_K = 64
PRINTABLE = np.frombuffer(
    b" \n0123456789ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz",
    dtype=np.uint8)
assert PRINTABLE.size == ZIPF_K

# The Zipf sampler draws a 20-bit uniform index into this many table slots.
_ZIPF_TABLE_BITS = 20


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform(n, seed):
    """n i.i.d. uniform bytes."""
    rng = _rng(seed)
    return np.frombuffer(rng.bytes(n), dtype=np.uint8).copy()


def zipf_probs(k=ZIPF_K, s=ZIPF_S):
    p = np.arange(1, k + 1, dtype=np.float64) ** (-s)
    return p / p.sum()


def zipf_table(symbols, k=ZIPF_K, s=ZIPF_S, bits=_ZIPF_TABLE_BITS):
    """A 2**bits-entry lookup table whose slot counts follow Zipf(s); a uniform
    slot index then samples a symbol (probabilities quantised to 2**-bits)."""
    size = 1 << bits
    counts = np.floor(zipf_probs(k, s) * size).astype(np.int64)
    counts[0] += size - counts.sum()
    return np.repeat(symbols, counts).astype(np.uint8)


def mixed_block_kinds(n_blocks, rng):
    n_rand = int(round(0.5 * n_blocks))
    n_zipf = int(round(0.3 * n_blocks))
    n_const = n_blocks - n_rand - n_zipf
    kinds = np.array([0] * n_rand + [1] * n_zipf + [2] * n_const, np.int8)
    rng.shuffle(kinds)
    return kinds


def mixed_stream(n_blocks, seed, block=BLOCK):
    """n_blocks blocks of ``block`` bytes: 50% uniform, 30% Zipf, 20% constant.

    Returns (data, kinds) where kinds[i] is 0 (uniform), 1 (Zipf) or
    2 (constant) for block i."""
    rng = _rng(seed)
    kinds = mixed_block_kinds(n_blocks, rng)
    symbols = PRINTABLE[rng.permutation(ZIPF_K)]
    table = zipf_table(symbols)
    const_vals = rng.integers(0, 256, n_blocks, dtype=np.uint8)
    out = np.empty(n_blocks * block, dtype=np.uint8)
    mask = (1 << _ZIPF_TABLE_BITS) - 1
    for b in range(n_blocks):
        dst = out[b * block:(b + 1) * block]
        if kinds[b] == 0:
            dst[:] = np.frombuffer(rng.bytes(block), dtype=np.uint8)
        elif kinds[b] == 1:
            idx = rng.integers(0, 1 << 32, block, dtype=np.uint32) & mask
            dst[:] = table[idx]
        else:
            dst[:] = const_vals[b]
    return out, kinds


def edit_version(prev, rng, region=4096, frac=0.01, max_len=512):
    """One new version of ``prev``: round(frac * R) distinct regions of
    ``region`` bytes (R = len // region) each get one edit, with operation
    uniform over insert / delete / overwrite, length uniform in [1, max_len]
    and offset uniform in the region.  Each edit is clipped to its own region,
    so edits never overlap and their order does not matter."""
    n = prev.size
    R = n // region
    k = int(round(frac * R))
    if k == 0:
        return prev.copy()
    regions = np.sort(rng.choice(R, size=k, replace=False))
    ops = rng.integers(0, 3, k)
    lens = rng.integers(1, max_len + 1, k)
    offs = regions * region + rng.integers(0, region, k)
    pieces = []
    pos = 0
    for r, op, ln, off in zip(regions, ops, lens, offs):
        end_region = (int(r) + 1) * region
        ln = int(min(ln, end_region - off)) if op != 0 else int(ln)
        pieces.append(prev[pos:off])
        if op == 0:                      # insert ln random bytes before off
            pieces.append(np.frombuffer(rng.bytes(ln), dtype=np.uint8))
            pos = off
        elif op == 1:                    # delete ln bytes at off
            pos = off + ln
        else:                            # overwrite ln bytes at off
            pieces.append(np.frombuffer(rng.bytes(ln), dtype=np.uint8))
            pos = off + ln
    pieces.append(prev[pos:])
    return np.concatenate(pieces)


def snapshot_versions(base_size, n_versions, seed, **edit_kw):
    """Yield the base (uniform random) and then n_versions edited versions."""
    rng = _rng(seed)
    cur = np.frombuffer(rng.bytes(base_size), dtype=np.uint8).copy()
    yield cur
    for _ in range(n_versions):
        cur = edit_version(cur, rng, **edit_kw)
        yield cur


def lognormal_sizes(n_files, seed, median=65536, sigma=2.0, lo=1024,
                    hi=256 << 20):
    """File sizes round(exp(N(ln median, sigma))) clipped to [lo, hi]."""
    rng = _rng(seed)
    z = rng.normal(np.log(median), sigma, n_files)
    return np.clip(np.round(np.exp(z)), lo, hi).astype(np.int64)


def many_files(sizes, seed):
    """One uniform random byte string per size, as a single contiguous buffer
    plus the start offset of each file."""
    sizes = np.asarray(sizes, dtype=np.int64)
    offs = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    return uniform(int(offs[-1]), seed), offs


def constant_blocks(n_blocks, seed, block=BLOCK):
    """n_blocks blocks of ``block`` bytes, each a run of one uniformly drawn
    byte value."""
    rng = _rng(seed)
    vals = rng.integers(0, 256, n_blocks, dtype=np.uint8)
    return np.repeat(vals, block)
