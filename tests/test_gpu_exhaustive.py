"""Every short string through the device path (GPU), element by element
against the oracle.

All strings of length 0..8 over the bytes {00, 7F, 80, FF} (87,381 strings;
the two middle values sit on either side of the signed-byte boundary, so a
signed compare anywhere changes some cut), under every window w in {1, 2, 3}
and maximum chunk M in {w+1, w+2, 2w+2, 16}: windows that fit inside the
tiny inputs, forced cuts, and the end-of-buffer rules of each chunker.  Each
(w, M) runs all four chunkers as one batch of 349,524 jobs; a seeded sample
also runs through single cdc_chunk calls at unaligned addresses.
"""
import itertools

import numpy as np
import pytest
import torch

import oracle
from paper_2508_05797_amd import binding

pytestmark = pytest.mark.gpu

ALGOS = ["ram", "ae", "maxp", "ae_min"]
SYMBOLS = np.array([0x00, 0x7F, 0x80, 0xFF], np.uint8)
MAX_LEN = 8


def say(*a):
    print(*a, flush=True)


def all_strings():
    """The strings packed back to back: (bytes, offsets, lengths)."""
    parts, offs, lens = [], [], []
    pos = 0
    for L in range(MAX_LEN + 1):
        k = 4 ** L
        digits = (np.arange(k)[:, None] // (4 ** np.arange(L))[None, :]) % 4
        s = SYMBOLS[digits].reshape(-1)
        parts.append(s)
        offs.append(pos + L * np.arange(k))
        lens.append(np.full(k, L))
        pos += k * L
    return (np.concatenate(parts).astype(np.uint8),
            np.concatenate(offs).astype(np.int64),
            np.concatenate(lens).astype(np.int64))


PARAMS = [(w, M) for w in (1, 2, 3) for M in sorted({w + 1, w + 2, 2 * w + 2, 16})]


@pytest.fixture(scope="module")
def strings():
    assert torch.cuda.is_available()
    binding.lib()
    x, offs, lens = all_strings()
    assert lens.size == (4 ** (MAX_LEN + 1) - 1) // 3
    # the bytes at an odd address, so every string starts unaligned somewhere
    d = torch.zeros(x.size + 64, dtype=torch.uint8, device="cuda")
    d[3:3 + x.size] = torch.from_numpy(x).cuda()
    yield x, offs, lens, d[3:3 + x.size]
    assert binding.device_errors() == 0


@pytest.mark.parametrize("w,M", PARAMS)
def test_all_strings_batched(strings, w, M):
    x, offs, lens, d = strings
    k = lens.size
    algos = [a for a in ALGOS for _ in range(k)]
    b = binding.Batch(d, np.tile(offs, 4), np.tile(lens, 4), algos, w, M)
    say("case exhaustive batch w=%d M=%d jobs=%d" % (w, M, b.n_jobs))
    b.run()
    torch.cuda.synchronize()
    st = b.statuses()
    assert (st == 0).all(), np.unique(st)
    nc = b.n_cuts.cpu().numpy()
    cuts = b.cuts.cpu().numpy().astype(np.uint64)
    for i, a in enumerate(ALGOS):
        base = b.cut_base[i * k:(i + 1) * k]
        exp, _b, cnt = oracle.chunk_many(a, x, offs, lens, w, M,
                                         base=base - base[0])
        got_n = nc[i * k:(i + 1) * k]
        bad = np.nonzero(got_n != cnt)[0]
        assert bad.size == 0, (a, w, M, "count differs for strings", bad[:5])
        # every cut slot that holds a cut, compared at once
        idx = np.repeat(base - base[0], cnt) + (
            np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt))
        got = cuts[int(base[0]):][idx.astype(np.int64)]
        want = exp[idx.astype(np.int64)]
        diff = np.nonzero(got != want)[0]
        assert diff.size == 0, (a, w, M, "cut differs at slot", idx[diff[:5]])


def test_sample_single_calls(strings):
    x, offs, lens, d = strings
    rng = np.random.default_rng(17)
    picks = rng.choice(lens.size, 300, replace=False)
    for j, (w, M), a in zip(picks, itertools.cycle(PARAMS), itertools.cycle(ALGOS)):
        o, n = int(offs[j]), int(lens[j])
        got = binding.chunk(d[o:o + n], a, w, M).cpu().numpy().astype(np.uint64)
        exp = oracle.chunk(a, x[o:o + n], w, M)
        assert np.array_equal(got, exp), (a, w, M, x[o:o + n])
