"""Resumable chunking of a stream pushed in pieces (GPU).

The offsets every push returns, concatenated, equal one cdc_chunk call over
the whole stream and the oracle, for all four chunkers: on the 1 GiB mixed
stream in seeded random pieces (1 byte to 64 MiB), and on a 16 MiB stream in
pieces smaller than a window, around the maximum chunk and mixed; each push
returns only cuts that later bytes cannot move, so the concatenation also
checks the prefix property of the definitions.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_05797_amd import binding, datagen

pytestmark = pytest.mark.gpu

W = {"ram": 4096, "ae": 4096, "maxp": 2048, "ae_min": 4096}
M = 65536


def say(*a):
    print(*a, flush=True)


def pieces(n, rng, lo, hi):
    out, pos = [], 0
    while pos < n:
        k = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        k = max(1, min(k, n - pos))
        out.append((pos, k))
        pos += k
    return out


def run_stream(d, algo, w, m, cuts_of, max_piece, last_empty=False):
    s = binding.Stream(algo, w, m, max_piece)
    got = []
    for i, (o, k) in enumerate(cuts_of):
        last = (i == len(cuts_of) - 1) and not last_empty
        got.append(s.push(d[o:o + k], last=last))
    if last_empty:
        got.append(s.push(d[:0], last=True))
    s.close()
    return torch.cat(got).cpu().numpy().astype(np.uint64)


@pytest.mark.parametrize("algo", ["ram", "ae", "maxp", "ae_min"])
def test_stream_small_pieces(algo):
    x, _ = datagen.mixed_stream(256, 61)
    x[5 << 20:(5 << 20) + 400000] = 33
    d = torch.from_numpy(x).cuda()
    rng = np.random.default_rng(62)
    w = W[algo] if algo != "ae_min" else 300
    exp = oracle.chunk(algo, x, w, M)
    for lo, hi, tag in ((1, 3000, "tiny"), (2000, 200000, "around M"),
                        (1, 4 << 20, "mixed")):
        cuts_of = pieces(x.size if tag != "tiny" else 2 << 20, rng, lo, hi)
        n = cuts_of[-1][0] + cuts_of[-1][1]
        e = exp if n == x.size else oracle.chunk(algo, x[:n], w, M)
        say("case stream", algo, tag, len(cuts_of), "pieces", n)
        got = run_stream(d, algo, w, M, cuts_of, max(k for _, k in cuts_of),
                         last_empty=(tag == "mixed"))
        assert got.size == e.size and np.array_equal(got, e), (algo, tag)


@pytest.mark.parametrize("algo", ["ram", "ae", "maxp", "ae_min"])
def test_stream_small_window_and_forced(algo):
    """Windows of 1..3 and max chunk w + 1 (every chunk forced), in pieces
    of 1..40 bytes."""
    rng = np.random.default_rng(63)
    x = rng.choice(np.array([0, 0x7F, 0x80, 0xFF], np.uint8), 20000)
    d = torch.from_numpy(x).cuda()
    for w, m in ((1, 2), (2, 6), (3, 16)):
        cuts_of = pieces(x.size, rng, 1, 40)
        say("case stream small", algo, w, m, len(cuts_of))
        got = run_stream(d, algo, w, m, cuts_of, 40)
        e = oracle.chunk(algo, x, w, m)
        assert np.array_equal(got, e), (algo, w, m)


@pytest.mark.slow
@pytest.mark.parametrize("algo", ["ram", "ae", "maxp", "ae_min"])
def test_stream_1gib(algo):
    x, _ = datagen.mixed_stream(16384, 2024)
    d = torch.from_numpy(x).cuda()
    rng = np.random.default_rng(64)
    cuts_of = pieces(x.size, rng, 1, 64 << 20)
    say("case stream 1 GiB", algo, len(cuts_of), "pieces")
    w = W[algo]
    got = run_stream(d, algo, w, M, cuts_of, 64 << 20)
    one = binding.chunk(d, algo, w, M).cpu().numpy().astype(np.uint64)
    assert np.array_equal(got, one), algo
    assert np.array_equal(got, oracle.chunk(algo, x, w, M)), algo
    del d
    torch.cuda.empty_cache()


def test_stream_refusals():
    s = binding.Stream("ram", 100, 1000, 4096)
    d = torch.zeros(8192, dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.CdcError):
        s.push(d)                          # longer than max_piece
    s.push(d[:4096], last=True)
    with pytest.raises(binding.CdcError):
        s.push(d[:10])                     # the stream has ended
    s.reset()
    got = s.push(d[:3000], last=True).cpu().numpy()
    assert got.tolist() == oracle.chunk("ram", np.zeros(3000, np.uint8), 100, 1000).tolist()
    s.close()
