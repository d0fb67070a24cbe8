"""Pins for the scalar CPU oracle (no GPU).

The oracle is checked against things other than itself:
  * worked examples derived by hand from the paper's prose (tests/golden);
  * closed forms for inputs whose chunking follows from the definitions;
  * textbook reductions built on library routines (numpy max / search,
    a monotonic-stack next-greater element, numpy sliding-window maxima);
  * exhaustive brute force over all short strings of a signed-trap alphabet;
  * invariants: tiling, chunk-length bounds, prefix property, the AE-Min /
    AE-Max complement identity, and edit locality.
"""
import itertools

import numpy as np
import pytest
from numpy.lib.stride_tricks import sliding_window_view

import oracle
from tests.golden.load import all_cases

ALGOS = ["ram", "ae", "maxp", "ae_min"]


# ---------------------------------------------------------------- golden

@pytest.mark.parametrize("case", all_cases(), ids=lambda c: c["name"])
def test_golden_worked_examples(case):
    got = oracle.chunk(case["algo"], case["data"], case["w"], case["M"])
    assert got.tolist() == case["cuts"]


# ---------------------------------------------------------- closed forms

def _arith(n, step):
    return list(range(step, n, step)) + [n] if n else []


@pytest.mark.parametrize("n", [0, 1, 5, 4097, 4098, 20000, 65536 * 3 + 7])
@pytest.mark.parametrize("val", [0, 0x7F, 0x80, 0xFF])
def test_constant_input(n, val):
    x = np.full(n, val, np.uint8)
    w, M = 4096, 65536
    lockstep = _arith(n, w + 1)
    assert oracle.chunk("ram", x, w, M).tolist() == lockstep
    assert oracle.chunk("ae", x, w, M).tolist() == lockstep
    assert oracle.chunk("ae_min", x, w, M).tolist() == lockstep
    assert oracle.chunk("maxp", x, 2048, M).tolist() == _arith(n, M)


@pytest.mark.parametrize("w,M", [(1, 2), (3, 7), (10, 11), (10, 40), (50, 64)])
def test_monotone_inputs(w, M):
    n = 256
    inc = np.arange(n, dtype=np.uint8)
    dec = inc[::-1].copy()
    # increasing: RAM's scan byte always beats its window, AE-Min's first byte
    # is its minimum; AE-Max keeps finding new targets; no strict local max.
    assert oracle.chunk("ram", inc, w, M).tolist() == _arith(n, w + 1)
    assert oracle.chunk("ae_min", inc, w, M).tolist() == _arith(n, w + 1)
    assert oracle.chunk("ae", inc, w, M).tolist() == _arith(n, M)
    assert oracle.chunk("maxp", inc, w, M).tolist() == _arith(n, M)
    # decreasing: the mirror image.
    assert oracle.chunk("ram", dec, w, M).tolist() == _arith(n, M)
    assert oracle.chunk("ae", dec, w, M).tolist() == _arith(n, w + 1)
    assert oracle.chunk("ae_min", dec, w, M).tolist() == _arith(n, M)
    assert oracle.chunk("maxp", dec, w, M).tolist() == _arith(n, M)


@pytest.mark.parametrize("seed", range(5))
def test_maxp_isolated_spikes(seed):
    """Zeros with 255-spikes spaced in (w, M]: every spike whose right window
    fits is a strict local maximum, and each ends a chunk right after it."""
    rng = np.random.default_rng(seed)
    w, M = 64, 1000
    gaps = rng.integers(w + 1, M + 1, 40)
    spikes = w + rng.integers(0, M - w) + np.concatenate([[0], np.cumsum(gaps)])
    n = int(spikes[-1]) + int(rng.integers(0, 2 * w))
    x = np.zeros(n, np.uint8)
    spikes = spikes[spikes < n]
    x[spikes] = 255
    cands = [int(q) for q in spikes if q + w <= n - 1]
    expect = [q + 1 for q in cands]
    s = expect[-1] if expect else 0
    expect += [s + c for c in _arith(n - s, M)]
    assert oracle.chunk("maxp", x, w, M).tolist() == expect


def test_ae_spikes_closed_form():
    """Zeros with 255-spikes: a chunk from s is w+1 bytes unless a spike q is
    among its bytes s..s+w, in which case it ends at q+w+1."""
    w, M = 16, 200
    x = np.zeros(3000, np.uint8)
    spikes = [40, 41, 100, 300, 317, 900, 1500, 2990]
    x[spikes] = 255
    n = x.size
    expect, s = [], 0
    while s < n:
        L = min(n, s + M)
        hit = [q for q in spikes if s <= q <= s + w]
        q = hit[0] if hit else s
        c = q + w + 1 if q + w + 1 <= L else L
        expect.append(c)
        s = c
    assert oracle.chunk("ae", x, w, M).tolist() == expect


# ------------------------------------------------------ textbook twins

def ram_twin(x, w, M):
    """numpy max over the window, then the first index of (scan >= T)."""
    n, s, out = x.size, 0, []
    while s < n:
        L = min(n, s + M)
        if s + w >= L:
            c = L
        else:
            T = x[s:s + w].max()
            hits = np.flatnonzero(x[s + w:L] >= T)
            c = s + w + int(hits[0]) + 1 if hits.size else L
        out.append(c)
        s = c
    return out


def next_greater(x, greater=True):
    """G[p] = first j > p with x[j] > x[p] (monotonic stack), else -1."""
    G = np.full(x.size, -1, np.int64)
    stack = []
    v = x.astype(np.int64) if greater else -x.astype(np.int64)
    for j in range(x.size):
        while stack and v[j] > v[stack[-1]]:
            G[stack.pop()] = j
        stack.append(j)
    return G


def ae_twin(x, w, M, greater=True):
    """The chain of strict records: from a target p, jump to its next-greater
    element if it lies within the window, else cut after the window."""
    G = next_greater(x, greater)
    n, s, out = x.size, 0, []
    while s < n:
        L = min(n, s + M)
        p = s
        while True:
            g = int(G[p])
            if g != -1 and g <= p + w:
                if g < L:
                    p = g
                    continue
                c = L
            else:
                c = p + w + 1 if p + w + 1 <= L else L
            break
        out.append(c)
        s = c
    return out


def maxp_candidates(x, w):
    """P[i]: x[i] above the max of x[i-w..i-1] and of x[i+1..i+w], from
    numpy sliding-window maxima."""
    n = x.size
    P = np.zeros(n, bool)
    if n < 2 * w + 1:
        return P
    win = sliding_window_view(x, w).max(axis=1)      # win[j] = max x[j..j+w)
    i = np.arange(w, n - w)
    P[i] = (x[i] > win[i - w]) & (x[i] > win[i + 1])
    return P


def maxp_twin(x, w, M):
    P = np.flatnonzero(maxp_candidates(x, w))
    n, s, out = x.size, 0, []
    while s < n:
        L = min(n, s + M)
        k = np.searchsorted(P, s + w)
        c = int(P[k]) + 1 if k < P.size and P[k] < L else L
        out.append(c)
        s = c
    return out


def twin(algo, x, w, M):
    if algo == "ram":
        return ram_twin(x, w, M)
    if algo == "ae":
        return ae_twin(x, w, M, True)
    if algo == "ae_min":
        return ae_twin(x, w, M, False)
    return maxp_twin(x, w, M)


def test_exhaustive_short_strings():
    """Every string of length 0..6 over {00, 7F, 80, FF} (the alphabet that
    exposes a signed compare), for several (w, M), all chunkers."""
    alphabet = [0x00, 0x7F, 0x80, 0xFF]
    params = [(1, 2), (1, 3), (2, 3), (2, 4), (2, 6), (3, 4), (3, 8)]
    checked = 0
    for length in range(0, 7):
        for tup in itertools.product(alphabet, repeat=length):
            x = np.array(tup, np.uint8)
            for w, M in params:
                for algo in ALGOS:
                    assert oracle.chunk(algo, x, w, M).tolist() == \
                        twin(algo, x, w, M), (algo, tup, w, M)
                    checked += 1
    assert checked == 5461 * len(params) * len(ALGOS)


def _inputs(seed, n):
    rng = np.random.default_rng(seed)
    kinds = {
        "uniform": rng.integers(0, 256, n).astype(np.uint8),
        "small_alpha": rng.choice([0, 1, 127, 128, 254, 255], n).astype(np.uint8),
        "zipf_text": rng.choice(np.frombuffer(b"etaoin shrdlu\n", np.uint8), n),
        "runs": np.repeat(rng.integers(0, 256, n // 50 + 1), 50)[:n].astype(np.uint8),
        "sawtooth": (np.arange(n) % 37).astype(np.uint8),
    }
    return kinds


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("w,M", [(1, 2), (5, 9), (16, 64), (40, 41), (100, 1000)])
def test_twins_random(seed, w, M):
    for name, x in _inputs(seed, 6000).items():
        for algo in ALGOS:
            assert oracle.chunk(algo, x, w, M).tolist() == twin(algo, x, w, M), \
                (name, algo, w, M)


# ------------------------------------------------------------ invariants

def _check_tiling(cuts, n, w, M):
    if n == 0:
        assert cuts.size == 0
        return
    assert cuts[-1] == n
    lens = np.diff(np.concatenate([[0], cuts.astype(np.int64)]))
    assert (lens >= 1).all() and (lens <= M).all()
    assert (lens[:-1] >= w + 1).all()
    assert cuts.size <= oracle.max_cuts(n, w)


@pytest.mark.parametrize("algo", ALGOS)
def test_invariants_tiling_and_prefix(algo):
    rng = np.random.default_rng(7)
    w, M = (48, 700)
    x = rng.integers(0, 256, 50000).astype(np.uint8)
    x[20000:26000] = 9                        # a constant run
    full = oracle.chunk(algo, x, w, M)
    _check_tiling(full, x.size, w, M)
    for m in [1, 100, 4097, 20500, 25999, 31234, 49999]:
        part = oracle.chunk(algo, x[:m], w, M)
        _check_tiling(part, m, w, M)
        if algo == "maxp":
            keep = set(full[full <= m - w].tolist())
            assert keep <= set(part.tolist())
        else:
            assert part.tolist() == [int(c) for c in full if c < m] + [m]


def test_complement_identity():
    rng = np.random.default_rng(3)
    for w, M in [(4, 9), (31, 500), (300, 4000)]:
        x = rng.integers(0, 256, 30000).astype(np.uint8)
        assert oracle.chunk("ae_min", x, w, M).tolist() == \
            oracle.chunk("ae", 255 - x, w, M).tolist()


@pytest.mark.parametrize("algo", ["ram", "ae", "maxp"])
@pytest.mark.parametrize("op", ["insert", "delete", "overwrite"])
def test_edit_locality(algo, op):
    """Cuts before an edit are unchanged (w bytes earlier for MAXP); after the
    first cut the two versions share, all later cuts coincide (shifted)."""
    rng = np.random.default_rng(11)
    w, M = (200, 5000) if algo != "maxp" else (60, 5000)
    x = rng.integers(0, 256, 200000).astype(np.uint8)
    e = 91234
    ins = rng.integers(0, 256, 77).astype(np.uint8)
    if op == "insert":
        y, d = np.concatenate([x[:e], ins, x[e:]]), 77
    elif op == "delete":
        y, d = np.concatenate([x[:e], x[e + 77:]]), -77
    else:
        y, d = np.concatenate([x[:e], ins, x[e + 77:]]), 0
    a = oracle.chunk(algo, x, w, M).astype(np.int64)
    b = oracle.chunk(algo, y, w, M).astype(np.int64)
    lim = e - (w if algo == "maxp" else 0)
    assert a[a <= lim].tolist() == b[b <= lim].tolist()
    after_a = a[a > e + 77]
    common = np.intersect1d(after_a + d, b)
    assert common.size > 0, "no resynchronisation"
    first = common[0]
    assert (a[a >= first - d] + d).tolist() == b[b >= first].tolist()


def test_next_cut_matches_chain():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 256, 20000).astype(np.uint8)
    for algo in ALGOS:
        cuts = oracle.chunk(algo, x, 30, 900)
        starts = np.concatenate([[0], cuts[:-1]])
        for s, c in zip(starts[::7], cuts[::7]):
            assert oracle.next_cut(algo, x, 30, 900, int(s)) == int(c)


def test_invalid_params():
    x = np.zeros(10, np.uint8)
    with pytest.raises(ValueError):
        oracle.chunk("ram", x, 0, 10)
    with pytest.raises(ValueError):
        oracle.chunk("ram", x, 5, 5)


def test_chunk_many_is_chunk_per_buffer():
    """The many-buffer driver equals one chunk() per buffer."""
    rng = np.random.default_rng(23)
    x = rng.integers(0, 256, 30000).astype(np.uint8)
    x[5000:12000] = 9
    offs = rng.integers(0, 20000, 40)
    lens = rng.integers(0, 10000, 40)
    lens[:3] = [0, 1, 7]
    for algo in ["ram", "ae", "maxp", "ae_min"]:
        cuts, base, cnt = oracle.chunk_many(algo, x, offs, lens, 31, 500)
        for j in range(40):
            exp = oracle.chunk(algo, x[offs[j]:offs[j] + lens[j]], 31, 500)
            got = cuts[int(base[j]):int(base[j]) + int(cnt[j])]
            assert np.array_equal(got, exp), (algo, j)


def test_pattern_bytes_exact_cases():
    """Bytes per pattern on inputs whose chains are known in closed form."""
    w, M = 50, 400
    # constant bytes: every chunk is w+1 long; RAM and AE search the w-byte
    # window (EBS) and take the one byte after it (RS); MAXP never cuts
    n = 20 * (w + 1)
    x = np.full(n, 9, np.uint8)
    for a in ("ram", "ae", "ae_min"):
        assert oracle.pattern_bytes(a, x, w, M) == (20 * w, 20)
    assert oracle.pattern_bytes("maxp", x, w, M) == (0, n)
    # spikes every 150 bytes from 60 on: MAXP cuts right after each spike
    # whose right window is complete; such a chunk searches both windows
    x = np.zeros(1000, np.uint8)
    spikes = list(range(60, 1000, 150))
    x[spikes] = 255
    cuts = oracle.chunk("maxp", x, w, M)
    ebs = 2 * w * sum(1 for q in spikes if q + w < 1000)
    assert oracle.pattern_bytes("maxp", x, w, M) == (ebs, 1000 + w * (ebs // (2 * w)) - ebs)
    assert [int(c) for c in cuts[:-1]] == [q + 1 for q in spikes if q + w < 1000]
    # strictly increasing bytes (AE-Max): every byte is a new target, so the
    # whole chunk is range-scanned up to each forced cut
    x = np.arange(256, dtype=np.uint8)
    assert oracle.pattern_bytes("ae", x, 20, 64) == (0, 256)
    # RAM where the window does not fit the last chunk: all of it is window
    x = np.full(3 * (w + 1) + 10, 4, np.uint8)
    assert oracle.pattern_bytes("ram", x, w, M) == (3 * w + 10, 3)


def test_pattern_bytes_ram_uniform_closed_form():
    """RAM on uniform bytes: the window (w bytes) almost surely holds a 255,
    and the scan after it stops at the first 255, about 256 bytes later
    (a geometric wait), so the window's share is w / (w + 256)."""
    x = np.random.default_rng(12).integers(0, 256, 48 << 20).astype(np.uint8)
    for w in (1024, 4096):
        e, r = oracle.pattern_bytes("ram", x, w, 1 << 20)
        share = e / (e + r)
        chunks = x.size / (w + 256)
        # the scan's mean has a standard error of about 256 / sqrt(chunks)
        tol = 4 * 256 / chunks ** 0.5 * w / (w + 256) ** 2
        assert abs(share - w / (w + 256)) < tol, (w, share)
