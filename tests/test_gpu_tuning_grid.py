"""Every value of the autotuner's grid gives the oracle's offsets (GPU).

The tuning (chain segment length, MAXP segment length, waves per workgroup)
changes only how the work is split.  Every grid value the autotuner can
choose runs here on a 16 MiB mixed stream with constant runs longer than a
segment, as single calls and as one batch of the four chunkers, each
compared element by element with the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_05797_amd import binding, datagen

pytestmark = pytest.mark.gpu

CHAIN_SEGS = [256 << 10, 512 << 10, 1 << 20, 2 << 20, 4 << 20]
MAXP_SEGS = [16 << 10, 32 << 10, 64 << 10, 128 << 10, 256 << 10, 512 << 10, 1 << 20]
WAVES = [1, 2, 4]
W = {"ram": 4096, "ae": 4096, "maxp": 2048, "ae_min": 4096}
M = 65536


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def stream16():
    assert torch.cuda.is_available()
    binding.lib()
    x, _ = datagen.mixed_stream(224, 31)
    runs = [np.full(5 << 20, 200, np.uint8), np.full(3 << 20, 0, np.uint8)]
    x = np.concatenate([x[:6 << 20], runs[0], x[6 << 20:], runs[1]])[:16 << 20]
    exp = {a: oracle.chunk(a, x, W[a], M) for a in W}
    d = torch.from_numpy(x).cuda()
    yield x, d, exp
    binding.set_tuning()
    assert binding.device_errors() == 0


def run_all(d, exp, tag):
    n = d.numel()
    for a in W:
        got = binding.chunk(d, a, W[a], M).cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, exp[a]), (tag, a, "single")
    b = binding.Batch(d, [0] * 4, [n] * 4, list(W), list(W.values()), M)
    b.run()
    torch.cuda.synchronize()
    assert (b.statuses() == 0).all(), tag
    for j, a in enumerate(W):
        got = b.result(j).cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, exp[a]), (tag, a, "batched")


@pytest.mark.parametrize("waves", WAVES)
@pytest.mark.parametrize("chain_seg", CHAIN_SEGS)
def test_chain_segments(stream16, chain_seg, waves):
    x, d, exp = stream16
    try:
        binding.set_tuning(chain_seg, waves, maxp_segment=0)
        say("case grid chain", chain_seg, waves)
        run_all(d, exp, (chain_seg, waves))
    finally:
        binding.set_tuning()


@pytest.mark.parametrize("waves", WAVES)
@pytest.mark.parametrize("maxp_seg", MAXP_SEGS)
def test_maxp_segments(stream16, maxp_seg, waves):
    x, d, exp = stream16
    try:
        binding.set_tuning(0, waves, maxp_segment=maxp_seg)
        say("case grid maxp", maxp_seg, waves)
        run_all(d, exp, (maxp_seg, waves))
    finally:
        binding.set_tuning()
