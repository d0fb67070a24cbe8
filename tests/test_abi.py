"""The C ABI library loads and exports every function include/*.h declares
(no GPU needed: nothing is called that touches a device)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
LIB = os.path.join(ROOT, "paper_2508_05797_amd", "libcdc.so")


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cdc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ["cdc_chunk", "cdc_chunk_batch", "cdc_max_cuts", "cdc_reserve",
                 "cdc_release", "cdc_status_string", "cdc_last_error",
                 "cdc_chunk_each", "cdc_autotune", "cdc_set_tuning", "cdc_serve"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcdc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcdc.so not built")
def test_host_only_entry_points():
    from paper_2508_05797_amd import binding
    L = binding.lib()
    assert L.cdc_status_string(0) == b"ok"
    assert L.cdc_status_string(-1) == b"invalid argument"
    p = binding.Params(4096, 65536, 0, 0)
    assert L.cdc_max_cuts(ctypes.byref(p), 0) == 0
    assert L.cdc_max_cuts(ctypes.byref(p), 1) == 1
    assert L.cdc_max_cuts(ctypes.byref(p), 4097) == 1
    assert L.cdc_max_cuts(ctypes.byref(p), 4098) == 2
    assert L.cdc_max_cuts(ctypes.byref(p), 1 << 30) == (((1 << 30) - 1) // 4097) + 1
    # invalid parameters are rejected before anything touches a device
    for w, M in [(0, 10), (10, 10), (10, (1 << 28) + 1)]:
        q = binding.Params(w, M, 0, 0)
        rc = L.cdc_chunk(0, ctypes.byref(q), ctypes.c_void_p(1), 100,
                         ctypes.c_void_p(1), ctypes.c_void_p(1), None)
        assert rc == -1
    q = binding.Params(16, 100, 0, 0)
    assert L.cdc_chunk(7, ctypes.byref(q), ctypes.c_void_p(1), 100,
                       ctypes.c_void_p(1), ctypes.c_void_p(1), None) == -1
    assert L.cdc_chunk(0, ctypes.byref(q), None, 100, ctypes.c_void_p(1),
                       ctypes.c_void_p(1), None) == -1
    T = binding.Tuning
    assert L.cdc_set_tuning(ctypes.byref(T(8, 0, 0, 0))) == -1
    assert L.cdc_set_tuning(ctypes.byref(T(0, (1 << 28) + 1, 0, 0))) == -1
    assert L.cdc_set_tuning(ctypes.byref(T(0, 0, 9, 0))) == -1
    assert L.cdc_set_tuning(ctypes.byref(T(0, 0, 0, 1))) == -1
    assert L.cdc_set_tuning(ctypes.byref(T(4096, 1 << 16, 2, 0))) == 0
    assert binding.get_tuning() == {"chain_segment": 4096, "maxp_segment": 65536,
                                    "waves_per_block": 2, "reserved": 0}
    assert L.cdc_set_tuning(None) == 0
    assert binding.get_tuning() == {"chain_segment": 1 << 19, "maxp_segment": 1 << 18,
                                    "waves_per_block": 4, "reserved": 0}
    assert L.cdc_autotune(None, 1, None, 1, None) == -1
    assert L.cdc_get_tuning(None) == -1
    # the serving loop validates before creating streams
    assert L.cdc_serve(None, 0, None, None, None, 0, None, None, None, None) == -1


def test_tuning_grid_test_covers_the_autotuner_grid():
    """The GPU grid test runs exactly the values the autotuner can choose."""
    import sys
    src = open(os.path.join(ROOT, "paper_2508_05797_amd", "csrc",
                            "autotune.cpp")).read()

    def grid(name):
        m = re.search(name + r"\s*=\s*\{([^}]*)\}", src)
        return sorted(eval(v.strip()) for v in m.group(1).split(",") if v.strip())

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import test_gpu_tuning_grid as t
    assert grid("chain_segs") == sorted(t.CHAIN_SEGS)
    assert grid("maxp_segs") == sorted(t.MAXP_SEGS)
    assert grid("waves") == sorted(t.WAVES)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcdc.so not built")
def test_noalloc_refuses_beyond_scratch_without_a_device():
    """cdc_chunk_noalloc checks its request against its fixed scratch before
    touching a device: a request that does not fit is refused with
    CDC_ENOMEM and a message naming the bytes it would need."""
    from paper_2508_05797_amd import binding
    L = binding.lib()
    p = binding.Params(1, 2, 0, 0)
    fake = ctypes.c_void_p(0x1000)
    rc = L.cdc_chunk_noalloc(0, ctypes.byref(p), fake, 1 << 30, fake, fake,
                             ctypes.c_void_p(0))
    assert rc == -2
    msg = L.cdc_last_error().decode()
    assert "scratch" in msg and str(64 << 20) in msg
    # invalid parameters are refused first
    bad = binding.Params(0, 2, 0, 0)
    assert L.cdc_chunk_noalloc(0, ctypes.byref(bad), fake, 10, fake, fake,
                               ctypes.c_void_p(0)) == -1


def test_sha256_constants_follow_their_definition():
    """The SHA-256 round constants and initial state in the fingerprint
    kernels are the first 32 bits of the fractional parts of the cube roots
    of the first 64 primes and of the square roots of the first 8 primes
    (FIPS 180-4, 4.2.2 and 5.3.3), recomputed here to 60 digits."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    src = open(os.path.join(ROOT, "paper_2508_05797_amd", "csrc",
                            "fingerprint_kernels.hip")).read()

    def table(name):
        m = re.search(name + r"\[\d+\]\s*=\s*\{([^}]*)\}", src)
        return [int(v.strip().rstrip("u"), 16) for v in m.group(1).split(",")]

    primes = []
    n = 2
    while len(primes) < 64:
        if all(n % p for p in primes):
            primes.append(n)
        n += 1

    def frac_bits(p, r):
        x = Decimal(p) ** (Decimal(1) / Decimal(r))
        return int((x - int(x)) * (1 << 32))

    assert table("kSha256K") == [frac_bits(p, 3) for p in primes]
    assert table("kSha256H0") == [frac_bits(p, 2) for p in primes[:8]]
