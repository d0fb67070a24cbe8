"""Python access to the scalar CPU oracle in ``cdc_oracle.c``.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this module; the product package never imports it.

The C file is compiled with the system ``gcc`` into ``liboracle.so`` next to
it (``build()``); it has no dependency beyond libc.
"""
import ctypes
import os
import subprocess

import numpy as np

RAM, AE, MAXP, AE_MIN = 0, 1, 2, 3
ALGOS = {"ram": RAM, "ae": AE, "maxp": MAXP, "ae_min": AE_MIN}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cdc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared"]

_lib = None


def build(force=True):
    """Compile the oracle with gcc (always, when force is true)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB)
                or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_chunk.restype = ctypes.c_int64
        lib.oracle_chunk.argtypes = [ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_void_p,
                                     ctypes.c_uint64]
        lib.oracle_chunk_many.restype = ctypes.c_int64
        lib.oracle_chunk_many.argtypes = [ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_pattern_bytes.restype = ctypes.c_int64
        lib.oracle_pattern_bytes.argtypes = [ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_uint64, ctypes.c_uint64,
                                             ctypes.c_uint64, ctypes.c_void_p]
        lib.oracle_next.restype = ctypes.c_uint64
        lib.oracle_next.argtypes = [ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_uint64]
        _lib = lib
    return _lib


def algo_id(algo):
    return ALGOS[algo] if isinstance(algo, str) else int(algo)


def max_cuts(n, w):
    """Every non-final chunk is at least w+1 bytes long."""
    return 0 if n == 0 else (n - 1) // (w + 1) + 1


def chunk(algo, data, w, max_chunk):
    """Exclusive chunk ends (uint64) of ``data`` under the given chunker."""
    x = np.ascontiguousarray(data, dtype=np.uint8)
    n = x.size
    out = np.empty(max(1, max_cuts(n, w)), dtype=np.uint64)
    k = _load().oracle_chunk(algo_id(algo), x.ctypes.data, n, w, max_chunk,
                             out.ctypes.data, out.size)
    if k < 0:
        raise ValueError("oracle_chunk failed with %d (w=%d, M=%d)"
                         % (k, w, max_chunk))
    return out[:k].copy()


def next_cut(algo, data, w, max_chunk, s):
    """One step of the chain: the end of the chunk that starts at ``s``."""
    x = np.ascontiguousarray(data, dtype=np.uint8)
    if w < 1 or max_chunk < w + 1 or not 0 <= s < x.size:
        raise ValueError("bad arguments")
    return int(_load().oracle_next(algo_id(algo), x.ctypes.data, x.size, w,
                                   max_chunk, s))


def chunk_many(algo, data, offsets, lengths, w, max_chunk, base=None):
    """Chunk every buffer data[offsets[j]:offsets[j]+lengths[j]] on its own.

    Returns (cuts, base, counts): the cuts of buffer j are
    cuts[base[j]:base[j]+counts[j]].  ``base`` may be given (uint64, one
    entry per buffer, each leaving room for max_cuts of its buffer)."""
    x = np.ascontiguousarray(data, dtype=np.uint8)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    ln = np.ascontiguousarray(lengths, dtype=np.uint64)
    assert off.size == ln.size
    assert x.size == 0 or int((off + ln).max(initial=0)) <= x.size
    room = np.where(ln > 0, (ln - 1) // np.uint64(w + 1) + 1, 0).astype(np.uint64)
    if base is None:
        base = np.zeros(ln.size, np.uint64)
        if ln.size > 1:
            np.cumsum(room[:-1], out=base[1:])
    base = np.ascontiguousarray(base, dtype=np.uint64)
    size = int((base + room).max(initial=0)) if ln.size else 0
    cuts = np.zeros(max(1, size), np.uint64)
    counts = np.zeros(ln.size, np.int64)
    rc = _load().oracle_chunk_many(algo_id(algo), x.ctypes.data, off.ctypes.data,
                                   ln.ctypes.data, ln.size, w, max_chunk,
                                   cuts.ctypes.data, base.ctypes.data,
                                   counts.ctypes.data)
    if rc < 0:
        raise ValueError("oracle_chunk_many failed with %d" % rc)
    return cuts, base, counts


def pattern_bytes(algo, data, w, max_chunk):
    """Bytes the chunker's chain hands to each pattern: (ebs, rs), as
    oracle_pattern_bytes defines the split of every chunk."""
    x = np.ascontiguousarray(data, dtype=np.uint8)
    out = np.zeros(2, np.uint64)
    k = _load().oracle_pattern_bytes(algo_id(algo), x.ctypes.data, x.size, w,
                                     max_chunk, out.ctypes.data)
    if k < 0:
        raise ValueError("oracle_pattern_bytes failed")
    return int(out[0]), int(out[1])
