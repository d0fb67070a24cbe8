"""ctypes binding of libcdc.so: argument marshalling only.

Every step of the chunking runs in the HIP kernels of the library; this
module passes device pointers, sizes and the current HIP stream of PyTorch.
It raises if the library has not been built (there is no CPU fallback).
"""
import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdc.so")

ALGOS = {"ram": 0, "ae": 1, "maxp": 2, "ae_min": 3}
STATUS = {0: "CDC_OK", -1: "CDC_EINVAL", -2: "CDC_ENOMEM", -3: "CDC_EHIP",
          -4: "CDC_ENOTSUP"}


class CdcError(RuntimeError):
    def __init__(self, rc, detail=""):
        super().__init__("%s (%d) %s" % (STATUS.get(rc, "?"), rc, detail))
        self.rc = rc


class Params(ctypes.Structure):
    _fields_ = [("window", ctypes.c_uint32), ("max_chunk", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    _fields_ = [("chain_segment", ctypes.c_uint64),
                ("maxp_segment", ctypes.c_uint64),
                ("waves_per_block", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Job(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("cut_offsets", ctypes.c_void_p), ("n_cuts", ctypes.c_void_p),
                ("algo", ctypes.c_uint32), ("window", ctypes.c_uint32),
                ("max_chunk", ctypes.c_uint32), ("status", ctypes.c_int32)]


_lib = None
_V, _U32, _U64, _SZ, _I = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64,
                           ctypes.c_size_t, ctypes.c_int)


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libcdc.so is not built (run paper_2508_05797_amd/build.py); "
                "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        L.cdc_max_cuts.restype = _SZ
        L.cdc_max_cuts.argtypes = [ctypes.POINTER(Params), _SZ]
        L.cdc_chunk.restype = _I
        L.cdc_chunk.argtypes = [_I, ctypes.POINTER(Params), _V, _SZ, _V, _V, _V]
        L.cdc_chunk_noalloc.restype = _I
        L.cdc_chunk_noalloc.argtypes = [_I, ctypes.POINTER(Params), _V, _SZ, _V, _V, _V]
        L.cdc_chunk_batch.restype = _I
        L.cdc_chunk_batch.argtypes = [_V, _U32, _V]
        L.cdc_reserve.restype = _I
        L.cdc_reserve.argtypes = [_V, _SZ, _U32, _U32, _U32]
        L.cdc_chunk_each.restype = _I
        L.cdc_chunk_each.argtypes = [_V, _U32, _V]
        L.cdc_release.restype = None
        L.cdc_release.argtypes = []
        L.cdc_status_string.restype = ctypes.c_char_p
        L.cdc_status_string.argtypes = [_I]
        L.cdc_last_error.restype = ctypes.c_char_p
        L.cdc_last_error.argtypes = []
        L.cdc_set_tuning.restype = _I
        L.cdc_set_tuning.argtypes = [_V]
        L.cdc_get_tuning.restype = _I
        L.cdc_get_tuning.argtypes = [_V]
        L.cdc_autotune.restype = _I
        L.cdc_autotune.argtypes = [_V, _U32, _V, _U32, _V]
        L.cdc_set_profiling.restype = _I
        L.cdc_set_profiling.argtypes = [_I]
        L.cdc_kernel_times.restype = _I
        L.cdc_kernel_times.argtypes = [_V, ctypes.POINTER(ctypes.c_char_p),
                                       ctypes.POINTER(ctypes.c_uint32),
                                       ctypes.POINTER(ctypes.c_double), _I]
        L.cdc_check_device_errors.restype = _I
        L.cdc_check_device_errors.argtypes = [_V]
        L.cdc_walk_stats.restype = _I
        L.cdc_walk_stats.argtypes = [_V, _V]
        L.cdc_stream_open.restype = _I
        L.cdc_stream_open.argtypes = [_I, ctypes.POINTER(Params), _SZ, _V,
                                      ctypes.POINTER(ctypes.c_void_p)]
        L.cdc_stream_max_cuts.restype = _SZ
        L.cdc_stream_max_cuts.argtypes = [_V, _SZ]
        L.cdc_stream_push.restype = _I
        L.cdc_stream_push.argtypes = [_V, _V, _SZ, _I, _V, _V, _V]
        L.cdc_stream_reset.restype = _I
        L.cdc_stream_reset.argtypes = [_V, _V]
        L.cdc_stream_close.restype = None
        L.cdc_stream_close.argtypes = [_V]
        L.cdc_fingerprint.restype = _I
        L.cdc_fingerprint.argtypes = [_V, _SZ, _V, _V, _SZ, _V, _V]
        L.cdc_dedup_create.restype = _I
        L.cdc_dedup_create.argtypes = [_U64, _V, ctypes.POINTER(ctypes.c_void_p)]
        L.cdc_dedup_add.restype = _I
        L.cdc_dedup_add.argtypes = [_V, _V, _V, _V, _SZ, _V]
        L.cdc_dedup_stats_get.restype = _I
        L.cdc_dedup_stats_get.argtypes = [_V, _V, _V]
        L.cdc_dedup_reset.restype = _I
        L.cdc_dedup_reset.argtypes = [_V, _V]
        L.cdc_dedup_destroy.restype = None
        L.cdc_dedup_destroy.argtypes = [_V]
        L.cdc_serve.restype = _I
        L.cdc_serve.argtypes = [_V, _U64, _V, _V, _V, _U32, _V, _V, _V, _V]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise CdcError(rc, lib().cdc_last_error().decode())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def algo_id(algo):
    return ALGOS[algo] if isinstance(algo, str) else int(algo)


def max_cuts(n, window):
    p = Params(window, window + 1, 0, 0)
    return int(lib().cdc_max_cuts(ctypes.byref(p), n))


def chunk_into(data, algo, window, max_chunk, cuts, n_cuts, stream=None):
    """Enqueue chunking of the uint8 device tensor ``data`` (contiguous) into
    the int64 device tensors ``cuts`` (>= max_cuts entries) and ``n_cuts``
    (one entry).  Asynchronous: nothing is synchronised."""
    assert data.dtype == torch.uint8 and data.is_cuda and data.is_contiguous()
    n = data.numel()
    p = Params(window, max_chunk, 0, 0)
    _check(lib().cdc_chunk(algo_id(algo), ctypes.byref(p),
                           ctypes.c_void_p(data.data_ptr() if n else 0), n,
                           ctypes.c_void_p(cuts.data_ptr()),
                           ctypes.c_void_p(n_cuts.data_ptr()), _stream(stream)))


def chunk_noalloc_into(data, algo, window, max_chunk, cuts, n_cuts, stream=None):
    """As chunk_into, through cdc_chunk_noalloc (the library's fixed scratch
    array instead of a per-stream workspace; nothing is allocated)."""
    assert data.dtype == torch.uint8 and data.is_cuda and data.is_contiguous()
    n = data.numel()
    p = Params(window, max_chunk, 0, 0)
    _check(lib().cdc_chunk_noalloc(algo_id(algo), ctypes.byref(p),
                                   ctypes.c_void_p(data.data_ptr() if n else 0), n,
                                   ctypes.c_void_p(cuts.data_ptr()),
                                   ctypes.c_void_p(n_cuts.data_ptr()),
                                   _stream(stream)))


def chunk(data, algo, window, max_chunk, stream=None):
    """Chunk boundaries (exclusive ends, int64 on the device) of ``data``.
    Synchronises to read the count."""
    n = data.numel()
    cuts = torch.empty(max(1, max_cuts(n, window)), dtype=torch.int64,
                       device=data.device)
    n_cuts = torch.empty(1, dtype=torch.int64, device=data.device)
    chunk_into(data, algo, window, max_chunk, cuts, n_cuts, stream)
    return cuts[:int(n_cuts.item())]


def set_tuning(segment_bytes=0, waves_per_block=0, maxp_segment=None):
    """Segment bytes for the chain search (and for MAXP unless maxp_segment
    is given) and waves per workgroup; 0 = built-in."""
    t = Tuning(segment_bytes, segment_bytes if maxp_segment is None else maxp_segment,
               waves_per_block, 0)
    _check(lib().cdc_set_tuning(ctypes.byref(t)))


def get_tuning():
    t = Tuning()
    _check(lib().cdc_get_tuning(ctypes.byref(t)))
    return t.as_dict()


def autotune(batch, reps=2, stream=None):
    """cdc_autotune on a Batch's device descriptors; returns the chosen
    tuning (now in effect, with the stream's workspace reserved)."""
    t = Tuning()
    _check(lib().cdc_autotune(ctypes.c_void_p(batch.jobs.data_ptr()),
                              batch.n_jobs, _stream(stream), reps,
                              ctypes.byref(t)))
    return t.as_dict()


def device_errors(stream=None):
    rc = lib().cdc_check_device_errors(_stream(stream))
    if rc < 0:
        _check(rc)
    return rc


def set_profiling(level):
    """0 off; 1 events around the main kernel of each call; 2 every kernel."""
    _check(lib().cdc_set_profiling(level))


def kernel_times(stream=None, max_kernels=16):
    """{kernel name: (calls, total ms)} recorded on the stream since the last
    report (synchronises the stream)."""
    names = (ctypes.c_char_p * max_kernels)()
    calls = (ctypes.c_uint32 * max_kernels)()
    tot = (ctypes.c_double * max_kernels)()
    k = lib().cdc_kernel_times(_stream(stream), names, calls, tot, max_kernels)
    if k < 0:
        _check(k)
    return {names[i].decode(): (int(calls[i]), float(tot[i])) for i in range(k)}


def walk_stats(stream=None):
    """How the last single RAM / AE call on the stream decided its chunks
    (synchronises the stream): segments, speculation steps by kind, tiles
    whose bytes each pattern read."""
    out = (ctypes.c_uint64 * 7)()
    _check(lib().cdc_walk_stats(_stream(stream), out))
    keys = ("segments", "steps_successor", "steps_fast", "steps_run",
            "steps_exact", "tiles_read_ebs", "tiles_read_rs")
    return {k: int(v) for k, v in zip(keys, out)}


def reserve(max_total_bytes, max_jobs, min_window, max_chunk, stream=None):
    """Pre-size the stream's workspace (needed before capturing batches)."""
    _check(lib().cdc_reserve(_stream(stream), max_total_bytes, max_jobs,
                             min_window, max_chunk))


JOB_DTYPE = np.dtype([("data", "<u8"), ("n", "<u8"), ("cut_offsets", "<u8"),
                      ("n_cuts", "<u8"), ("algo", "<u4"), ("window", "<u4"),
                      ("max_chunk", "<u4"), ("status", "<i4")])
assert JOB_DTYPE.itemsize == ctypes.sizeof(Job) == 48


class Batch:
    """Many buffers inside one uint8 device tensor, with one output area.

    ``offsets``/``lengths`` (host integer arrays) locate each buffer in
    ``data``; ``algo``, ``window`` and ``max_chunk`` are scalars or per-job
    arrays.  The job descriptors live in device memory (``jobs``) and, for the
    plain path, in host memory (``host_jobs``)."""

    def __init__(self, data, offsets, lengths, algo, window, max_chunk):
        assert data.dtype == torch.uint8 and data.is_cuda
        n_jobs = len(lengths)
        lengths = np.asarray(lengths, dtype=np.uint64)
        offsets = np.asarray(offsets, dtype=np.uint64)
        algos = np.broadcast_to(np.asarray(
            [algo_id(a) for a in np.atleast_1d(algo)], np.uint32), (n_jobs,))
        windows = np.broadcast_to(np.asarray(window, np.uint32), (n_jobs,))
        maxc = np.broadcast_to(np.asarray(max_chunk, np.uint32), (n_jobs,))
        room = np.where(lengths > 0,
                        (lengths - 1) // (windows.astype(np.uint64) + 1) + 1, 0)
        room = np.maximum(room, 1).astype(np.uint64)
        self.cut_base = np.zeros(n_jobs + 1, np.uint64)
        np.cumsum(room, out=self.cut_base[1:])
        dev = data.device
        self.data = data
        self.cuts = torch.empty(int(self.cut_base[-1]), dtype=torch.int64,
                                device=dev)
        self.n_cuts = torch.zeros(n_jobs, dtype=torch.int64, device=dev)
        t = np.zeros(n_jobs, JOB_DTYPE)
        t["data"] = data.data_ptr() + offsets
        t["n"] = lengths
        t["cut_offsets"] = self.cuts.data_ptr() + 8 * self.cut_base[:-1]
        t["n_cuts"] = self.n_cuts.data_ptr() + 8 * np.arange(n_jobs, dtype=np.uint64)
        t["algo"] = algos
        t["window"] = windows
        t["max_chunk"] = maxc
        self.host_jobs = t
        self.jobs = torch.from_numpy(t.view(np.uint8).copy()).to(dev)
        self.n_jobs = n_jobs
        self.total_bytes = int(lengths.sum())

    def run(self, stream=None):
        """cdc_chunk_batch on the device job table (asynchronous)."""
        _check(lib().cdc_chunk_batch(ctypes.c_void_p(self.jobs.data_ptr()),
                                     self.n_jobs, _stream(stream)))

    def run_each(self, stream=None):
        """One cdc_chunk call per job (the plain path; asynchronous)."""
        rc = lib().cdc_chunk_each(self.host_jobs.ctypes.data, self.n_jobs,
                                  _stream(stream))
        if rc != 0:
            _check(rc)

    def statuses(self):
        return self.jobs.cpu().numpy().view(JOB_DTYPE)["status"].copy()

    def result(self, j, n_cuts_host=None):
        """Cut offsets of job j (int64 device tensor)."""
        k = int(self.n_cuts[j].item()) if n_cuts_host is None else int(n_cuts_host[j])
        b = int(self.cut_base[j])
        return self.cuts[b:b + k]


REQUEST_DTYPE = np.dtype([("offset", "<u8"), ("n", "<u8"), ("cut_base", "<u8"),
                          ("algo", "<u4"), ("window", "<u4"),
                          ("max_chunk", "<u4"), ("reserved", "<u4"),
                          ("arrival", "<f8")])
assert REQUEST_DTYPE.itemsize == 48


class ServeConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("max_batch", ctypes.c_uint32),
                ("slots", ctypes.c_uint32), ("min_window", ctypes.c_uint32),
                ("max_chunk", ctypes.c_uint32)]


class ServeStats(ctypes.Structure):
    _fields_ = [("elapsed", ctypes.c_double), ("launches", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("bytes_done", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64), ("max_queue", ctypes.c_uint32),
                ("max_inflight", ctypes.c_uint32)]


def requests(offsets, sizes, algos, windows, max_chunk, arrivals):
    """Request table (host) with each request's output area laid out
    back to back; returns (table, total offset slots)."""
    n = len(sizes)
    r = np.zeros(n, REQUEST_DTYPE)
    r["offset"] = offsets
    r["n"] = sizes
    r["algo"] = [algo_id(a) for a in algos]
    r["window"] = windows
    r["max_chunk"] = max_chunk
    r["arrival"] = arrivals
    w = r["window"].astype(np.uint64)
    sz = r["n"]
    room = np.where(sz > 0, (sz - 1) // np.maximum(w + 1, 2) + 1, 0)
    room = np.maximum(room, 1).astype(np.uint64)
    base = np.zeros(n + 1, np.uint64)
    np.cumsum(room, out=base[1:])
    r["cut_base"] = base[:-1]
    return r, int(base[-1])


def serve(pool, reqs, total_slots, budget_bytes=0, max_batch=1024, slots=4,
          min_window=None, max_chunk=None):
    """Run the request loop (cdc_serve) over ``reqs`` (REQUEST_DTYPE, host),
    whose bytes are in the uint8 device tensor ``pool``.  Returns
    (cuts, n_cuts, latency, status, stats): cuts/n_cuts int64 device tensors,
    latency (seconds) and status host arrays, stats a dict."""
    assert pool.dtype == torch.uint8 and pool.is_cuda and pool.is_contiguous()
    reqs = np.ascontiguousarray(reqs, REQUEST_DTYPE)
    n = len(reqs)
    cuts = torch.empty(max(total_slots, 1), dtype=torch.int64, device=pool.device)
    n_cuts = torch.full((n,), -1, dtype=torch.int64, device=pool.device)
    lat = np.zeros(n, np.float64)
    st = np.zeros(n, np.int32)
    cfg = ServeConfig(budget_bytes, max_batch, slots,
                      int(reqs["window"].min()) if min_window is None else min_window,
                      int(reqs["max_chunk"].max()) if max_chunk is None else max_chunk)
    stats = ServeStats()
    torch.cuda.synchronize()          # the pool and outputs are ready
    rc = lib().cdc_serve(ctypes.c_void_p(pool.data_ptr()), pool.numel(),
                         ctypes.c_void_p(cuts.data_ptr()),
                         ctypes.c_void_p(n_cuts.data_ptr()),
                         reqs.ctypes.data, n, ctypes.byref(cfg), lat.ctypes.data,
                         st.ctypes.data, ctypes.byref(stats))
    _check(rc)
    return cuts, n_cuts, lat, st, {f: getattr(stats, f) for f, _ in ServeStats._fields_}


def release():
    lib().cdc_release()


def fingerprint_into(data, cuts, n_cuts, digests, stream=None):
    """Enqueue SHA-256 of every chunk of the cut list (int64 device tensors
    ``cuts`` and ``n_cuts`` as chunk_into fills them) into the uint8 device
    tensor ``digests`` (32 bytes per slot of ``cuts``)."""
    assert data.dtype == torch.uint8 and data.is_cuda and data.is_contiguous()
    assert digests.dtype == torch.uint8 and digests.numel() >= 32 * cuts.numel()
    _check(lib().cdc_fingerprint(ctypes.c_void_p(data.data_ptr()), data.numel(),
                                 ctypes.c_void_p(cuts.data_ptr()),
                                 ctypes.c_void_p(n_cuts.data_ptr()), cuts.numel(),
                                 ctypes.c_void_p(digests.data_ptr()),
                                 _stream(stream)))


def fingerprint(data, cuts, stream=None):
    """SHA-256 digests (uint8 device tensor, K x 32) of the chunks that end at
    the offsets ``cuts`` (an int64 device tensor holding exactly the cuts)."""
    k = cuts.numel()
    n_cuts = torch.tensor([k], dtype=torch.int64, device=cuts.device)
    dg = torch.empty((max(k, 1), 32), dtype=torch.uint8, device=cuts.device)
    fingerprint_into(data, cuts, n_cuts, dg, stream)
    return dg[:k]


class Dedup:
    """A device table of distinct chunks (cdc_dedup_*)."""

    FIELDS = ("total_bytes", "chunks", "unique_bytes", "unique_chunks",
              "collisions", "flags")

    def __init__(self, max_chunks, stream=None):
        h = ctypes.c_void_p()
        _check(lib().cdc_dedup_create(max_chunks, _stream(stream), ctypes.byref(h)))
        self.h = h

    def add(self, digests, cuts, n_cuts, stream=None):
        _check(lib().cdc_dedup_add(self.h, ctypes.c_void_p(digests.data_ptr()),
                                   ctypes.c_void_p(cuts.data_ptr()),
                                   ctypes.c_void_p(n_cuts.data_ptr()),
                                   cuts.numel(), _stream(stream)))

    def stats(self, stream=None):
        out = (ctypes.c_uint64 * 6)()
        _check(lib().cdc_dedup_stats_get(self.h, _stream(stream), out))
        return dict(zip(self.FIELDS, [int(v) for v in out]))

    def reset(self, stream=None):
        _check(lib().cdc_dedup_reset(self.h, _stream(stream)))

    def close(self):
        if self.h:
            lib().cdc_dedup_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    """A stream chunked in pieces (cdc_stream_*), on one torch stream."""

    def __init__(self, algo, window, max_chunk, max_piece, stream=None):
        self.torch_stream = stream
        p = Params(window, max_chunk, 0, 0)
        h = ctypes.c_void_p()
        _check(lib().cdc_stream_open(algo_id(algo), ctypes.byref(p), max_piece,
                                     _stream(stream), ctypes.byref(h)))
        self.h = h

    def max_cuts(self, n):
        return int(lib().cdc_stream_max_cuts(self.h, n))

    def push_into(self, piece, cuts, n_cuts, last=False):
        """Enqueue a piece (uint8 device tensor); decided offsets go to the
        int64 device tensors cuts / n_cuts.  Asynchronous."""
        assert piece.dtype == torch.uint8 and piece.is_cuda and piece.is_contiguous()
        n = piece.numel()
        _check(lib().cdc_stream_push(self.h, ctypes.c_void_p(piece.data_ptr() if n else 0),
                                     n, 1 if last else 0,
                                     ctypes.c_void_p(cuts.data_ptr()),
                                     ctypes.c_void_p(n_cuts.data_ptr()),
                                     _stream(self.torch_stream)))

    def push(self, piece, last=False):
        """The offsets this piece decides (int64 device tensor; synchronises)."""
        cuts = torch.empty(self.max_cuts(piece.numel()), dtype=torch.int64,
                           device=piece.device)
        nc = torch.empty(1, dtype=torch.int64, device=piece.device)
        self.push_into(piece, cuts, nc, last)
        return cuts[:int(nc.item())]

    def reset(self):
        _check(lib().cdc_stream_reset(self.h, _stream(self.torch_stream)))

    def close(self):
        if self.h:
            lib().cdc_stream_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
