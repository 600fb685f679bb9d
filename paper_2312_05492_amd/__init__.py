"""MI355X-native G-Interp error-bounded compressor (cuSZ-i, arXiv 2312.05492).

A thin ctypes binding of ``libszi.so`` (the C ABI in ``include/szi.h``):
argument marshalling only.  Every step of compression and decompression runs
in the library's HIP kernels (and, for the Huffman codebook, in its native
host code, as the paper builds the codebook on the CPU).  PyTorch supplies
device memory and the current stream.

    import torch, paper_2312_05492_amd as szi
    ctx = szi.Context()
    res = ctx.compress(x_cuda_f32, eb=1e-3)          # relative bound
    y = ctx.decompress(res)                           # torch tensor on the GPU
    blob = res.blob()                                 # bytes
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libszi.so")

STAGES = ["range", "profile", "plan", "interp", "codebook", "huff_stats", "scan", "encode",
          "decode", "scatter", "replay", "elide"]
SZ_OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "NONFINITE", -3: "OOM", -4: "DEVICE", -5: "CORRUPT",
          -6: "UNSUPPORTED", -7: "CAPACITY"}
EB_ABS, EB_REL = 0, 1
LINEAR, CUBIC_NAK, CUBIC_NATURAL, CUBIC_AUTO = 0, 1, 2, 3
SEC_ANCHORS, SEC_CODES, SEC_OUTLIER_IDX, SEC_OUTLIER_VAL, SEC_WORDS, SEC_CHUNK_BITS, \
    SEC_HIST, SEC_CODE_LEN = range(8)
_SEC_DTYPE = {SEC_ANCHORS: np.float32, SEC_CODES: np.uint16, SEC_OUTLIER_IDX: np.uint32,
              SEC_OUTLIER_VAL: np.float32, SEC_WORDS: np.uint32, SEC_CHUNK_BITS: np.uint16,
              SEC_HIST: np.uint32, SEC_CODE_LEN: np.uint8}


class SzDims(C.Structure):
    _fields_ = [("ndim", C.c_uint32), ("reserved", C.c_uint32), ("n", C.c_uint64 * 3)]


class SzParams(C.Structure):
    _fields_ = [("eb_mode", C.c_int32), ("reserved0", C.c_int32), ("eb", C.c_double),
                ("interp", C.c_int32 * 3), ("order", C.c_int32 * 3), ("alpha", C.c_double),
                ("radius", C.c_uint32), ("huff_chunk", C.c_uint32),
                ("anchor_stride", C.c_uint32), ("window", C.c_uint32 * 3)]


class SzResult(C.Structure):
    _fields_ = [("anchors", C.c_void_p), ("n_anchors", C.c_uint64),
                ("codes", C.c_void_p), ("n", C.c_uint64),
                ("outlier_idx", C.c_void_p), ("outlier_val", C.c_void_p),
                ("n_outliers", C.c_uint64),
                ("words", C.c_void_p), ("n_words", C.c_uint64),
                ("chunk_bits", C.c_void_p), ("n_chunks", C.c_uint64),
                ("hist", C.c_void_p), ("code_len", C.c_void_p),
                ("compressed_bytes", C.c_uint64), ("header", C.c_uint8 * 256),
                ("internal", C.c_void_p)]


class SzRequest(C.Structure):
    _fields_ = [("kind", C.c_int32), ("book", C.c_int32), ("tag", C.c_uint64),
                ("d_in", C.c_void_p), ("dims", SzDims), ("params", SzParams),
                ("src", C.POINTER(SzResult)), ("d_out", C.c_void_p)]


class SzCompletion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("slot", C.c_int32),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("result", SzResult)]


REQ_COMPRESS, REQ_DECOMPRESS = 0, 1


class SzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


_lib = None


def lib():
    """Load libszi.so; raises when it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libszi.so is not built: run `python -m paper_2312_05492_amd.build`"
                               " (or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        L.sz_params_default.restype = None
        L.sz_params_default.argtypes = [P(SzParams)]
        L.sz_ctx_create.restype = C.c_int
        L.sz_ctx_create.argtypes = [P(vp), C.c_int, C.c_uint64]
        L.sz_ctx_destroy.restype = C.c_int
        L.sz_ctx_destroy.argtypes = [vp]
        L.sz_last_error.restype = C.c_char_p
        L.sz_last_error.argtypes = [vp]
        L.sz_ctx_bytes_in_use.restype = C.c_uint64
        L.sz_ctx_bytes_in_use.argtypes = [vp]
        L.sz_ctx_set_grid.restype = C.c_int
        L.sz_ctx_set_grid.argtypes = [vp, C.c_int]
        L.sz_ctx_set_graphs.restype = C.c_int
        L.sz_ctx_set_graphs.argtypes = [vp, C.c_int]
        L.sz_ctx_set_tuning.restype = C.c_int
        L.sz_ctx_set_tuning.argtypes = [vp, C.c_int]
        L.sz_ctx_set_shape.restype = C.c_int
        L.sz_ctx_set_shape.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.sz_ctx_get_shape.restype = C.c_int
        L.sz_ctx_get_shape.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.sz_ctx_set_timing.restype = C.c_int
        L.sz_ctx_set_timing.argtypes = [vp, C.c_int]
        L.sz_ctx_read_timing.restype = C.c_int
        L.sz_ctx_read_timing.argtypes = [vp, P(C.c_double), P(C.c_uint64), C.c_int]
        L.sz_compress.restype = C.c_int
        L.sz_compress.argtypes = [vp, vp, P(SzDims), P(SzParams), vp, P(SzResult)]
        L.sz_compress_with_code.restype = C.c_int
        L.sz_compress_with_code.argtypes = [vp, vp, P(SzDims), P(SzParams), vp, vp, P(SzResult)]
        L.sz_code_lengths.restype = C.c_int
        L.sz_code_lengths.argtypes = [vp, C.c_uint32, vp]
        L.sz_compress_batch.restype = C.c_int
        L.sz_compress_batch.argtypes = [vp, C.c_uint32, P(vp), P(SzDims), P(SzParams), vp,
                                        P(SzResult)]
        L.sz_compress_batch_with_code.restype = C.c_int
        L.sz_compress_batch_with_code.argtypes = [vp, C.c_uint32, P(vp), P(SzDims), P(SzParams),
                                                  P(vp), vp, P(SzResult)]
        L.sz_decompress.restype = C.c_int
        L.sz_decompress.argtypes = [vp, P(SzResult), vp, vp]
        L.sz_decompress_batch.restype = C.c_int
        L.sz_decompress_batch.argtypes = [vp, C.c_uint32, P(SzResult), P(vp), vp]
        L.sz_decompress_noalloc.restype = C.c_int
        L.sz_decompress_noalloc.argtypes = [vp, P(SzResult), vp, vp]
        L.sz_serialize.restype = C.c_int
        L.sz_serialize.argtypes = [vp, P(SzResult), vp, C.c_uint64, P(C.c_uint64)]
        L.sz_upload.restype = C.c_int
        L.sz_upload.argtypes = [vp, vp, C.c_uint64, vp, P(SzResult)]
        L.sz_result_free.restype = C.c_int
        L.sz_result_free.argtypes = [vp, P(SzResult)]
        L.sz_result_read.restype = C.c_int
        L.sz_result_read.argtypes = [vp, P(SzResult), C.c_int32, vp, C.c_uint64,
                                     P(C.c_uint64)]
        L.sz_server_create.restype = C.c_int
        L.sz_server_create.argtypes = [P(vp), C.c_int, C.c_int, C.c_uint64]
        L.sz_server_submit.restype = C.c_int
        L.sz_server_submit.argtypes = [vp, P(SzRequest)]
        L.sz_server_poll.restype = C.c_int
        L.sz_server_poll.argtypes = [vp, P(SzCompletion), C.c_uint32, P(C.c_uint32), C.c_int]
        L.sz_server_result_free.restype = C.c_int
        L.sz_server_result_free.argtypes = [vp, P(SzResult)]
        L.sz_server_stats.restype = C.c_int
        L.sz_server_stats.argtypes = [vp, P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
        L.sz_server_last_error.restype = C.c_char_p
        L.sz_server_last_error.argtypes = [vp]
        L.sz_server_destroy.restype = C.c_int
        L.sz_server_destroy.argtypes = [vp]
        _lib = L
    return _lib


def make_dims(shape) -> SzDims:
    d = SzDims()
    d.ndim = len(shape)
    for ax, s in enumerate(shape):
        d.n[len(shape) - 1 - ax] = int(s)
    return d


def make_params(ndim, eb=1e-3, eb_mode=EB_REL, interp=None, order=None, alpha=0.0, radius=512,
                chunk=1024, S=0, window=None) -> SzParams:
    """interp, order and window are given per numpy axis (slowest first), as
    in the oracle's Params; they are stored per dimension index (0 =
    fastest).  S: anchor stride (0 = the default of the dimensionality)."""
    p = SzParams()
    lib().sz_params_default(C.byref(p))
    p.eb_mode = eb_mode
    p.eb = float(eb)
    if interp is not None:
        for ax, v in enumerate(interp):
            p.interp[ndim - 1 - ax] = int(v)
    if order is not None:
        for k, ax in enumerate(order):
            p.order[k] = ndim - 1 - int(ax)
    p.alpha = float(alpha)
    p.radius = int(radius)
    p.huff_chunk = int(chunk)
    p.anchor_stride = int(S)
    if window is not None:
        for ax, w in enumerate(window):
            p.window[ndim - 1 - ax] = int(w)
    return p


def code_lengths(hist) -> np.ndarray:
    """Code lengths for Context.compress_with_code from a histogram of 2R
    bins: the length-limited Huffman lengths of the counts plus one, so that
    every symbol has a code (host only)."""
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    out = np.zeros(h.size, dtype=np.uint8)
    rc = lib().sz_code_lengths(h.ctypes.data_as(C.c_void_p), h.size, out.ctypes.data_as(C.c_void_p))
    if rc != SZ_OK:
        raise SzError(rc, "sz_code_lengths: histogram of %d bins" % h.size)
    return out


def _stream(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Result:
    """A compressed field held in device memory by its context."""

    def __init__(self, ctx: "Context", raw: SzResult, shape):
        self.ctx = ctx
        self.raw = raw
        self.shape = tuple(shape)

    @property
    def compressed_bytes(self):
        return self.raw.compressed_bytes

    @property
    def n_outliers(self):
        return self.raw.n_outliers

    def ratio(self):
        return 4.0 * self.raw.n / self.raw.compressed_bytes

    def read(self, section) -> np.ndarray:
        L = lib()
        need = C.c_uint64(0)
        L.sz_result_read(self.ctx.h, C.byref(self.raw), section, None, 0, C.byref(need))
        out = np.zeros(max(need.value, 1), dtype=np.uint8)
        self.ctx._check(L.sz_result_read(self.ctx.h, C.byref(self.raw), section,
                                         out.ctypes.data_as(C.c_void_p), out.size,
                                         C.byref(need)))
        return out[:need.value].view(_SEC_DTYPE[section]).copy()

    def blob(self) -> bytes:
        buf = (C.c_uint8 * self.raw.compressed_bytes)()
        w = C.c_uint64(0)
        self.ctx._check(lib().sz_serialize(self.ctx.h, C.byref(self.raw), buf,
                                           self.raw.compressed_bytes, C.byref(w)))
        return bytes(buf)

    def header(self) -> bytes:
        return bytes(self.raw.header)

    def free(self):
        if self.raw.internal:
            lib().sz_result_free(self.ctx.h, C.byref(self.raw))

    def __del__(self):
        try:
            if self.ctx.h and self.raw.internal:
                self.free()
        except Exception:
            pass


class Context:
    """A libszi context on one GPU (device memory pool, staging buffers)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        import torch
        self.torch = torch
        self.device = device
        h = C.c_void_p()
        rc = lib().sz_ctx_create(C.byref(h), device, hbm_budget)
        if rc != SZ_OK:
            raise SzError(rc, "sz_ctx_create failed")
        self.h = h

    def _check(self, rc):
        if rc != SZ_OK:
            raise SzError(rc, lib().sz_last_error(self.h).decode())

    def close(self):
        if self.h:
            lib().sz_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bytes_in_use(self):
        return lib().sz_ctx_bytes_in_use(self.h)

    def set_grid(self, per_cu: int):
        self._check(lib().sz_ctx_set_grid(self.h, per_cu))

    def set_tuning(self, on: bool):
        """Launch-shape tuning of the window kernels on the first plain call
        per (kind, ndim, radius); results are unchanged."""
        self._check(lib().sz_ctx_set_tuning(self.h, 1 if on else 0))

    def set_shape(self, kind: int, ndim: int, radius: int, variant: int, per_cu: int):
        """Pin the launch shape of a window kernel (kind 0 compression, 1 replay)."""
        self._check(lib().sz_ctx_set_shape(self.h, kind, ndim, radius, variant, per_cu))

    def shape(self, kind: int, ndim: int, radius: int = 512):
        """(variant, workgroups per CU, known) in use for a key."""
        v, g, k = C.c_int(), C.c_int(), C.c_int()
        self._check(lib().sz_ctx_get_shape(self.h, kind, ndim, radius, C.byref(v), C.byref(g),
                                           C.byref(k)))
        return v.value, g.value, bool(k.value)

    def set_graphs(self, on: bool):
        self._check(lib().sz_ctx_set_graphs(self.h, 1 if on else 0))

    def set_timing(self, on: bool):
        self._check(lib().sz_ctx_set_timing(self.h, 1 if on else 0))

    def read_timing(self, reset: bool = False) -> dict:
        ms = (C.c_double * len(STAGES))()
        n = (C.c_uint64 * len(STAGES))()
        self._check(lib().sz_ctx_read_timing(self.h, ms, n, 1 if reset else 0))
        return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}

    def _field(self, x):
        t = self.torch
        if not (isinstance(x, t.Tensor) and x.is_cuda and x.dtype == t.float32):
            raise TypeError("expected a float32 CUDA tensor")
        if not x.is_contiguous():
            raise ValueError("field must be contiguous")
        return x

    def compress(self, x, **kw) -> Result:
        x = self._field(x)
        d = make_dims(x.shape)
        p = make_params(x.dim(), **kw)
        r = SzResult()
        self._check(lib().sz_compress(self.h, C.c_void_p(x.data_ptr()), C.byref(d), C.byref(p),
                                      _stream(self.torch, x.device), C.byref(r)))
        return Result(self, r, x.shape)

    def compress_with_code(self, x, code_len, **kw) -> Result:
        """Compression with a given code book: 2R code lengths (uint8, each
        1..24, Kraft sum <= 1), e.g. code_lengths(earlier.read(SEC_HIST))."""
        x = self._field(x)
        d = make_dims(x.shape)
        p = make_params(x.dim(), **kw)
        cl = np.ascontiguousarray(code_len, dtype=np.uint8)
        if cl.size != 2 * p.radius:
            raise ValueError("code_len needs %d entries (2R), got %d" % (2 * p.radius, cl.size))
        r = SzResult()
        self._check(lib().sz_compress_with_code(self.h, C.c_void_p(x.data_ptr()), C.byref(d),
                                                C.byref(p), cl.ctypes.data_as(C.c_void_p),
                                                _stream(self.torch, x.device), C.byref(r)))
        return Result(self, r, x.shape)

    def compress_batch(self, xs, params=None) -> list:
        xs = [self._field(x) for x in xs]
        n = len(xs)
        params = params or [{}] * n
        ins = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        dims = (SzDims * n)(*[make_dims(x.shape) for x in xs])
        ps = (SzParams * n)(*[make_params(x.dim(), **kw) for x, kw in zip(xs, params)])
        outs = (SzResult * n)()
        self._check(lib().sz_compress_batch(self.h, n, ins, dims, ps,
                                            _stream(self.torch, xs[0].device), outs))
        return [Result(self, outs[i], xs[i].shape) for i in range(n)]

    def compress_batch_with_code(self, xs, code_lens, params=None) -> list:
        """A batch with a given code book per field (2R uint8 lengths each)."""
        xs = [self._field(x) for x in xs]
        n = len(xs)
        params = params or [{}] * n
        ps = (SzParams * n)(*[make_params(x.dim(), **kw) for x, kw in zip(xs, params)])
        cls = [np.ascontiguousarray(c, dtype=np.uint8) for c in code_lens]
        for p, cl in zip(ps, cls):
            if cl.size != 2 * p.radius:
                raise ValueError("code_len needs %d entries (2R), got %d" % (2 * p.radius, cl.size))
        ins = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        dims = (SzDims * n)(*[make_dims(x.shape) for x in xs])
        books = (C.c_void_p * n)(*[cl.ctypes.data for cl in cls])
        outs = (SzResult * n)()
        self._check(lib().sz_compress_batch_with_code(self.h, n, ins, dims, ps, books,
                                                      _stream(self.torch, xs[0].device), outs))
        return [Result(self, outs[i], xs[i].shape) for i in range(n)]

    def decompress(self, res: Result, out=None):
        t = self.torch
        if out is None:
            out = t.empty(res.shape, dtype=t.float32, device="cuda:%d" % self.device)
        self._check(lib().sz_decompress(self.h, C.byref(res.raw), C.c_void_p(out.data_ptr()),
                                        _stream(t, out.device)))
        return out

    def decompress_noalloc(self, res: Result, out):
        """sz_decompress_noalloc: the library allocates nothing; the work is
        only enqueued on the current stream (synchronise before reading)."""
        self._check(lib().sz_decompress_noalloc(self.h, C.byref(res.raw),
                                                C.c_void_p(out.data_ptr()),
                                                _stream(self.torch, out.device)))
        return out

    def decompress_batch(self, results, outs=None):
        t = self.torch
        n = len(results)
        if outs is None:
            outs = [t.empty(r.shape, dtype=t.float32, device="cuda:%d" % self.device)
                    for r in results]
        raw = (SzResult * n)(*[r.raw for r in results])
        ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        self._check(lib().sz_decompress_batch(self.h, n, raw, ptrs, _stream(t, outs[0].device)))
        return outs

    def upload(self, blob: bytes, shape=None) -> Result:
        buf = (C.c_uint8 * len(blob)).from_buffer_copy(blob)
        r = SzResult()
        self._check(lib().sz_upload(self.h, buf, len(blob), _stream(self.torch, self.device),
                                    C.byref(r)))
        if shape is None:
            import struct
            ndim = struct.unpack_from("<I", blob, 8)[0]
            n = struct.unpack_from("<3Q", blob, 16)
            shape = tuple(reversed(n[:ndim]))
        return Result(self, r, shape)


class ServerResult(Result):
    """A compression result produced by a Server (freed through it)."""

    def __init__(self, server: "Server", raw: SzResult, shape):
        super().__init__(server.reader, raw, shape)
        self.server = server

    def free(self):
        if self.raw.internal and self.server.h:
            lib().sz_server_result_free(self.server.h, C.byref(self.raw))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Request server (continuous batching): `slots` workers with their own
    context and stream admit queued compress/decompress requests in arrival
    order as slots and the HBM budget allow.  Inputs stay referenced here
    until their completion is polled."""

    def __init__(self, device: int = 0, slots: int = 4, hbm_budget: int = 0):
        import torch
        self.torch = torch
        self.device = device
        self.reader = Context(device)   # for reading results back
        h = C.c_void_p()
        rc = lib().sz_server_create(C.byref(h), device, slots, hbm_budget)
        if rc != SZ_OK:
            raise SzError(rc, "sz_server_create failed")
        self.h = h
        self._keep = {}   # tag -> objects that must outlive the request
        self._shape = {}
        self._bufs = {}   # poll's completion arrays (poll from one thread at a time)

    def _check(self, rc):
        if rc != SZ_OK:
            raise SzError(rc, lib().sz_server_last_error(self.h).decode())

    def submit_compress(self, x, tag: int, book: int = 0, **kw):
        """book > 0: use (or, the first time, leave) the server's resident
        code book of that number."""
        x = self.reader._field(x)
        r = SzRequest()
        r.kind = REQ_COMPRESS
        r.book = book
        r.tag = tag
        r.d_in = x.data_ptr()
        r.dims = make_dims(x.shape)
        r.params = make_params(x.dim(), **kw)
        self._check(lib().sz_server_submit(self.h, C.byref(r)))
        self._keep[tag] = x
        self._shape[tag] = tuple(x.shape)

    def submit_decompress(self, res: Result, out, tag: int):
        if not (out.is_cuda and out.is_contiguous() and out.numel() == res.raw.n):
            raise ValueError("output must be a contiguous CUDA tensor of the field's size")
        r = SzRequest()
        r.kind = REQ_DECOMPRESS
        r.tag = tag
        r.src = C.pointer(res.raw)
        r.d_out = out.data_ptr()
        self._check(lib().sz_server_submit(self.h, C.byref(r)))
        self._keep[tag] = (res, out, r)

    def poll(self, wait: bool = True, cap: int = 256) -> list:
        """Completed requests, oldest first: dicts with tag, status, slot,
        t_submit, t_start, t_done (seconds) and, for a compression, result."""
        buf = self._bufs.get(cap)
        if buf is None:   # one completion array per size, reused
            buf = self._bufs[cap] = (SzCompletion * cap)()
        n = C.c_uint32(0)
        self._check(lib().sz_server_poll(self.h, buf, cap, C.byref(n), 1 if wait else 0))
        out = []
        for i in range(n.value):
            c = buf[i]
            d = dict(tag=c.tag, status=c.status, slot=c.slot, t_submit=c.t_submit,
                     t_start=c.t_start, t_done=c.t_done, result=None)
            shape = self._shape.pop(c.tag, None)
            if c.result.internal:
                raw = SzResult()
                C.pointer(raw)[0] = c.result
                d["result"] = ServerResult(self, raw, shape)
            self._keep.pop(c.tag, None)
            out.append(d)
        return out

    def stats(self):
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        self._check(lib().sz_server_stats(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(charged=a.value, queued=b.value, running=c.value)

    def close(self):
        if self.h:
            lib().sz_server_destroy(self.h)
            self.h = None
        self._keep.clear()
        if self.reader is not None:
            self.reader.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

