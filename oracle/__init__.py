"""CPU oracle for the G-Interp compressor (cuSZ-i, arXiv 2312.05492).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package.

The arithmetic lives in ``szo.c`` (plain scalar C, built with gcc and FP
contraction off).  This module marshals numpy arrays through ctypes and
assembles the compressed blob with ``struct`` and ``zlib.crc32``.

The blob layout (little-endian) is the format the library writes too; both
sides implement it independently:

    256-byte header (see ``_HEADER`` below), then the sections
    anchors f32[n_anchors], code_len u8[2R], chunk_bits u16[n_chunks],
    words u32[n_words], outlier_idx u32[n_outliers], outlier_val f32[n_outliers],
    each zero-padded to a multiple of 8 bytes.  Header bytes 224..247 hold
    the CRC-32 of each unpadded section; bytes 252..255 the CRC-32 of
    header bytes 0..251.
"""
from __future__ import annotations

import ctypes as C
import os
import struct
import subprocess
import zlib
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "szo.c")
_LIB = os.path.join(_HERE, "libszo.so")

LIN, NAK, NAT, AUTO = 0, 1, 2, 3
EB_ABS, EB_REL = 0, 1
ST_ONE, ST_LINEAR, ST_QUAD_LEFT, ST_QUAD_RIGHT, ST_NAK, ST_NAT = range(6)
CLS_NONE, CLS_ANCHOR, CLS_ONE, CLS_LINEAR, CLS_QUAD, CLS_CUBIC = range(6)
LMAX = 24
MAGIC = b"SZI1"
VERSION = 1


def build(force: bool = True, plant: int = 0, out: str = None) -> str:
    """Compile szo.c into libszo.so with gcc (no contraction, IEEE).

    plant > 0 builds, into `out`, a copy with one deliberate mistake
    (SZO_PLANT in szo.c) so that tests can show the pins catch it; the
    library the oracle itself loads is always built with plant = 0."""
    target = out or _LIB
    if plant and target == _LIB:
        raise ValueError("a planted build needs its own output path")
    if not force and os.path.exists(target) and os.path.getmtime(target) >= os.path.getmtime(_SRC):
        return target
    tmp = target + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wno-unused-function", "-DSZO_PLANT=%d" % plant,
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, target)
    return target


class _Params(C.Structure):
    _fields_ = [("ndim", C.c_uint32), ("S", C.c_uint32), ("n", C.c_uint64 * 3),
                ("w", C.c_uint32 * 3), ("R", C.c_uint32), ("eb_mode", C.c_int32),
                ("pad0", C.c_int32), ("eb", C.c_double), ("interp", C.c_int32 * 3),
                ("order", C.c_int32 * 3), ("alpha", C.c_double)]


class _Config(C.Structure):
    _fields_ = [("vmin", C.c_float), ("vmax", C.c_float), ("range", C.c_double),
                ("eps", C.c_double), ("e_abs", C.c_double), ("e", C.c_float),
                ("levels", C.c_int32), ("alpha", C.c_double),
                ("el", C.c_float * 16), ("ebx2", C.c_float * 16), ("inv", C.c_float * 16),
                ("spline", C.c_int32 * 3), ("order", C.c_int32 * 3),
                ("prof", (C.c_double * 3) * 3), ("profiled", C.c_int32), ("pad1", C.c_int32)]


_lib = None


def load(path: str):
    """Open an oracle library at `path` and declare its entry points."""
    L = C.CDLL(path)
    P = C.POINTER
    L.szo_alpha.restype = C.c_double
    L.szo_alpha.argtypes = [C.c_double]
    L.szo_round_down.restype = C.c_float
    L.szo_round_down.argtypes = [C.c_double]
    L.szo_stencil.restype = C.c_float
    L.szo_stencil.argtypes = [C.c_int, C.c_float, C.c_float, C.c_float, C.c_float]
    L.szo_plan.restype = C.c_int
    L.szo_plan.argtypes = [C.c_void_p, P(_Params), P(_Config)]
    L.szo_num_anchors.restype = C.c_uint64
    L.szo_num_anchors.argtypes = [P(_Params)]
    L.szo_compress.restype = C.c_int
    L.szo_compress.argtypes = [C.c_void_p, P(_Params), P(_Config), C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, P(C.c_uint64), C.c_void_p]
    L.szo_compress_windowed.restype = C.c_int
    L.szo_compress_windowed.argtypes = [C.c_void_p, P(_Params), P(_Config), C.c_void_p,
                                        C.c_void_p]
    L.szo_decompress.restype = C.c_int
    L.szo_decompress.argtypes = [P(_Params), P(_Config), C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_uint64, C.c_void_p]
    L.szo_histogram.restype = None
    L.szo_histogram.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_void_p]
    L.szo_huffman_lengths.restype = C.c_int
    L.szo_huffman_lengths.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p]
    L.szo_canonical_codes.restype = None
    L.szo_canonical_codes.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p]
    L.szo_encode.restype = C.c_uint64
    L.szo_encode.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_uint32,
                             C.c_void_p, C.c_void_p]
    L.szo_decode.restype = C.c_int
    L.szo_decode.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_uint32,
                             C.c_void_p, C.c_uint32, C.c_void_p]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = load(_LIB)
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed with status %d" % (what, code))
        self.code = code


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class Params:
    """Compression parameters.  ``shape`` is C-order (slowest first), as for
    a numpy array; internally n[0] is the fastest dimension."""
    shape: tuple
    eb: float = 1e-3
    eb_mode: int = EB_REL
    interp: tuple = None        # per numpy axis; default AUTO everywhere
    order: tuple = None         # processing order as numpy axes; None = auto
    alpha: float = 0.0          # <= 0: Eq. 1
    R: int = 512
    S: int = None               # default 8 (3D) / 16 (2D)
    window: tuple = None        # per numpy axis; default (8,8,32) / (16,64)
    chunk: int = 1024           # Huffman symbols per chunk

    def ndim(self):
        return len(self.shape)

    def c_struct(self) -> _Params:
        D = self.ndim()
        if D not in (1, 2, 3):
            raise ValueError("ndim must be 1, 2 or 3")
        # Sec. V-A: chunks of 8^3, 16^2 or 512 points; the window spans four
        # chunks along x and one along the other dimensions
        S = self.S or {3: 8, 2: 16, 1: 512}[D]
        win = self.window or {3: (S, S, 4 * S), 2: (S, 4 * S), 1: (4 * S,)}[D]
        interp = self.interp or (AUTO,) * D
        p = _Params()
        p.ndim = D
        p.S = S
        for ax in range(D):
            d = D - 1 - ax          # numpy axis -> dimension index (0 = fastest)
            p.n[d] = int(self.shape[ax])
            p.w[d] = int(win[ax])
            p.interp[d] = int(interp[ax])
        p.R = self.R
        p.eb_mode = self.eb_mode
        p.eb = float(self.eb)
        if self.order is None:
            for k in range(3):
                p.order[k] = -1
        else:
            for k, ax in enumerate(self.order):
                p.order[k] = D - 1 - int(ax)
        p.alpha = float(self.alpha)
        return p


@dataclass
class Config:
    vmin: float
    vmax: float
    range: float
    eps: float
    e_abs: float
    e: float
    levels: int
    alpha: float
    el: np.ndarray
    ebx2: np.ndarray
    inv: np.ndarray
    spline: tuple      # per dimension index (0 = fastest)
    order: tuple       # dimension indices
    prof: np.ndarray
    profiled: bool
    raw: _Config = field(repr=False, default=None)


def _to_config(c: _Config, D: int) -> Config:
    L = c.levels
    return Config(vmin=c.vmin, vmax=c.vmax, range=c.range, eps=c.eps, e_abs=c.e_abs, e=c.e,
                  levels=L, alpha=c.alpha,
                  el=np.array(c.el[:L], dtype=np.float32),
                  ebx2=np.array(c.ebx2[:L], dtype=np.float32),
                  inv=np.array(c.inv[:L], dtype=np.float32),
                  spline=tuple(c.spline[:D]), order=tuple(c.order[:D]),
                  prof=np.array([[c.prof[d][k] for k in range(3)] for d in range(3)]),
                  profiled=bool(c.profiled), raw=c)


def alpha(eps: float) -> float:
    return lib().szo_alpha(eps)


def round_down(v: float) -> np.float32:
    return np.float32(lib().szo_round_down(v))


def stencil(kind, a, b, c, d) -> np.float32:
    return np.float32(lib().szo_stencil(kind, a, b, c, d))


def _check_field(x: np.ndarray, p: Params):
    x = np.ascontiguousarray(x, dtype=np.float32)
    if tuple(x.shape) != tuple(p.shape):
        raise ValueError("shape mismatch")
    return x


def plan(x: np.ndarray, p: Params) -> Config:
    x = _check_field(x, p)
    cp, cc = p.c_struct(), _Config()
    rc = lib().szo_plan(_ptr(x), C.byref(cp), C.byref(cc))
    if rc:
        raise OracleError(rc, "szo_plan")
    return _to_config(cc, p.ndim())


def histogram(codes: np.ndarray, nsym: int) -> np.ndarray:
    codes = np.ascontiguousarray(codes, dtype=np.uint16).ravel()
    h = np.zeros(nsym, dtype=np.uint32)
    lib().szo_histogram(_ptr(codes), codes.size, nsym, _ptr(h))
    return h


def huffman_lengths(h: np.ndarray, lmax: int = LMAX) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.uint32)
    ln = np.zeros(h.size, dtype=np.uint8)
    rc = lib().szo_huffman_lengths(_ptr(h), h.size, lmax, _ptr(ln))
    if rc < 0:
        raise OracleError(rc, "szo_huffman_lengths")
    return ln


def canonical_codes(lengths: np.ndarray) -> np.ndarray:
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    code = np.zeros(lengths.size, dtype=np.uint32)
    lib().szo_canonical_codes(_ptr(lengths), lengths.size, _ptr(code))
    return code


def encode(sym: np.ndarray, lengths: np.ndarray, codes: np.ndarray, chunk: int):
    sym = np.ascontiguousarray(sym, dtype=np.uint16).ravel()
    n = sym.size
    nchunks = (n + chunk - 1) // chunk
    bits_cap = int(np.sum(lengths[sym].astype(np.uint64))) if n else 0
    words = np.zeros(bits_cap // 32 + nchunks + 1, dtype=np.uint32)
    cb = np.zeros(max(nchunks, 1), dtype=np.uint16)
    nw = lib().szo_encode(_ptr(sym), n, _ptr(np.ascontiguousarray(lengths, dtype=np.uint8)),
                          _ptr(np.ascontiguousarray(codes, dtype=np.uint32)), chunk,
                          _ptr(cb), _ptr(words))
    if nw == 2 ** 64 - 1:
        raise OracleError(-1, "szo_encode (symbol without code)")
    return cb[:nchunks].copy(), words[:nw].copy()


def decode(words, chunk_bits, n, chunk, lengths) -> np.ndarray:
    words = np.ascontiguousarray(words, dtype=np.uint32)
    chunk_bits = np.ascontiguousarray(chunk_bits, dtype=np.uint16)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    out = np.zeros(max(n, 1), dtype=np.uint16)
    rc = lib().szo_decode(_ptr(words), words.size, _ptr(chunk_bits), n, chunk, _ptr(lengths),
                          lengths.size, _ptr(out))
    if rc:
        raise OracleError(rc, "szo_decode")
    return out[:n]


@dataclass
class Compressed:
    params: Params
    config: Config
    anchors: np.ndarray
    codes: np.ndarray          # shaped like the field
    recon: np.ndarray          # the reconstruction the decompressor reproduces
    outlier_idx: np.ndarray
    outlier_val: np.ndarray
    hist: np.ndarray
    code_len: np.ndarray
    codewords: np.ndarray
    chunk_bits: np.ndarray
    words: np.ndarray
    cls: np.ndarray = None     # stencil class per point (optional)

    def blob(self) -> bytes:
        return serialize(self)


def compress(x: np.ndarray, p: Params, want_cls: bool = False, cfg: Config = None,
             lengths: np.ndarray = None) -> Compressed:
    """Whole pipeline: plan, traversal, histogram, codebook, chunked encode.

    lengths: a code book to use instead of the one the histogram gives
    (Sec. VI-A builds it from the histogram; any prefix code whose lengths
    cover every symbol encodes the same quant-codes)."""
    x = _check_field(x, p)
    cp = p.c_struct()
    if cfg is None:
        cfg = plan(x, p)
    N = x.size
    na = lib().szo_num_anchors(C.byref(cp))
    anchors = np.zeros(na, dtype=np.float32)
    codes = np.zeros(x.shape, dtype=np.uint16)
    recon = np.zeros(x.shape, dtype=np.float32)
    oidx = np.zeros(max(N, 1), dtype=np.uint32)
    oval = np.zeros(max(N, 1), dtype=np.float32)
    nout = C.c_uint64(0)
    cls = np.zeros(x.shape, dtype=np.uint8) if want_cls else None
    rc = lib().szo_compress(_ptr(x), C.byref(cp), C.byref(cfg.raw), _ptr(anchors), _ptr(codes),
                            _ptr(recon), _ptr(oidx), _ptr(oval), C.byref(nout),
                            _ptr(cls) if want_cls else None)
    if rc:
        raise OracleError(rc, "szo_compress")
    m = nout.value
    nsym = 2 * p.R
    h = histogram(codes, nsym)
    if lengths is None:
        ln = huffman_lengths(h)
    else:
        ln = np.ascontiguousarray(lengths, dtype=np.uint8)
        used = ln[ln > 0].astype(np.int64)
        if ln.size != nsym or np.any(ln[h > 0] == 0) or ln.max() > LMAX or \
                float(np.sum(np.ldexp(1.0, -used))) > 1.0:
            raise ValueError("code book: %d lengths of at most %d bits, one for every symbol "
                             "that occurs, with Kraft sum <= 1 needed" % (nsym, LMAX))
    cw = canonical_codes(ln)
    cb, words = encode(codes, ln, cw, p.chunk)
    return Compressed(params=p, config=cfg, anchors=anchors, codes=codes, recon=recon,
                      outlier_idx=oidx[:m].copy(), outlier_val=oval[:m].copy(), hist=h,
                      code_len=ln, codewords=cw, chunk_bits=cb, words=words, cls=cls)


def compress_windowed(x: np.ndarray, p: Params, cfg: Config):
    """Second formulation of the traversal, window by window."""
    x = _check_field(x, p)
    cp = p.c_struct()
    codes = np.zeros(x.shape, dtype=np.uint16)
    recon = np.zeros(x.shape, dtype=np.float32)
    rc = lib().szo_compress_windowed(_ptr(x), C.byref(cp), C.byref(cfg.raw), _ptr(codes),
                                     _ptr(recon))
    if rc:
        raise OracleError(rc, "szo_compress_windowed")
    return codes, recon


def decompress_parts(p: Params, cfg: Config, anchors, codes, oidx, oval) -> np.ndarray:
    cp = p.c_struct()
    out = np.zeros(p.shape, dtype=np.float32)
    anchors = np.ascontiguousarray(anchors, dtype=np.float32)
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    oidx = np.ascontiguousarray(oidx, dtype=np.uint32)
    oval = np.ascontiguousarray(oval, dtype=np.float32)
    rc = lib().szo_decompress(C.byref(cp), C.byref(cfg.raw), _ptr(anchors), _ptr(codes),
                              _ptr(oidx), _ptr(oval), oidx.size, _ptr(out))
    if rc:
        raise OracleError(rc, "szo_decompress")
    return out


# ---------------------------------------------------------------- blob format
_HEADER = struct.Struct("<4sIII3Q3IIIIII dd fff 3i 3i I 16f QQQQ 6I I I")
assert _HEADER.size == 256


def _pad8(b: bytes) -> bytes:
    return b + b"\0" * ((-len(b)) % 8)


FLAG_WORDS_ELIDED = 1


def elide_zero_words(words: np.ndarray):
    """The Huffman words without their zero words: a bitmap of u32 words,
    bit k % 32 of bitmap word k // 32 set when word k is non-zero, followed
    by the non-zero words in order.  Returns that array when it is shorter
    than the words themselves, else None (the words are stored as they are).
    An open stand-in for the closed de-redundancy pass that follows Huffman
    coding in the paper (Sec. VI-B); runs of zero words are what a smooth
    field's one-bit centre code leaves."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    nbm = (w.size + 31) // 32
    nz = w != 0
    if nbm + int(nz.sum()) >= w.size:
        return None
    flags = np.zeros(nbm * 32, dtype=np.uint64)
    flags[:w.size] = nz
    weights = np.left_shift(np.uint64(1), np.arange(32, dtype=np.uint64))
    bitmap = (flags.reshape(nbm, 32) * weights).sum(axis=1).astype(np.uint32)
    return np.concatenate([bitmap, w[nz]])


def restore_zero_words(section: np.ndarray, n_words: int) -> np.ndarray:
    """Inverse of elide_zero_words; raises on a malformed section."""
    sec = np.ascontiguousarray(section, dtype=np.uint32)
    nbm = (n_words + 31) // 32
    if sec.size < nbm:
        raise OracleError(-5, "restore_zero_words (bitmap)")
    bits = ((sec[:nbm, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(bool).ravel()
    if bits[n_words:].any():
        raise OracleError(-5, "restore_zero_words (bits past the words)")
    pos = np.flatnonzero(bits[:n_words])
    vals = sec[nbm:]
    if vals.size != pos.size or (vals == 0).any():
        raise OracleError(-5, "restore_zero_words (values)")
    w = np.zeros(n_words, dtype=np.uint32)
    w[pos] = vals
    return w


def serialize(c: Compressed) -> bytes:
    p, cfg = c.params, c.config
    cp = p.c_struct()
    D = p.ndim()
    el = list(cfg.el) + [0.0] * (16 - cfg.levels)
    elided = elide_zero_words(c.words)
    wsec = c.words if elided is None else elided
    sections = [c.anchors.astype("<f4").tobytes(), c.code_len.astype(np.uint8).tobytes(),
                c.chunk_bits.astype("<u2").tobytes(), wsec.astype("<u4").tobytes(),
                c.outlier_idx.astype("<u4").tobytes(), c.outlier_val.astype("<f4").tobytes()]
    crcs = [zlib.crc32(s) & 0xFFFFFFFF for s in sections]
    spline = list(cfg.spline) + [0] * (3 - D)
    order = list(cfg.order) + [-1] * (3 - D)
    fields = ([MAGIC, VERSION, D, cp.S] + [cp.n[i] for i in range(3)] +
              [cp.w[i] for i in range(3)] + [p.R, LMAX, p.chunk, p.eb_mode, cfg.levels] +
              [float(p.eb), float(cfg.alpha), cfg.vmin, cfg.vmax, cfg.e] + spline + order +
              [0 if elided is None else FLAG_WORDS_ELIDED] + el +
              [c.anchors.size, c.chunk_bits.size, c.words.size,
                          c.outlier_idx.size] + crcs + [0, 0])
    head = bytearray(_HEADER.pack(*fields))
    struct.pack_into("<I", head, 252, zlib.crc32(bytes(head[:252])) & 0xFFFFFFFF)
    return bytes(head) + b"".join(_pad8(s) for s in sections)


def parse(blob: bytes) -> dict:
    """Header fields and sections of a blob, with both CRC levels checked."""
    if len(blob) < 256:
        raise OracleError(-5, "parse (short blob)")
    head = blob[:256]
    if zlib.crc32(head[:252]) & 0xFFFFFFFF != struct.unpack_from("<I", head, 252)[0]:
        raise OracleError(-5, "parse (header crc)")
    f = _HEADER.unpack(head)
    if f[0] != MAGIC or f[1] != VERSION:
        raise OracleError(-5, "parse (magic)")
    flags = struct.unpack_from("<I", head, 124)[0]
    if flags & ~FLAG_WORDS_ELIDED or struct.unpack_from("<I", head, 248)[0]:
        raise OracleError(-5, "parse (reserved words)")
    i = 0
    out = {}
    names = ["magic", "version", "ndim", "S", "n0", "n1", "n2", "w0", "w1", "w2", "R", "lmax",
             "chunk", "eb_mode", "levels", "eb", "alpha", "vmin", "vmax", "e", "sp0", "sp1", "sp2",
             "or0", "or1", "or2", "res0"] + ["el%d" % k for k in range(16)] + \
            ["n_anchors", "n_chunks", "n_words", "n_outliers"] + ["crc%d" % k for k in range(6)] + \
            ["res1", "hcrc"]
    for nm, v in zip(names, f):
        out[nm] = v
    sizes = [(out["n_anchors"], "<f4"), (2 * out["R"], np.uint8), (out["n_chunks"], "<u2"),
             (out["n_words"], "<u4"), (out["n_outliers"], "<u4"), (out["n_outliers"], "<f4")]
    pos = 256
    secs = []
    for k, (cnt, dt) in enumerate(sizes):
        if k == 3 and flags & FLAG_WORDS_ELIDED:
            # bitmap, then one word per set bit
            nbm = (int(cnt) + 31) // 32
            bm = np.frombuffer(blob[pos:pos + 4 * nbm], dtype="<u4")
            if bm.size != nbm:
                raise OracleError(-5, "parse (bitmap)")
            cnt = nbm + int(sum(bin(int(v)).count("1") for v in bm))
        nb = int(cnt) * np.dtype(dt).itemsize
        raw = blob[pos:pos + nb]
        if len(raw) != nb or zlib.crc32(raw) & 0xFFFFFFFF != out["crc%d" % k]:
            raise OracleError(-5, "parse (section %d crc)" % k)
        if any(blob[pos + nb:pos + nb + ((-nb) % 8)]):
            raise OracleError(-5, "parse (section %d padding)" % k)
        secs.append(np.frombuffer(raw, dtype=dt).copy())
        pos += nb + ((-nb) % 8)
    if pos != len(blob):
        raise OracleError(-5, "parse (length)")
    if flags & FLAG_WORDS_ELIDED:
        secs[3] = restore_zero_words(secs[3], int(out["n_words"]))
    out["anchors"], out["code_len"], out["chunk_bits"], out["words"], out["outlier_idx"], \
        out["outlier_val"] = secs
    out["flags"] = flags
    return out


def decompress_blob(blob: bytes) -> np.ndarray:
    """Decode a blob from either implementation with the oracle alone."""
    h = parse(blob)
    D = h["ndim"]
    n = [h["n0"], h["n1"], h["n2"]][:D]
    shape = tuple(reversed(n))
    N = int(np.prod(n))
    codes = decode(h["words"], h["chunk_bits"], N, h["chunk"], h["code_len"])
    p = Params(shape=shape, eb=h["eb"], eb_mode=h["eb_mode"], R=h["R"], S=h["S"],
               window=tuple(reversed([h["w0"], h["w1"], h["w2"]][:D])), chunk=h["chunk"])
    cp = p.c_struct()
    cc = _Config()
    cc.levels = h["levels"]
    for l in range(h["levels"]):
        el = np.float32(h["el%d" % l])
        cc.el[l] = el
        cc.ebx2[l] = np.float32(2.0) * el
    for d in range(D):
        cc.spline[d] = [h["sp0"], h["sp1"], h["sp2"]][d]
        cc.order[d] = [h["or0"], h["or1"], h["or2"]][d]
    out = np.zeros(shape, dtype=np.float32)
    rc = lib().szo_decompress(C.byref(cp), C.byref(cc), _ptr(h["anchors"]),
                              _ptr(np.ascontiguousarray(codes.reshape(shape))),
                              _ptr(h["outlier_idx"]), _ptr(h["outlier_val"]),
                              h["outlier_idx"].size, _ptr(out))
    if rc:
        raise OracleError(rc, "szo_decompress")
    return out


def psnr(x: np.ndarray, y: np.ndarray) -> float:
    """Value-range PSNR: 20 log10(range) - 10 log10(MSE), FP64."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    rng = float(x.max() - x.min())
    mse = float(np.mean((x - y) ** 2))
    if mse == 0.0:
        return float("inf")
    if rng == 0.0:
        return float("-inf")
    return 20.0 * np.log10(rng) - 10.0 * np.log10(mse)
