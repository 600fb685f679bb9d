"""Compression with a caller's code book on the GPU (sz_compress_with_code),
bit-exact with the oracle given the same book: every section, the blob and
both decompressions.  Includes a field with more outliers than the first
outlier allocation, which the call finds at its end and encodes again."""
import numpy as np
import pytest

import oracle as O
import paper_2312_05492_amd as szi
from paper_2312_05492_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    c = szi.Context(0)
    yield c
    c.close()


def _gpu(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def _check(ctx, x, book, kw):
    m = dict(kw)
    if "radius" in m:
        m["R"] = m.pop("radius")
    print("\n[given code] shape=%s params=%s" % (x.shape, kw), flush=True)
    ref = O.compress(x, O.Params(shape=x.shape, **m), lengths=book)
    res = ctx.compress_with_code(_gpu(x), book, **kw)
    try:
        assert np.array_equal(res.read(szi.SEC_CODES), ref.codes.ravel()), "codes"
        assert np.array_equal(res.read(szi.SEC_HIST), ref.hist), "histogram"
        assert np.array_equal(res.read(szi.SEC_CODE_LEN), book), "code lengths"
        assert res.n_outliers == ref.outlier_idx.size
        assert np.array_equal(res.read(szi.SEC_OUTLIER_IDX), ref.outlier_idx), "outlier idx"
        assert np.array_equal(_bits(res.read(szi.SEC_OUTLIER_VAL)), _bits(ref.outlier_val))
        assert np.array_equal(res.read(szi.SEC_CHUNK_BITS), ref.chunk_bits), "chunk bits"
        assert np.array_equal(res.read(szi.SEC_WORDS), ref.words), "huffman words"
        assert res.blob() == ref.blob(), "blob"
        y = ctx.decompress(res).cpu().numpy()
        assert np.array_equal(_bits(y), _bits(ref.recon)), "decompressed field"
        assert np.array_equal(_bits(O.decompress_blob(res.blob())), _bits(ref.recon))
    finally:
        res.free()
    return ref


def test_book_of_another_field(ctx):
    a = synth.spectral_field((40, 56, 72), seed=41, mean=3.0)
    b = synth.spectral_field((40, 56, 72), seed=42, beta=3.0)
    other = ctx.compress(_gpu(b))
    book = szi.code_lengths(other.read(szi.SEC_HIST))
    other.free()
    ref = _check(ctx, a, book, {})
    # the same quant-codes as with the field's own book
    own = O.compress(a, O.Params(shape=a.shape))
    assert np.array_equal(ref.codes, own.codes)


def test_book_of_the_field_itself_2d(ctx):
    x = synth.climate_field(901, shape=(150, 260))
    first = ctx.compress(_gpu(x))
    book = szi.code_lengths(first.read(szi.SEC_HIST))
    first.free()
    _check(ctx, x, book, {})


def test_more_outliers_than_the_first_guess(ctx):
    # radius 2: almost every point of a rough field is an outlier, far more
    # than the n / 32 the lists first get
    rng = np.random.default_rng(7)
    x = rng.standard_normal((48, 48, 64)).astype(np.float32)
    book = np.array([2, 2, 2, 2], dtype=np.uint8)
    ref = _check(ctx, x, book, dict(radius=2, eb=1e-4))
    assert ref.outlier_idx.size > x.size // 32


def test_incomplete_book_rejected(ctx):
    x = synth.spectral_field((16, 16, 40), seed=43)
    book = np.full(1024, 10, dtype=np.uint8)
    book[5] = 0
    with pytest.raises(szi.SzError) as e:
        ctx.compress_with_code(_gpu(x), book)
    assert e.value.code == -1
    book[5] = 25
    with pytest.raises(szi.SzError):
        ctx.compress_with_code(_gpu(x), book)
    with pytest.raises(szi.SzError):
        ctx.compress_with_code(_gpu(x), np.full(1024, 9, dtype=np.uint8))   # Kraft sum 2


def test_nonfinite_rejected_with_book(ctx):
    x = synth.spectral_field((16, 16, 40), seed=44)
    x[3, 4, 5] = np.nan
    with pytest.raises(szi.SzError) as e:
        ctx.compress_with_code(_gpu(x), np.full(1024, 10, dtype=np.uint8))
    assert e.value.code == -2


def test_book_with_graph_mode_on(ctx):
    # a given code book runs the plain launch path even when the context
    # replays graphs; the result is the same
    x = synth.spectral_field((24, 40, 72), seed=45, mean=1.0)
    first = ctx.compress(_gpu(x))
    book = szi.code_lengths(first.read(szi.SEC_HIST))
    first.free()
    a = ctx.compress_with_code(_gpu(x), book)
    ctx.set_graphs(True)
    try:
        b = ctx.compress_with_code(_gpu(x), book)
        c = ctx.compress(_gpu(x))   # a graph replay in between
        d = ctx.compress_with_code(_gpu(x), book)
        assert a.blob() == b.blob() == d.blob()
        c.free()
        b.free()
        d.free()
    finally:
        ctx.set_graphs(False)
        a.free()
