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
    # a given code book replays both graphs back to back; the result is the
    # plain path's
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


def _batch_case():
    xs = [synth.spectral_field((40, 56, 72), seed=46, mean=3.0),
          synth.climate_field(902, shape=(150, 260)),
          synth.spectral_field((33, 47, 65), seed=47, beta=3.0),
          synth.spectral_field((30, 40, 50), seed=48)]
    kws = [{}, {}, dict(eb=1e-4), dict(radius=64, chunk=256)]
    return xs, kws


@pytest.mark.parametrize("graphs", [False, True])
def test_batch_with_given_books(ctx, graphs):
    """sz_compress_batch_with_code: every field's blob is the oracle's with
    the same book, and the single call's; one field takes another field's
    book, one its own, one has more outliers than the first lists hold."""
    xs, kws = _batch_case()
    books = []
    for x, kw in zip(xs, kws):
        r = ctx.compress(_gpu(x), **kw)
        books.append(szi.code_lengths(r.read(szi.SEC_HIST)))
        r.free()
    books[0], books[2] = books[2].copy(), books[0].copy()   # both R = 512
    # radius 2 on a rough field: nearly every point an outlier
    rng = np.random.default_rng(9)
    xs.append(rng.standard_normal((24, 32, 48)).astype(np.float32))
    kws.append(dict(radius=2, eb=1e-4))
    books.append(np.array([2, 2, 2, 2], dtype=np.uint8))
    refs = []
    for x, kw, book in zip(xs, kws, books):
        m = dict(kw)
        if "radius" in m:
            m["R"] = m.pop("radius")
        refs.append(O.compress(x, O.Params(shape=x.shape, **m), lengths=book).blob())
    print("\n[given books batch] graphs=%s fields=%d" % (graphs, len(xs)), flush=True)
    ctx.set_graphs(graphs)
    try:
        for rep in range(3):   # graph capture, then replays
            res = ctx.compress_batch_with_code([_gpu(x) for x in xs], books, kws)
            try:
                for k, (r, ref) in enumerate(zip(res, refs)):
                    assert r.blob() == ref, (rep, k)
                y = ctx.decompress(res[1]).cpu().numpy()
                assert np.array_equal(_bits(y), _bits(O.decompress_blob(refs[1])))
            finally:
                for r in res:
                    r.free()
        one = ctx.compress_with_code(_gpu(xs[3]), books[3], **kws[3])
        assert one.blob() == refs[3]
        one.free()
    finally:
        ctx.set_graphs(False)


def test_server_resident_books(ctx):
    """Requests naming a resident book: the first ones build it, the later
    ones use it (every code then has a length, which only a book made by
    sz_code_lengths gives); each blob is the oracle's with the lengths it
    holds, and decompresses to the plain reconstruction."""
    import torch
    fields = [synth.spectral_field((40, 48, 64), seed=80 + k, mean=5.0) for k in range(4)]
    xs = [_gpu(f) for f in fields]
    plain = [O.compress(f, O.Params(shape=f.shape)) for f in fields]
    srv = szi.Server(0, slots=4)
    try:
        for i in range(12):
            srv.submit_compress(xs[i % 4], tag=i, book=1)
        got = []
        while len(got) < 12:
            comp = srv.poll(wait=True)
            assert comp, "server stalled"
            got.extend(comp)
        used = 0
        for c in got:
            assert c["status"] == 0
            r = c["result"]
            k = c["tag"] % 4
            lens = r.read(szi.SEC_CODE_LEN)
            used += int(np.all(lens > 0))
            ref = O.compress(fields[k], O.Params(shape=fields[k].shape), lengths=lens)
            assert r.blob() == ref.blob(), c["tag"]
            out = torch.empty_like(xs[k])
            ctx.decompress(r, out)
            assert np.array_equal(_bits(out.cpu().numpy()), _bits(plain[k].recon))
            r.free()
        print("\n[server books] %d of 12 results used the resident book" % used, flush=True)
        # requests 5..12 wait for a free slot, so a completion (and its book)
        # came before each of them
        assert used >= 8
    finally:
        srv.close()
