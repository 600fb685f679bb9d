"""Zero-word elision of the blob's Huffman words on the GPU path: the flag,
the section and the blob bytes equal the oracle's; elided blobs upload,
decompress and serialize again to the same bytes.  A smooth 2D field (the
centre code takes one bit, so most words are zero) elides; a rough 3D
field keeps its words as they are."""
import struct

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


def _flags(blob):
    return struct.unpack_from("<I", blob, 124)[0]


@pytest.mark.parametrize("name,gen,kw,elided", [
    ("climate_smooth", lambda: synth.climate_field(911, shape=(360, 720)), dict(eb=1e-3), True),
    ("climate_e2", lambda: synth.climate_field(912, shape=(200, 300)), dict(eb=1e-2), True),
    ("spectral_rough", lambda: synth.spectral_field((48, 64, 80), seed=913), dict(eb=1e-3), False),
])
def test_elision_matches_oracle(ctx, name, gen, kw, elided):
    x = gen()
    print("\n[elision] %s shape=%s %s" % (name, x.shape, kw), flush=True)
    ref = O.compress(x, O.Params(shape=x.shape, **kw))
    res = ctx.compress(_gpu(x), **kw)
    try:
        blob = res.blob()
        assert _flags(blob) == (O.FLAG_WORDS_ELIDED if elided else 0)
        assert blob == ref.blob()
        assert res.compressed_bytes == len(blob)
        assert _flags(res.header()) == _flags(blob)
        if elided:   # smaller than the words as they are
            assert len(blob) < 256 + 4 * res.read(szi.SEC_WORDS).size
        up = ctx.upload(blob)
        try:
            assert np.array_equal(up.read(szi.SEC_WORDS), ref.words)
            assert up.blob() == blob
            y = ctx.decompress(up).cpu().numpy()
            assert np.array_equal(y.view(np.uint32), ref.recon.view(np.uint32))
        finally:
            up.free()
    finally:
        res.free()


def test_large_elided_blob_in_large_tiles(ctx):
    """A smooth 8000 x 9600 field whose words (about 2.4 M) exceed the bound
    below which the elision and the upload's restore use 2048-word tiles: the
    blob, the restored words and the reconstruction equal the oracle's with
    8192-word tiles on both sides."""
    x = synth.climate_field(931, shape=(8000, 9600))
    print("\n[elision large] shape=%s" % (x.shape,), flush=True)
    ref = O.compress(x, O.Params(shape=x.shape, eb=1e-3))
    assert ref.words.size >= 1024 * 2048   # the large tiles
    res = ctx.compress(_gpu(x), eb=1e-3)
    try:
        blob = res.blob()
        assert _flags(blob) == O.FLAG_WORDS_ELIDED
        assert blob == ref.blob()
        up = ctx.upload(blob)
        try:
            assert np.array_equal(up.read(szi.SEC_WORDS), ref.words)
            y = ctx.decompress(up).cpu().numpy()
            assert np.array_equal(y.view(np.uint32), ref.recon.view(np.uint32))
        finally:
            up.free()
    finally:
        res.free()


def test_elided_blob_with_a_flipped_bitmap_bit_is_rejected(ctx):
    x = synth.climate_field(914, shape=(120, 240))
    res = ctx.compress(_gpu(x))
    blob = bytearray(res.blob())
    res.free()
    assert _flags(blob) == O.FLAG_WORDS_ELIDED
    h = O.parse(bytes(blob))
    at = 256 + sum((n + (-n) % 8) for n in (4 * h["n_anchors"], 2 * h["R"], 2 * h["n_chunks"]))
    blob[at] ^= 0x02
    with pytest.raises(szi.SzError) as e:
        ctx.upload(bytes(blob))
    assert e.value.code == -5


@pytest.mark.parametrize("graphs", [False, True])
def test_batch_elision_mixed_fields(ctx, graphs):
    """One elision launch covers every field of a batch: fields that elide
    and fields that keep their words, most spanning several tiles (of 2048
    words at these sizes), give the oracle's blobs; elided ones restore on
    upload."""
    xs = [synth.climate_field(921, shape=(900, 1800)),
          synth.spectral_field((40, 56, 72), seed=922),
          synth.climate_field(923, shape=(700, 1200)),
          synth.climate_field(924, shape=(7, 9))]
    kws = [dict(eb=1e-3), dict(eb=1e-3), dict(eb=1e-2), dict(eb=1e-3)]
    refs = [O.compress(x, O.Params(shape=x.shape, **kw)) for x, kw in zip(xs, kws)]
    assert [_flags(r.blob()) for r in refs[:3]] == [O.FLAG_WORDS_ELIDED, 0, O.FLAG_WORDS_ELIDED]
    print("\n[elision batch] graphs=%s shapes=%s" % (graphs, [x.shape for x in xs]), flush=True)
    ctx.set_graphs(graphs)
    try:
        for rep in range(2):
            res = ctx.compress_batch([_gpu(x) for x in xs], kws)
            try:
                for x, ref, r in zip(xs, refs, res):
                    blob = r.blob()
                    assert blob == ref.blob(), (rep, x.shape)
                    up = ctx.upload(blob)
                    try:
                        assert np.array_equal(up.read(szi.SEC_WORDS), ref.words)
                    finally:
                        up.free()
            finally:
                for r in res:
                    r.free()
    finally:
        ctx.set_graphs(False)
