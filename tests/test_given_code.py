"""Compression with a caller's code book (host side and oracle; CPU only).

sz_code_lengths (host code of the library, no GPU work) must give the
oracle's length-limited Huffman lengths of the counts plus one; the
oracle's compression with a given code book must equal its own pipeline
when the book is the histogram's, and round-trip with any other complete
prefix code."""
import numpy as np
import pytest

import oracle as O
import paper_2312_05492_amd as szi
from paper_2312_05492_amd import synth


def test_code_lengths_are_the_oracle_lengths_of_counts_plus_one():
    rng = np.random.default_rng(11)
    for t in range(200):
        nsym = int(rng.choice([4, 64, 1024, 2048]))
        h = np.zeros(nsym, dtype=np.uint32)
        k = int(rng.integers(0, nsym + 1))
        idx = rng.choice(nsym, size=k, replace=False)
        h[idx] = rng.integers(1, [5, 1000, 1 << 30][t % 3], size=k).astype(np.uint32)
        got = szi.code_lengths(h)
        want = O.huffman_lengths(h.astype(np.uint64).clip(0, 2**32 - 2).astype(np.uint32) + 1)
        assert np.array_equal(got, want), "histogram %d" % t
        assert got.min() >= 1 and got.max() <= O.LMAX
        assert np.sum(np.ldexp(1.0, -got.astype(np.int64))) <= 1.0


def test_code_lengths_rejects_bad_sizes():
    with pytest.raises(szi.SzError):
        szi.code_lengths(np.zeros(1, dtype=np.uint32))
    with pytest.raises(szi.SzError):
        szi.code_lengths(np.zeros(4096, dtype=np.uint32))


@pytest.fixture(scope="module")
def fields():
    O.build(force=False)
    a = synth.spectral_field((24, 32, 40), seed=31, mean=5.0)
    b = synth.spectral_field((24, 32, 40), seed=32, beta=3.0)
    return a, b


def test_oracle_given_own_book_equals_pipeline(fields):
    a, _ = fields
    p = O.Params(shape=a.shape)
    ref = O.compress(a, p)
    got = O.compress(a, p, lengths=ref.code_len)
    assert got.blob() == ref.blob()


def test_oracle_given_other_book_round_trips(fields):
    a, b = fields
    p = O.Params(shape=a.shape)
    other = O.compress(b, p)
    book = O.huffman_lengths(other.hist + 1)
    got = O.compress(a, p, lengths=book)
    ref = O.compress(a, p)
    # the same quant-codes and reconstruction, another bitstream
    assert np.array_equal(got.codes, ref.codes)
    assert np.array_equal(got.code_len, book)
    assert np.array_equal(O.decode(got.words, got.chunk_bits, a.size, p.chunk, book),
                          got.codes.ravel())
    y = O.decompress_blob(got.blob())
    assert np.array_equal(y.view(np.uint32), ref.recon.view(np.uint32))


def test_oracle_rejects_incomplete_book(fields):
    a, _ = fields
    p = O.Params(shape=a.shape)
    book = np.full(2 * p.R, 10, dtype=np.uint8)
    book[p.R] = 0   # the centre code occurs (anchors take it)
    with pytest.raises(ValueError):
        O.compress(a, p, lengths=book)
    book[p.R] = 25
    with pytest.raises(ValueError):
        O.compress(a, p, lengths=book)
    with pytest.raises(ValueError):
        O.compress(a, p, lengths=np.full(2 * p.R, 9, dtype=np.uint8))   # Kraft sum 2
