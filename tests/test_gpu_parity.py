"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact for everything: anchors, quant-codes, outlier lists, histogram,
code lengths, chunk bit counts, Huffman words, the serialized blob, and the
decompressed field.  Runs on an MI355X only (marker ``gpu``)."""
import math
import sys

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


def _to_gpu(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _oracle_params(shape, kw):
    m = dict(kw)
    if "radius" in m:
        m["R"] = m.pop("radius")
    return O.Params(shape=shape, **m)


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def check_case(ctx, name, x, kw):
    print("\n[parity] %s shape=%s params=%s" % (name, x.shape, kw), flush=True)
    ref = O.compress(x, _oracle_params(x.shape, kw))
    res = ctx.compress(_to_gpu(x), **kw)
    try:
        # section by section first, for a readable failure
        assert np.array_equal(res.read(szi.SEC_ANCHORS), ref.anchors), "anchors"
        codes = res.read(szi.SEC_CODES)
        want = ref.codes.ravel()
        if not np.array_equal(codes, want):
            bad = np.flatnonzero(codes != want)
            raise AssertionError("codes differ at %d points, first %s: gpu %s oracle %s" % (
                bad.size, np.unravel_index(bad[:5], x.shape), codes[bad[:5]], want[bad[:5]]))
        assert np.array_equal(res.read(szi.SEC_HIST), ref.hist), "histogram"
        assert np.array_equal(res.read(szi.SEC_CODE_LEN), ref.code_len), "code lengths"
        assert np.array_equal(res.read(szi.SEC_OUTLIER_IDX), ref.outlier_idx), "outlier idx"
        assert np.array_equal(_bits(res.read(szi.SEC_OUTLIER_VAL)), _bits(ref.outlier_val)), \
            "outlier values"
        assert np.array_equal(res.read(szi.SEC_CHUNK_BITS), ref.chunk_bits), "chunk bits"
        assert np.array_equal(res.read(szi.SEC_WORDS), ref.words), "huffman words"
        blob = res.blob()
        oblob = ref.blob()
        if blob != oblob:
            diff = [i for i in range(min(len(blob), len(oblob))) if blob[i] != oblob[i]][:8]
            raise AssertionError("blobs differ (len %d vs %d) at bytes %s" % (
                len(blob), len(oblob), diff))
        # decompression replays the oracle's reconstruction bit for bit
        y = ctx.decompress(res).cpu().numpy()
        assert np.array_equal(_bits(y), _bits(ref.recon)), "decompressed field"
        err = np.abs(y.astype(np.float64) - x.astype(np.float64)).max() if x.size else 0.0
        assert err <= float(ref.config.el[0])
        # the oracle's blob decompresses on the GPU; the GPU blob in the oracle
        up = ctx.upload(oblob)
        y2 = ctx.decompress(up).cpu().numpy()
        up.free()
        assert np.array_equal(_bits(y2), _bits(ref.recon)), "decompress of the oracle blob"
        y3 = O.decompress_blob(blob)
        assert np.array_equal(_bits(y3), _bits(ref.recon)), "oracle decode of the gpu blob"
    finally:
        res.free()
    return ref


def _spec(shape, seed, beta=5.0 / 3.0, mean=0.0):
    return lambda: synth.spectral_field(shape, beta=beta, seed=seed, mean=mean)


def _const(shape, v):
    return lambda: np.full(shape, v, dtype=np.float32)


def _signed_zeros(shape, seed):
    def gen():
        rng = np.random.default_rng(seed)
        return np.where(rng.random(shape) < 0.5, np.float32(-0.0), np.float32(0.0)).astype(np.float32)
    return gen


CASES = [
    ("small64_bumps", synth.workload_small, {}),
    ("odd_17_33_65", _spec((17, 33, 65), 3), {}),
    ("ragged_100_37_53_e4", _spec((100, 37, 53), 4, mean=10.0), dict(eb=1e-4)),
    ("linear_all", _spec((40, 48, 70), 5), dict(interp=(0, 0, 0))),
    ("mixed_zlin", _spec((40, 48, 70), 5), dict(interp=(0, 3, 3))),
    ("nak_order_xyz", _spec((24, 40, 66), 6), dict(interp=(1, 1, 1), order=(2, 1, 0))),
    ("natural", _spec((24, 40, 66), 6, beta=3.0), dict(interp=(2, 2, 2))),
    ("abs_bound", _spec((31, 29, 47), 7), dict(eb=0.01, eb_mode=0)),
    ("alpha_one", _spec((31, 29, 47), 7), dict(eb=1e-2, alpha=1.0)),
    ("eb_1e2", _spec((31, 29, 47), 8, beta=3.0), dict(eb=1e-2)),
    ("tiny_bound_all_outliers", _spec((19, 21, 37), 9), dict(eb=1e-30, eb_mode=0)),
    ("zero_bound", _spec((19, 21, 37), 9), dict(eb=0.0, eb_mode=0)),
    ("constant_zero_range", _const((20, 30, 40), 2.5), {}),
    ("constant_abs0", _const((20, 30, 40), 3.0), dict(eb=0.0, eb_mode=0)),
    ("denormal_values", lambda: (synth.spectral_field((18, 20, 40), seed=10) * np.float32(1e-40)),
     dict(eb=1e-44, eb_mode=0)),
    ("radius_64", _spec((30, 30, 60), 11, beta=1.0), dict(eb=1e-4, radius=64)),
    # odd radii: the decode tables start off a 16-byte boundary in the result
    ("radius_odd_37", _spec((30, 30, 60), 15, beta=1.0), dict(eb=1e-4, radius=37)),
    ("radius_odd_3", _spec((24, 40, 50), 16, beta=1.0), dict(eb=1e-3, radius=3)),
    ("chunk_256", _spec((30, 30, 60), 12), dict(chunk=256)),
    ("chunk_2048", _spec((30, 30, 60), 12), dict(chunk=2048)),
    ("thin_1x9x100", _spec((1, 9, 100), 13), {}),
    ("line_1x1x3000", _spec((1, 1, 3000), 14), {}),
    ("column_70x1x1", _spec((70, 1, 1), 15), {}),
    ("single_point_3d", _const((1, 1, 1), 1.5), {}),
    ("multi_window_33_17_129", _spec((33, 17, 129), 16), {}),
    ("front_3d", lambda: synth.front_field((30, 40, 50), seed=17), dict(eb=1e-2)),
    ("climate_2d", lambda: synth.climate_field(301, shape=(90, 180)), {}),
    ("spectral_2d_e4", _spec((77, 131), 18, beta=3.0), dict(eb=1e-4)),
    ("line_2d_1x5000", _spec((1, 5000), 19), {}),
    ("column_2d_300x1", _spec((300, 1), 20), {}),
    ("single_point_2d", _const((1, 1), -4.0), {}),
    ("linear_2d", _spec((65, 129), 21), dict(interp=(0, 0))),
    # natural cubic on values near 1e-38: numerators below 2^-123 take the
    # exact division instead of the reciprocal multiply
    ("natural_tiny_values", lambda: synth.spectral_field((30, 40, 70), seed=22) * np.float32(1e-38),
     dict(interp=(2, 2, 2), eb=2e-39, eb_mode=0)),
    ("natural_tiny_2d", lambda: synth.spectral_field((70, 140), seed=24) * np.float32(3e-38),
     dict(interp=(2, 2), eb=2e-39, eb_mode=0)),
    # +0 and -0 mixed: the sign of zero survives prediction and quantisation
    ("signed_zeros_zero_bound", _signed_zeros((20, 24, 40), 23),
     dict(interp=(2, 2, 2), eb=0.0, eb_mode=0)),
    ("signed_zeros_abs_bound", _signed_zeros((20, 24, 40), 25),
     dict(interp=(1, 2, 0), eb=0.5, eb_mode=0)),
    # Huffman codes up to the 24-bit length limit, decoded past the look-up
    # table (Fibonacci code counts give the deepest tree; the oracle pins
    # check the lengths)
    ("long_codes_3d", lambda: synth.fib_spikes((100, 100, 100)),
     dict(interp=(0, 0, 0), eb=0.5, eb_mode=0)),
    ("long_codes_2d", lambda: synth.fib_spikes((700, 700), seed=27),
     dict(interp=(0, 0), eb=0.5, eb_mode=0)),
    # 1D fields (Sec. V-A: anchors every 512 points, windows of 2048)
    ("line1d_100003", _spec((100003,), 40, mean=10.0), {}),
    ("line1d_e4_nat", _spec((65537,), 41, beta=3.0), dict(eb=1e-4, interp=(2,))),
    ("line1d_linear", _spec((4097,), 42), dict(interp=(0,))),
    ("line1d_nak_e2", _spec((20000,), 43), dict(eb=1e-2, interp=(1,))),
    ("line1d_short_700", _spec((700,), 44), {}),
    ("line1d_exact_window_2048", _spec((2048,), 45), {}),
    ("line1d_2049", _spec((2049,), 46), {}),
    ("line1d_single", _const((1,), 2.0), {}),
    ("line1d_tiny_bound", _spec((5000,), 47), dict(eb=1e-30, eb_mode=0)),
    ("line1d_zero_bound_signed", _signed_zeros((3000,), 48), dict(eb=0.0, eb_mode=0)),
    ("line1d_radius_odd", _spec((30000,), 49, beta=1.0), dict(eb=1e-4, radius=37, chunk=256)),
    # other windows and strides (Sec. V-D): the generic window kernels
    ("window3d_16x16x8", _spec((40, 50, 70), 60, mean=3.0), dict(window=(16, 16, 8))),
    ("window3d_8x8x48_e4", _spec((33, 41, 130), 61), dict(eb=1e-4, window=(8, 8, 48))),
    ("stride4_3d", _spec((30, 37, 45), 62, beta=3.0), dict(S=4, interp=(2, 1, 0))),
    ("stride2_3d", _spec((17, 20, 31), 63), dict(S=2, eb=1e-2)),
    ("window2d_32x32", _spec((100, 130), 64), dict(window=(32, 32))),
    ("stride8_2d", _spec((90, 77), 65, beta=3.0), dict(S=8, eb=1e-4)),
    ("window1d_512", _spec((30001,), 66), dict(window=(512,))),
    ("stride64_1d", _spec((10000,), 67, beta=3.0), dict(S=64, eb=1e-4, interp=(2,))),
    ("window3d_tiny_bound", _spec((20, 24, 40), 68), dict(window=(16, 8, 16), eb=1e-30, eb_mode=0)),
]


@pytest.mark.parametrize("name,gen,kw", CASES, ids=[c[0] for c in CASES])
def test_parity(ctx, name, gen, kw):
    check_case(ctx, name, gen(), kw)


def test_batch_equals_single_calls(ctx):
    fields = [synth.spectral_field((20, 30, 70), seed=31), synth.climate_field(302, shape=(60, 130)),
              synth.spectral_field((9, 17, 33), seed=32, beta=3.0),
              synth.spectral_field((50, 70), seed=33)]
    params = [dict(eb=1e-3), dict(eb=1e-4), dict(eb=1e-2, interp=(0, 3, 3)), dict(eb=0.05, eb_mode=0)]
    print("\n[parity] batch of %d fields" % len(fields), flush=True)
    outs = ctx.compress_batch([_to_gpu(f) for f in fields], params)
    for f, kw, r in zip(fields, params, outs):
        ref = O.compress(f, _oracle_params(f.shape, kw))
        assert r.blob() == ref.blob()
    ys = ctx.decompress_batch(outs)
    for f, kw, y in zip(fields, params, ys):
        ref = O.compress(f, _oracle_params(f.shape, kw))
        assert np.array_equal(_bits(y.cpu().numpy()), _bits(ref.recon))
    for r in outs:
        r.free()


def test_batch_of_all_dimensionalities(ctx):
    # 3D, 2D and 1D fields and other windows in one call: four window-kernel groups
    fields = [synth.spectral_field((300001,), seed=51), synth.spectral_field((20, 30, 70), seed=52),
              synth.spectral_field((5000,), seed=53, beta=3.0), synth.climate_field(303, shape=(60, 130)),
              synth.spectral_field((1,), seed=54), synth.spectral_field((30, 40, 50), seed=55),
              synth.spectral_field((70, 90), seed=56)]
    params = [dict(eb=1e-3), dict(eb=1e-4), dict(eb=1e-2, interp=(2,)), {}, {},
              dict(window=(8, 16, 16)), dict(S=8, window=(8, 16))]
    refs = [O.compress(f, _oracle_params(f.shape, kw)) for f, kw in zip(fields, params)]
    print("\n[parity] batch of 3D, 2D and 1D fields", flush=True)
    for rep in range(2):
        outs = ctx.compress_batch([_to_gpu(f) for f in fields], params)
        for r, ref in zip(outs, refs):
            assert r.blob() == ref.blob()
        ys = ctx.decompress_batch(outs)
        for y, ref in zip(ys, refs):
            assert np.array_equal(_bits(y.cpu().numpy()), _bits(ref.recon))
        for r in outs:
            r.free()


@pytest.mark.parametrize("shape,seed", [((24, 40, 64), 61), ((96, 200), 62), ((9001,), 63)])
def test_field_and_output_off_16_byte_alignment(ctx, shape, seed):
    """A field and an output buffer one float past a 16-byte boundary: the
    range kernel's scalar loop, the window kernels' per-slot block loads
    (not the 16-byte ones) and the replay's per-value writes; the blob and
    the reconstruction are the oracle's."""
    import torch
    x = synth.spectral_field(shape, seed=seed)
    print("\n[parity] unaligned shape=%s" % (shape,), flush=True)
    ref = O.compress(x, _oracle_params(x.shape, {}))
    n = x.size
    buf = torch.empty(n + 4, dtype=torch.float32, device="cuda")
    xin = buf[1:1 + n].view(shape)
    xin.copy_(torch.from_numpy(x))
    assert xin.data_ptr() % 16 == 4
    res = ctx.compress(xin)
    try:
        assert res.blob() == ref.blob()
        obuf = torch.zeros(n + 4, dtype=torch.float32, device="cuda")
        out = obuf[1:1 + n].view(shape)
        ctx.decompress(res, out)
        y = obuf.cpu().numpy()
        assert np.array_equal(_bits(y[1:1 + n]), _bits(ref.recon.ravel()))
        assert y[0] == 0.0 and not np.any(y[1 + n:])   # nothing written outside
    finally:
        res.free()


def test_pointers_off_4_byte_alignment_are_rejected(ctx):
    """A field or output pointer that is not 4-byte aligned (no float array
    is) is an argument error, found before any work is queued."""
    import ctypes as C
    import torch
    x = synth.spectral_field((16, 16, 16), seed=64)
    buf = torch.zeros(x.size + 4, dtype=torch.float32, device="cuda")
    buf[:x.size].copy_(torch.from_numpy(x.ravel()))
    d = szi.make_dims(x.shape)
    p = szi.make_params(3)
    r = szi.SzResult()
    rc = szi.lib().sz_compress(ctx.h, C.c_void_p(buf.data_ptr() + 2), C.byref(d), C.byref(p),
                               C.c_void_p(0), C.byref(r))
    assert rc == -1
    res = ctx.compress(buf[:x.size].view(x.shape))
    try:
        rc = szi.lib().sz_decompress(ctx.h, C.byref(res.raw), C.c_void_p(buf.data_ptr() + 2),
                                     C.c_void_p(0))
        assert rc == -1
    finally:
        res.free()


def test_window_limits(ctx):
    # the generic kernels hold a block of at most 4096 points in LDS; a
    # window must be a multiple of the stride
    x = _to_gpu(synth.spectral_field((40, 40, 40), seed=57))
    with pytest.raises(szi.SzError) as e:
        ctx.compress(x, window=(16, 16, 16))   # 17^3 block points
    assert e.value.code == -6
    with pytest.raises(szi.SzError) as e:
        ctx.compress(x, window=(8, 8, 36))
    assert e.value.code == -6
    with pytest.raises(szi.SzError) as e:
        ctx.compress(x, S=3)
    assert e.value.code == -6


def test_larger_batch_twice_equals_oracle(ctx):
    # twelve fields of mixed dimensionality, radius and chunk size (several
    # encode groups; the context's host workers build the code books), run
    # twice on one context
    rng = np.random.default_rng(91)
    fields, params = [], []
    for k in range(12):
        if k % 3 == 2:
            fields.append(synth.climate_field(920 + k, shape=(int(rng.integers(40, 160)), int(rng.integers(60, 240)))))
        else:
            fields.append(synth.spectral_field(tuple(int(v) for v in rng.integers(9, 45, size=3)),
                                               seed=930 + k, beta=5.0 / 3.0 if k % 2 else 3.0))
        kw = dict(eb=[1e-2, 1e-3, 1e-4][k % 3])
        if k % 4 == 1:
            kw["chunk"] = 512
        if k % 5 == 3:
            kw["radius"] = 128
        params.append(kw)
    refs = [O.compress(f, _oracle_params(f.shape, kw)) for f, kw in zip(fields, params)]
    for rep in range(2):
        print("\n[parity] batch of %d fields, pass %d" % (len(fields), rep), flush=True)
        outs = ctx.compress_batch([_to_gpu(f) for f in fields], params)
        for r, ref in zip(outs, refs):
            assert r.blob() == ref.blob()
        ys = ctx.decompress_batch(outs)
        for y, ref in zip(ys, refs):
            assert np.array_equal(_bits(y.cpu().numpy()), _bits(ref.recon))
        for r in outs:
            r.free()


def test_launch_shape_is_arithmetic_neutral(ctx):
    x = synth.spectral_field((40, 50, 90), seed=41)
    print("\n[parity] grid sweep", flush=True)
    blobs = []
    for per_cu in (1, 2, 8, 16):
        ctx.set_grid(per_cu)
        r = ctx.compress(_to_gpu(x))
        blobs.append(r.blob())
        r.free()
    ctx.set_grid(0)
    assert all(b == blobs[0] for b in blobs)


def test_window_order_over_grids_equals_oracle(ctx):
    # The order in which workgroups take groups of windows, the wave slots
    # within a group and the issue-priority tiers all follow from the grid.
    # A ragged field of 1920 groups (240 per L2 domain, partial windows on
    # three faces) with grids of 1, 2, 3 and 5 workgroups per CU (5 is more
    # than fit at once) gives 7.5, 3.75, 2.5 and 1.5 rounds per workgroup
    # and one to four priority tiers; each must give the oracle's blob and
    # reconstruction.
    x = synth.spectral_field((120, 250, 500), seed=43)
    ref = O.compress(x, _oracle_params(x.shape, {}))
    want = ref.blob()
    d = _to_gpu(x)
    try:
        for per_cu in (1, 2, 3, 5):
            print("\n[parity] window order, %d workgroups per CU" % per_cu, flush=True)
            ctx.set_grid(per_cu)
            r = ctx.compress(d)
            try:
                assert r.blob() == want, "blob, %d workgroups per CU" % per_cu
                y = ctx.decompress(r).cpu().numpy()
                assert np.array_equal(_bits(y), _bits(ref.recon)), \
                    "reconstruction, %d workgroups per CU" % per_cu
            finally:
                r.free()
    finally:
        ctx.set_grid(0)


def test_tuned_shapes_are_arithmetic_neutral():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    plain = szi.Context(0)
    tuned = szi.Context(0)
    tuned.set_tuning(True)
    cases = [synth.spectral_field((70, 90, 130), seed=81), synth.climate_field(351, shape=(300, 500))]
    for x in cases:
        nd = x.ndim
        print("\n[parity] tuner, %dD %s" % (nd, x.shape), flush=True)
        d = _to_gpu(x)
        a = plain.compress(d)
        ya = plain.decompress(a)
        b = tuned.compress(d)   # times the candidate shapes on this call
        assert b.blob() == a.blob()
        yb = tuned.decompress(b)
        assert torch.equal(yb.view(torch.int32), ya.view(torch.int32))
        assert tuned.shape(0, nd)[2] and tuned.shape(1, nd)[2]
        b.free()
        # every candidate, pinned, gives the same bytes
        cands = [(0, 0), (0, 2)] if nd == 3 else [(0, 0), (1, 0), (1, 3)]
        for v, g in cands:
            p = szi.Context(0)
            p.set_shape(0, nd, 512, v, g)
            p.set_shape(1, nd, 512, v, g)
            r = p.compress(d)
            assert r.blob() == a.blob(), "shape %s" % ((v, g),)
            y = p.decompress(r)
            assert torch.equal(y.view(torch.int32), ya.view(torch.int32)), "shape %s" % ((v, g),)
            r.free()
            p.close()
        a.free()
    with pytest.raises(szi.SzError):
        tuned.set_shape(0, 3, 512, 1, 0)   # no four-wave variant in 3D
    tuned.close()
    plain.close()


def test_repeat_is_deterministic(ctx):
    x = synth.bumps_field((64, 64, 64), seed=3)
    print("\n[parity] repeat", flush=True)
    g = _to_gpu(x)
    r1 = ctx.compress(g)
    r2 = ctx.compress(g)
    assert r1.blob() == r2.blob()
    r1.free()
    r2.free()


def test_nonfinite_input_rejected(ctx):
    x = synth.spectral_field((16, 16, 40), seed=5)
    x[3, 4, 5] = np.inf
    print("\n[errors] non-finite", flush=True)
    with pytest.raises(szi.SzError) as e:
        ctx.compress(_to_gpu(x))
    assert e.value.code == -2


def test_corrupt_blob_rejected(ctx):
    x = synth.spectral_field((16, 16, 40), seed=6)
    r = ctx.compress(_to_gpu(x))
    blob = bytearray(r.blob())
    r.free()
    print("\n[errors] corrupt blob", flush=True)
    for pos in (20, 300, len(blob) - 3):
        bad = bytearray(blob)
        bad[pos] ^= 0x04
        with pytest.raises(szi.SzError) as e:
            ctx.upload(bytes(bad))
        assert e.value.code == -5
    with pytest.raises(szi.SzError) as e:
        ctx.upload(bytes(blob[:-8]))
    assert e.value.code == -5


def test_budget_exceeded_is_oom():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = szi.Context(0, hbm_budget=64 << 10)   # below the 512 KiB code array
    x = synth.spectral_field((64, 64, 64), seed=7)
    print("\n[errors] budget", flush=True)
    with pytest.raises(szi.SzError) as e:
        c.compress(_to_gpu(x))
    assert e.value.code == -3
    c.close()


def test_full_size_512_cube(ctx):
    # the benchmark's workload at its full size: 512^3, rel 1e-3, AUTO
    print("\n[parity] 512^3 full size", flush=True)
    x = synth.workload_large()
    ref = O.compress(x, O.Params(shape=x.shape, eb=1e-3))
    res = ctx.compress(_to_gpu(x), eb=1e-3)
    assert res.blob() == ref.blob()
    y = ctx.decompress(res).cpu().numpy()
    assert np.array_equal(_bits(y), _bits(ref.recon))
    res.free()


@pytest.mark.parametrize("case", ["climate_1800x3600", "spectral_100x500x500_e4",
                                  "front_256x384x384_e2"])
def test_full_size_batch_shapes(ctx, case):
    # one field at each full shape of the batched workloads, against the
    # oracle: a climate field (2D, 5 % fill), a k^-3 field of the uneven
    # batch at rel 1e-4 and its tanh front at rel 1e-2
    print("\n[parity] full shape %s" % case, flush=True)
    if case.startswith("climate"):
        x, eb = synth.climate_field(300), 1e-3
    elif case.startswith("spectral"):
        x, eb = synth.spectral_field((100, 500, 500), beta=3.0, seed=401), 1e-4
    else:
        x, eb = synth.front_field((256, 384, 384), 413), 1e-2
    ref = O.compress(x, O.Params(shape=x.shape, eb=eb))
    res = ctx.compress(_to_gpu(x), eb=eb)
    assert res.blob() == ref.blob()
    y = ctx.decompress(res).cpu().numpy()
    assert np.array_equal(_bits(y), _bits(ref.recon))
    res.free()


def test_graph_mode_replays_equal_eager(ctx):
    # graph mode against the default mode: several replays of the same
    # signature with eager work and synchronizations between them, a new
    # signature (re-capture) in the middle, and a batch
    import torch
    a = synth.spectral_field((40, 50, 90), seed=81)
    b = synth.climate_field(381, shape=(120, 250))
    fields = [synth.spectral_field((20, 30, 70), seed=82), synth.climate_field(382, shape=(60, 130))]
    print("\n[graphs] replays vs eager", flush=True)
    ctx.set_graphs(False)
    ref = {}
    for name, x, kw in (("a", a, {}), ("b", b, dict(eb=1e-4))):
        r = ctx.compress(_to_gpu(x), **kw)
        ref[name] = (r.blob(), _bits(ctx.decompress(r).cpu().numpy()), kw)
        r.free()
    rb = ctx.compress_batch([_to_gpu(f) for f in fields])
    ref_batch = [r.blob() for r in rb]
    ref_batch_y = [_bits(y.cpu().numpy()) for y in ctx.decompress_batch(rb)]
    for r in rb:
        r.free()
    ctx.set_graphs(True)
    try:
        for rep, name in enumerate(["a", "a", "a", "b", "b", "a", "a"]):
            x = a if name == "a" else b
            g = _to_gpu(x)
            g2 = g * 2.0   # eager work on the caller's stream between replays
            r = ctx.compress(g, **ref[name][2])
            assert r.blob() == ref[name][0], "compression replay %d (%s)" % (rep, name)
            y = ctx.decompress(r)
            assert np.array_equal(_bits(y.cpu().numpy()), ref[name][1]), "decompression replay %d" % rep
            torch.cuda.synchronize()
            del g2
            r.free()
        for rep in range(3):
            rb = ctx.compress_batch([_to_gpu(f) for f in fields])
            assert [r.blob() for r in rb] == ref_batch, "batch replay %d" % rep
            ys = ctx.decompress_batch(rb)
            assert all(np.array_equal(_bits(y.cpu().numpy()), e) for y, e in zip(ys, ref_batch_y))
            for r in rb:
                r.free()
    finally:
        ctx.set_graphs(False)
