"""Seeded random sweep of shapes and parameters against the oracle: every
blob byte-identical and the reconstruction bit-identical.  Sides are
mostly not multiples of the window, so most windows are ragged; 2D and 3D
alternate; bounds, splines, orders, radius and chunk vary."""
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


def _cases(n=48, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        three = k % 2 == 0
        if three:
            shape = tuple(int(v) for v in rng.integers(9, 70, size=3))
        else:
            shape = tuple(int(v) for v in rng.integers(17, 400, size=2))
        D = len(shape)
        kw = {"eb": float(rng.choice([1e-2, 3e-3, 1e-3, 1e-4, 1e-5]))}
        r = rng.random()
        if r < 0.3:
            kw["interp"] = tuple(int(v) for v in rng.integers(0, 4, size=D))
        if rng.random() < 0.3:
            kw["order"] = tuple(int(v) for v in rng.permutation(D))
        if rng.random() < 0.25:
            kw["radius"] = int(rng.choice([2, 16, 100, 1024]))
        if rng.random() < 0.25:
            kw["chunk"] = int(rng.choice([256, 512, 2048]))
        gen = int(rng.integers(0, 3))
        out.append(("case%02d" % k, shape, kw, gen, int(rng.integers(1, 10**6))))
    return out


def _field(shape, gen, seed):
    if gen == 0:
        return synth.spectral_field(shape, beta=5.0 / 3.0, seed=seed, mean=float(seed % 7))
    if gen == 1:
        return synth.spectral_field(shape, beta=3.0, seed=seed)
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) * 3.0 + 100.0).astype(np.float32)


@pytest.mark.parametrize("name,shape,kw,gen,seed", _cases())
def test_random_case(ctx, name, shape, kw, gen, seed):
    import torch
    x = _field(shape, gen, seed)
    print("\n[random] %s shape=%s params=%s gen=%d" % (name, shape, kw, gen), flush=True)
    m = dict(kw)
    if "radius" in m:
        m["R"] = m.pop("radius")
    ref = O.compress(x, O.Params(shape=x.shape, **m))
    res = ctx.compress(torch.from_numpy(x).cuda(), **kw)
    try:
        assert res.blob() == ref.blob()
        y = ctx.decompress(res).cpu().numpy()
        assert np.array_equal(y.view(np.uint32), ref.recon.view(np.uint32))
    finally:
        res.free()
