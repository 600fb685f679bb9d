"""The request server (continuous batching): every result is the one a plain
call gives, alone or in the mix, and admission keeps the charged device
memory within the budget.  Runs on an MI355X only (marker ``gpu``)."""
import numpy as np
import pytest

import oracle as O
import paper_2312_05492_amd as szi
from paper_2312_05492_amd import synth

pytestmark = pytest.mark.gpu


def _gpu(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _skip_without_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mix():
    return [
        (synth.workload_small(), dict(eb=1e-3)),
        (synth.spectral_field((70, 90, 130), seed=51), dict(eb=1e-4)),
        (synth.climate_field(351, shape=(300, 500)), dict(eb=1e-3)),
        (synth.spectral_field((40, 50, 60), seed=52, beta=3.0), dict(eb=1e-2, interp=(0, 2, 1))),
        (synth.front_field((33, 47, 65), seed=53), dict(eb=1e-2)),
        (synth.spectral_field((200, 350), seed=54), dict(eb=0.05, eb_mode=0)),
        (synth.spectral_field((96, 96, 96), seed=55, mean=10.0), dict(eb=1e-3)),
        (synth.spectral_field((1, 9, 3000), seed=56), dict(eb=1e-3)),
    ]


def test_server_results_equal_plain_calls():
    _skip_without_gpu()
    import torch
    print("\n[server] mix of %d compressions + %d decompressions" % (8, 8), flush=True)
    fields = _mix()
    xs = [_gpu(f) for f, _ in fields]
    ctx = szi.Context(0)
    plain = [ctx.compress(x, **kw) for x, (_, kw) in zip(xs, fields)]
    ref_blobs = [r.blob() for r in plain]
    ref_out = [ctx.decompress(r) for r in plain]
    # the plain path itself is the oracle's (the parity tests); tie one case here too
    ref0 = O.compress(fields[0][0], O.Params(shape=fields[0][0].shape, eb=1e-3))
    assert ref_blobs[0] == ref0.blob()

    srv = szi.Server(0, slots=4)
    outs = [torch.empty_like(x) for x in xs]
    # everything at once: compressions and decompressions of the plain results
    for i, (x, (_, kw)) in enumerate(zip(xs, fields)):
        srv.submit_compress(x, tag=i, **kw)
        srv.submit_decompress(plain[i], outs[i], tag=100 + i)
    got = {}
    while len(got) < 2 * len(xs):
        comp = srv.poll(wait=True)
        assert comp, "server stalled"
        for c in comp:
            got[c["tag"]] = c
    for i in range(len(xs)):
        c = got[i]
        assert c["status"] == 0
        assert c["result"].blob() == ref_blobs[i], "compression %d differs in the mix" % i
        d = got[100 + i]
        assert d["status"] == 0
        assert torch.equal(outs[i].view(torch.int32), ref_out[i].view(torch.int32)), \
            "decompression %d differs in the mix" % i
    # the server's own results replay on the server, again identically
    outs2 = [torch.empty_like(x) for x in xs]
    for i in range(len(xs)):
        srv.submit_decompress(got[i]["result"], outs2[i], tag=200 + i)
    left = set(range(200, 200 + len(xs)))
    while left:
        for c in srv.poll(wait=True):
            assert c["status"] == 0
            left.discard(c["tag"])
    for i in range(len(xs)):
        assert torch.equal(outs2[i].view(torch.int32), ref_out[i].view(torch.int32))
    # work of different slots overlapped in time
    spans = sorted((c["t_start"], c["t_done"], c["slot"]) for c in got.values())
    assert any(b[0] < a[1] and b[2] != a[2] for a, b in zip(spans, spans[1:]))
    for i in range(len(xs)):
        got[i]["result"].free()
    assert srv.stats()["charged"] == 0
    srv.close()
    for r in plain:
        r.free()
    ctx.close()


def test_server_budget_admission():
    _skip_without_gpu()
    import torch
    fields = [(synth.spectral_field((96, 128, 128), seed=60 + k), dict(eb=1e-3)) for k in range(6)]
    n = 96 * 128 * 128
    words = 3 * n + 4 * (n // 256 + 10)                     # the documented compression bound
    need = 2 * n + words + (words + words // 32 + 4) + 8 * n + n // 16 + (2 << 20)
    budget = need + need // 2                               # one compression at a time
    print("\n[server] budget %d bytes, request bound %d" % (budget, need), flush=True)
    xs = [_gpu(f) for f, _ in fields]
    ctx = szi.Context(0)
    ref = [ctx.compress(x, **kw).blob() for x, (_, kw) in zip(xs, fields)]
    ctx.close()
    torch.cuda.synchronize()
    srv = szi.Server(0, slots=4, hbm_budget=budget)
    # the device memory the server holds (free memory is read around the
    # requests; the driver hands out memory in pages, hence the slack)
    free0 = torch.cuda.mem_get_info()[0]
    slack = 16 << 20
    peak = 0
    for i, (x, (_, kw)) in enumerate(zip(xs, fields)):
        srv.submit_compress(x, tag=i, **kw)
    done = 0
    while done < len(xs):
        st = srv.stats()
        assert st["charged"] <= budget
        assert st["running"] <= 1
        peak = max(peak, free0 - torch.cuda.mem_get_info()[0])
        assert peak <= budget + slack, (peak, budget)
        comp = srv.poll(wait=True)
        assert comp, "server stalled"
        for c in comp:
            assert c["status"] == 0
            assert c["result"].blob() == ref[c["tag"]]
            c["result"].free()   # returns the bytes, the next request is admitted
            done += 1
    # what the workers still cache stays within the budget too
    assert free0 - torch.cuda.mem_get_info()[0] <= budget + slack
    print("[server] peak device memory %d of budget %d" % (peak, budget), flush=True)
    # a request larger than the whole budget is refused at submission
    big = _gpu(synth.spectral_field((256, 256, 256), seed=70))
    with pytest.raises(szi.SzError) as e:
        srv.submit_compress(big, tag=99)
    assert e.value.code == -3
    srv.close()
