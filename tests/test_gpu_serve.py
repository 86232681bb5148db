"""The request server on the GPU: each request's result is the same alone and
in the mix.  A mix of compression requests (3D and 2D, FP32 and FP64, some
with fault plans) and decompression requests (some with RECON faults)
arrives within ten milliseconds and is served by two workers with
continuous batching; every result must equal, byte for byte (streams) or bit
for bit (values), with equal fault counts, the result of the same request
run by itself through the single-field calls."""
import numpy as np
import pytest

from paper_2010_03144_amd import sdcsz, serve, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _fields():
    out = []
    for i in range(14):
        if i % 3 == 0:
            shape, block = (40 + i, 37, 33), (6, 6, 6)
        elif i % 3 == 1:
            shape, block = (300 + 7 * i, 211), (16, 16)
        else:
            shape, block = (25, 26, 27 + i), (6, 6, 6)
        dtype = np.float64 if i % 4 == 3 else np.float32
        x = synth.grf_field(shape, seed=100 + i, slope=-2.0 - 0.15 * i, dtype=dtype)
        eb = float(10 ** (-2 - 3 * (i % 5) / 4))
        out.append((x, block, eb))
    return out


def _requests(fields, streams):
    reqs = []
    for i, (x, block, eb) in enumerate(fields):
        faults = None
        if i % 4 == 2:
            faults = synth.fault_plan(x.shape, block, x.dtype, {"input": 1, "coef": 1, "code": 1}, seed=300 + i)
        reqs.append(serve.Request("compress", torch.from_numpy(x).cuda(), block, eb, faults=faults, tag=("c", i)))
    for i, (s, x, block) in enumerate(streams):
        faults = None
        if i % 3 == 1:
            faults = synth.fault_plan(x.shape, block, x.dtype, {"recon": 2}, seed=400 + i)
        reqs.append(serve.Request("decompress", s, faults=faults, geom=(x.shape, x.dtype == np.float32, block),
                                  tag=("d", i)))
    rng = np.random.default_rng(7)
    for r in reqs:
        r.t_arrival = float(rng.uniform(0, 0.01))
    return reqs


def _alone(codec, r):
    if r.kind == "compress":
        rc, s, rep = codec.compress(r.data, r.block, r.eb, faults=r.faults)
        return rc, s.clone() if s is not None else None, rep
    return codec.decompress(r.data, faults=r.faults)


def _same(r, alone):
    rc, res, rep = alone
    assert r.rc == rc == 0, (r.tag, r.rc, rc)
    for t in sdcsz.TARGETS:
        assert r.report[t] == rep[t], (r.tag, t, r.report[t], rep[t])
    if r.kind == "compress":
        assert r.result.numel() == res.numel() and torch.equal(r.result, res), r.tag
    else:
        a = r.result.view(torch.int32 if r.result.dtype == torch.float32 else torch.int64)
        b = res.view(torch.int32 if res.dtype == torch.float32 else torch.int64)
        assert torch.equal(a, b), r.tag


@pytest.fixture(scope="module")
def mix():
    codec = sdcsz.Codec("cuda:0")
    fields = _fields()
    streams = []
    for x, block, eb in fields[:8]:
        rc, s, _ = codec.compress(torch.from_numpy(x).cuda(), block, eb)
        assert rc == 0
        streams.append((s.clone(), x, block))
    return codec, fields, streams


@pytest.mark.parametrize("workers,budget,max_batch", [(2, 200e9, 8), (3, None, 64)])
def test_each_result_same_alone_and_in_the_mix(mix, workers, budget, max_batch):
    codec, fields, streams = mix
    reqs = _requests(fields, streams)
    if budget is None:  # tight: only about two requests fit at a time
        budget = 2.2 * max(serve.device_footprint(r) for r in reqs)
    print(f"case workers={workers} budget={budget:.3g} max_batch={max_batch} requests={len(reqs)}", flush=True)
    with serve.Server("cuda:0", workers=workers, hbm_budget=budget, max_batch=max_batch) as srv:
        t0 = srv.clock()
        serve.replay(srv, reqs, t0)
        assert srv.peak_in_use <= budget
        batches = list(srv.batches)
    torch.cuda.synchronize()
    assert sum(batches) == len(reqs)
    for r in reqs:
        assert r.t_done >= r.t_arrival
        _same(r, _alone(codec, r))
    if max_batch > 1 and workers == 2:
        assert max(batches) > 1  # some requests were served together


class _Capturing(serve.GpuExecutor):
    """Keeps a copy of each result before the server releases it."""

    def run(self, ctx, batch, now):
        super().run(ctx, batch, now)
        # on the worker's stream, finished before its next batch reuses the buffers
        with torch.cuda.stream(ctx["stream"]):
            for r in batch:
                r.kept = r.result.clone() if r.result is not None else None
        ctx["stream"].synchronize()


def test_released_results_come_from_reused_buffers_and_match(mix):
    """keep_results=False: a batch's outputs are views into per-worker
    buffers reused by the next batches; each result, copied before release,
    still equals the request run alone."""
    codec, fields, streams = mix
    for rep in range(2):  # the second round reuses the buffers the first grew
        reqs = _requests(fields, streams)
        ex = _Capturing("cuda:0")
        print(f"case released results round={rep} requests={len(reqs)}", flush=True)
        with serve.Server("cuda:0", workers=2, hbm_budget=200e9, max_batch=8, executor=ex,
                          keep_results=False) as srv:
            assert ex.reuse_outputs
            serve.replay(srv, reqs, srv.clock())
        torch.cuda.synchronize()
        for r in reqs:
            assert r.result is None and r.result_bytes > 0
            r.result = r.kept
            _same(r, _alone(codec, r))
