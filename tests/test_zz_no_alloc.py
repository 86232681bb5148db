"""sdcsz_decompress_noalloc, the decompression entry point that allocates
nothing, against sdcsz_decompress through the C ABI: the same values bit for
bit and the same reports, over calls in a row whose inputs shrink and grow
(the library's device array keeps the previous call's contents), and a clear
error for a stream whose workspace exceeds the array."""
import numpy as np
import pytest

from paper_2010_03144_amd import sdcsz, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def codec():
    return sdcsz.Codec(DEV)


def compressed(codec, x, block, eb, **kw):
    print(f"case shape={x.shape} dtype={x.dtype} block={block} eb={eb} {kw}", flush=True)
    rc, s, _ = codec.compress(torch.from_numpy(np.ascontiguousarray(x)).to(DEV), block, eb, **kw)
    assert rc == sdcsz.OK, sdcsz.strerror(rc)
    return s.clone()  # out of the codec's reusable buffer


def bits(t):
    return t.view(torch.int32 if t.dtype == torch.float32 else torch.int64)


def same_as_workspace_call(codec, stream, shape, dtype, faults=None):
    rc_a, y_a, rep_a = codec.decompress(stream, faults=faults)
    out = torch.full(shape, float("nan"), dtype=dtype, device=DEV)
    rc_b, rep_b = codec.decompress_noalloc(stream, out, faults=faults)
    assert rc_a == rc_b == sdcsz.OK, (rc_a, rc_b)
    assert torch.equal(bits(y_a), bits(out))
    assert rep_a == rep_b


def test_calls_in_a_row_match_the_workspace_entry_point(codec):
    # a field of 8,360 6x6x6 blocks (more than the 4,096 re-execution slots
    # the array's small recon area holds), then smaller and differently
    # shaped ones, then the first again
    big = synth.grf_field((130, 120, 110), seed=21)
    small = synth.grf_field((40, 36, 30), seed=22)
    flat = synth.grf_field((700, 1013), seed=23, dtype=np.float64)
    s_big = compressed(codec, big, (6, 6, 6), 1e-3)
    s_small = compressed(codec, small, (6, 6, 6), 1e-4)
    s_flat = compressed(codec, flat, (16, 16), 1e-3)
    same_as_workspace_call(codec, s_big, big.shape, torch.float32)
    same_as_workspace_call(codec, s_small, small.shape, torch.float32)
    same_as_workspace_call(codec, s_flat, flat.shape, torch.float64)
    same_as_workspace_call(codec, s_big, big.shape, torch.float32)


def test_fault_plans_and_generic_shapes(codec):
    x = synth.grf_field((45, 40, 37), seed=24)
    s = compressed(codec, x, (6, 6, 6), 1e-3)
    plan = [(3, 30, 5, 17), (3, 7, 90, 0), (3, 31, 211, 100)]  # RECON flips
    same_as_workspace_call(codec, s, x.shape, torch.float32, faults=plan)
    same_as_workspace_call(codec, s, x.shape, torch.float32)
    g = synth.grf_field((50, 44, 41), seed=25, dtype=np.float64)
    s_g = compressed(codec, g, (8, 8, 8), 1e-3)
    same_as_workspace_call(codec, s_g, g.shape, torch.float64)


def test_stream_beyond_the_array_is_rejected(codec):
    # 8x8x8 blocks take the generic decoder, which stages every block's
    # values: 20,480 blocks of 512 FP64 values need 84 MB > 64 MiB
    x = synth.grf_field((256, 256, 160), seed=26, dtype=np.float64)
    s = compressed(codec, x, (8, 8, 8), 1e-2)
    out = torch.zeros(x.shape, dtype=torch.float64, device=DEV)
    rc, _ = codec.decompress_noalloc(s, out)
    assert rc == sdcsz.ENOSPC
    assert int(torch.count_nonzero(out)) == 0  # nothing written
    # the next call still works
    y = synth.grf_field((40, 36, 30), seed=27)
    same_as_workspace_call(codec, compressed(codec, y, (6, 6, 6), 1e-3), y.shape, torch.float32)
