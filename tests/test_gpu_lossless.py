"""GPU parity of the lossless stage (frame-of-reference packing of the block
table and sum_dc per chunk of 256 blocks): the packed streams of
sdcsz_pack equal the oracle's byte for byte, sdcsz_unpack gives back the
plain stream byte for byte, and every error code equals the oracle's on
the same corrupt or short inputs."""
import ctypes as C

import numpy as np
import pytest

from oracle import ref
from paper_2010_03144_amd import sdcsz, synth
from tests.gpu_util import first_difference, sections

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def codec():
    return sdcsz.Codec("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def check_both_ways(codec, s):
    """s: a plain stream (host bytes).  GPU pack == oracle pack; GPU unpack
    of either packed form == s."""
    rc_r, p_r = ref.pack(s)
    rc_g, p_g = codec.pack(dev(s))
    assert rc_r == rc_g == 0, (rc_r, rc_g)
    p_g = host(p_g)
    assert np.array_equal(p_r, p_g), first_difference(p_r, p_g)
    rc, back = codec.unpack(dev(p_g))
    assert rc == 0
    back = host(back)
    assert np.array_equal(back, s), first_difference(s, back)
    return p_g


@pytest.mark.parametrize("shape,block,dtype,abft", [
    ((48, 42, 36), (6, 6, 6), np.float32, True),
    ((48, 42, 36), (6, 6, 6), np.float64, False),
    ((300, 257), (16, 16), np.float64, True),
    ((5000,), (64,), np.float32, True),
    ((7, 13, 5), (6, 6, 6), np.float32, True),      # 12 blocks: one partial chunk
    ((96, 96, 96), (6, 6, 6), np.float32, True),    # 4096 blocks: 16 full chunks
    ((97, 96, 96), (6, 6, 6), np.float32, False),   # 4352 blocks: 17 chunks
    ((64, 64, 64), (8, 8, 8), np.float64, True),
])
def test_pack_and_unpack_match_oracle(codec, shape, block, dtype, abft):
    print(f"case shape={shape} block={block} dtype={np.dtype(dtype).name} abft={abft}", flush=True)
    x = synth.grf_field(shape, seed=31, dtype=dtype)
    rc, s_g, _ = codec.compress(dev(x), block, 1e-3, abft=abft)
    assert rc == 0
    s = host(s_g)
    p = check_both_ways(codec, s)
    # the oracle decompresses what the GPU unpacked
    rc, back = codec.unpack(dev(p))
    rc_g, y_g, _ = codec.decompress(back)
    rc_r, y_r, _ = ref.decompress(s)
    assert rc_g == rc_r == 0
    assert np.array_equal(host(y_g).view(np.uint8), y_r.view(np.uint8))


def test_stream_without_blocks(codec):
    print("case empty field (0, 5)", flush=True)
    rc, s, _ = ref.compress(np.zeros((0, 5), np.float32), (16, 16), 1e-3)
    assert rc == 0
    check_both_ways(codec, s)


@pytest.fixture(scope="module")
def full_field():
    print("generating 512^3 field (seed 2)", flush=True)
    return dev(synth.grf_field((512, 512, 512), seed=2))


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4])
def test_full_size_matches_oracle(codec, full_field, eb):
    print(f"case 512^3 FP32 6^3 eb={eb} ABFT", flush=True)
    rc, s_g, _ = codec.compress(full_field, (6, 6, 6), eb)
    assert rc == 0
    s = host(s_g)
    p = check_both_ways(codec, s)
    assert p.size < s.size


def _corruptions(s):
    """(name, packed stream) pairs: the oracle's own corruption pins and
    seeded byte flips inside the packed sections."""
    rc, p = ref.pack(s)
    assert rc == 0
    sec = sections(p)
    t0, s0 = sec["table"], sec["sumdc"]
    nch = -(-int(np.frombuffer(p[80:88].tobytes(), "<u8")[0]) // 256)
    data = t0 + 4 * (nch + 1)
    out = []
    bad = p.copy()
    bad[data + 8:data + 12] = np.frombuffer(np.uint32(65).tobytes(), np.uint8)
    out.append(("width 65", bad))
    bad = p.copy()
    bad[data + 8:data + 12] = np.frombuffer(np.uint32(33).tobytes(), np.uint8)
    out.append(("table width 33", bad))
    bad = p.copy()
    bad[t0 + 4:t0 + 8] = np.frombuffer(np.uint32(10 ** 6).tobytes(), np.uint8)
    out.append(("chunk past the section", bad))
    bad = p.copy()
    bad[t0:t0 + 4] = np.frombuffer(np.uint32(1).tobytes(), np.uint8)
    out.append(("first offset not 0", bad))
    out.append(("truncated", p[:s0].copy()))
    bad = p.copy()
    bad[s0 + 4 * (nch + 1) + 12] ^= 0x01
    out.append(("flipped checksum bit", bad))
    rng = np.random.default_rng(7)
    for k in range(24):
        bad = p.copy()
        at = int(rng.integers(t0, p.size))
        bad[at] ^= np.uint8(1 << int(rng.integers(0, 8)))
        out.append((f"flip byte {at}", bad))
    return out


def test_corrupt_packed_streams_match_oracle(codec):
    x = synth.grf_field((48, 42, 36), seed=31)
    rc, s, _ = ref.compress(x, (6, 6, 6), 1e-3)
    assert rc == 0
    for name, bad in _corruptions(s):
        print(f"case {name}", flush=True)
        rc_r, back_r = ref.unpack(bad)
        rc_g, back_g = codec.unpack(dev(bad))
        assert rc_r == rc_g, (name, rc_r, rc_g)
        if rc_r == 0:
            back_g = host(back_g)
            assert np.array_equal(back_r, back_g), (name, first_difference(back_r, back_g))
            rc_dr, y_r, rep_r = ref.decompress(back_r)
            rc_dg, y_g, rep_g = codec.decompress(dev(back_g))
            assert rc_dr == rc_dg, (name, rc_dr, rc_dg)
            if rc_dr == sdcsz.EFORMAT:
                continue
            for t in sdcsz.TARGETS:
                assert rep_r[t] == rep_g[t], (name, t)


def _raw(fn, src, cap, ws_bytes):
    L = sdcsz.lib()
    out = torch.zeros(max(cap, 8), dtype=torch.uint8, device="cuda")
    ws = torch.zeros(ws_bytes, dtype=torch.uint8, device="cuda")
    size = C.c_uint64(0)
    rc = getattr(L, fn)(C.c_void_p(src.data_ptr()), src.numel(), C.c_void_p(out.data_ptr()), cap,
                        C.byref(size), C.c_void_p(ws.data_ptr()), ws.numel(), None)
    torch.cuda.synchronize()
    return rc, int(size.value), out


def test_short_outputs_and_wrong_versions(codec):
    x = synth.grf_field((48, 42, 36), seed=31)
    rc, s, _ = ref.compress(x, (6, 6, 6), 1e-3)
    rc, p = ref.pack(s)
    sd, pd = dev(s), dev(p)
    ws = int(sdcsz.lib().sdcsz_pack_workspace_size(s.size // 8))
    rc, size, out = _raw("sdcsz_pack", sd, p.size - 8, ws)
    assert rc == sdcsz.ENOSPC and size == p.size
    assert not out.any()  # nothing written
    rc, size, out = _raw("sdcsz_unpack", pd, s.size - 8, 256)
    assert rc == sdcsz.ENOSPC and size == s.size
    assert not out.any()
    rc, size, _ = _raw("sdcsz_unpack", pd, s.size, 64)
    assert rc == sdcsz.ENOSPC  # workspace too small
    # a corrupt packed stream with a short output: the oracle's EFORMAT
    bad = p.copy()
    t0 = sections(p)["table"]
    bad[t0 + 4:t0 + 8] = np.frombuffer(np.uint32(10 ** 6).tobytes(), np.uint8)
    assert ref.unpack(bad)[0] == ref.EFORMAT
    rc, _, _ = _raw("sdcsz_unpack", dev(bad), 16, 256)
    assert rc == sdcsz.EFORMAT
    # versions are not mixed
    assert codec.unpack(sd)[0] == sdcsz.EFORMAT
    assert codec.pack(pd)[0] == sdcsz.EFORMAT
    assert codec.decompress(pd)[0] == sdcsz.EFORMAT
