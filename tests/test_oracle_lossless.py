"""Pins of the oracle's lossless stage (frame-of-reference packing of the
block table and sum_dc per chunk of 256 blocks), checked against values
worked out by hand from the definition and against round trips; CPU only."""
import numpy as np
import pytest

from oracle import ref
from paper_2010_03144_amd import synth
from tests.gpu_util import sections

M32 = 0xFFFFFFFF


@pytest.mark.parametrize("values,words", [
    # minimum 5; differences 0, 2, 1 in 2 bits, least significant first:
    # 00 | 10 << 2 | 01 << 4 = 0x18
    ([5, 7, 6], [5, 0, 2, 0x18]),
    # equal values: width 0, no packed words
    ([9, 9], [9, 0, 0]),
    ([], [0, 0, 0]),
    # the widest difference takes 64 bits, so value 1 fills words 2 and 3
    ([0, 2**64 - 1], [0, 0, 64, 0, 0, M32, M32]),
    # minimum 1: nibbles 0, e, 2, 7, e, e, e, e then 1 in the next word
    ([1, 15, 3, 8, 15, 15, 15, 15, 2], [1, 0, 4, 0xEEEE72E0, 1]),
    # 3-bit value 101 at bits 30..32 straddles two words
    ([0] * 10 + [5], [0, 0, 3, 0x40000000, 1]),
    # a base above 32 bits keeps its high word
    ([2**40 + 3, 2**40], [0, 2**8, 2, 3]),
])
def test_frame_of_reference_column(values, words):
    assert [int(w) for w in ref.pack_column(values)] == words


def _stream(shape, block, eb, dtype=np.float32, abft=True):
    x = synth.grf_field(shape, seed=31, dtype=dtype) if all(shape) else np.zeros(shape, dtype)
    rc, s, _ = ref.compress(x, block, eb, abft=abft)
    assert rc == 0
    return s


@pytest.mark.parametrize("shape,block,dtype,abft", [
    ((48, 42, 36), (6, 6, 6), np.float32, True),
    ((48, 42, 36), (6, 6, 6), np.float64, False),
    ((300, 257), (16, 16), np.float64, True),
    ((5000,), (64,), np.float32, True),
    ((7, 13, 5), (6, 6, 6), np.float32, True),   # 12 blocks: one partial chunk
    ((0, 5), (16, 16), np.float32, True),         # no blocks at all
])
def test_pack_round_trip(shape, block, dtype, abft):
    s = _stream(shape, block, 1e-3, dtype, abft)
    rc, p = ref.pack(s)
    assert rc == 0
    assert bytes(p[:8]) == b"SDCSZ\x00v2"
    rc, back = ref.unpack(p)
    assert rc == 0 and np.array_equal(back, s)


def test_packed_stream_is_smaller_and_decodes_the_same():
    s = _stream((96, 90, 84), (6, 6, 6), 1e-2)
    rc, p = ref.pack(s)
    assert rc == 0 and p.size < s.size
    sec = sections(s)
    meta = (sec["coef"] - sec["table"]) + (sec["outliers"] - sec["sumdc"])
    assert s.size - p.size > meta // 3  # table and sum_dc shrink by more than a third
    rc, back = ref.unpack(p)
    rc1, y1, _ = ref.decompress(back)
    rc0, y0, _ = ref.decompress(s)
    assert rc0 == rc1 == 0 and np.array_equal(y0.view(np.uint32), y1.view(np.uint32))


def test_versions_are_not_mixed():
    s = _stream((24, 24, 24), (6, 6, 6), 1e-3)
    assert ref.unpack(s)[0] == ref.EFORMAT
    rc, p = ref.pack(s)
    assert ref.pack(p)[0] == ref.EFORMAT
    assert ref.decompress(p)[0] == ref.EFORMAT


def test_corrupt_packed_sections():
    s = _stream((48, 42, 36), (6, 6, 6), 1e-3)
    rc, p = ref.pack(s)
    hdr = sections(p)
    t0, s0 = hdr["table"], hdr["sumdc"]
    n_chunks = -(-int(np.frombuffer(p[80:88].tobytes(), "<u8")[0]) // 256)
    data = t0 + 4 * (n_chunks + 1)
    bad = p.copy()
    bad[data + 8:data + 12] = np.frombuffer(np.uint32(65).tobytes(), np.uint8)  # width 65
    assert ref.unpack(bad)[0] == ref.EFORMAT
    bad = p.copy()
    bad[t0 + 4:t0 + 8] = np.frombuffer(np.uint32(10**6).tobytes(), np.uint8)  # chunk past the section
    assert ref.unpack(bad)[0] == ref.EFORMAT
    assert ref.unpack(p[:s0])[0] == ref.EFORMAT  # truncated
    # a flipped bit in a packed checksum: unpacking succeeds, and the
    # decompressor's checksum finds the block and cannot correct it (the
    # re-execution from the stream meets the same checksum)
    sdata = s0 + 4 * (n_chunks + 1)
    bad = p.copy()
    bad[sdata + 12] ^= 0x01
    rc, back = ref.unpack(bad)
    assert rc == 0
    rc, _, rep = ref.decompress(back)
    assert rc == ref.ESDC and rep["recon"]["detected"] >= 1 and rep["recon"]["uncorrectable"] >= 1
