"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Integer outputs (codes, predictor choices, Huffman streams, fault counters)
and the reconstructed values must match bit for bit: both sides evaluate the
same IEEE operations in the same order (no contraction, no fast math).
"""
import numpy as np
import pytest

from oracle import ref
from paper_2010_03144_amd import sdcsz, synth
from tests.gpu_util import first_difference

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def codec():
    return sdcsz.Codec("cuda:0")


def both(codec, x, block, eb, **kw):
    print(f"case shape={x.shape} dtype={x.dtype} block={block} eb={eb} {kw}", flush=True)
    rc_r, s_r, rep_r = ref.compress(x, block, eb, **kw)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    rc_g, s_g, rep_g = codec.compress(xd, block, eb, **kw)
    s_g = s_g.cpu().numpy() if s_g is not None else None
    return (rc_r, s_r, rep_r), (rc_g, s_g, rep_g)


def same_counts(a, b):
    for t in sdcsz.TARGETS:
        assert a[t] == b[t], (t, a[t], b[t])


def check_roundtrip(codec, x, block, eb, **kw):
    (rc_r, s_r, rep_r), (rc_g, s_g, rep_g) = both(codec, x, block, eb, **kw)
    assert rc_r == rc_g == 0, (rc_r, rc_g)
    assert np.array_equal(s_r, s_g), first_difference(s_r, s_g)
    same_counts(rep_r, rep_g)
    assert rep_r["eb_abs"] == rep_g["eb_abs"]
    rc, y_r, _ = ref.decompress(s_r)
    rc2, y_g, rep_d = codec.decompress(torch.from_numpy(s_g).cuda())
    assert rc == rc2 == 0
    y_g = y_g.cpu().numpy()
    assert np.array_equal(y_r.view(np.uint8), y_g.view(np.uint8))
    fin = np.isfinite(x)
    if x.size:
        err = np.abs(x[fin].astype(np.float64) - y_g[fin].astype(np.float64))
        assert err.size == 0 or err.max() <= rep_g["eb_abs"]
    return s_g, rep_g


def test_config1_bumps_64cube(codec):
    x = synth.bumps_field((64, 64, 64), seed=1)
    check_roundtrip(codec, x, (6, 6, 6), 1e-3)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("eb", [1e-2, 1e-4])
@pytest.mark.parametrize("abft", [True, False])
def test_grf_tiles_and_ragged_tail(codec, dtype, eb, abft):
    x = synth.grf_field((50, 47, 44), seed=2, dtype=dtype)
    check_roundtrip(codec, x, (6, 6, 6), eb, abft=abft)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("eb", [1e-2, 1e-5])
@pytest.mark.parametrize("abft", [True, False])
def test_grf_2d_tiles_and_ragged_tail(codec, dtype, eb, abft):
    # 44 x 64 blocks of 16x16 (12-row and 5-column partial edges): 11 work-groups
    # of full blocks and one of the partial shell in the 2D row-streaming kernels
    x = synth.grf_field((700, 1013), seed=12, slope=-2.5, front=True, dtype=dtype)
    check_roundtrip(codec, x, (16, 16), eb, abft=abft)


@pytest.mark.parametrize("predictor", ["lorenzo", "regression"])
def test_2d_forced_predictors(codec, predictor):
    x = synth.grf_field((333, 517), seed=13)
    check_roundtrip(codec, x, (16, 16), 1e-3, predictor=predictor)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_2d_fault_counts_match_oracle(codec, dtype):
    shape, block = (400, 390), (16, 16)
    x = synth.grf_field(shape, seed=14, dtype=dtype)
    plan = synth.fault_plan(shape, block, dtype, {"input": 5, "coef": 5, "code": 5, "dup_pred": 5,
                                                  "dup_recon": 5}, seed=41)
    (rc_r, s_r, rep_r), (rc_g, s_g, rep_g) = both(codec, x, block, 1e-4, faults=plan)
    assert rc_r == rc_g == 0, (rc_r, rc_g)
    same_counts(rep_r, rep_g)
    assert rep_g["generic_plan_blocks"] == 0  # every flip applied by the specialised kernels
    assert np.array_equal(s_r, s_g), first_difference(s_r, s_g)
    rplan = synth.fault_plan(shape, block, dtype, {"recon": 9}, seed=42)
    rc_r, y_r, rep_dr = ref.decompress(s_r, faults=rplan)
    rc_g, y_g, rep_dg = codec.decompress(torch.from_numpy(s_g).cuda(), faults=rplan)
    assert rc_r == rc_g == 0
    same_counts(rep_dr, rep_dg)
    assert rep_dg["generic_plan_blocks"] == 0
    assert rep_dg["recon"]["detected"] == rep_dg["recon"]["corrected"] == 9
    assert np.array_equal(y_r.view(np.uint8), y_g.cpu().numpy().view(np.uint8))


@pytest.mark.parametrize("predictor", ["lorenzo", "regression"])
def test_forced_predictors(codec, predictor):
    x = synth.grf_field((30, 31, 32), seed=7)
    check_roundtrip(codec, x, (6, 6, 6), 1e-3, predictor=predictor)


@pytest.mark.parametrize("shape,block", [((300, 257), (16, 16)), ((5000,), (64,)), ((7, 13, 5), (6, 6, 6)),
                                         ((33, 20), (8, 5)), ((1, 1, 1), (6, 6, 6)), ((9, 9, 9), (4, 4, 4)),
                                         ((40, 40, 40), (10, 10, 10)), ((35, 33, 37), (8, 8, 8)),
                                         ((45, 41, 43), (20, 20, 20)), ((26, 27, 25), (12, 12, 12))])
def test_shapes(codec, shape, block):
    x = synth.grf_field(shape, seed=4, dtype=np.float32)
    check_roundtrip(codec, x, block, 1e-3)
    check_roundtrip(codec, x.astype(np.float64), block, 0.05, eb_mode="abs")


def test_scan_of_more_than_a_million_blocks(codec):
    """Over 2^20 blocks a scan thread takes more than two blocks (here 3):
    offsets and totals must still match the oracle's stream."""
    x = synth.grf_field((2_200_000,), seed=12, dtype=np.float32)
    check_roundtrip(codec, x, (2,), 1e-3)


def test_special_values(codec):
    x = synth.bumps_field((20, 20, 20), seed=3)
    x[1, 2, 3] = np.nan
    x[7, 7, 7] = np.inf
    x[19, 0, 5] = -np.inf
    x[10, 10, 10] = 1e-42  # FP32 denormal
    check_roundtrip(codec, x, (6, 6, 6), 1e-3)
    c = np.full((9, 8, 7), 3.25, np.float32)
    check_roundtrip(codec, c, (6, 6, 6), 1e-3)


def test_empty_field(codec):
    x = np.zeros((0, 5), np.float32)
    (rc_r, s_r, _), (rc_g, s_g, _) = both(codec, x, (16, 16), 1e-3)
    assert rc_r == rc_g == 0 and np.array_equal(s_r, s_g)


def test_invalid_arguments(codec):
    x = torch.zeros((8, 8), device="cuda")
    assert codec.compress(x, (0, 8), 1e-3)[0] == sdcsz.EINVAL
    assert codec.compress(x, (8, 8), -1.0)[0] == sdcsz.EINVAL
    bad = torch.zeros(256, dtype=torch.uint8, device="cuda")
    assert codec.decompress(bad)[0] == sdcsz.EFORMAT


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_compression_fault_counts_match_oracle(codec, dtype):
    shape, block = (48, 42, 36), (6, 6, 6)
    x = synth.grf_field(shape, seed=3, dtype=dtype)
    plan = synth.fault_plan(shape, block, dtype, {"input": 6, "coef": 6, "code": 6, "dup_pred": 6,
                                                  "dup_recon": 6}, seed=31)
    for abft in (True, False):
        (rc_r, s_r, rep_r), (rc_g, s_g, rep_g) = both(codec, x, block, 1e-4, abft=abft, faults=plan)
        assert rc_r == rc_g, (rc_r, rc_g)
        same_counts(rep_r, rep_g)
        assert rep_g["generic_plan_blocks"] == 0  # every flip applied by the specialised kernels
        if rc_r == 0:
            assert np.array_equal(s_r, s_g), first_difference(s_r, s_g)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,block", [((48, 42, 36), (6, 6, 6)), ((400, 390), (16, 16))])
def test_every_coefficient_word_is_repaired(codec, dtype, shape, block):
    # one flip on each coefficient word (the four coefficients' words, low
    # word first in FP64), on distinct blocks, at low, middle and top bits:
    # every flip is located and repaired, as in the oracle (a flip of the
    # FP64 mean's words was once left uncorrectable by the compiled kernel)
    x = synth.grf_field(shape, seed=41, dtype=dtype)
    per = 1 if dtype == np.float32 else 2
    rows = []
    for wd in range(4 * per):
        for t, bit in enumerate((0, 17, 31)):
            rows.append((1, bit, 3 + 7 * wd + 2 * t, wd))
    plan = np.array(sorted(rows, key=lambda r: r[2]), dtype=np.int64)
    (rc_r, s_r, rep_r), (rc_g, s_g, rep_g) = both(codec, x, block, 1e-4, faults=plan)
    assert rc_r == rc_g == 0, (rc_r, rc_g)
    same_counts(rep_r, rep_g)
    assert rep_g["coef"]["corrected"] == len(rows), rep_g["coef"]
    assert rep_g["generic_plan_blocks"] == 0
    assert np.array_equal(s_r, s_g), first_difference(s_r, s_g)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,block", [((48, 42, 36), (6, 6, 6)), ((400, 390), (16, 16))])
def test_several_flips_in_one_block_match_oracle(codec, dtype, shape, block):
    # input, coefficient and prediction flips together, or coefficient and
    # reconstruction flips together, stay on the specialised kernels; two of
    # a kind, or a reconstruction flip after an input flip, send the block to
    # the generic routine
    x = synth.grf_field(shape, seed=16, dtype=dtype)
    per = 1 if dtype == np.float32 else 2
    bits = 32 * per
    rows = [(0, 30, 3, 7), (1, 29, 3, 2), (4, bits - 2, 3, 11),  # block 3: INPUT, COEF, DUP_PRED
            (1, 31, 5, 3), (5, 20, 5, 40),                      # block 5: COEF, DUP_RECON
            (0, 31, 9, 5), (0, 4, 9, 60),                       # block 9: two INPUT
            (4, 3, 12, 0), (4, bits - 1, 12, 1),                # block 12: two DUP_PRED
            (0, 27, 14, 9), (5, 6, 14, 30),                     # block 14: INPUT, DUP_RECON
            (2, 9, 20, 4), (2, 3, 20, 5)]                       # block 20: two CODE
    plan = np.array(sorted(rows, key=lambda r: r[2]), dtype=np.int64)
    for abft in (True, False):
        (rc_r, s_r, rep_r), (rc_g, s_g, rep_g) = both(codec, x, block, 1e-3, abft=abft, faults=plan)
        assert rc_r == rc_g, (rc_r, rc_g)
        same_counts(rep_r, rep_g)
        assert rep_g["generic_plan_blocks"] == 3
        if rc_r == 0:
            assert np.array_equal(s_r, s_g), first_difference(s_r, s_g)


def test_reexecution_queue_overflow_is_an_error(codec):
    # 5,000 blocks whose duplicated predictions disagree: the oracle corrects
    # them all, the library queues at most 4,096 re-executions and reports
    # the call as uncorrectable instead of keeping the others' results
    shape, block = (108, 108, 108), (6, 6, 6)
    x = synth.grf_field(shape, seed=17)
    plan = synth.fault_plan(shape, block, np.float32, {"dup_pred": 5000}, seed=18)
    rc, _, rep = codec.compress(torch.from_numpy(x).cuda(), block, 1e-3, faults=plan)
    assert rc == sdcsz.ESDC
    assert rep["dup_pred"]["detected"] == 5000
    rc, _, _ = codec.compress(torch.from_numpy(x).cuda(), block, 1e-3,
                              faults=synth.fault_plan(shape, block, np.float32, {"dup_pred": 4000}, seed=18))
    assert rc == sdcsz.OK


def test_decompression_faults_and_verify(codec):
    shape, block = (48, 42, 36), (6, 6, 6)
    x = synth.grf_field(shape, seed=3)
    rc, s, _ = ref.compress(x, block, 1e-4)
    plan = synth.fault_plan(shape, block, np.float32, {"recon": 25}, seed=8)
    rc_r, y_r, rep_r = ref.decompress(s, faults=plan)
    sd = torch.from_numpy(s).cuda()
    rc_g, y_g, rep_g = codec.decompress(sd, faults=plan)
    assert rc_r == rc_g == 0
    same_counts(rep_r, rep_g)
    assert rep_g["generic_plan_blocks"] == 0
    assert np.array_equal(y_r.view(np.uint32), y_g.cpu().numpy().view(np.uint32))
    z = y_g.clone()
    rc_v, rep_v = codec.verify(sd, z, faults=plan)
    assert rc_v == 0 and rep_v["recon"]["corrected"] == 25
    assert torch.equal(z, y_g)


def test_corrupt_stream_is_reported(codec):
    x = synth.grf_field((24, 24, 24), seed=3)
    rc, s, _ = ref.compress(x, (6, 6, 6), 1e-4)
    from tests.gpu_util import sections
    bad = s.copy()
    bad[sections(s)["payload"] + 40] ^= 0x10
    rc_r, _, rep_r = ref.decompress(bad)
    rc_g, _, rep_g = codec.decompress(torch.from_numpy(bad).cuda())
    assert rc_r == rc_g == sdcsz.ESDC
    same_counts(rep_r, rep_g)


def test_region(codec):
    x = synth.grf_field((30, 26, 20), seed=6)
    rc, s, _ = ref.compress(x, (6, 6, 6), 1e-3)
    lo, hi = (5, 3, 7), (17, 26, 13)
    rc_r, part_r, _ = ref.decompress_region(s, lo, hi)
    rc_g, part_g, _ = codec.decompress_region(torch.from_numpy(s).cuda(), lo, hi)
    assert rc_r == rc_g == 0
    assert np.array_equal(part_r.view(np.uint32), part_g.cpu().numpy().view(np.uint32))


def _regions(shape, block, rng, n):
    """Regions of a field: the whole field, single values at the corners,
    regions aligned to blocks, regions inside one block, slabs, regions
    touching the partial blocks at the upper faces, and random boxes."""
    nd = len(shape)
    out = [((0,) * nd, tuple(shape)), ((0,) * nd, (1,) * nd),
           (tuple(v - 1 for v in shape), tuple(shape)),
           (tuple(block), tuple(min(2 * b, v) for b, v in zip(block, shape))),
           (tuple(1 for _ in shape), tuple(min(b - 1, v) for b, v in zip(block, shape))),
           (tuple(v // 2 for v in shape), tuple(shape)),
           ((0,) * (nd - 1) + (shape[-1] // 3,), tuple(shape[:-1]) + (shape[-1] // 3 + 1,))]
    for _ in range(n):
        lo = [int(rng.integers(0, v)) for v in shape]
        hi = [int(rng.integers(a + 1, v + 1)) for a, v in zip(lo, shape)]
        out.append((tuple(lo), tuple(hi)))
    return out


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,block", [((40, 37, 35), (6, 6, 6)), ((70, 83), (16, 16)), ((5000,), (64,))])
def test_regions_match_oracle(codec, dtype, shape, block):
    """Region decompression on the specialised decoder (6x6x6, 16x16) and
    the generic one (1D): every region equals the oracle's, and the slice of
    full decompression."""
    x = synth.grf_field(shape, seed=8, dtype=dtype)
    rc, s, _ = ref.compress(x, block, 1e-3)
    assert rc == 0
    sd = torch.from_numpy(s).cuda()
    rc, full, _ = codec.decompress(sd)
    assert rc == 0
    full = full.cpu().numpy()
    u = np.uint32 if dtype == np.float32 else np.uint64
    for lo, hi in _regions(shape, block, np.random.default_rng(3), 12):
        print(f"case region shape={shape} dtype={np.dtype(dtype).name} lo={lo} hi={hi}", flush=True)
        rc_r, part_r, _ = ref.decompress_region(s, lo, hi)
        rc_g, part_g, _ = codec.decompress_region(sd, lo, hi)  # the stream's state, built once
        rc_1, part_1, _ = codec.decompress_region(sd, lo, hi, cache=False)  # tables rebuilt in the call
        assert rc_r == rc_g == rc_1 == 0, (rc_r, rc_g, rc_1)
        part_g = part_g.cpu().numpy()
        assert np.array_equal(part_r.view(u), part_g.view(u))
        assert np.array_equal(part_1.cpu().numpy().view(u), part_g.view(u))
        assert np.array_equal(full[tuple(slice(a, b) for a, b in zip(lo, hi))].view(u), part_g.view(u))


def test_region_state_is_checked_against_the_stream(codec):
    """A region state answers only for the stream it was built from: a
    different stream in the same buffer, or a wrong header from the caller,
    is a format error, and the codec's cache rebuilds the state for the new
    stream."""
    import ctypes as C
    xa = synth.grf_field((30, 30, 30), seed=21)
    xb = synth.grf_field((30, 30, 30), seed=22)
    rc, sa, _ = ref.compress(xa, (6, 6, 6), 1e-3)
    rc2, sb, _ = ref.compress(xb, (6, 6, 6), 1e-3)
    assert rc == rc2 == 0
    n = max(sa.size, sb.size)
    buf = torch.zeros(n, dtype=torch.uint8, device="cuda")
    buf[:sa.size] = torch.from_numpy(sa).cuda()
    view = buf[:sa.size]
    lo, hi = (3, 4, 5), (20, 21, 30)
    rc, state = codec.prepare_region(view)
    assert rc == 0
    rc, part, _ = codec.decompress_region(view, lo, hi, state=state)
    assert rc == 0
    assert np.array_equal(part.cpu().numpy().view(np.uint32), ref.decompress_region(sa, lo, hi)[1].view(np.uint32))
    L = sdcsz.lib()
    lo_a = (C.c_uint64 * 3)(*lo)
    hi_a = (C.c_uint64 * 3)(*hi)
    out = torch.empty(part.shape, dtype=torch.float32, device="cuda")

    def prepared(stream, header):
        hb = C.create_string_buffer(header, sdcsz.HEADER_BYTES)
        return L.sdcsz_decompress_region_prepared(
            C.c_void_p(stream.data_ptr()), stream.numel(), C.cast(hb, C.c_void_p), lo_a, hi_a,
            C.c_void_p(out.data_ptr()), out.numel() * 4, None, C.c_void_p(state.ws.data_ptr()), state.ws.numel(),
            None)
    bad_header = bytearray(state.header)
    bad_header[100] ^= 1
    assert prepared(view, bytes(bad_header)) == sdcsz.EFORMAT
    # stream B in the same buffer: its header differs from the state's
    buf[:sb.size] = torch.from_numpy(sb).cuda()
    view_b = buf[:sb.size]
    assert prepared(view_b, bytes(sb[:192])) == sdcsz.EFORMAT
    # the codec's cache (keyed by address) notices and rebuilds
    buf[:sa.size] = torch.from_numpy(sa).cuda()
    rc, _, _ = codec.decompress_region(buf[:sa.size], lo, hi)
    assert rc == 0
    buf[:sb.size] = torch.from_numpy(sb).cuda()
    rc, part_b, _ = codec.decompress_region(buf[:sb.size], lo, hi)
    assert rc == 0
    assert np.array_equal(part_b.cpu().numpy().view(np.uint32), ref.decompress_region(sb, lo, hi)[1].view(np.uint32))


def test_region_invalid_bounds(codec):
    x = synth.grf_field((20, 20, 20), seed=9)
    rc, s, _ = codec.compress(torch.from_numpy(x).cuda(), (6, 6, 6), 1e-3)
    assert rc == 0
    for lo, hi in (((0, 0, 0), (21, 20, 20)), ((5, 5, 5), (5, 6, 6)), ((3, 3, 3), (2, 9, 9))):
        rc, _, _ = codec.decompress_region(s, lo, hi)
        assert rc == sdcsz.EINVAL, (lo, hi, rc)


def _codebook(s):
    n_sym = int(np.frombuffer(s[76:80].tobytes(), "<u4")[0])
    return n_sym, s[192:192 + 4 * n_sym].view("<u4")


def _decode_both(codec, s):
    rc_r, y_r, rep_r = ref.decompress(s)
    rc_g, y_g, rep_g = codec.decompress(torch.from_numpy(s).cuda())
    assert rc_r == rc_g, (rc_r, rc_g)
    if rc_r in (0, sdcsz.ESDC):
        same_counts(rep_r, rep_g)
        assert np.array_equal(y_r.view(np.uint32), y_g.cpu().numpy().view(np.uint32))
    return rc_r


def test_codebook_entries_in_any_order(codec):
    # the format names used symbols with their lengths; codes follow from
    # (length, symbol) whatever order the entries are listed in
    x = synth.grf_field((30, 24, 18), seed=4)
    rc, s, _ = ref.compress(x, (6, 6, 6), 1e-3)
    n_sym, cb = _codebook(s)
    assert n_sym > 8
    shuffled = s.copy()
    perm = np.random.default_rng(5).permutation(n_sym)
    shuffled[192:192 + 4 * n_sym] = cb[perm].view(np.uint8)
    assert _decode_both(codec, shuffled) == 0
    rc0, y0, _ = ref.decompress(s)
    rc1, y1, _ = codec.decompress(torch.from_numpy(shuffled).cuda())
    assert np.array_equal(y0.view(np.uint32), y1.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("edit", ["duplicate", "zero_length", "too_long", "symbol_range"])
def test_invalid_codebook_is_a_format_error(codec, edit):
    x = synth.grf_field((24, 24, 24), seed=4)
    rc, s, _ = ref.compress(x, (6, 6, 6), 1e-3)
    n_sym, cb = _codebook(s)
    bad = s.copy()
    e = bad[192:192 + 4 * n_sym].view("<u4")
    if edit == "duplicate":
        e[1] = (e[0] & ~np.uint32(0xFF)) | (e[1] & np.uint32(0xFF))
    elif edit == "zero_length":
        e[2] &= ~np.uint32(0xFF)
    elif edit == "too_long":
        e[2] = (e[2] & ~np.uint32(0xFF)) | np.uint32(25)
    else:
        e[3] = (np.uint32(70000) << np.uint32(8)) | (e[3] & np.uint32(0xFF))
    assert _decode_both(codec, bad) == sdcsz.EFORMAT


def test_oversubscribed_codebook_decodes_like_the_oracle(codec):
    # a length edited shorter breaks the prefix property: both sides still
    # take, bit by bit, the shortest codeword that matches
    x = synth.grf_field((24, 24, 24), seed=4)
    rc, s, _ = ref.compress(x, (6, 6, 6), 1e-3)
    n_sym, cb = _codebook(s)
    for t, new_len in ((n_sym // 2, 2), (n_sym - 1, 1), (0, 3)):
        bad = s.copy()
        e = bad[192:192 + 4 * n_sym].view("<u4")
        e[t] = (e[t] & ~np.uint32(0xFF)) | np.uint32(new_len)
        _decode_both(codec, bad)


def test_block_table_total_mismatch_is_a_format_error(codec):
    x = synth.grf_field((24, 24, 24), seed=4)
    rc, s, _ = ref.compress(x, (6, 6, 6), 1e-3)
    from tests.gpu_util import sections
    bad = s.copy()
    tab = bad[sections(s)["table"]:].view("<u4")
    tab[0] += 1
    assert _decode_both(codec, bad) == sdcsz.EFORMAT


def test_output_too_small_writes_nothing(codec):
    import ctypes as C
    x = synth.grf_field((30, 24, 18), seed=4)
    xd = torch.from_numpy(x).cuda()
    rc, s_r, _ = ref.compress(x, (6, 6, 6), 1e-3)
    L = sdcsz.lib()
    p = sdcsz.make_params(x.shape, True, (6, 6, 6), 1e-3)
    ws = torch.empty(L.sdcsz_compress_workspace_size(C.byref(p)), dtype=torch.uint8, device="cuda")
    out = torch.full((s_r.size + 64,), 0xA5, dtype=torch.uint8, device="cuda")
    size = C.c_uint64(0)
    rep = sdcsz.Report()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.sdcsz_compress(C.c_void_p(xd.data_ptr()), C.byref(p), C.c_void_p(out.data_ptr()), s_r.size - 8,
                          C.byref(size), C.byref(rep), C.c_void_p(ws.data_ptr()), ws.numel(), st)
    assert rc == sdcsz.ENOSPC and size.value == s_r.size
    assert bool((out == 0xA5).all())
    rc = L.sdcsz_compress(C.c_void_p(xd.data_ptr()), C.byref(p), C.c_void_p(out.data_ptr()), s_r.size,
                          C.byref(size), C.byref(rep), C.c_void_p(ws.data_ptr()), ws.numel(), st)
    assert rc == 0 and size.value == s_r.size
    assert np.array_equal(out[: s_r.size].cpu().numpy(), s_r)
    assert bool((out[s_r.size:] == 0xA5).all())


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("abft", [True, False])
def test_one_pass_encoding_matches_two_pass(codec, dtype, abft):
    # an output that holds the largest stream takes the one-pass code check
    # and encoding (k_checkenc_fast); a smaller one the check, scans and
    # encoding in three passes: both give the oracle's stream, code flips
    # (repaired with ABFT) included, over several tiles of 256 blocks
    import ctypes as C
    shape = (60, 66, 54)  # 10 x 11 x 9 blocks: 990, four tiles, the last partial
    x = synth.grf_field(shape, seed=44, dtype=dtype)
    plan = synth.fault_plan(shape, (6, 6, 6), dtype, {"code": 8}, seed=45) if abft else None
    rc_r, s_r, rep_r = ref.compress(x, (6, 6, 6), 1e-4, abft=abft, faults=plan)
    assert rc_r == 0
    xd = torch.from_numpy(x).cuda()
    rc, s_one, rep_one = codec.compress(xd, (6, 6, 6), 1e-4, abft=abft, faults=plan)
    assert rc == 0 and np.array_equal(s_one.cpu().numpy(), s_r), first_difference(s_r, s_one.cpu().numpy())
    same_counts(rep_r, rep_one)
    L = sdcsz.lib()
    p = sdcsz.make_params(x.shape, dtype == np.float32, (6, 6, 6), 1e-4, abft=abft, faults=plan)
    ws = torch.empty(L.sdcsz_compress_workspace_size(C.byref(p)), dtype=torch.uint8, device="cuda")
    assert s_r.size < L.sdcsz_max_compressed_size(C.byref(p))
    out = torch.zeros(s_r.size, dtype=torch.uint8, device="cuda")
    size = C.c_uint64(0)
    rep = sdcsz.Report()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.sdcsz_compress(C.c_void_p(xd.data_ptr()), C.byref(p), C.c_void_p(out.data_ptr()), out.numel(),
                          C.byref(size), C.byref(rep), C.c_void_p(ws.data_ptr()), ws.numel(), st)
    assert rc == 0 and size.value == s_r.size
    assert np.array_equal(out.cpu().numpy(), s_r)
    same_counts(rep_r, sdcsz.report_dict(rep))


@pytest.mark.parametrize("shape,eb", [((48, 42, 36), 2e-5), ((102, 102, 102), 1e-5),
                                      ((102, 102, 102), 1e-6)])
def test_large_codebooks_decode_like_the_oracle(codec, shape, eb):
    # tens of thousands of symbols: the specialised decoder's second-level
    # table outgrows its LDS share (entries past it come from the global
    # table), and at 1e-6 (65,529 symbols, 65,830 second-level entries) it
    # exceeds the 65,536 entries built, so the long prefixes take the length
    # search
    x = synth.grf_field(shape, seed=9)
    s, rep = check_roundtrip(codec, x, (6, 6, 6), eb)
    n_sym = int(np.frombuffer(s[76:80].tobytes(), "<u4")[0])
    assert n_sym > 8000, n_sym


def _config4_like_fields(n, seed):
    """Fields of uneven shapes, dtypes and bounds, as in a batch of mixed
    2D/3D outputs (GRF, spectral slope U[-4,-2]); small sizes for the oracle."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        two_d = i % 2 == 1
        dtype = np.float64 if i % 4 == 3 else np.float32
        if two_d:
            shape = tuple(int(v) for v in rng.integers(40, 160, size=2))
            block = (16, 16)
        else:
            shape = tuple(int(v) for v in rng.integers(14, 44, size=3))
            block = (6, 6, 6)
        eb = float(10 ** rng.uniform(-5, -2))
        x = synth.grf_field(shape, seed=int(rng.integers(1 << 30)), slope=float(rng.uniform(-4, -2)),
                            dtype=dtype)
        out.append((x, block, eb))
    return out


def test_batch_matches_single_calls_and_oracle(codec):
    fields = _config4_like_fields(12, seed=4)
    xs = [torch.from_numpy(x).cuda() for x, _, _ in fields]
    rc, res = codec.compress_batch(xs, [b for _, b, _ in fields], [e for _, _, e in fields])
    assert rc == 0, rc
    for (x, block, eb), (rc_i, s_g, rep_g) in zip(fields, res):
        print(f"case batch field shape={x.shape} dtype={x.dtype} eb={eb:.3g}", flush=True)
        assert rc_i == 0
        rc_r, s_r, rep_r = ref.compress(x, block, eb)
        s_g = s_g.cpu().numpy()
        assert np.array_equal(s_r, s_g), first_difference(s_r, s_g)
        same_counts(rep_r, rep_g)
    # decompress the whole batch in one call
    streams = [s for _, s, _ in res]
    rc, dres = codec.decompress_batch(streams)
    assert rc == 0, rc
    for (x, block, eb), (rc_i, y, rep) in zip(fields, dres):
        assert rc_i == 0
        rc_r, y_r, _ = ref.decompress(ref.compress(x, block, eb)[1])
        assert np.array_equal(y_r.view(np.uint8), y.cpu().numpy().view(np.uint8))


def test_batch_item_errors_stay_per_item(codec):
    good = torch.from_numpy(synth.grf_field((20, 20, 20), seed=5)).cuda()
    rc, res = codec.compress_batch([good, good], [(6, 6, 6), (0, 6, 6)], 1e-3)
    assert rc == sdcsz.EINVAL
    assert res[0][0] == 0 and res[1][0] == sdcsz.EINVAL
    rc_r, s_r, _ = ref.compress(good.cpu().numpy(), (6, 6, 6), 1e-3)
    assert np.array_equal(res[0][1].cpu().numpy(), s_r)


def test_caller_header_is_checked_against_the_stream(codec):
    """Compression returns the stream header; decompression given that copy
    matches decompression that reads it back, and a copy that differs from
    the stream (here only in the stored bound, which the host cannot tell)
    is a format error that writes nothing."""
    x = synth.grf_field((30, 26, 22), seed=21)
    rc, s, rep = codec.compress(torch.from_numpy(x).cuda(), (6, 6, 6), 1e-3)
    assert rc == 0
    s = s.clone()  # not the codec's own buffer: nothing cached for it
    hdr = rep["header"]
    assert hdr == bytes(s[: sdcsz.HEADER_BYTES].cpu().numpy())
    rc_r, y_r, _ = ref.decompress(s.cpu().numpy())
    for h in (None, hdr):
        print(f"case header given={h is not None}", flush=True)
        rc, y, _ = codec.decompress(s, header=h)
        assert rc == rc_r == 0
        assert np.array_equal(y_r.view(np.uint8), y.cpu().numpy().view(np.uint8))
    bad = bytearray(hdr)
    bad[56] ^= 1  # lowest mantissa bit of the stored bound
    out = torch.full(x.shape, 7.0, device="cuda:0")
    rc, y, _ = codec.decompress(s, out=out, header=bytes(bad))
    assert rc == sdcsz.EFORMAT
    assert bool((out == 7.0).all())
    # a batch mixing items with a correct header, a wrong one and none
    print("case header batch", flush=True)
    rc, res = codec.decompress_batch([s, s, s], headers=[hdr, bytes(bad), None])
    assert rc == sdcsz.EFORMAT
    assert [r[0] for r in res] == [0, sdcsz.EFORMAT, 0]
    for i in (0, 2):
        assert np.array_equal(y_r.view(np.uint8), res[i][1].cpu().numpy().view(np.uint8))


@pytest.mark.parametrize("lanes", [64, 128])
def test_launch_shape_does_not_change_results(codec, lanes):
    from paper_2010_03144_amd import tune
    cases = [(synth.grf_field((50, 47, 44), seed=21), (6, 6, 6)),
             (synth.grf_field((50, 47, 44), seed=22, dtype=np.float64), (6, 6, 6)),
             (synth.grf_field((300, 417), seed=23), (16, 16)),
             (synth.grf_field((300, 417), seed=24, dtype=np.float64), (16, 16))]
    ref_out = []
    for x, block in cases:
        rc, s, _ = codec.compress(torch.from_numpy(x).cuda(), block, 1e-3)
        assert rc == 0
        rc, y, _ = codec.decompress(s)
        ref_out.append((s.cpu().numpy(), y.cpu().numpy()))
    try:
        for si in range(len(sdcsz.TUNE_STAGES)):
            for ci in range(len(sdcsz.SHAPE_CLASSES)):
                for dt in (0, 1):
                    assert sdcsz.tune_set(si, ci, dt, [(tune.UNBOUNDED, lanes)]) == sdcsz.OK
        for (x, block), (s_ref, y_ref) in zip(cases, ref_out):
            print(f"case lanes={lanes} shape={x.shape} dtype={x.dtype}", flush=True)
            rc, s, _ = codec.compress(torch.from_numpy(x).cuda(), block, 1e-3)
            assert rc == 0
            assert np.array_equal(s.cpu().numpy(), s_ref), first_difference(s_ref, s.cpu().numpy())
            rc, y, _ = codec.decompress(s)
            assert rc == 0 and np.array_equal(y.cpu().numpy().view(np.uint8), y_ref.view(np.uint8))
    finally:
        tune.reset()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,block", [((48, 42, 36), (6, 6, 6)), ((400, 390), (16, 16))])
def test_preparation_fault_counts_and_streams_match_oracle(codec, dtype, shape, block):
    x = synth.grf_field(shape, seed=15, dtype=dtype)
    plan = synth.fault_plan(shape, block, dtype, {"prep_input": 6, "prep_coef": 6, "prep_sample": 6,
                                                  "input": 3, "coef": 3}, seed=45)
    for abft in (True, False):
        (rc_r, s_r, rep_r), (rc_g, s_g, rep_g) = both(codec, x, block, 1e-3, abft=abft, faults=plan)
        assert rc_r == rc_g, (rc_r, rc_g)
        same_counts(rep_r, rep_g)
        assert rep_g["generic_plan_blocks"] == 18  # the preparation errors; INPUT and COEF stay specialised
        if rc_r == 0:
            assert np.array_equal(s_r, s_g), first_difference(s_r, s_g)

