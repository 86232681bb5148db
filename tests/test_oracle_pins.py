"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the ABFT
algebra of Sec. 3.2 by exhaustive bit flips, the checksum capacity of Sec. 5.4,
the closed-form least-squares plane against numpy's lstsq, the Lorenzo
predictor against mixed finite differences on exact integers, the Huffman code
against a textbook heap-based construction, the error bound of every element,
and the fault-tolerance outcomes of Algorithms 1 and 2.
"""
import heapq
import json
import os

import numpy as np
import pytest

from oracle import ref
from paper_2010_03144_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


def blocks_of(x, block):
    """Yield (block index, view) in C order of blocks (partial blocks at the edges)."""
    grid = synth.block_grid(x.shape, block)
    for b, idx in enumerate(np.ndindex(*grid)):
        sl = tuple(slice(i * s, min((i + 1) * s, n)) for i, s, n in zip(idx, block, x.shape))
        yield b, x[sl]


# --------------------------------------------------------------------------- checksums
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_checksum_locates_and_repairs_every_single_bit_flip(dtype):
    """Sec. 3.2: j = (isum' - isum) / (sum' - sum) locates the corrupted word;
    Sec. 5.4: FP64 values are two 32-bit words.  Exhaustive over a 6^3 block."""
    rng = np.random.default_rng(7)
    vals = rng.standard_normal(216).astype(dtype)
    words = vals.view(np.uint32).copy()
    s, i = ref.checksums(words)
    n = words.size
    for j in range(n):
        for bit in range(32):
            w = words.copy()
            w[j] ^= np.uint32(1 << bit)
            assert ref.correct(w, s, i, 32) == 1
            assert np.array_equal(w, words), (j, bit)
    assert ref.correct(words.copy(), s, i, 32) == 0


def test_checksum_codes_16bit_flips():
    """Same algebra on the bin array (16-bit codes)."""
    rng = np.random.default_rng(8)
    codes = rng.integers(1, 65536, 216).astype(np.uint32)
    s, i = ref.checksums(codes)
    for j in range(216):
        for bit in range(16):
            w = codes.copy()
            w[j] ^= np.uint32(1 << bit)
            assert ref.correct(w, s, i, 16) == 1
            assert np.array_equal(w, codes)


def test_checksum_paper_example_and_capacity():
    g = json.load(open(GOLDEN))
    ex = g["abft_example"]
    a = np.array(ex["array"], dtype=np.uint32)
    s0, i0 = ref.checksums(a)
    b = a.copy()
    b[ex["corrupt_index"]] = ex["corrupt_value"]
    s1, i1 = ref.checksums(b)
    assert (i1 - i0) // (s1 - s0) == ex["corrupt_index"]
    assert ref.correct(b, s0, i0, 32) == 1 and np.array_equal(a, b)
    cap = g["checksum_capacity_words"]["value"]
    assert (2**64 - 1) // (2**32 - 1) == cap
    # no wrap at the largest block the library accepts: all-ones words
    n = 8192 * 2
    ones = np.full(n, 0xFFFFFFFF, np.uint32)
    s, i = ref.checksums(ones)
    assert s == n * (2**32 - 1)
    assert i == (n * (n - 1) // 2) * (2**32 - 1)


def test_checksum_zero_sum_difference_is_uncorrectable():
    w = np.array([5, 9, 1, 7], np.uint32)
    s, i = ref.checksums(w)
    w2 = w.copy()
    w2[0] += 1
    w2[1] -= 1  # sum unchanged, isum changed
    assert ref.correct(w2, s, i, 32) == -1


# --------------------------------------------------------------------------- regression
@pytest.mark.parametrize("shape", [(6, 6, 6), (4, 6, 2), (2, 6, 5), (16, 16), (7, 3), (64,), (5,)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_regression_matches_lstsq(shape, dtype):
    """Alg. 1, regression coefficients: the closed form equals the least-squares plane."""
    rng = np.random.default_rng(11)
    x = (rng.standard_normal(shape) + 3.0).astype(dtype)
    coef = ref.regression(x)
    full = (1,) * (3 - len(shape)) + shape
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) - (n - 1) / 2 for n in full], indexing="ij")
    cols = [g.ravel() for a, g in enumerate(grids) if full[a] > 1]
    A = np.stack(cols + [np.ones(x.size)], axis=1)
    sol = np.linalg.lstsq(A, x.astype(np.float64).ravel(), rcond=None)[0]
    want = np.zeros(4)
    at = 0
    for a in range(3):
        if full[a] > 1:
            want[a] = sol[at]
            at += 1
    want[3] = sol[at]
    tol = 2e-5 if dtype == np.float32 else 1e-12
    np.testing.assert_allclose(coef.astype(np.float64), want, rtol=tol, atol=tol * 4)


@pytest.mark.parametrize("shape,block", [((30, 24, 18), (6, 6, 6)), ((40, 33), (16, 16)),
                                         ((17, 11, 9), (6, 6, 6))])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_linear_field_gives_zero_codes(shape, block, dtype):
    """A field linear inside every block is predicted exactly by regression:
    every block picks regression and every code is the zero residual (32768)."""
    f = synth.linear_field(shape, [0.3, -0.2, 0.1][: len(shape)], 5.0, dtype)
    rc, stream, rep, dbg = ref.compress(f, block, 1e-3, debug=True)
    assert rc == 0
    assert dbg["is_regression"].all()
    assert (dbg["codes"] == 32768).all()
    assert rep["n_outliers"] == 0


def test_selection_prefers_lorenzo_without_three_way_interaction():
    """Alg. 1, sampling loop: a field f(i, j) with no dependence on k and strong
    curvature is predicted exactly by Lorenzo away from the block's k = 0 face,
    while no plane fits it; every full block must pick Lorenzo."""
    i, j, k = np.meshgrid(np.arange(24), np.arange(24), np.arange(24), indexing="ij")
    f = (40.0 * np.sin(1.3 * i) * np.cos(0.9 * j) + 0.0 * k).astype(np.float32)
    rc, s, rep, dbg = ref.compress(f, (6, 6, 6), 1e-4, debug=True)
    assert rc == 0
    assert not dbg["is_regression"].any()


# --------------------------------------------------------------------------- Lorenzo
@pytest.mark.parametrize("shape,block", [((5, 7, 4), (3, 3, 3)), ((3, 3, 3), (3, 3, 3)),
                                         ((2, 2, 2), (2, 2, 2)), ((1, 1, 1), (6, 6, 6)),
                                         ((9, 10), (4, 4)), ((13,), (5,))])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_lorenzo_residual_is_mixed_difference(shape, block, dtype):
    """Lorenzo prediction inside independent blocks (zero outside the block).
    With integer data and eb = 1/2 the reconstruction is exact, so each code
    minus 32768 must equal the mixed backward difference of the block."""
    rng = np.random.default_rng(5)
    x = rng.integers(-8, 9, shape).astype(dtype)
    rc, stream, rep, dbg = ref.compress(x, block, 0.5, eb_mode="abs", predictor="lorenzo",
                                        debug=True)
    assert rc == 0
    codes = dbg["codes"].astype(np.int64) - 32768
    at = 0
    for b, xb in blocks_of(x.astype(np.int64), block):
        r = xb
        for a in range(xb.ndim):
            r = np.diff(r, axis=a, prepend=0)
        n = xb.size
        assert np.array_equal(codes[at:at + n], r.ravel()), b
        at += n
    rc, y, _ = ref.decompress(stream)
    assert rc == 0 and np.array_equal(x, y)


# --------------------------------------------------------------------------- Huffman
def heap_huffman(counts):
    """Textbook Huffman by a binary heap: (optimal cost, deepest leaf)."""
    h = [(int(c), 0) for c in counts if c > 0]
    if len(h) <= 1:
        return sum(c for c, _ in h), len(h)
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, da = heapq.heappop(h)
        b, db = heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, (a + b, max(da, db) + 1))
    return cost, h[0][1]


def heap_cost(counts):
    return heap_huffman(counts)[0]


@pytest.mark.parametrize("seed", range(6))
def test_huffman_cost_is_optimal(seed):
    rng = np.random.default_rng(seed)
    hist = np.zeros(65536, np.uint64)
    nsym = [2, 3, 17, 300, 4000, 20000][seed]
    syms = rng.choice(65536, nsym, replace=False)
    hist[syms] = rng.geometric(0.01, nsym) * rng.integers(1, 50, nsym)
    lens = ref.huffman_lengths(hist)
    assert ((lens > 0) == (hist > 0)).all()
    cost = int((hist.astype(object) * lens.astype(object)).sum())
    best, depth = heap_huffman(hist)
    if depth <= 24:
        assert cost == best
    else:  # the 24-bit limit reshaped the tree: never better than optimal
        assert lens.max() <= 24 and cost >= best
    kraft = sum(2.0 ** -int(l) for l in lens if l)
    assert kraft == 1.0


def test_huffman_single_symbol_and_length_limit():
    hist = np.zeros(65536, np.uint64)
    hist[32768] = 1000
    lens = ref.huffman_lengths(hist)
    assert lens[32768] == 1 and lens.sum() == 1
    # Fibonacci weights build a 39-deep tree; the limit caps it at 24
    hist = np.zeros(65536, np.uint64)
    a, b = 1, 1
    for s in range(40):
        hist[100 + s] = a
        a, b = b, a + b
    lens = ref.huffman_lengths(hist)
    assert lens.max() <= 24
    assert sum(2.0 ** -int(l) for l in lens if l) == 1.0
    assert int((hist.astype(object) * lens.astype(object)).sum()) >= heap_cost(hist)


# --------------------------------------------------------------------------- error bound
def max_err(x, y):
    return float(np.max(np.abs(x.astype(np.float64) - y.astype(np.float64)))) if x.size else 0.0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4])
@pytest.mark.parametrize("abft", [True, False])
def test_error_bound_every_element(dtype, eb, abft):
    x = synth.bumps_field((40, 36, 30), seed=1, dtype=dtype)
    rc, s, rep = ref.compress(x, (6, 6, 6), eb, abft=abft)
    assert rc == 0
    rc, y, _ = ref.decompress(s)
    assert rc == 0
    assert max_err(x, y) <= rep["eb_abs"]
    assert rep["eb_abs"] == eb * (float(x.max()) - float(x.min()))
    # a rounding quantizer almost never needs the verbatim fallback on a smooth
    # field; truncation or a sign slip would turn about half the points into outliers
    assert rep["n_outliers"] <= 1e-3 * x.size


@pytest.mark.parametrize("shape,block", [((7, 13, 5), (6, 6, 6)), ((300, 7), (16, 16)),
                                         ((1000,), (64,)), ((1, 1, 1), (6, 6, 6)),
                                         ((33, 20), (8, 5))])
def test_error_bound_odd_shapes(shape, block):
    x = synth.grf_field(shape, seed=4, front=False, dtype=np.float32)
    for mode, eb in (("rel", 1e-3), ("abs", 0.05)):
        rc, s, rep = ref.compress(x, block, eb, eb_mode=mode)
        assert rc == 0
        rc, y, _ = ref.decompress(s)
        assert rc == 0 and max_err(x, y) <= rep["eb_abs"]


def test_constant_field_is_lossless():
    x = np.full((9, 8, 7), 3.25, np.float32)
    rc, s, rep = ref.compress(x, (6, 6, 6), 1e-3)
    assert rc == 0 and rep["eb_abs"] == 0.0 and rep["n_outliers"] == x.size
    rc, y, _ = ref.decompress(s)
    assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


def test_non_finite_values_survive_bit_exact():
    x = synth.bumps_field((12, 12, 12), seed=3)
    x[1, 2, 3] = np.nan
    x[7, 7, 7] = np.inf
    x[11, 0, 5] = -np.inf
    rc, s, rep = ref.compress(x, (6, 6, 6), 1e-3)
    assert rc == 0
    rc, y, _ = ref.decompress(s)
    bad = ~np.isfinite(x)
    assert np.array_equal(x[bad].view(np.uint32), y[bad].view(np.uint32))
    assert max_err(x[~bad], y[~bad]) <= rep["eb_abs"]


def test_empty_field():
    x = np.zeros((0, 5), np.float32)
    rc, s, rep = ref.compress(x, (16, 16), 1e-3)
    assert rc == 0 and s.size == 192
    rc, y, _ = ref.decompress(s)
    assert rc == 0 and y.shape == (0, 5)


def test_invalid_params():
    x = np.zeros((4, 4), np.float32)
    assert ref.compress(x, (4, 4), 0.0, eb_mode="abs")[0] == ref.EINVAL
    assert ref.compress(x, (4, 4), float("nan"))[0] == ref.EINVAL
    assert ref.compress(x, (0, 4), 1e-3)[0] == ref.EINVAL
    assert ref.decompress(np.zeros(64, np.uint8))[0] == ref.EFORMAT


# --------------------------------------------------------------------------- ABFT behaviour
def sections(stream):
    import struct
    h = stream[:192].tobytes()
    offs = struct.unpack_from("<7Q", h, 112)
    return dict(zip(["codebook", "table", "coef", "sumdc", "outliers", "payload", "total"], offs))


def test_abft_on_off_differ_only_in_flag_and_sum_dc():
    x = synth.bumps_field((30, 30, 30), seed=9)
    rc1, s1, _ = ref.compress(x, (6, 6, 6), 1e-3, abft=True)
    rc0, s0, _ = ref.compress(x, (6, 6, 6), 1e-3, abft=False)
    o1, o0 = sections(s1), sections(s0)
    assert o1["outliers"] - o1["sumdc"] == 8 * 125 and o0["outliers"] == o0["sumdc"]
    assert np.array_equal(s1[192:o1["sumdc"]], s0[192:o0["sumdc"]])
    assert np.array_equal(s1[o1["outliers"]:], s0[o0["outliers"]:])
    assert ref.decompress(s1)[1].tobytes() == ref.decompress(s0)[1].tobytes()


def test_deterministic():
    x = synth.grf_field((24, 24, 24), seed=2)
    a = ref.compress(x, (6, 6, 6), 1e-4)[1]
    b = ref.compress(x, (6, 6, 6), 1e-4)[1]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_compression_faults_are_corrected_bit_for_bit(dtype):
    """Mode-A memory errors in input, coefficients and codes, and computation
    errors in the duplicated prediction/reconstruction: with ABFT every one is
    detected and corrected, and the stream equals the fault-free stream."""
    shape, block = (36, 30, 24), (6, 6, 6)
    x = synth.grf_field(shape, seed=3, dtype=dtype)
    rc, clean, _ = ref.compress(x, block, 1e-4)
    assert rc == 0
    plan = synth.fault_plan(shape, block, dtype,
                            {"input": 12, "coef": 12, "code": 12, "dup_pred": 12, "dup_recon": 12},
                            seed=21)
    rc, s, rep = ref.compress(x, block, 1e-4, faults=plan)
    assert rc == 0
    assert np.array_equal(s, clean)
    for t in ("input", "coef", "code", "dup_pred"):
        assert rep[t]["injected"] == 12, t
        assert rep[t]["detected"] == rep[t]["corrected"] == 12, t
        assert rep[t]["uncorrectable"] == 0
    r = rep["dup_recon"]
    assert r["detected"] == r["corrected"] == r["injected"] and r["uncorrectable"] == 0


def test_decompression_faults_are_reexecuted():
    shape, block = (36, 30, 24), (6, 6, 6)
    x = synth.grf_field(shape, seed=3)
    rc, s, _ = ref.compress(x, block, 1e-4)
    rc, clean, _ = ref.decompress(s)
    plan = synth.fault_plan(shape, block, np.float32, {"recon": 20}, seed=5)
    rc, y, rep = ref.decompress(s, faults=plan)
    assert rc == 0 and np.array_equal(clean.view(np.uint32), y.view(np.uint32))
    assert rep["recon"]["injected"] == rep["recon"]["detected"] == rep["recon"]["corrected"] == 20
    # stand-alone verification of a caller buffer repairs it in place
    z = clean.copy()
    rc, rep = ref.verify(s, z, faults=plan)
    assert rc == 0 and np.array_equal(clean.view(np.uint32), z.view(np.uint32))
    assert rep["recon"]["corrected"] == 20


def test_corrupt_stream_reports_sdc():
    x = synth.grf_field((24, 24, 24), seed=3)
    rc, s, _ = ref.compress(x, (6, 6, 6), 1e-4)
    o = sections(s)
    bad = s.copy()
    bad[o["payload"] + 40] ^= 0x10  # a flipped payload bit survives re-execution
    rc, y, rep = ref.decompress(bad)
    assert rc == ref.ESDC and rep["recon"]["uncorrectable"] >= 1


def test_without_abft_an_input_error_breaks_the_bound():
    """The unprotected outcome of Table 3: an exponent-bit flip in the input
    after the checksums would be taken escapes the bound; with ABFT it does not."""
    shape, block = (24, 24, 24), (6, 6, 6)
    x = synth.bumps_field(shape, seed=2)
    plan = np.array([[0, 30, 17, 100]], np.int64)  # input word 100 of block 17, bit 30
    for abft in (True, False):
        rc, s, rep = ref.compress(x, block, 1e-3, abft=abft, faults=plan)
        assert rc == 0
        y = ref.decompress(s)[1]
        err = max_err(x, y)
        if abft:
            assert err <= rep["eb_abs"] and rep["input"]["corrected"] == 1
        else:
            assert err > rep["eb_abs"] and rep["input"]["detected"] == 0


def test_region_equals_slice_of_full_decompression():
    x = synth.grf_field((30, 26, 20), seed=6)
    rc, s, _ = ref.compress(x, (6, 6, 6), 1e-3)
    full = ref.decompress(s)[1]
    lo, hi = (5, 3, 7), (17, 26, 13)
    rc, part, _ = ref.decompress_region(s, lo, hi)
    assert rc == 0
    assert np.array_equal(part, full[5:17, 3:26, 7:13])


def test_cr_decrease_bound_example():
    """Sec. 5.5: one block falling to CR 1 costs at most (R0-1)/(R0+n-1)."""
    g = json.load(open(GOLDEN))["cr_bound_example"]
    n = g["input_bytes"] // g["value_bytes"] // int(np.prod(g["block"]))
    assert n == g["n_blocks"]
    r0 = g["cr"]
    # exact decrease when one of n equal blocks is stored raw
    size0 = n / r0
    size1 = (n - 1) / r0 + 1
    dec = 1 - size0 / size1
    assert abs(dec - (r0 - 1) / (r0 + n - 1)) < 1e-15
    assert dec < g["bound_below"]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_prediction_preparation_errors_keep_the_bound_and_stay_local(dtype):
    """Sec. 4.1-4.2: an error in the regression, in the sampled estimates, or
    in the input as those two read it can change only the struck block's
    coefficients, predictor and codes (so the compression ratio), never the
    error bound; with ABFT the input error is still found and repaired before
    the prediction reads the input."""
    shape, block = (36, 30, 24), (6, 6, 6)  # 6 x 5 x 4 = 120 full blocks
    x = synth.grf_field(shape, seed=3, dtype=dtype)
    rc, clean, rep0, d0 = ref.compress(x, block, 1e-3, debug=True)
    assert rc == 0
    plan = synth.fault_plan(shape, block, dtype, {"prep_input": 8, "prep_coef": 8, "prep_sample": 8}, seed=44)
    rc, s, rep, d1 = ref.compress(x, block, 1e-3, faults=plan, debug=True)
    assert rc == 0
    assert rep["prep_input"]["injected"] == rep["prep_input"]["detected"] == rep["prep_input"]["corrected"] == 8
    for t in ("prep_coef", "prep_sample"):
        assert rep[t]["injected"] == 8 and rep[t]["detected"] == 0, t
    assert rep["input"]["detected"] == 0
    struck = {int(b) for b in plan[:, 2]}
    for b in range(120):
        c0, c1 = d0["codes"][216 * b:216 * (b + 1)], d1["codes"][216 * b:216 * (b + 1)]
        if b not in struck:
            assert np.array_equal(c0, c1), b
            assert d0["is_regression"][b] == d1["is_regression"][b]
            assert np.array_equal(d0["coef"][4 * b:4 * b + 4].view(np.uint8), d1["coef"][4 * b:4 * b + 4].view(np.uint8))
    for row in plan:
        if row[0] == synth.TARGET_IDS["prep_coef"]:  # the corrupted coefficient is the one kept
            b = int(row[2])
            assert not np.array_equal(d0["coef"][4 * b:4 * b + 4].view(np.uint8),
                                      d1["coef"][4 * b:4 * b + 4].view(np.uint8))
    rc, y, _ = ref.decompress(s)
    assert rc == 0 and max_err(x, y) <= rep["eb_abs"]


def test_sampling_error_can_flip_the_predictor_only():
    """A flip of the top bit of one estimate reverses the comparison: the
    block takes the other predictor, and its values still respect the bound."""
    shape, block = (12, 12, 12), (6, 6, 6)
    x = synth.grf_field(shape, seed=8)
    rc, _, _, d0 = ref.compress(x, block, 1e-3, debug=True)
    for b in range(8):
        word = 1 if d0["is_regression"][b] else 0  # inflate the winner's estimate
        plan = np.array([[synth.TARGET_IDS["prep_sample"], 62, b, word]], np.int64)
        rc, s, rep, d1 = ref.compress(x, block, 1e-3, faults=plan, debug=True)
        assert rc == 0 and rep["prep_sample"]["injected"] == 1
        assert d1["is_regression"][b] != d0["is_regression"][b]
        others = [c for c in range(8) if c != b]
        assert all(d1["is_regression"][c] == d0["is_regression"][c] for c in others)
        assert max_err(x, ref.decompress(s)[1]) <= rep["eb_abs"]


def test_without_abft_a_preparation_input_error_reaches_the_output():
    shape, block = (24, 24, 24), (6, 6, 6)
    x = synth.bumps_field(shape, seed=2)
    plan = np.array([[synth.TARGET_IDS["prep_input"], 30, 17, 100]], np.int64)
    rc, s, rep = ref.compress(x, block, 1e-3, abft=False, faults=plan)
    assert rc == 0 and rep["prep_input"]["detected"] == 0
    assert max_err(x, ref.decompress(s)[1]) > rep["eb_abs"]


class _OracleCodec:
    """The oracle behind the Codec calls the block-size tools make."""

    def compress(self, x, block, eb, eb_mode="rel", abft=True):
        import torch
        rc, s, rep = ref.compress(x.numpy(), block, eb, eb_mode=eb_mode, abft=abft)
        return rc, torch.from_numpy(s), rep

    def decompress(self, s):
        import torch
        rc, y, rep = ref.decompress(s.numpy())
        return rc, torch.from_numpy(y), rep


def test_block_size_tools_on_the_oracle():
    """PSNR and bit-rate as defined in the paper's evaluation, and the block
    chosen is the one with the fewest bits at the same absolute bound."""
    torch = pytest.importorskip("torch")
    from paper_2010_03144_amd import blocksize
    x = torch.from_numpy(synth.grf_field((40, 36, 32), seed=9))
    y = x + 1e-3 * torch.from_numpy(np.random.default_rng(1).standard_normal(x.shape).astype(np.float32))
    xd, yd = x.double().numpy(), y.double().numpy()
    want = 20 * np.log10(xd.max() - xd.min()) - 10 * np.log10(np.mean((xd - yd) ** 2))
    assert abs(blocksize.psnr(x, y) - want) < 1e-9
    rd = blocksize.rate_distortion(_OracleCodec(), x, [1e-2, 1e-3], edges=(4, 8))
    for e, rows in rd.items():
        (eb1, b1, p1, _), (eb2, b2, p2, _) = rows
        assert b2 > b1 and p2 > p1  # a tighter bound costs bits and buys PSNR
    best, rates = blocksize.best_block(_OracleCodec(), x, 1e-3, edges=(4, 6, 10), side=16, count=2,
                                       fast_only=False)
    assert best == min(rates, key=rates.get) and set(rates) == {4, 6, 10}
    # by default the pick stays among shapes with specialised kernels (6^3 in 3D)
    best, rates2 = blocksize.best_block(_OracleCodec(), x, 1e-3, edges=(4, 6, 10), side=16, count=2)
    assert best == 6 and rates2 == rates
    assert blocksize.best_block(_OracleCodec(), x, 1e-3, edges=(4, 10), side=16, count=2)[0] == \
        min((4, 10), key=rates.get)
    eb_abs = 1e-3 * float(x.max() - x.min())
    v = blocksize.sample_views(x, 16, 2)[0]
    rc, s, _ = ref.compress(v.numpy(), (6, 6, 6), eb_abs, eb_mode="abs")
    assert rc == 0
