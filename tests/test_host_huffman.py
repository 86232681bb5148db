"""The library's host-side codebook builder against the oracle's Huffman
code lengths, and its codewords against the canonical-code definition.

The builder is compiled here with the host compiler (it is plain C++ without
device code) into a small driver, so these run without a GPU.  The
histograms have the shapes that matter for the length limit: heavy-tailed
counts whose unconstrained tree is deeper than 24 (several halvings, many
tied halved counts), Fibonacci counts, many equal counts, one and two symbols.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_03144_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("huff") / "huffman_host_driver")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "huffman_host_driver.cpp"),
                    "-o", exe], check=True)
    return exe


def run_driver(exe, hists):
    data = b"".join(np.ascontiguousarray(h, dtype=np.uint64).tobytes() for h in hists)
    out = subprocess.run([exe], input=data, stdout=subprocess.PIPE, check=True).stdout
    per = 65536 * 5
    assert len(out) == per * len(hists)
    res = []
    for i in range(len(hists)):
        chunk = out[i * per:(i + 1) * per]
        res.append((np.frombuffer(chunk[:65536], np.uint8), np.frombuffer(chunk[65536:], np.uint32)))
    return res


def canonical(lens):
    """Codewords from the definition: within a length, consecutive in symbol
    order; the first code of length l is (first code of l-1 + count of l-1) << 1."""
    count = np.bincount(lens[lens > 0], minlength=26)  # count[0] == 0
    first, c = {}, 0
    for l in range(1, 25):
        c = (c + int(count[l - 1])) << 1 if l > 1 else 0
        first[l] = c
    code = np.zeros(65536, np.uint32)
    nxt = dict(first)
    for s in np.nonzero(lens)[0]:
        code[s] = nxt[int(lens[s])]
        nxt[int(lens[s])] += 1
    return code


def histograms(seed):
    rng = np.random.default_rng(seed)
    out = []
    for kind in range(8):
        h = np.zeros(65536, np.uint64)
        n = int(rng.integers(2, 30000))
        syms = rng.choice(65536, n, replace=False)
        if kind == 0:    # two-sided geometric tail around the zero residual, as quantization codes
            z = np.arange(65536, dtype=np.float64) - 32768
            h = np.floor(2e7 * np.exp(-np.abs(z) / float(rng.uniform(30, 3000)))).astype(np.uint64)
        elif kind == 1:  # log-uniform counts over 9 decades: deep unconstrained trees
            h[syms] = np.exp(rng.uniform(0, 21, n)).astype(np.uint64) + 1
        elif kind == 2:  # mostly tiny counts with ties
            h[syms] = rng.integers(1, 4, n)
        elif kind == 3:  # powers of two
            h[syms] = (1 << rng.integers(0, 31, n)).astype(np.uint64)
        elif kind == 4:  # a few symbols, one of them rare
            k = int(rng.integers(2, 6))
            h[syms[:k]] = rng.integers(2, 1 << 30, k)
            h[syms[1]] = 1
        elif kind == 5:  # one symbol
            h[syms[0]] = int(rng.integers(1, 1 << 31))
        elif kind == 6:  # Fibonacci counts plus a tail of ones
            a, b = 1, 1
            for s in syms[:45]:
                h[s] = a
                a, b = b, min(a + b, (1 << 32) - 1)
            h[syms[45:200]] = 1
        else:            # all counts equal
            h[syms] = 7
        out.append(h)
    return out


@pytest.mark.parametrize("seed", range(4))
def test_host_lengths_match_oracle_and_codes_are_canonical(driver, seed):
    hists = histograms(seed)
    got = run_driver(driver, hists)
    for h, (lens, codes) in zip(hists, got):
        want = ref.huffman_lengths(h)
        assert np.array_equal(lens, want), (seed, int(np.count_nonzero(h)))
        assert np.array_equal(codes, canonical(want))


def test_host_lengths_at_the_limit_need_halving(driver):
    # log-uniform counts over 9 decades on 20000 symbols: deeper than 24 before halving
    rng = np.random.default_rng(99)
    h = np.zeros(65536, np.uint64)
    syms = rng.choice(65536, 20000, replace=False)
    h[syms] = np.exp(rng.uniform(0, 21, 20000)).astype(np.uint64) + 1
    (lens, _), = run_driver(driver, [h])
    assert lens.max() == 24
    assert np.array_equal(lens, ref.huffman_lengths(h))
