"""Seeded synthetic inputs and fault plans.

This module holds only input generation: smooth and turbulent test fields of
the shapes and value distributions the paper's evaluation uses (Sec. 6:
512^3 cosmology fields, 100x500x500 climate fields, 2D images), and bit-flip
plans in the style of its evaluation mode A (one flip per struck block, a
uniformly drawn word and bit).  It contains none of the compressor's
arithmetic; the HIP library and the CPU oracle both consume its output.
"""
import math

import numpy as np

try:
    import scipy.fft as _fft
    _FFT_KW = {"workers": 16}
except Exception:  # pragma: no cover - scipy is part of the image
    _fft = np.fft
    _FFT_KW = {}


def bumps_field(shape=(64, 64, 64), seed=1, dtype=np.float32, n_bumps=16, n_waves=3,
                noise=1e-3):
    """Sum of Gaussian bumps + sinusoids + white noise (smooth field with texture)."""
    rng = np.random.default_rng(seed)
    nd = len(shape)
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    f = np.zeros(shape, dtype=np.float64)
    for _ in range(n_bumps):
        c = rng.uniform(0, 1, nd) * np.array(shape)
        amp = rng.uniform(0.5, 2.0)
        w = rng.uniform(4.0, 16.0)
        g = 1.0
        for a in range(nd):
            sh = [1] * nd
            sh[a] = shape[a]
            g = g * np.exp(-((axes[a] - c[a]) ** 2) / (2 * w * w)).reshape(sh)
        f += amp * g
    for _ in range(n_waves):
        amp = rng.uniform(0.1, 0.5)
        k = np.zeros(nd, dtype=np.int64)
        while not k.any():
            k = rng.integers(-4, 5, nd)
        phase = rng.uniform(0, 2 * math.pi)
        arg = phase
        for a in range(nd):
            sh = [1] * nd
            sh[a] = shape[a]
            arg = arg + (2 * math.pi * k[a] / shape[a]) * axes[a].reshape(sh)
        f += amp * np.sin(arg)
    f += rng.normal(0.0, noise, shape)
    return f.astype(dtype)


def grf_field(shape=(512, 512, 512), seed=2, slope=-3.0, front=True, dtype=np.float32,
              front_halfwidth=2.56):
    """Gaussian random field with power spectrum P(k) ~ k^slope, standardised,
    plus (optionally) a sharp tanh front on ~1% of the cells."""
    rng = np.random.default_rng(seed)
    nd = len(shape)
    spec = _fft.rfftn(rng.standard_normal(shape), **_FFT_KW)
    k2 = np.zeros(spec.shape, dtype=np.float64)
    for a, n in enumerate(shape):
        if a == nd - 1:
            kk = np.arange(spec.shape[a], dtype=np.float64)
        else:
            kk = np.fft.fftfreq(n) * n
        sh = [1] * nd
        sh[a] = spec.shape[a]
        k2 = k2 + (kk * kk).reshape(sh)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)  # sqrt(P) = k^(slope/2)
    del k2
    spec *= amp
    del amp
    f = _fft.irfftn(spec, s=shape, **_FFT_KW)
    del spec
    f -= f.mean()
    sd = f.std()
    if sd > 0:
        f /= sd
    if front:
        nvec = rng.standard_normal(nd)
        nvec /= np.linalg.norm(nvec)
        p0 = rng.uniform(0.25, 0.75, nd) * np.array(shape)
        d = float(nvec @ p0)
        s = -d
        for a in range(nd):
            sh = [1] * nd
            sh[a] = shape[a]
            s = s + nvec[a] * np.arange(shape[a], dtype=np.float64).reshape(sh)
        s = np.broadcast_to(s, shape)
        mask = np.abs(s) < front_halfwidth
        f[mask] = 4.0 * np.tanh(s[mask])
    return f.astype(dtype)


def linear_field(shape, coeffs, offset=0.0, dtype=np.float32):
    """f = offset + sum_a coeffs[a] * x_a (exactly linear on every block)."""
    f = np.full(shape, offset, dtype=np.float64)
    for a, n in enumerate(shape):
        sh = [1] * len(shape)
        sh[a] = n
        f = f + coeffs[a] * np.arange(n, dtype=np.float64).reshape(sh)
    return f.astype(dtype)


# ---------------------------------------------------------------------------
# block geometry (index bookkeeping only) and fault plans
# ---------------------------------------------------------------------------
TARGET_IDS = {"input": 0, "coef": 1, "code": 2, "recon": 3, "dup_pred": 4, "dup_recon": 5}


def block_grid(shape, block):
    return tuple(-(-int(n) // int(b)) for n, b in zip(shape, block))


def block_points(shape, block, blk):
    """Number of points of linear block `blk` (partial blocks at the upper edges)."""
    grid = block_grid(shape, block)
    pts = 1
    rem = int(blk)
    coords = []
    for g in reversed(grid):
        coords.append(rem % g)
        rem //= g
    coords.reverse()
    for a, c in enumerate(coords):
        pts *= min(int(block[a]), int(shape[a]) - c * int(block[a]))
    return pts


def fault_plan(shape, block, dtype, counts, seed=3):
    """Plan of single-bit flips, one per struck block (distinct blocks overall).

    counts: {target name: number of flips}.  Returns an int64 array of rows
    (target, bit, block, word) in the layout of the library's fault record.
    word ranges: input/recon -> 32-bit words of the block; coef -> the 4
    coefficients' words; code/dup_* -> point index.  Bits are drawn from the
    32-bit word (codes use the bit modulo 16); dup_* draw from the whole value.
    """
    rng = np.random.default_rng(seed)
    per = 1 if np.dtype(dtype) == np.float32 else 2
    nblk = int(np.prod(block_grid(shape, block)))
    total = sum(counts.values())
    if total == 0:
        return np.zeros((0, 4), dtype=np.int64)
    if total > nblk:
        raise ValueError("more faults than blocks")
    blocks = rng.choice(nblk, size=total, replace=False)
    rows = []
    at = 0
    for name in sorted(counts, key=lambda t: TARGET_IDS[t]):
        tid = TARGET_IDS[name]
        for _ in range(counts[name]):
            blk = int(blocks[at])
            at += 1
            pts = block_points(shape, block, blk)
            if name in ("input", "recon"):
                nwords = pts * per
            elif name == "coef":
                nwords = 4 * per
            else:
                nwords = pts
            word = int(rng.integers(0, nwords))
            bit = int(rng.integers(0, 32 * per if name.startswith("dup") else 32))
            rows.append((tid, bit, blk, word))
    return np.array(rows, dtype=np.int64)
