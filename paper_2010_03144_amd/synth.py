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
TARGET_IDS = {"input": 0, "coef": 1, "code": 2, "recon": 3, "dup_pred": 4, "dup_recon": 5,
              "prep_input": 6, "prep_coef": 7, "prep_sample": 8}


def _word_bit_range(name, pts, per):
    """(words, bits) a flip of this target is drawn from."""
    if name in ("input", "recon", "prep_input"):
        return pts * per, 32
    if name in ("coef", "prep_coef"):
        return 4 * per, 32
    if name == "prep_sample":
        return 2, 64
    if name.startswith("dup"):
        return pts, 32 * per
    return pts, 32  # code


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
    word ranges: input/prep_input/recon -> 32-bit words of the block;
    coef/prep_coef -> the 4 coefficients' words; code/dup_* -> point index;
    prep_sample -> 0 (Lorenzo estimate) or 1 (regression estimate).  Bits are
    drawn from the 32-bit word (codes use the bit modulo 16); dup_* draw from
    the whole value, prep_sample from the 64-bit estimate.
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
            nwords, nbits = _word_bit_range(name, pts, per)
            word = int(rng.integers(0, nwords))
            bit = int(rng.integers(0, nbits))
            rows.append((tid, bit, blk, word))
    return np.array(rows, dtype=np.int64)


# ---------------------------------------------------------------------------
# Mixed-field workloads (many fields of uneven shapes, dtypes and bounds)
# ---------------------------------------------------------------------------
SLOPES = (-2.0, -2.5, -3.0, -3.5, -4.0)


class FieldPool:
    """Base volumes of Gaussian random fields, one per spectral slope in
    SLOPES (3D and 2D), from which fields of any shape up to the base shape
    are cut.  A crop of a stationary random field is a field of the same
    spectrum, so many fields of uneven shapes cost a handful of FFTs."""

    def __init__(self, shape3=(384, 384, 256), shape2=(4096, 4096), seed=40):
        self.shape3, self.shape2 = tuple(shape3), tuple(shape2)
        self.seed = seed
        self._v = {}

    def base(self, nd, slope_idx):
        key = (nd, slope_idx)
        if key not in self._v:
            shape = self.shape3 if nd == 3 else self.shape2
            self._v[key] = grf_field(shape, seed=self.seed + 10 * nd + slope_idx,
                                     slope=SLOPES[slope_idx], front=False, dtype=np.float64)
        return self._v[key]

    def field(self, shape, slope_idx, dtype, rng):
        b = self.base(len(shape), slope_idx)
        lo = [int(rng.integers(0, b.shape[a] - shape[a] + 1)) for a in range(len(shape))]
        sl = tuple(slice(l, l + n) for l, n in zip(lo, shape))
        return np.ascontiguousarray(b[sl]).astype(dtype)


def log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_specs(n=192, seed=4, frac_2d=0.5, frac_f64=0.25, shape3_hi=(384, 384, 256), shape2_hi=4096):
    """Field descriptions of a mixed batch: 3D shapes log-uniform per axis in
    [32, 384] x [32, 384] x [32, 256] with 6x6x6 blocks, 2D shapes in
    [256, 4096]^2 with 16x16 blocks, FP64 with probability frac_f64, spectral
    slope index uniform over SLOPES, value-range-relative bound log-uniform in
    [1e-5, 1e-2].  Returns a list of dicts (shape, block, dtype, slope, eb)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        if rng.uniform() < frac_2d:
            shape = tuple(log_uniform_int(rng, 256, shape2_hi) for _ in range(2))
            block = (16, 16)
        else:
            shape = (log_uniform_int(rng, 32, shape3_hi[0]), log_uniform_int(rng, 32, shape3_hi[1]),
                     log_uniform_int(rng, 32, shape3_hi[2]))
            block = (6, 6, 6)
        dtype = np.float64 if rng.uniform() < frac_f64 else np.float32
        out.append({"shape": shape, "block": block, "dtype": dtype,
                    "slope": int(rng.integers(len(SLOPES))),
                    "eb": float(math.exp(rng.uniform(math.log(1e-5), math.log(1e-2))))})
    return out


def batch_fields(specs, pool, seed=5):
    rng = np.random.default_rng(seed)
    return [pool.field(s["shape"], s["slope"], s["dtype"], rng) for s in specs]


def request_stream(rate=200.0, duration=60.0, seed=5, size_lo=1 << 20, size_hi=1 << 30,
                   frac_decompress=0.5, frac_f64=0.25, frac_faults=0.2):
    """Poisson arrivals of compress/decompress requests: arrival time,
    kind, value bytes (log-uniform in [size_lo, size_hi]), dtype, bound
    (log-uniform in [1e-5, 1e-2]) and whether the request carries a fault
    plan.  Shapes are 3D with 6x6x6 blocks, the axes as equal as the size
    allows."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        dtype = np.float64 if rng.uniform() < frac_f64 else np.float32
        nbytes = math.exp(rng.uniform(math.log(size_lo), math.log(size_hi)))
        nvals = max(216, int(nbytes / np.dtype(dtype).itemsize))
        e = max(6, int(round(nvals ** (1.0 / 3.0))))
        shape = (e, e, max(6, nvals // (e * e)))
        out.append({"t": t, "kind": "decompress" if rng.uniform() < frac_decompress else "compress",
                    "shape": shape, "dtype": dtype,
                    "eb": float(math.exp(rng.uniform(math.log(1e-5), math.log(1e-2)))),
                    "faults": bool(rng.uniform() < frac_faults), "seed": int(rng.integers(1 << 30))})
    return out


def sparse_fault_plan(shape, block, dtype, counts, seed):
    """fault_plan for a few flips on a large grid: the struck blocks are drawn
    one at a time (distinct, uniform) instead of by a permutation of all
    blocks, so a plan costs O(flips)."""
    rng = np.random.default_rng(seed)
    per = 1 if np.dtype(dtype) == np.float32 else 2
    nblk = int(np.prod(block_grid(shape, block)))
    total = sum(counts.values())
    if total > nblk:
        raise ValueError("more faults than blocks")
    taken, rows = set(), []
    for name in sorted(counts, key=lambda t: TARGET_IDS[t]):
        tid = TARGET_IDS[name]
        for _ in range(counts[name]):
            while True:
                blk = int(rng.integers(0, nblk))
                if blk not in taken:
                    taken.add(blk)
                    break
            pts = block_points(shape, block, blk)
            nwords, nbits = _word_bit_range(name, pts, per)
            word = int(rng.integers(0, nwords))
            bit = int(rng.integers(0, nbits))
            rows.append((tid, bit, blk, word))
    if not rows:
        return np.zeros((0, 4), dtype=np.int64)
    return np.array(rows, dtype=np.int64)
