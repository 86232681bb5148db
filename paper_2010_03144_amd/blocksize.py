"""Block-size exploration (Sec. 6.2): rate-distortion per block size, and a
block-size autotuner.

The paper picks its block size from rate-distortion curves (PSNR against
bit-rate) measured for cubic blocks from 4 to 20 points a side: small blocks
pay relatively more for their regression coefficients, large ones fit a
plane less well.  `rate_distortion` measures those curves for a field on the
GPU; `best_block` picks, for one error bound, the block size that gives the
fewest bits per value (at a fixed bound the distortion is bounded alike, so
the rate decides), measured on a few sub-volumes of the field so that the
choice costs a small fraction of compressing the field.

Bit-rate = stream bits / values.  PSNR = 20 log10(value range) - 10 log10(MSE),
with the range over the original values and the MSE in double precision.
"""
import math

CUBES = (4, 6, 8, 10, 12, 16, 20)


def psnr(x, y):
    """PSNR (dB) of y against x (tensors of one shape)."""
    xd, yd = x.double(), y.double()
    rng = float(xd.max() - xd.min())
    mse = float(((xd - yd) ** 2).mean())
    if mse == 0.0:
        return math.inf
    return 20.0 * math.log10(rng) - 10.0 * math.log10(mse)


def measure(codec, x, block, eb, abft=True):
    """(bits per value, PSNR dB, compression ratio) of one compression."""
    rc, s, _ = codec.compress(x, block, eb, abft=abft)
    if rc != 0:
        raise RuntimeError(f"compress failed: {rc}")
    nbytes = int(s.numel())
    rc, y, _ = codec.decompress(s)
    if rc != 0:
        raise RuntimeError(f"decompress failed: {rc}")
    n = x.numel()
    return 8.0 * nbytes / n, psnr(x, y), n * x.element_size() / nbytes


def rate_distortion(codec, x, ebs, edges=CUBES):
    """{edge: [(eb, bits per value, PSNR, CR), ...]} for cubic (or square)
    blocks of each edge."""
    nd = x.dim()
    out = {}
    for e in edges:
        out[e] = []
        for eb in ebs:
            bpv, p, cr = measure(codec, x, (e,) * nd, eb)
            out[e].append((eb, bpv, p, cr))
    return out


def sample_views(x, side=64, count=4):
    """Up to `count` contiguous sub-volumes of edge `side` spread along the
    diagonal of the field."""
    nd = x.dim()
    side = min([side] + list(x.shape))
    views = []
    for t in range(count):
        f = (t + 0.5) / count
        sl = tuple(slice(int(f * (n - side)), int(f * (n - side)) + side) for n in x.shape)
        views.append(x[sl].contiguous())
    return views


def fast_edges(nd):
    """Edges of the cubic (square) block shapes with specialised kernels in
    `nd` dimensions; other shapes run the wave-per-block and one-thread
    kernels, tens of times slower on a large field."""
    from .sdcsz import SHAPE_CLASSES
    return {blk[0] for blk, d in SHAPE_CLASSES if d == nd and len(set(blk)) == 1}


def best_block(codec, x, eb, edges=CUBES, side=64, count=4, fast_only=True):
    """The block edge with the lowest bit-rate at the value-range-relative
    bound eb of x (applied to the samples as the same absolute bound) on
    samples of x, and the measured bits per value per edge (every edge of
    `edges`).  With fast_only the pick is made among the edges whose shape
    has specialised kernels (when `edges` holds any), since a slightly lower
    rate does not pay for a many times slower compressor."""
    views = sample_views(x, side, count)
    nd = x.dim()
    eb_abs = eb * float(x.max().double() - x.min().double())
    rates = {}
    for e in edges:
        bits = 0.0
        for v in views:
            rc, s, _ = codec.compress(v, (e,) * nd, eb_abs, eb_mode="abs")
            if rc != 0:
                raise RuntimeError(f"compress failed: {rc}")
            bits += 8.0 * int(s.numel())
        rates[e] = bits / sum(v.numel() for v in views)
    pool = [e for e in rates if e in fast_edges(nd)] if fast_only else []
    best = min(pool or rates, key=rates.get)
    return best, rates
