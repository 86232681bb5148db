"""Autotuner of the launch shapes of the block-shape-specialised kernels.

The specialised kernels run one block per lane; what a launch can choose is
the number of lanes per work-group (64, 128 or 256).  Large launches favour
256 (the per-work-group LDS tables and histogram window are shared by more
blocks); small ones (a single small field, a batch of few blocks) favour
smaller work-groups, which spread the same blocks over more compute units.

For each shape class (6x6x6 3D, 16x16 2D) and data type, the tuner compresses
and decompresses synthetic Gaussian random fields of several sizes once per
candidate work-group size, reads each stage's device time from the library's
phase timers, and keeps, per stage, the fastest candidate at each size (256
lanes unless another candidate is faster by more than MARGIN).  Size
ranges between two measured sizes split at their geometric mean; the largest
measured size's choice extends to every larger launch.  `apply` installs a
table in the library (sdcsz_tune_set); `save` and `load` keep it as JSON.
The launch shape never changes a result, only the time.
"""
import json
import math

from . import sdcsz

LANES = (64, 128, 256)
STAGE_PHASE = {"predict": "predict_quantize", "check": "code_check", "encode": "encode", "decode": "decode"}
SIZES = (1 << 8, 1 << 11, 1 << 14, 1 << 17)  # blocks per launch
MARGIN = 0.05  # a smaller work-group must beat 256 lanes by this fraction to be chosen
UNBOUNDED = 1 << 62


def pick(times):
    """times: {lanes: ms} -> the lanes to use: 256 unless another candidate
    is faster by more than MARGIN (timing noise does not flip choices)."""
    fastest = min(times, key=times.get)
    return fastest if times[fastest] < (1 - MARGIN) * times[256] else 256


def entries_from_best(best):
    """best: {blocks: lanes} at the measured sizes -> ascending
    [(max_blocks, lanes)] with equal neighbours merged."""
    sizes = sorted(best)
    out = []
    for i, n in enumerate(sizes):
        bound = UNBOUNDED if i + 1 == len(sizes) else int(math.sqrt(n * sizes[i + 1]))
        if out and out[-1][1] == best[n]:
            out[-1] = (bound, best[n])
        else:
            out.append((bound, best[n]))
    return out


def device_field(torch, shape, seed, dtype, slope=-3.0, device="cuda:0"):
    """Gaussian random field with P(k) ~ k^slope, made on the device."""
    g = torch.Generator(device=device).manual_seed(seed)
    w = torch.randn(shape, generator=g, device=device, dtype=torch.float32)
    spec = torch.fft.rfftn(w)
    k2 = torch.zeros(spec.shape, device=device)
    for a, n in enumerate(shape):
        if a == len(shape) - 1:
            kk = torch.arange(spec.shape[a], device=device, dtype=torch.float32)
        else:
            kk = torch.fft.fftfreq(n, device=device) * n
        sh = [1] * len(shape)
        sh[a] = -1
        k2 = k2 + kk.reshape(sh) ** 2
    amp = torch.where(k2 > 0, k2.clamp_min(1e-12) ** (slope / 4), torch.zeros_like(k2))
    x = torch.fft.irfftn(spec * amp, s=shape)
    x = (x - x.mean()) / x.std()
    return x.to(dtype).contiguous()


def class_shape(block, nblocks):
    """A field shape of about nblocks blocks of the given block, near-cubic,
    with a partial block along every axis."""
    nd = len(block)
    e = max(1, round(nblocks ** (1.0 / nd)))
    per = [e] * nd
    per[0] = max(1, round(nblocks / e ** (nd - 1)))
    return tuple(p * b - (b // 3 if p > 1 else 0) for p, b in zip(per, block))


def autotune(device="cuda:0", sizes=SIZES, eb=1e-3, reps=2, log=None):
    """Measure and install; returns (table, times) where table maps
    "stage/class/dtype" to entries and times holds the measured ms."""
    import time
    import torch
    codec = sdcsz.Codec(device)
    table, times = {}, {}
    for ci, (block, _) in enumerate(sdcsz.SHAPE_CLASSES):
        for dt, tdt in ((0, torch.float32), (1, torch.float64)):
            t0 = time.perf_counter()
            t = {s: {} for s in STAGE_PHASE}
            for n in sizes:
                x = device_field(torch, class_shape(block, n), seed=11 + n % 97, dtype=tdt, device=device)
                for lanes in LANES:
                    for si in range(len(sdcsz.TUNE_STAGES)):
                        sdcsz.tune_set(si, ci, dt, [(UNBOUNDED, lanes)])
                    rc, s, _ = codec.compress(x, block, eb)  # warm-up
                    assert rc == sdcsz.OK, rc
                    rc, _, _ = codec.decompress(s)
                    assert rc == sdcsz.OK, rc
                    sdcsz.timing_enable(True)
                    for _ in range(reps):
                        codec.compress(x, block, eb)
                        codec.decompress(s)
                    ph = sdcsz.timing_read()
                    sdcsz.timing_enable(False)
                    for stage, phase in STAGE_PHASE.items():
                        t[stage].setdefault(n, {})[lanes] = ph[phase][0] / reps
                del x
            for si, stage in enumerate(sdcsz.TUNE_STAGES):
                best = {n: pick(t[stage][n]) for n in sizes}
                table[f"{stage}/{ci}/{dt}"] = entries_from_best(best)
                times[f"{stage}/{ci}/{dt}"] = {str(n): {str(ln): round(v, 5) for ln, v in d.items()}
                                               for n, d in t[stage].items()}
            if log:
                log(f"tuned class {ci} dtype {dt} in {time.perf_counter() - t0:.1f} s: " +
                    ", ".join(f"{s}={table[f'{s}/{ci}/{dt}']}" for s in sdcsz.TUNE_STAGES))
    apply(table)
    return table, times


def apply(table):
    for key, entries in table.items():
        stage, ci, dt = (sdcsz.TUNE_STAGES.index(key.split("/")[0]),) + tuple(int(v) for v in key.split("/")[1:])
        rc = sdcsz.tune_set(stage, ci, dt, [tuple(e) for e in entries])
        if rc != sdcsz.OK:
            raise sdcsz.SdcszError(rc, f"sdcsz_tune_set {key}")


def reset():
    for si in range(len(sdcsz.TUNE_STAGES)):
        for ci in range(len(sdcsz.SHAPE_CLASSES)):
            for dt in (0, 1):
                sdcsz.tune_set(si, ci, dt, [])


def save(table, path):
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load(path):
    with open(path) as f:
        table = json.load(f)
    apply(table)
    return table
