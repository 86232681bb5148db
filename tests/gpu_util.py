"""Helpers of the GPU tests: run both sides, compare streams section by section."""
import struct

import numpy as np

NAMES = ["codebook", "table", "coef", "sumdc", "outliers", "payload", "total"]


def sections(stream):
    return dict(zip(NAMES, struct.unpack_from("<7Q", stream[:192].tobytes(), 112)))


def first_difference(a, b):
    """Human-readable location of the first differing byte of two streams."""
    if a.size != b.size:
        return f"sizes differ: {a.size} vs {b.size}; header {sections(a)} vs {sections(b)}"
    d = np.nonzero(a != b)[0]
    if d.size == 0:
        return "identical"
    at = int(d[0])
    if at < 192:
        return f"header byte {at}"
    s = sections(a)
    order = sorted((v, k) for k, v in s.items() if k != "total")
    name = "codebook"
    for off, k in order:
        if at >= off:
            name = k
    rel = at - s[name]
    extra = ""
    if name == "table":
        extra = f" (block {rel // 8})"
    return f"{d.size} bytes differ, first at {at} in {name} +{rel}{extra}"
