"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this module.  It loads oracle/libsdcsz_ref.so (built by
oracle/build_oracle.py) and works on numpy arrays in host memory.
"""
import ctypes as C
import os

import numpy as np

from . import build_oracle

TARGETS = ["input", "coef", "code", "recon", "dup_pred", "dup_recon", "prep_input", "prep_coef", "prep_sample"]
T_INPUT, T_COEF, T_CODE, T_RECON, T_DUP_PRED, T_DUP_RECON, T_PREP_INPUT, T_PREP_COEF, T_PREP_SAMPLE = range(9)
OK, EINVAL, ENOSPC, EFORMAT, ESDC = 0, -1, -2, -3, -4


class Fault(C.Structure):
    _fields_ = [("target", C.c_uint32), ("bit", C.c_uint32), ("block", C.c_uint64),
                ("word", C.c_uint64)]


class Params(C.Structure):
    _fields_ = [("dtype", C.c_uint32), ("ndim", C.c_uint32), ("dims", C.c_uint64 * 3),
                ("block", C.c_uint32 * 3), ("eb_mode", C.c_uint32), ("predictor", C.c_uint32),
                ("eb", C.c_double), ("abft", C.c_uint32), ("n_faults", C.c_uint32),
                ("faults", C.POINTER(Fault))]


class Report(C.Structure):
    _fields_ = [("n_blocks", C.c_uint64), ("injected", C.c_uint64 * len(TARGETS)),
                ("detected", C.c_uint64 * len(TARGETS)), ("corrected", C.c_uint64 * len(TARGETS)),
                ("uncorrectable", C.c_uint64 * len(TARGETS)), ("n_outliers", C.c_uint64),
                ("n_regression", C.c_uint64), ("payload_words", C.c_uint64),
                ("stream_size", C.c_uint64), ("eb_abs", C.c_double)]


class Debug(C.Structure):
    _fields_ = [("codes", C.c_void_p), ("is_regression", C.c_void_p), ("coef", C.c_void_p),
                ("hist", C.c_void_p), ("lengths", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(build_oracle.LIB):
            build_oracle.build()
        L = C.CDLL(build_oracle.LIB)
        P = C.POINTER
        L.sdcsz_ref_max_stream_size.restype = C.c_uint64
        L.sdcsz_ref_max_stream_size.argtypes = [P(Params)]
        L.sdcsz_ref_compress.argtypes = [C.c_void_p, P(Params), C.c_void_p, C.c_uint64,
                                         P(C.c_uint64), P(Report), P(Debug)]
        L.sdcsz_ref_decompress.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64,
                                           P(Fault), C.c_uint32, P(Report)]
        L.sdcsz_ref_pack.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, P(C.c_uint64)]
        L.sdcsz_ref_unpack.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, P(C.c_uint64)]
        L.sdcsz_ref_pack_column.restype = C.c_uint64
        L.sdcsz_ref_pack_column.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p]
        L.sdcsz_ref_decompress_region.argtypes = [C.c_void_p, C.c_uint64, P(C.c_uint64),
                                                  P(C.c_uint64), C.c_void_p, C.c_uint64,
                                                  P(Report)]
        L.sdcsz_ref_verify.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, P(Fault),
                                       C.c_uint32, P(Report)]
        L.sdcsz_ref_checksums.argtypes = [C.c_void_p, C.c_uint64, P(C.c_uint64), P(C.c_uint64)]
        L.sdcsz_ref_correct.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64,
                                        C.c_uint32]
        L.sdcsz_ref_regression.argtypes = [C.c_void_p, C.c_uint32, P(C.c_uint32), C.c_void_p]
        L.sdcsz_ref_huffman_lengths.argtypes = [C.c_void_p, C.c_void_p]
        L.sdcsz_ref_read_header.argtypes = [C.c_void_p, C.c_uint64, P(Params), P(C.c_double),
                                            P(C.c_uint64)]
        _lib = L
    return _lib


def report_dict(r):
    d = {"n_blocks": r.n_blocks, "n_outliers": r.n_outliers, "n_regression": r.n_regression,
         "payload_words": r.payload_words, "stream_size": r.stream_size, "eb_abs": r.eb_abs}
    for i, t in enumerate(TARGETS):
        d[t] = {"injected": r.injected[i], "detected": r.detected[i],
                "corrected": r.corrected[i], "uncorrectable": r.uncorrectable[i]}
    return d


def fault_array(faults):
    """faults: numpy structured/int array of rows (target, bit, block, word) or None."""
    if faults is None or len(faults) == 0:
        return None, 0
    arr = (Fault * len(faults))()
    for i, f in enumerate(faults):
        arr[i].target, arr[i].bit, arr[i].block, arr[i].word = (int(f[0]), int(f[1]),
                                                                int(f[2]), int(f[3]))
    return arr, len(faults)


def make_params(shape, dtype, block, eb, eb_mode="rel", abft=True, predictor="auto",
                faults=None):
    p = Params()
    p.dtype = 0 if np.dtype(dtype) == np.float32 else 1
    p.ndim = len(shape)
    for a, n in enumerate(shape):
        p.dims[a] = int(n)
        p.block[a] = int(block[a])
    p.eb_mode = {"abs": 0, "rel": 1}[eb_mode]
    p.predictor = {"auto": 0, "lorenzo": 1, "regression": 2}[predictor]
    p.eb = float(eb)
    p.abft = 1 if abft else 0
    arr, n = fault_array(faults)
    p.n_faults = n
    p.faults = C.cast(arr, C.POINTER(Fault)) if arr is not None else None
    p._keep = arr
    return p


def compress(x, block, eb, eb_mode="rel", abft=True, predictor="auto", faults=None,
             debug=False):
    """Returns (rc, stream uint8 array, report dict[, debug dict])."""
    L = lib()
    x = np.ascontiguousarray(x)
    p = make_params(x.shape, x.dtype, block, eb, eb_mode, abft, predictor, faults)
    cap = L.sdcsz_ref_max_stream_size(C.byref(p))
    out = np.zeros(max(cap, 8), dtype=np.uint8)
    size = C.c_uint64(0)
    rep = Report()
    dbg = None
    dbg_arrays = None
    if debug:
        nb = 1
        for a, n in enumerate(x.shape):
            nb *= -(-n // block[a])
        dbg_arrays = {"codes": np.zeros(x.size, np.uint16), "is_regression": np.zeros(nb, np.uint8),
                      "coef": np.zeros(4 * nb, x.dtype), "hist": np.zeros(65536, np.uint64),
                      "lengths": np.zeros(65536, np.uint8)}
        dbg = Debug(*(dbg_arrays[k].ctypes.data for k in
                      ("codes", "is_regression", "coef", "hist", "lengths")))
    rc = L.sdcsz_ref_compress(x.ctypes.data if x.size else None, C.byref(p), out.ctypes.data,
                              cap, C.byref(size), C.byref(rep),
                              C.byref(dbg) if dbg is not None else None)
    stream = out[: size.value].copy() if rc == OK else out[:0]
    if debug:
        return rc, stream, report_dict(rep), dbg_arrays
    return rc, stream, report_dict(rep)


def read_header(stream):
    L = lib()
    p = Params()
    eb_abs = C.c_double(0)
    nb = C.c_uint64(0)
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    rc = L.sdcsz_ref_read_header(stream.ctypes.data, stream.size, C.byref(p), C.byref(eb_abs),
                                 C.byref(nb))
    if rc != OK:
        return rc, None
    shape = tuple(int(p.dims[a]) for a in range(p.ndim))
    return OK, {"dtype": np.float32 if p.dtype == 0 else np.float64, "shape": shape,
                "block": tuple(int(p.block[a]) for a in range(p.ndim)), "eb": p.eb,
                "eb_mode": p.eb_mode, "abft": p.abft, "eb_abs": eb_abs.value,
                "n_blocks": nb.value, "predictor": p.predictor}


def decompress(stream, faults=None):
    """Returns (rc, array, report dict)."""
    L = lib()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    rc, h = read_header(stream)
    if rc != OK:
        return rc, None, None
    out = np.zeros(h["shape"], dtype=h["dtype"])
    arr, n = fault_array(faults)
    rep = Report()
    rc = L.sdcsz_ref_decompress(stream.ctypes.data, stream.size,
                                out.ctypes.data if out.size else None, out.nbytes,
                                C.cast(arr, C.POINTER(Fault)) if arr is not None else None, n,
                                C.byref(rep))
    return rc, out, report_dict(rep)


def decompress_region(stream, lo, hi):
    L = lib()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    rc, h = read_header(stream)
    if rc != OK:
        return rc, None, None
    nd = len(h["shape"])
    ext = tuple(int(hi[a]) - int(lo[a]) for a in range(nd))
    out = np.zeros([max(e, 0) for e in ext], dtype=h["dtype"])
    lo_a = (C.c_uint64 * 3)(*[int(v) for v in lo] + [0] * (3 - nd))
    hi_a = (C.c_uint64 * 3)(*[int(v) for v in hi] + [0] * (3 - nd))
    rep = Report()
    rc = L.sdcsz_ref_decompress_region(stream.ctypes.data, stream.size, lo_a, hi_a,
                                       out.ctypes.data if out.size else None, out.nbytes,
                                       C.byref(rep))
    return rc, out, report_dict(rep)


def verify(stream, data, faults=None):
    """Checks `data` (repaired in place) against the stream's checksums."""
    L = lib()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    assert data.flags.c_contiguous
    arr, n = fault_array(faults)
    rep = Report()
    rc = L.sdcsz_ref_verify(stream.ctypes.data, stream.size, data.ctypes.data, data.nbytes,
                            C.cast(arr, C.POINTER(Fault)) if arr is not None else None, n,
                            C.byref(rep))
    return rc, report_dict(rep)


def checksums(words):
    L = lib()
    w = np.ascontiguousarray(words, dtype=np.uint32)
    s, i = C.c_uint64(0), C.c_uint64(0)
    L.sdcsz_ref_checksums(w.ctypes.data, w.size, C.byref(s), C.byref(i))
    return s.value, i.value


def correct(words, s, i, width=32):
    """Repairs `words` (uint32 array) in place; returns 0 clean, 1 fixed, -1 not."""
    L = lib()
    assert words.dtype == np.uint32 and words.flags.c_contiguous
    return L.sdcsz_ref_correct(words.ctypes.data, words.size, s, i, width)


def regression(block_vals):
    L = lib()
    v = np.ascontiguousarray(block_vals)
    shape = (1,) * (3 - v.ndim) + v.shape
    ext = (C.c_uint32 * 3)(*shape)
    coef = np.zeros(4, v.dtype)
    L.sdcsz_ref_regression(v.ctypes.data, 0 if v.dtype == np.float32 else 1, ext,
                           coef.ctypes.data)
    return coef


def huffman_lengths(hist):
    L = lib()
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    assert h.size == 65536
    lens = np.zeros(65536, np.uint8)
    L.sdcsz_ref_huffman_lengths(h.ctypes.data, lens.ctypes.data)
    return lens


def _transform(fn, src):
    """Run pack or unpack on a uint8 stream: (rc, output array or None)."""
    src = np.ascontiguousarray(src, dtype=np.uint8)
    need = C.c_uint64(0)
    rc = fn(src.ctypes.data, src.size, None, 0, C.byref(need))
    if rc not in (OK, ENOSPC):
        return rc, None
    out = np.zeros(max(int(need.value), 1), np.uint8)
    rc = fn(src.ctypes.data, src.size, out.ctypes.data, out.size, C.byref(need))
    return rc, (out[: int(need.value)] if rc == OK else None)


def pack(stream):
    """Lossless stage: the plain stream's block table and sum_dc packed per
    chunk of 256 blocks (frame of reference); (rc, packed stream)."""
    return _transform(lib().sdcsz_ref_pack, stream)


def unpack(packed):
    """The plain stream of a packed one: (rc, stream)."""
    return _transform(lib().sdcsz_ref_unpack, packed)


def pack_column(values):
    """Frame-of-reference words of a column of unsigned 64-bit values."""
    v = np.ascontiguousarray(values, dtype=np.uint64)
    n = int(lib().sdcsz_ref_pack_column(v.ctypes.data if v.size else None, v.size, None))
    out = np.zeros(max(n, 1), np.uint32)
    lib().sdcsz_ref_pack_column(v.ctypes.data if v.size else None, v.size, out.ctypes.data)
    return out[:n]

