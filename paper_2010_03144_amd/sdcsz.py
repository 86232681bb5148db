"""Python binding of libsdcsz.so (the C ABI declared in include/sdcsz.h).

Argument marshalling only: PyTorch provides device memory and the current
HIP stream; every step of compression and decompression runs in the
library's HIP kernels.  Importing works without a GPU; calling needs the
built library (paper_2010_03144_amd/libsdcsz.so) and fails loudly if it is
missing.
"""
import ctypes as C
import os


HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdcsz.so")

OK, EINVAL, ENOSPC, EFORMAT, ESDC, EHIP = 0, -1, -2, -3, -4, -5
TARGETS = ["input", "coef", "code", "recon", "dup_pred", "dup_recon", "prep_input", "prep_coef", "prep_sample"]
ERRORS = {OK: "ok", EINVAL: "EINVAL", ENOSPC: "ENOSPC", EFORMAT: "EFORMAT", ESDC: "ESDC", EHIP: "EHIP"}
FUNCTIONS = ["sdcsz_max_compressed_size", "sdcsz_compress_workspace_size", "sdcsz_compress",
             "sdcsz_stream_info", "sdcsz_decompress_workspace_size", "sdcsz_decompress",
             "sdcsz_verify", "sdcsz_decompress_region", "sdcsz_compress_batch_workspace_size",
             "sdcsz_compress_batch", "sdcsz_decompress_batch_workspace_size",
             "sdcsz_decompress_batch", "sdcsz_strerror", "sdcsz_timing_enable",
             "sdcsz_timing_read", "sdcsz_phase_name", "sdcsz_tune_set", "sdcsz_tune_get",
             "sdcsz_decompress_noalloc", "sdcsz_pack_workspace_size", "sdcsz_pack", "sdcsz_unpack",
             "sdcsz_region_prepare", "sdcsz_decompress_region_prepared"]
N_PHASES = 11
HEADER_BYTES = 192
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024  # device array of sdcsz_decompress_noalloc
UNPACK_WORKSPACE_BYTES = 256
PACKED_MAGIC = b"SDCSZ\x00v2"
TUNE_MAX = 8
TUNE_STAGES = ["predict", "check", "encode", "decode"]
SHAPE_CLASSES = [((6, 6, 6), 3), ((16, 16), 2)]  # (block, ndim) of the specialised kernels
DEVICE_PHASES = 8  # phases 0..7 are device (kernel) time, 8.. host wall time


class SdcszError(RuntimeError):
    def __init__(self, rc, what=""):
        super().__init__(f"{what}: {ERRORS.get(rc, rc)}")
        self.rc = rc


class Fault(C.Structure):
    _fields_ = [("target", C.c_uint32), ("bit", C.c_uint32), ("block", C.c_uint64),
                ("word", C.c_uint64)]


class Params(C.Structure):
    _fields_ = [("dtype", C.c_uint32), ("ndim", C.c_uint32), ("dims", C.c_uint64 * 3),
                ("block", C.c_uint32 * 3), ("eb_mode", C.c_uint32), ("predictor", C.c_uint32),
                ("eb", C.c_double), ("abft", C.c_uint32), ("n_faults", C.c_uint32),
                ("faults", C.POINTER(Fault))]


class Timing(C.Structure):
    _fields_ = [("ms", C.c_double * N_PHASES), ("launches", C.c_uint64 * N_PHASES)]


class Report(C.Structure):
    _fields_ = [("n_blocks", C.c_uint64), ("injected", C.c_uint64 * len(TARGETS)),
                ("detected", C.c_uint64 * len(TARGETS)), ("corrected", C.c_uint64 * len(TARGETS)),
                ("uncorrectable", C.c_uint64 * len(TARGETS)), ("n_outliers", C.c_uint64),
                ("n_regression", C.c_uint64), ("payload_words", C.c_uint64),
                ("stream_size", C.c_uint64), ("eb_abs", C.c_double),
                ("generic_plan_blocks", C.c_uint64)]


class CompItem(C.Structure):
    _fields_ = [("d_in", C.c_void_p), ("params", Params), ("d_out", C.c_void_p),
                ("out_cap", C.c_uint64), ("out_size", C.c_uint64), ("rc", C.c_int),
                ("rep", Report), ("header", C.c_uint8 * HEADER_BYTES)]


class DecItem(C.Structure):
    _fields_ = [("d_stream", C.c_void_p), ("stream_size", C.c_uint64), ("d_out", C.c_void_p),
                ("out_cap", C.c_uint64), ("faults", C.POINTER(Fault)), ("n_faults", C.c_uint32),
                ("h_header", C.c_void_p), ("rc", C.c_int), ("rep", Report)]


_lib = None


def lib():
    """Load libsdcsz.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2010_03144_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        L.sdcsz_max_compressed_size.restype = C.c_uint64
        L.sdcsz_max_compressed_size.argtypes = [P(Params)]
        L.sdcsz_compress_workspace_size.restype = C.c_uint64
        L.sdcsz_compress_workspace_size.argtypes = [P(Params)]
        L.sdcsz_decompress_workspace_size.restype = C.c_uint64
        L.sdcsz_decompress_workspace_size.argtypes = [P(Params)]
        L.sdcsz_compress.argtypes = [vp, P(Params), vp, C.c_uint64, P(C.c_uint64), P(Report), vp,
                                     C.c_uint64, vp]
        L.sdcsz_stream_info.argtypes = [vp, C.c_uint64, P(Params), P(C.c_uint64), P(C.c_double), vp]
        L.sdcsz_decompress.argtypes = [vp, C.c_uint64, vp, C.c_uint64, P(Fault), C.c_uint32, P(Report),
                                       vp, C.c_uint64, vp]
        L.sdcsz_decompress_noalloc.argtypes = [vp, C.c_uint64, vp, C.c_uint64, P(Fault), C.c_uint32,
                                               P(Report), vp]
        L.sdcsz_verify.argtypes = [vp, C.c_uint64, vp, C.c_uint64, P(Fault), C.c_uint32, P(Report), vp,
                                   C.c_uint64, vp]
        L.sdcsz_decompress_region.argtypes = [vp, C.c_uint64, P(C.c_uint64), P(C.c_uint64), vp,
                                              C.c_uint64, P(Report), vp, C.c_uint64, vp]
        L.sdcsz_region_prepare.argtypes = [vp, C.c_uint64, vp, vp, C.c_uint64, vp]
        L.sdcsz_decompress_region_prepared.argtypes = [vp, C.c_uint64, vp, P(C.c_uint64), P(C.c_uint64), vp,
                                                       C.c_uint64, P(Report), vp, C.c_uint64, vp]
        L.sdcsz_compress_batch_workspace_size.restype = C.c_uint64
        L.sdcsz_compress_batch_workspace_size.argtypes = [P(CompItem), C.c_uint32]
        L.sdcsz_compress_batch.argtypes = [P(CompItem), C.c_uint32, vp, C.c_uint64, vp]
        L.sdcsz_decompress_batch_workspace_size.restype = C.c_uint64
        L.sdcsz_decompress_batch_workspace_size.argtypes = [P(Params), C.c_uint32]
        L.sdcsz_decompress_batch.argtypes = [P(DecItem), C.c_uint32, vp, C.c_uint64, vp]
        L.sdcsz_pack_workspace_size.restype = C.c_uint64
        L.sdcsz_pack_workspace_size.argtypes = [C.c_uint64]
        L.sdcsz_pack.argtypes = [vp, C.c_uint64, vp, C.c_uint64, P(C.c_uint64), vp, C.c_uint64, vp]
        L.sdcsz_unpack.argtypes = [vp, C.c_uint64, vp, C.c_uint64, P(C.c_uint64), vp, C.c_uint64, vp]
        L.sdcsz_strerror.restype = C.c_char_p
        L.sdcsz_strerror.argtypes = [C.c_int]
        L.sdcsz_timing_enable.argtypes = [C.c_int]
        L.sdcsz_timing_enable.restype = None
        L.sdcsz_timing_read.argtypes = [P(Timing)]
        L.sdcsz_timing_read.restype = None
        L.sdcsz_phase_name.argtypes = [C.c_int]
        L.sdcsz_phase_name.restype = C.c_char_p
        L.sdcsz_tune_set.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint32, P(C.c_uint64), P(C.c_uint32)]
        L.sdcsz_tune_get.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_uint32), P(C.c_uint64), P(C.c_uint32)]
        _lib = L
    return _lib


def report_dict(r):
    inj, det, cor, unc = r.injected[:], r.detected[:], r.corrected[:], r.uncorrectable[:]
    d = {"n_blocks": r.n_blocks, "n_outliers": r.n_outliers, "n_regression": r.n_regression,
         "payload_words": r.payload_words, "stream_size": r.stream_size, "eb_abs": r.eb_abs,
         "generic_plan_blocks": r.generic_plan_blocks}
    for i, t in enumerate(TARGETS):
        d[t] = {"injected": inj[i], "detected": det[i], "corrected": cor[i], "uncorrectable": unc[i]}
    return d


def _faults(faults):
    if faults is None or len(faults) == 0:
        return None, 0, None
    arr = (Fault * len(faults))()
    for i, f in enumerate(faults):
        arr[i].target, arr[i].bit, arr[i].block, arr[i].word = (int(f[0]), int(f[1]), int(f[2]),
                                                                int(f[3]))
    return C.cast(arr, C.POINTER(Fault)), len(faults), arr


def make_params(shape, is_f32, block, eb, eb_mode="rel", abft=True, predictor="auto", faults=None):
    p = Params()
    p.dtype = 0 if is_f32 else 1
    p.ndim = len(shape)
    for a, n in enumerate(shape):
        p.dims[a] = int(n)
        p.block[a] = int(block[a])
    p.eb_mode = {"abs": 0, "rel": 1}[eb_mode]
    p.predictor = {"auto": 0, "lorenzo": 1, "regression": 2}[predictor]
    p.eb = float(eb)
    p.abft = 1 if abft else 0
    ptr, n, keep = _faults(faults)
    p.n_faults = n
    p.faults = ptr
    p._keep = keep
    return p


def max_compressed_size(shape, is_f32, block):
    """Upper bound of the stream size of a field (bytes)."""
    p = make_params(tuple(shape), is_f32, block, 1.0)
    return int(lib().sdcsz_max_compressed_size(C.byref(p)))


def workspace_sizes(shape, is_f32, block, n_faults=0):
    """(compress, decompress) device workspace bytes of one field."""
    L = lib()
    p = make_params(tuple(shape), is_f32, block, 1.0)
    p.n_faults = n_faults
    return int(L.sdcsz_compress_workspace_size(C.byref(p))), int(L.sdcsz_decompress_workspace_size(C.byref(p)))


def _stream_handle(device):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Codec:
    """Compress/decompress torch tensors on one GPU.  Workspaces are cached
    per size (torch allocations), so repeated calls allocate nothing new."""

    def __init__(self, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self._ws = {}
        # streams this codec wrote into its own buffers: pointer -> (size, shape, dtype, block)
        self._meta = {}
        # region-decoding states of recently used streams: pointer -> RegionState
        self._regions = {}
        # parameters and sizes of recent call shapes without fault plans
        self._cp = {}  # compress: (shape, dtype, block, eb, mode, abft, predictor) -> (Params, ws, cap)
        self._dp = {}  # decompress: (shape, is_f32, block) -> (Params, ws)

    def workspace(self, nbytes, tag):
        """A device buffer of at least nbytes kept under `tag`.  It grows by
        half at least, and a large one it replaces goes back to the device
        (not to torch's cache, where blocks of outgrown sizes would pile up
        until allocations fail and the allocator's retries stall every
        stream)."""
        t = self._ws.get(tag)
        if t is None or t.numel() < nbytes:
            old = 0
            if t is not None:
                old = t.numel()
                self._meta.pop(t.data_ptr(), None)  # its memory may be reused
                self._ws[tag] = t = None
                if old >= 1 << 30:
                    self.torch.cuda.empty_cache()
            t = self.torch.empty(max(int(nbytes), old + old // 2, 256), dtype=self.torch.uint8, device=self.device)
            self._ws[tag] = t
        return t

    # ------------------------------------------------------------------ compress
    def compress(self, x, block, eb, eb_mode="rel", abft=True, predictor="auto", faults=None,
                 out=None):
        """Returns (rc, stream uint8 tensor on the device, report dict).
        Without `out`, the stream is a view into a buffer this codec reuses:
        its next compression overwrites it, so clone the stream to keep it
        (decompress and region decompression know a stream still there)."""
        torch = self.torch
        L = lib()
        assert x.is_cuda and x.is_contiguous() and x.dtype in (torch.float32, torch.float64)
        plain = faults is None or len(faults) == 0
        key = (tuple(x.shape), x.dtype, tuple(block), float(eb), eb_mode, bool(abft), predictor) if plain else None
        ent = self._cp.get(key) if key else None
        if ent is None:
            p = make_params(tuple(x.shape), x.dtype == torch.float32, block, eb, eb_mode, abft,
                            predictor, faults)
            ent = (p, L.sdcsz_compress_workspace_size(C.byref(p)), L.sdcsz_max_compressed_size(C.byref(p)))
            if key and ent[1]:
                if len(self._cp) >= 64:
                    self._cp.clear()
                self._cp[key] = ent
        p, ws_n, cap = ent
        if ws_n == 0:
            return EINVAL, None, None
        if out is None or out.numel() < cap:
            out = self.workspace(cap, "stream_out")
        ws = self.workspace(ws_n, "compress")
        item = (CompItem * 1)()  # one field through the batch entry: it also returns the header
        item[0].d_in = x.data_ptr()
        item[0].params = p
        item[0].d_out = out.data_ptr()
        item[0].out_cap = out.numel()
        rc = L.sdcsz_compress_batch(item, 1, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(self.device))
        rc = item[0].rc if rc in (OK, item[0].rc) else rc
        size = int(item[0].out_size)
        stream = out[:size] if rc == OK else None
        header = bytes(item[0].header) if rc == OK else None
        self._remember(out, rc, size, tuple(x.shape), p.dtype, block, header)
        rep = report_dict(item[0].rep)
        rep["header"] = header
        return rc, stream, rep

    def _remember(self, buf, rc, size, shape, dtype, block, header=None):
        self._regions.pop(buf.data_ptr(), None)  # the buffer now holds another stream
        own = any(t.data_ptr() == buf.data_ptr() for t in self._ws.values())
        if rc == OK and own:
            self._meta[buf.data_ptr()] = (size, shape, dtype, tuple(int(b) for b in block), header)
        else:
            self._meta.pop(buf.data_ptr(), None)

    def _header(self, stream):
        """The header bytes of a stream this codec wrote into its own buffer
        (the library checks them against the stream on the device)."""
        m = self._meta.get(stream.data_ptr())
        if m is not None and m[0] == stream.numel():
            return m[4]
        return None

    def _geometry(self, stream):
        """(rc, params, shape) of a stream: from the last compression when the
        stream is that call's output, still in this codec's buffer (only
        compress writes there; the library validates the header anyway),
        else read from the stream's header on the device."""
        m = self._meta.get(stream.data_ptr())
        if m is not None and m[0] == stream.numel():
            return OK, self._dec_params(m[1], m[2] == 0, m[3])[0], m[1]
        return self.info(stream)

    def _dec_params(self, shape, is_f32, block):
        """(Params, workspace bytes without fault plans) of a decompression;
        the Params are shared: callers must not change them."""
        key = (tuple(shape), bool(is_f32), tuple(int(b) for b in block))
        ent = self._dp.get(key)
        if ent is None:
            p = make_params(key[0], is_f32, key[2], 1.0)
            ent = (p, int(lib().sdcsz_decompress_workspace_size(C.byref(p))))
            if len(self._dp) >= 64:
                self._dp.clear()
            self._dp[key] = ent
        return ent

    def info(self, stream):
        L = lib()
        p = Params()
        nb = C.c_uint64(0)
        eb_abs = C.c_double(0)
        rc = L.sdcsz_stream_info(C.c_void_p(stream.data_ptr()), stream.numel(), C.byref(p),
                                 C.byref(nb), C.byref(eb_abs), _stream_handle(self.device))
        if rc != OK:
            return rc, None, None
        shape = tuple(int(p.dims[a]) for a in range(p.ndim))
        return rc, p, shape

    def _dec_ws(self, p, n_faults):
        if n_faults == 0:
            n = self._dec_params(tuple(p.dims[a] for a in range(p.ndim)), p.dtype == 0,
                                 tuple(p.block[a] for a in range(p.ndim)))[1]
        else:
            q = Params.from_buffer_copy(p)  # p may be shared
            q.n_faults = n_faults
            n = lib().sdcsz_decompress_workspace_size(C.byref(q))
        return self.workspace(n, "decompress")

    # ---------------------------------------------------------------- decompress
    def decompress(self, stream, faults=None, out=None, geom=None, header=None):
        """Returns (rc, tensor, report dict).  geom: (shape, is_f32, block)
        when the caller knows them (the library checks them against the
        header), else they are taken from the stream.  header: the stream's
        header bytes (from its compression report; a stream this codec wrote
        into its own buffer brings its own), which spares the read-back of
        the header (the library checks it against the stream on the device)."""
        torch = self.torch
        L = lib()
        if geom is not None:
            rc, p, shape = OK, self._dec_params(geom[0], geom[1], geom[2])[0], tuple(geom[0])
        else:
            rc, p, shape = self._geometry(stream)
        if rc != OK:
            return rc, None, None
        if header is None:
            header = self._header(stream)
        dt = torch.float32 if p.dtype == 0 else torch.float64
        if out is None:
            out = torch.empty(shape, dtype=dt, device=self.device)
        fptr, nf, keep = _faults(faults)
        ws = self._dec_ws(p, nf)
        if header is not None:
            hbuf = C.create_string_buffer(bytes(header), HEADER_BYTES)
            item = (DecItem * 1)()
            item[0].d_stream = stream.data_ptr()
            item[0].stream_size = stream.numel()
            item[0].d_out = out.data_ptr()
            item[0].out_cap = out.numel() * out.element_size()
            item[0].faults = fptr
            item[0].n_faults = nf
            item[0].h_header = C.cast(hbuf, C.c_void_p)
            rc = L.sdcsz_decompress_batch(item, 1, C.c_void_p(ws.data_ptr()), ws.numel(),
                                          _stream_handle(self.device))
            del keep, hbuf
            return item[0].rc if rc in (OK, item[0].rc) else rc, out, report_dict(item[0].rep)
        rep = Report()
        rc = L.sdcsz_decompress(C.c_void_p(stream.data_ptr()), stream.numel(),
                                C.c_void_p(out.data_ptr()), out.numel() * out.element_size(), fptr,
                                nf, C.byref(rep), C.c_void_p(ws.data_ptr()), ws.numel(),
                                _stream_handle(self.device))
        del keep
        return rc, out, report_dict(rep)

    # ------------------------------------------------------------ lossless stage
    def pack(self, stream, out=None):
        """The packed form of a plain stream: (rc, packed uint8 tensor), a
        view of `out` when given (uint8, on this device, large enough), else
        of a new tensor.  Sizes are bounded from the stream's size alone (a
        plain stream holds 8 bytes of block table per block), so no header
        is read here."""
        torch = self.torch
        L = lib()
        nb_max = stream.numel() // 8
        ws = self.workspace(L.sdcsz_pack_workspace_size(nb_max), "pack")
        size = C.c_uint64(0)

        def call(o):
            return L.sdcsz_pack(C.c_void_p(stream.data_ptr()), stream.numel(), C.c_void_p(o.data_ptr()),
                                o.numel(), C.byref(size), C.c_void_p(ws.data_ptr()), ws.numel(),
                                _stream_handle(self.device))
        if out is None:
            # a chunk column adds 3 words and at most one partial word
            out = torch.empty(stream.numel() + 64 * (nb_max // 256 + 2), dtype=torch.uint8, device=self.device)
        rc = call(out)
        if rc == ENOSPC:
            out = torch.empty(int(size.value), dtype=torch.uint8, device=self.device)
            rc = call(out)
        return rc, (out[:int(size.value)] if rc == OK else None)

    def unpack(self, packed, out=None):
        """The plain stream of a packed one: (rc, uint8 tensor), a view of
        `out` when given and large enough, else of a new tensor."""
        torch = self.torch
        L = lib()
        ws = self.workspace(UNPACK_WORKSPACE_BYTES, "unpack")
        size = C.c_uint64(0)

        def call(o):
            ptr, cap = (o.data_ptr(), o.numel()) if o is not None else (None, 0)
            return L.sdcsz_unpack(C.c_void_p(packed.data_ptr()), packed.numel(), C.c_void_p(ptr), cap,
                                  C.byref(size), C.c_void_p(ws.data_ptr()), ws.numel(),
                                  _stream_handle(self.device))
        rc = call(out)  # out None: a size query
        if rc == ENOSPC and (out is None or out.numel() < int(size.value)):
            out = torch.empty(int(size.value), dtype=torch.uint8, device=self.device)
            rc = call(out)
        return rc, (out[:int(size.value)] if rc == OK else None)

    def decompress_noalloc(self, stream, out, faults=None):
        """sdcsz_decompress_noalloc: decompress `stream` into the caller's
        `out` (a contiguous tensor of the field's size) with the library's
        fixed device array as workspace; nothing is allocated.  Returns
        (rc, report dict)."""
        fptr, nf, keep = _faults(faults)
        rep = Report()
        rc = lib().sdcsz_decompress_noalloc(C.c_void_p(stream.data_ptr()), stream.numel(),
                                            C.c_void_p(out.data_ptr()), out.numel() * out.element_size(),
                                            fptr, nf, C.byref(rep), _stream_handle(self.device))
        del keep
        return rc, report_dict(rep)

    def verify(self, stream, data, faults=None):
        """Check `data` (repaired in place) against the stream's checksums."""
        L = lib()
        rc, p, shape = self.info(stream)
        if rc != OK:
            return rc, None
        fptr, nf, keep = _faults(faults)
        ws = self._dec_ws(p, nf)
        rep = Report()
        rc = L.sdcsz_verify(C.c_void_p(stream.data_ptr()), stream.numel(),
                            C.c_void_p(data.data_ptr()), data.numel() * data.element_size(), fptr,
                            nf, C.byref(rep), C.c_void_p(ws.data_ptr()), ws.numel(),
                            _stream_handle(self.device))
        del keep
        return rc, report_dict(rep)

    # ------------------------------------------------------------------ batches
    def compress_batch(self, fields, block, eb, eb_mode="rel", abft=True, predictor="auto",
                       faults=None, outs=None):
        """Compress several fields in one call.  Each of `block` (a tuple),
        `eb`, `eb_mode`, `abft` and `predictor` is one value for every field or
        a list with one value per field; `faults` is None or a list with one
        plan (or None) per field.  Returns (rc, [(rc, stream, report)]); the
        streams are views into `outs` (one buffer per field) or into buffers
        this codec keeps per batch slot."""
        torch = self.torch
        L = lib()
        n = len(fields)
        pick = lambda v, i: v[i] if isinstance(v, list) else v
        items = (CompItem * max(n, 1))()
        keep = []
        caps = []
        for i, x in enumerate(fields):
            assert x.is_cuda and x.is_contiguous() and x.dtype in (torch.float32, torch.float64)
            fl = faults[i] if faults is not None else None
            p = make_params(tuple(x.shape), x.dtype == torch.float32, pick(block, i), pick(eb, i),
                            pick(eb_mode, i), pick(abft, i), pick(predictor, i), fl)
            keep.append(p)
            items[i].d_in = x.data_ptr()
            items[i].params = p
            caps.append(L.sdcsz_max_compressed_size(C.byref(p)))
        bufs = []
        for i in range(n):
            if outs is not None:
                out = outs[i]
            else:
                out = self.workspace(caps[i], f"batch_out_{i}")
            bufs.append(out)
            items[i].d_out = out.data_ptr()
            items[i].out_cap = out.numel()
        ws_n = L.sdcsz_compress_batch_workspace_size(items, n)
        ws = self.workspace(ws_n, "compress_batch")
        rc = L.sdcsz_compress_batch(items, n, C.c_void_p(ws.data_ptr()), ws.numel(),
                                    _stream_handle(self.device))
        res = []
        for i in range(n):
            it = items[i]
            header = bytes(it.header) if it.rc == OK else None
            self._remember(bufs[i], it.rc, int(it.out_size), tuple(fields[i].shape), it.params.dtype,
                           pick(block, i), header)
            rep = report_dict(it.rep)
            rep["header"] = header
            res.append((it.rc, bufs[i][: it.out_size] if it.rc == OK else None, rep))
        return rc, res

    def decompress_batch(self, streams, outs=None, faults=None, geoms=None, headers=None):
        """Decompress several streams in one call (faults: None or one RECON
        plan or None per stream; geoms: None or (shape, is_f32, block) per
        stream when the caller knows them, which saves reading the headers
        here: the library checks them against the headers anyway; headers:
        None or the header bytes (or None) per stream, which spare the
        header read-back when every stream has one).  Returns
        (rc, [(rc, tensor, report)])."""
        torch = self.torch
        L = lib()
        n = len(streams)
        items = (DecItem * max(n, 1))()
        params = (Params * max(n, 1))()
        outs = list(outs) if outs is not None else [None] * n
        keep = []
        for i, s in enumerate(streams):
            if geoms is not None and geoms[i] is not None:
                shape, is_f32, blk = geoms[i]
                rc, p, shape = OK, make_params(tuple(shape), is_f32, blk, 1.0), tuple(shape)
            else:
                rc, p, shape = self._geometry(s)
            if rc != OK:
                return rc, None
            fptr, nf, k = _faults(faults[i] if faults is not None else None)
            keep.append(k)
            items[i].faults = fptr
            items[i].n_faults = nf
            hb = headers[i] if headers is not None else None
            if hb is None:
                hb = self._header(s)
            if hb is not None:
                hbuf = C.create_string_buffer(bytes(hb), HEADER_BYTES)
                keep.append(hbuf)
                items[i].h_header = C.cast(hbuf, C.c_void_p)
            params[i] = p  # a copy (p may be shared)
            params[i].n_faults = nf
            dt = torch.float32 if p.dtype == 0 else torch.float64
            if outs[i] is None:
                outs[i] = torch.empty(shape, dtype=dt, device=self.device)
            items[i].d_stream = s.data_ptr()
            items[i].stream_size = s.numel()
            items[i].d_out = outs[i].data_ptr()
            items[i].out_cap = outs[i].numel() * outs[i].element_size()
        ws_n = L.sdcsz_decompress_batch_workspace_size(params, n)
        ws = self.workspace(ws_n, "decompress_batch")
        rc = L.sdcsz_decompress_batch(items, n, C.c_void_p(ws.data_ptr()), ws.numel(),
                                      _stream_handle(self.device))
        return rc, [(items[i].rc, outs[i], report_dict(items[i].rep)) for i in range(n)]

    def prepare_region(self, stream, header=None):
        """(rc, RegionState): the stream's decoding tables and per-block
        offsets built once in a workspace of their own, for repeated
        decompress_region calls on the unchanged stream."""
        torch = self.torch
        L = lib()
        rc, p, shape = self._geometry(stream)
        if rc != OK:
            return rc, None
        if header is None:
            header = self._header(stream)
        if header is None:
            header = bytes(stream[:HEADER_BYTES].cpu().numpy())
        q = Params.from_buffer_copy(p)  # p may be shared
        q.n_faults = 0
        ws = torch.empty(int(L.sdcsz_decompress_workspace_size(C.byref(q))), dtype=torch.uint8,
                         device=self.device)
        hbuf = C.create_string_buffer(bytes(header), HEADER_BYTES)
        rc = L.sdcsz_region_prepare(C.c_void_p(stream.data_ptr()), stream.numel(), C.cast(hbuf, C.c_void_p),
                                    C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(self.device))
        if rc != OK:
            return rc, None
        return rc, RegionState(stream.data_ptr(), stream.numel(), bytes(header), p.dtype, shape, ws)

    def decompress_region(self, stream, lo, hi, state=None, cache=True):
        """Values of the box [lo, hi) of a stream's field: (rc, tensor of the
        box's shape, report).  Only the blocks the box touches are decoded.
        With a RegionState (prepare_region), or with cache (the codec keeps
        the states of its last few streams, dropped when it writes another
        stream into that buffer), the tables and block offsets are not
        rebuilt; cache=False rebuilds them inside the call."""
        torch = self.torch
        L = lib()
        cached = False
        if state is None and cache:
            state = self._regions.get(stream.data_ptr())
            cached = state is not None
            if state is not None and state.size != stream.numel():
                state = None
            if state is None:
                rc, state = self.prepare_region(stream)
                if rc != OK:
                    return rc, None, None
                if len(self._regions) >= 4:
                    self._regions.pop(next(iter(self._regions)))
                self._regions[stream.data_ptr()] = state
        if state is not None:
            dtype, shape = state.dtype, state.shape
        else:
            rc, p, shape = self._geometry(stream)
            if rc != OK:
                return rc, None, None
            dtype = p.dtype
        dt = torch.float32 if dtype == 0 else torch.float64
        ext = [int(h) - int(l) for l, h in zip(lo, hi)]
        out = torch.empty([max(e, 0) for e in ext], dtype=dt, device=self.device)
        lo_a = (C.c_uint64 * 3)(*([int(v) for v in lo] + [0] * (3 - len(lo))))
        hi_a = (C.c_uint64 * 3)(*([int(v) for v in hi] + [0] * (3 - len(hi))))
        rep = Report()
        optr = C.c_void_p(out.data_ptr()) if out.numel() else None
        obytes = out.numel() * out.element_size()
        if state is not None:
            hbuf = C.create_string_buffer(state.header, HEADER_BYTES)
            rc = L.sdcsz_decompress_region_prepared(C.c_void_p(stream.data_ptr()), stream.numel(),
                                                    C.cast(hbuf, C.c_void_p), lo_a, hi_a, optr, obytes,
                                                    C.byref(rep), C.c_void_p(state.ws.data_ptr()),
                                                    state.ws.numel(), _stream_handle(self.device))
            if rc == EFORMAT and cached:
                # another stream now sits at this address: build its state afresh
                self._regions.pop(stream.data_ptr(), None)
                return self.decompress_region(stream, lo, hi)
        else:
            ws = self._dec_ws(p, 0)
            rc = L.sdcsz_decompress_region(C.c_void_p(stream.data_ptr()), stream.numel(), lo_a, hi_a, optr,
                                           obytes, C.byref(rep), C.c_void_p(ws.data_ptr()), ws.numel(),
                                           _stream_handle(self.device))
        return rc, out, report_dict(rep)


class RegionState:
    """A stream's region-decoding state on the device (Codec.prepare_region):
    decoding tables, per-block offsets and a copy of the header they were
    built from, in a workspace of its own."""

    def __init__(self, ptr, size, header, dtype, shape, ws):
        self.ptr, self.size, self.header, self.dtype, self.shape, self.ws = ptr, size, header, dtype, shape, ws

def timing_enable(on=True):
    lib().sdcsz_timing_enable(1 if on else 0)


def timing_read():
    """{phase name: (accumulated device ms, launches)} of the enabled period."""
    L = lib()
    t = Timing()
    L.sdcsz_timing_read(C.byref(t))
    return {L.sdcsz_phase_name(i).decode(): (t.ms[i], t.launches[i]) for i in range(N_PHASES)}


def tune_set(stage, shape_class, dtype, entries):
    """entries: [(max_blocks, lanes), ...] ascending; [] restores the default."""
    m = max(len(entries), 1)
    mb = (C.c_uint64 * m)(*[int(e[0]) for e in entries])
    ln = (C.c_uint32 * m)(*[int(e[1]) for e in entries])
    return lib().sdcsz_tune_set(stage, shape_class, dtype, len(entries), mb, ln)


def tune_get(stage, shape_class, dtype):
    n = C.c_uint32(0)
    mb = (C.c_uint64 * TUNE_MAX)()
    ln = (C.c_uint32 * TUNE_MAX)()
    rc = lib().sdcsz_tune_get(stage, shape_class, dtype, C.byref(n), mb, ln)
    if rc != OK:
        raise SdcszError(rc, "sdcsz_tune_get")
    return [(int(mb[i]), int(ln[i])) for i in range(n.value)]


def strerror(rc):
    return lib().sdcsz_strerror(rc).decode()
