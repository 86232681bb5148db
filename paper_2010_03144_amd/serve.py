"""Serving: compress and decompress requests on one GPU with continuous batching.

Requests enter one FIFO queue as they arrive.  Each of `workers` host threads
owns a HIP stream (default priority) and a Codec; a worker that becomes free
takes, in arrival order, every queued request whose device footprint still
fits the HBM budget (up to `max_batch` requests and `max_batch_bytes` of
field data), runs them as one batched compression call and one batched
decompression call (every kernel of a call covers all of its fields), and
completes them.  Requests that arrive while batches run wait only until a
worker is free and memory allows; the batches of different workers overlap
on the device (one worker's kernels run while another builds its codebooks
on the host or waits for its histogram).  Streams, codebooks and decoder
tables stay in device memory throughout: a compression request's result is a
device stream, a decompression request reads a device stream and builds its
decoder tables on the device.

Batching does not change any result: each field's kernels see only that
field's data and parameters, so a request gives the same stream (or values)
and the same fault counts alone and in any mix.

The execution backend is replaceable (`executor`), so the queueing and
admission logic can run without a GPU.
"""
import collections
import math
import threading
import time

from . import sdcsz

ENOMEM = -6  # a request whose footprint exceeds the whole budget
EEXEC = -7   # the batch's execution raised (the exception is kept in req.error)


class Request:
    """One request.  kind is "compress" (data: a device field) or
    "decompress" (data: a device stream; geom = (shape, is_f32, block) and
    header = the stream's header bytes when known, which spares reading them
    back).  After completion: rc, result (stream or field tensor), report,
    and the times t_arrival, t_start, t_done (time.perf_counter seconds)."""

    def __init__(self, kind, data, block=None, eb=None, eb_mode="rel", abft=True, predictor="auto",
                 faults=None, geom=None, footprint=None, nbytes=None, tag=None, header=None):
        assert kind in ("compress", "decompress")
        self.kind, self.data, self.block, self.eb = kind, data, block, eb
        self.eb_mode, self.abft, self.predictor, self.faults = eb_mode, abft, predictor, faults
        self.geom, self.footprint, self.nbytes, self.tag = geom, footprint, nbytes, tag
        self.header = header
        self.rc = None
        self.result = None
        self.result_bytes = None  # size of the result (bytes), kept when the result is dropped
        self.report = None
        self.t_arrival = self.t_start = self.t_done = None
        self.error = None
        self.done = threading.Event()

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


def field_bytes(req):
    """Bytes of the field a request compresses or reconstructs."""
    if req.nbytes is not None:
        return req.nbytes
    if req.kind == "compress":
        return req.data.numel() * req.data.element_size()
    shape, is_f32, _ = req.geom
    n = 1
    for d in shape:
        n *= int(d)
    return n * (4 if is_f32 else 8)


def device_footprint(req):
    """Device bytes the server allocates for a request: its output buffer
    and its share of the library workspace."""
    import torch
    if req.kind == "compress":
        x = req.data
        is_f32 = x.dtype == torch.float32
        nf = 0 if req.faults is None else len(req.faults)
        ws, _ = sdcsz.workspace_sizes(x.shape, is_f32, req.block, nf)
        return sdcsz.max_compressed_size(x.shape, is_f32, req.block) + ws
    shape, is_f32, block = req.geom
    nf = 0 if req.faults is None else len(req.faults)
    _, ws = sdcsz.workspace_sizes(shape, is_f32, block, nf)
    return field_bytes(req) + ws


class GpuExecutor:
    """Runs a batch on one worker's stream through the batched C-ABI calls."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        # True when results are released as soon as they are measured: the
        # outputs of a batch are then views into one buffer per worker and
        # kind, reused by its next batches.  Fresh outputs of every size
        # for every batch leave torch's caching allocator with hundreds of GB
        # of blocks of the wrong sizes, and its out-of-memory retries (which
        # free and reallocate everything) cut the throughput several-fold.
        self.reuse_outputs = False

    def worker_context(self):
        torch = self.torch
        stream = torch.cuda.Stream(device=self.device)  # default priority
        return {"stream": stream, "codec": sdcsz.Codec(self.device)}

    def _outputs(self, ctx, key, sizes):
        """Byte views of the given sizes (256-byte aligned), fresh tensors
        unless outputs are reused, else views into the worker's buffer for
        `key` (grown by at least half when too small)."""
        torch = self.torch
        if not self.reuse_outputs:
            return [torch.empty(n, dtype=torch.uint8, device=self.device) for n in sizes]
        offs, total = [], 0
        for n in sizes:
            offs.append(total)
            total += (int(n) + 255) // 256 * 256
        buf = ctx.get(key)
        if buf is None or buf.numel() < total:
            old = 0 if buf is None else buf.numel()
            ctx[key] = buf = None  # released, and returned to the device, before the larger one is taken
            if old >= 1 << 30:
                torch.cuda.empty_cache()
            buf = ctx[key] = torch.empty(max(total, old + old // 2, 1), dtype=torch.uint8, device=self.device)
        return [buf[o:o + int(n)] for o, n in zip(offs, sizes)]

    def run(self, ctx, batch, now):
        torch = self.torch
        codec = ctx["codec"]
        comp = [r for r in batch if r.kind == "compress"]
        dec = [r for r in batch if r.kind == "decompress"]
        groups = sorted([g for g in (comp, dec) if g], key=lambda g: sum(field_bytes(r) for r in g))
        with torch.cuda.stream(ctx["stream"]):
            for g in groups:  # the group with less data first
                if g is comp:
                    outs = self._outputs(ctx, "compress", [sdcsz.max_compressed_size(
                        r.data.shape, r.data.dtype == torch.float32, r.block) for r in g])
                    rc, res = codec.compress_batch([r.data for r in g], [tuple(r.block) for r in g],
                                                   [r.eb for r in g], [r.eb_mode for r in g],
                                                   [r.abft for r in g], [r.predictor for r in g],
                                                   faults=[r.faults for r in g], outs=outs)
                else:
                    outs = None
                    if self.reuse_outputs and all(r.geom is not None for r in g):
                        dts = [torch.float32 if r.geom[1] else torch.float64 for r in g]
                        nbs = [math.prod(r.geom[0]) * (4 if r.geom[1] else 8) for r in g]
                        outs = [v.view(dt).view(tuple(r.geom[0]))
                                for v, dt, r in zip(self._outputs(ctx, "decompress", nbs), dts, g)]
                    rc, res = codec.decompress_batch([r.data for r in g], outs=outs, faults=[r.faults for r in g],
                                                     geoms=[r.geom for r in g], headers=[r.header for r in g])
                t = now()
                for i, r in enumerate(g):
                    if res is None:
                        r.rc, r.result, r.report = rc, None, None
                    else:
                        r.rc, r.result, r.report = res[i]
                    r.t_done = t


class Server:
    def __init__(self, device="cuda:0", workers=2, hbm_budget=200e9, max_batch=64,
                 max_batch_bytes=8 << 30, executor=None, clock=time.perf_counter, keep_results=True):
        self.budget = float(hbm_budget)
        self.max_batch = int(max_batch)
        self.max_batch_bytes = int(max_batch_bytes)
        self.executor = executor if executor is not None else GpuExecutor(device)
        if hasattr(self.executor, "reuse_outputs"):
            self.executor.reuse_outputs = not keep_results
        self.clock = clock
        self.keep_results = keep_results  # False: results are measured, then released
        self._q = collections.deque()
        self._cv = threading.Condition()
        self._in_use = 0
        self._running = 0
        self._closed = False
        self.peak_in_use = 0
        self.batches = []  # sizes of the batches run
        self._threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(workers)]
        for t in self._threads:
            t.start()

    # ------------------------------------------------------------------ client
    def submit(self, req):
        if req.t_arrival is None:
            req.t_arrival = self.clock()
        if req.footprint is None:
            req.footprint = device_footprint(req)
        with self._cv:
            if self._closed:
                raise RuntimeError("server closed")
            self._q.append(req)
            self._cv.notify()
        return req

    def drain(self):
        """Wait until every submitted request has completed."""
        with self._cv:
            while self._q or self._running:
                self._cv.wait()

    def close(self):
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ workers
    def _admit(self):
        """Requests for one batch, in arrival order, within the budget (called
        with the lock held).  The head of the queue is never overtaken."""
        batch, data = [], 0
        while self._q and len(batch) < self.max_batch:
            r = self._q[0]
            if r.footprint > self.budget:  # can never fit: fail it
                self._q.popleft()
                r.rc, r.t_done = ENOMEM, self.clock()
                r.done.set()
                self._cv.notify_all()
                continue
            if self._in_use + r.footprint > self.budget:
                break
            nb = field_bytes(r)
            if batch and data + nb > self.max_batch_bytes:
                break
            self._q.popleft()
            batch.append(r)
            self._in_use += r.footprint
            data += nb
        self.peak_in_use = max(self.peak_in_use, self._in_use)
        return batch

    def _worker(self):
        ctx = self.executor.worker_context()
        while True:
            with self._cv:
                while True:
                    batch = self._admit() if self._q else []
                    if batch:
                        self._running += 1
                        break
                    if self._closed and not self._q:
                        return
                    self._cv.wait()
            t = self.clock()
            for r in batch:
                r.t_start = t
            try:
                self.executor.run(ctx, batch, self.clock)
            except Exception as e:  # noqa: BLE001 - reported per request, the worker stays up
                for r in batch:
                    if r.rc is None:
                        r.rc, r.error = EEXEC, e
            finally:
                with self._cv:
                    self._in_use -= sum(r.footprint for r in batch)
                    self._running -= 1
                    self.batches.append(len(batch))
                    self._cv.notify_all()
                for r in batch:
                    if r.t_done is None:
                        r.t_done = self.clock()
                    _finish(r, self.keep_results)
                    r.done.set()


def _finish(r, keep):
    if r.result is not None and hasattr(r.result, "numel"):
        r.result_bytes = r.result.numel() * r.result.element_size()
        if not keep:
            r.result = None


def replay(server, requests, t0):
    """Client side of a timed run: submits each request at t0 + its arrival
    offset (req.t_arrival on entry, seconds), which becomes its arrival time,
    then waits for all of them."""
    for r in sorted(requests, key=lambda r: r.t_arrival):
        at = t0 + r.t_arrival
        wait = at - server.clock()
        if wait > 0:
            time.sleep(wait)
        r.t_arrival = at
        server.submit(r)
    server.drain()


def serve_one_at_a_time(requests, t0, device="cuda:0", clock=time.perf_counter, keep_results=True):
    """The plain loop: requests in arrival order (offsets req.t_arrival from
    t0, as in replay), each by itself through the single-field calls and
    started no earlier than its arrival."""
    import torch
    codec = sdcsz.Codec(device)
    for r in sorted(requests, key=lambda r: r.t_arrival):
        r.t_arrival = t0 + r.t_arrival
        wait = r.t_arrival - clock()
        if wait > 0:
            time.sleep(wait)
        r.t_start = clock()
        if r.kind == "compress":
            out = torch.empty(sdcsz.max_compressed_size(r.data.shape, r.data.dtype == torch.float32, r.block),
                              dtype=torch.uint8, device=device)
            r.rc, r.result, r.report = codec.compress(r.data, r.block, r.eb, r.eb_mode, r.abft, r.predictor,
                                                      faults=r.faults, out=out)
        else:
            r.rc, r.result, r.report = codec.decompress(r.data, faults=r.faults, geom=r.geom, header=r.header)
        r.t_done = clock()
        _finish(r, keep_results)
        r.done.set()
