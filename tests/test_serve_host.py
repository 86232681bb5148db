"""Queueing and admission of the request server, on the CPU (a stand-in
executor replaces the GPU): arrival order is kept, the HBM budget is never
exceeded, requests that cannot fit fail, and requests arriving while batches
run are admitted as memory frees up."""
import threading
import time

from paper_2010_03144_amd import serve


class FakeExecutor:
    def __init__(self, delay=0.01):
        self.delay = delay
        self.lock = threading.Lock()
        self.admitted = []  # batches in the order they started
        self.running = 0
        self.max_running = 0

    def worker_context(self):
        return {}

    def run(self, ctx, batch, now):
        with self.lock:
            self.admitted.append([r.tag for r in batch])
            self.running += 1
            self.max_running = max(self.max_running, self.running)
        time.sleep(self.delay)
        t = now()
        for r in batch:
            r.rc, r.result, r.t_done = 0, ("done", r.tag), t
        with self.lock:
            self.running -= 1


def make(footprints, nbytes=10):
    return [serve.Request("compress", None, footprint=f, nbytes=nbytes, tag=i) for i, f in enumerate(footprints)]


def test_budget_fifo_and_oversized_requests():
    ex = FakeExecutor()
    reqs = make([30, 30, 50, 90, 10, 10, 200, 5])
    with serve.Server(workers=3, hbm_budget=100, max_batch=4, executor=ex) as srv:
        for r in reqs:
            srv.submit(r)
        srv.drain()
        assert srv.peak_in_use <= 100
    assert all(r.done.is_set() for r in reqs)
    assert reqs[6].rc == serve.ENOMEM and reqs[6].result is None
    assert all(r.rc == 0 and r.result == ("done", r.tag) for r in reqs if r.tag != 6)
    order = [t for b in ex.admitted for t in b]
    assert order == sorted(order)  # batches are taken from the head of the queue
    for b in ex.admitted:
        assert sum(reqs[t].footprint for t in b) <= 100


def test_batch_limits():
    ex = FakeExecutor(delay=0.05)
    reqs = make([1] * 10, nbytes=100)
    with serve.Server(workers=1, hbm_budget=1e9, max_batch=4, max_batch_bytes=250, executor=ex) as srv:
        for r in reqs:
            srv.submit(r)
        srv.drain()
    assert all(len(b) <= 2 for b in ex.admitted)  # 250 bytes hold two 100-byte fields
    assert sorted(t for b in ex.admitted for t in b) == list(range(10))


def test_arrivals_during_a_batch_join_the_next_one():
    ex = FakeExecutor(delay=0.1)
    with serve.Server(workers=1, hbm_budget=1e9, max_batch=64, executor=ex) as srv:
        first = srv.submit(make([1])[0])
        time.sleep(0.03)  # the first batch is running
        late = make([1, 1, 1])
        for i, r in enumerate(late):
            r.tag = 10 + i
            srv.submit(r)
        srv.drain()
    assert ex.admitted[0] == [0]
    assert ex.admitted[1] == [10, 11, 12]  # admitted together once the worker was free
    assert first.latency < late[0].latency + 0.1


def test_workers_overlap():
    ex = FakeExecutor(delay=0.05)
    reqs = make([60] * 4)
    with serve.Server(workers=2, hbm_budget=130, max_batch=1, executor=ex) as srv:
        for r in reqs:
            srv.submit(r)
        srv.drain()
    assert ex.max_running == 2  # two 60-byte requests fit the 130-byte budget at once


def test_replay_sets_arrival_times():
    ex = FakeExecutor(delay=0.0)
    reqs = make([1, 1, 1])
    for i, r in enumerate(reqs):
        r.t_arrival = 0.02 * i
    with serve.Server(workers=1, hbm_budget=10, executor=ex) as srv:
        t0 = srv.clock()
        serve.replay(srv, reqs, t0)
    for i, r in enumerate(reqs):
        assert abs(r.t_arrival - (t0 + 0.02 * i)) < 1e-9
        assert r.t_done >= r.t_arrival


class RaisingExecutor(FakeExecutor):
    def run(self, ctx, batch, now):
        if any(r.tag == 1 for r in batch):
            raise RuntimeError("device error")
        super().run(ctx, batch, now)


def test_a_failing_batch_fails_its_requests_only():
    ex = RaisingExecutor()
    reqs = make([1, 1, 1])
    with serve.Server(workers=1, hbm_budget=10, max_batch=1, executor=ex) as srv:
        for r in reqs:
            srv.submit(r)
        srv.drain()
    assert reqs[1].rc == serve.EEXEC and isinstance(reqs[1].error, RuntimeError)
    assert reqs[0].rc == reqs[2].rc == 0
