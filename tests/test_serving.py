"""The serving scheduler on the CPU, against a fake backend with a manual
clock: admission by memory, per-rig order, continuous batching, expiry,
failure isolation, latency report, and a threaded run."""
import threading
import time

import numpy as np
import pytest

from paper_1910_03517_amd.serving import Backend, BackendError, Server


class Clock:
    def __init__(self):
        self.now = 0.0

    def __call__(self):
        return self.now


class FakeBackend(Backend):
    """Launch = the batch completes `duration` after it was enqueued (after
    the previous launch, like a device stream)."""

    def __init__(self, n_rigs, clock, bytes_per=None, duration=0.01, refuse=(), device_error=False):
        self.n_rigs = n_rigs
        self.clock = clock
        self.bytes_per = bytes_per or [100] * n_rigs
        self.duration = duration
        self.refuse = set(refuse)
        self.device_error = device_error
        self.launches = []
        self.live_out = 0
        self.max_live_out = 0
        self.stream_free_at = 0.0
        self.outstanding = 0
        self.max_outstanding = 0

    def frameset_bytes(self, rig):
        return self.bytes_per[rig]

    def rig_pixels(self, rig):
        return 1000 * (rig + 1)

    def alloc_out(self, rig):
        self.live_out += 1
        self.max_live_out = max(self.max_live_out, self.live_out)
        return ["out", rig]

    def free_out(self, rig, out):
        assert out == ["out", rig]
        self.live_out -= 1

    def launch(self, batch):
        rigs = [r.rig for r in batch]
        assert len(rigs) == len(set(rigs)), "two frame-sets of one rig in a batch"
        bad = [r for r in rigs if r in self.refuse]
        if bad:
            raise BackendError(bad, f"refused {bad}")
        if self.device_error:
            raise RuntimeError("device lost")
        self.launches.append([(r.rig, r.seq) for r in batch])
        self.ready_seen = getattr(self, "ready_seen", []) + [r.ready for r in batch]
        start = max(self.clock(), self.stream_free_at)
        self.stream_free_at = start + self.duration
        self.outstanding += 1
        self.max_outstanding = max(self.max_outstanding, self.outstanding)
        return [self.stream_free_at, False]

    def ready(self, token):
        ok = self.clock() >= token[0]
        if ok and not token[1]:
            token[1] = True
            self.outstanding -= 1
        return ok

    def wait(self, token):
        self.clock.now = max(self.clock.now, token[0])


def run_until_idle(srv, clock, step=0.001, limit=10_000):
    for _ in range(limit):
        srv.poll()
        if not srv.pending():
            return
        clock.now += step
    raise AssertionError("server did not drain")


def launched_order(fake, rig):
    return [seq for batch in fake.launches for (r, seq) in batch if r == rig]


def test_order_one_per_rig_and_full_batches():
    clock = Clock()
    fake = FakeBackend(3, clock)
    srv = Server(fake, mem_budget=10_000, max_batches_in_flight=2, clock=clock)
    for i in range(5):
        for r in range(3):
            srv.submit(r, [f"f{r}.{i}"])
    run_until_idle(srv, clock)
    for r in range(3):
        assert launched_order(fake, r) == list(range(5))
    assert all(len(b) == 3 for b in fake.launches)
    assert fake.max_outstanding <= 2
    rep = srv.report()
    assert rep["done"] == 15 and rep["failed"] == rep["expired"] == rep["rejected"] == 0
    assert fake.live_out == 0 and srv.mem_used == 0


def test_continuous_batching_takes_whatever_is_ready():
    clock = Clock()
    fake = FakeBackend(3, clock, duration=0.01)
    srv = Server(fake, mem_budget=10_000, max_batches_in_flight=1, clock=clock)
    srv.submit(0, ["a"])
    srv.poll()                                   # launches rig 0 alone
    srv.submit(1, ["b"])
    srv.submit(2, ["c"])
    srv.submit(0, ["a2"])
    srv.poll()                                   # one launch in flight: nothing new yet
    assert fake.launches == [[(0, 0)]]
    clock.now += 0.01
    srv.poll()                                   # retire, then one batch of all three rigs
    assert fake.launches[1] == [(0, 1), (1, 0), (2, 0)]
    run_until_idle(srv, clock)


def test_memory_admission_bounds_reservations():
    clock = Clock()
    fake = FakeBackend(2, clock, bytes_per=[300, 100], duration=0.005)
    srv = Server(fake, mem_budget=600, max_batches_in_flight=4, clock=clock)
    for i in range(6):
        srv.submit(0, [i])
    for _ in range(200):
        srv.poll()
        assert srv.mem_used <= 600
        assert fake.live_out <= 2
        clock.now += 0.001
    assert srv.report()["done"] == 6
    assert srv.mem_peak == 600


def test_admission_is_fifo_without_overtaking():
    clock = Clock()
    fake = FakeBackend(2, clock, bytes_per=[500, 100], duration=0.01)
    srv = Server(fake, mem_budget=600, max_batches_in_flight=4, clock=clock)
    a = srv.submit(0, ["a"])
    b = srv.submit(0, ["b"])     # does not fit while `a` holds 500
    c = srv.submit(1, ["c"])     # would fit, but arrived after `b`
    srv.poll()
    assert a.status == "running" and b.status == "queued" and c.status == "queued"
    clock.now += 0.01
    srv.poll()
    assert b.status == "running" and c.status == "running"
    run_until_idle(srv, clock)


def test_queue_limit_rejects():
    clock = Clock()
    fake = FakeBackend(1, clock)
    srv = Server(fake, mem_budget=100, queue_limit=2, clock=clock)
    reqs = [srv.submit(0, [i]) for i in range(4)]
    assert [r.status for r in reqs] == ["queued", "queued", "rejected", "rejected"]
    run_until_idle(srv, clock)
    assert srv.report()["rejected"] == 2 and srv.report()["done"] == 2


def test_stale_requests_expire():
    clock = Clock()
    fake = FakeBackend(1, clock, duration=0.1)
    srv = Server(fake, mem_budget=100, max_wait=0.05, clock=clock)
    first = srv.submit(0, ["a"])
    srv.poll()                   # admitted, holds all memory
    stale = srv.submit(0, ["b"])
    clock.now += 0.06
    srv.poll()
    assert stale.status == "expired"
    run_until_idle(srv, clock)
    assert first.status == "done"


def test_failure_isolation_and_closing_a_rig():
    clock = Clock()
    fake = FakeBackend(3, clock, refuse={1})
    srv = Server(fake, mem_budget=10_000, max_failures=2, clock=clock)
    for i in range(3):
        for r in range(3):
            srv.submit(r, [i])
    run_until_idle(srv, clock)
    by = {}
    for q in srv.finished:
        by.setdefault(q.rig, []).append(q.status)
    assert by[0] == ["done"] * 3 and by[2] == ["done"] * 3
    assert by[1].count("failed") == 2 and by[1].count("rejected") == 1
    assert 1 in srv.closed_rigs
    assert srv.submit(1, ["x"]).status == "rejected"
    assert all(1 not in [r for r, _ in b] for b in fake.launches)
    assert srv.mem_used == 0 and fake.live_out == 0


def test_device_error_stops_the_server():
    clock = Clock()
    fake = FakeBackend(2, clock, device_error=True)
    srv = Server(fake, mem_budget=1000, clock=clock)
    a, b = srv.submit(0, [0]), srv.submit(1, [0])
    srv.poll()
    assert srv.broken is not None
    assert a.status == b.status == "failed"
    assert srv.submit(0, [1]).status == "rejected"
    assert srv.mem_used == 0


def test_latency_report():
    clock = Clock()
    fake = FakeBackend(1, clock, duration=0.004)
    srv = Server(fake, mem_budget=10_000, max_batches_in_flight=1, queue_limit=10, clock=clock)
    for i in range(10):
        srv.submit(0, [i], t_arrival=0.0)
    run_until_idle(srv, clock, step=0.001)
    lat = np.array([r.latency for r in srv.finished])
    rep = srv.report()
    assert rep["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert rep["p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)
    # one frame-set every 4 ms, back to back: the i-th completes at 4 (i + 1) ms
    assert np.allclose(np.sort(lat), 0.004 * np.arange(1, 11), atol=1.5e-3)
    assert rep["pixels"] == 10 * 1000


def test_oversized_rig_is_refused_at_construction():
    with pytest.raises(ValueError):
        Server(FakeBackend(1, Clock(), bytes_per=[1000]), mem_budget=999)


def test_threaded_run_with_arrival_thread():
    class RealFake(FakeBackend):
        def launch(self, batch):
            super().launch(batch)
            return time.perf_counter() + 0.0005

        def ready(self, token):
            return time.perf_counter() >= token

    fake = RealFake(3, time.perf_counter)
    srv = Server(fake, mem_budget=1000, max_batches_in_flight=2)
    srv.start()

    def producer(rig):
        for i in range(20):
            srv.submit(rig, [i])
            time.sleep(0.0003 * (rig + 1))

    th = [threading.Thread(target=producer, args=(r,)) for r in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.stop(drain=True)
    assert srv.report()["done"] == 60
    for r in range(3):
        assert launched_order(fake, r) == list(range(20))
    assert srv.mem_peak <= 1000


def test_ready_events_reach_the_backend():
    """A producer's ready event travels with its request to the launch."""
    clock = Clock()
    fake = FakeBackend(2, clock)
    srv = Server(fake, mem_budget=10_000, clock=clock)
    srv.submit(0, ["a"], ready="ev-a")
    srv.submit(1, ["b"])
    run_until_idle(srv, clock)
    assert sorted(fake.ready_seen, key=str) == [None, "ev-a"]


class Token:
    """A launch event of FakeShard: completes when the test says so."""

    def __init__(self):
        self.done = False

    def query(self):
        return self.done

    def synchronize(self):
        self.done = True


class FakeShard:
    """One context's backend for ShardedBackend (a rig: its list of cameras)."""

    made = []

    def __init__(self, rigs, opts=None, refuse=(), **kw):
        self.rigs = [len(r) for r in rigs]
        self.refuse = set(refuse)
        self.kw = kw
        self.launches = []
        FakeShard.made.append(self)

    def rig_cams(self, rig):
        return ["cam"] * self.rigs[rig]

    def frameset_bytes(self, rig):
        return 10 * self.rigs[rig]

    def rig_pixels(self, rig):
        return 100 * self.rigs[rig]

    def alloc_out(self, rig):
        return ("out", id(self), rig)

    def free_out(self, rig, out):
        assert out == ("out", id(self), rig)

    def check(self, req):
        return "bad frames" if self.rigs[req.rig] in self.refuse else ""

    def launch(self, batch):
        tok = Token()
        self.launches.append(([r.rig for r in batch], tok))
        return tok

    def close(self):
        self.closed = True


def test_sharded_backend_splits_rigs_and_batches():
    """Rigs fill contexts in order up to max_cams cameras; a batch becomes one
    launch per context with the rigs' local indices; it is ready when every
    context's launch is; a refused frame-set refuses before any launch,
    with the global rig index; and the server runs over it unchanged."""
    from paper_1910_03517_amd.serving import ShardedBackend
    FakeShard.made = []
    cams = [3, 2, 4, 1, 5]                     # rigs' camera counts
    rigs = [["cam"] * n for n in cams]
    sb = ShardedBackend(rigs, None, max_cams=5, shard_cls=FakeShard, refuse=(), lanes=2)
    shards = FakeShard.made
    assert [s.rigs for s in shards] == [[3, 2], [4, 1], [5]]
    assert all(s.kw == {"lanes": 2} and s.refuse == set() for s in shards)
    assert [len(sb.rig_cams(r)) for r in range(5)] == cams
    assert [sb.frameset_bytes(r) for r in range(5)] == [30, 20, 40, 10, 50]
    assert sb.alloc_out(3) == ("out", id(shards[1]), 1)
    clock = Clock()
    srv = Server(sb, mem_budget=10_000, clock=clock)
    reqs = [srv.submit(r, ["f"] * cams[r]) for r in (4, 0, 3, 1)]
    srv.poll()
    assert shards[0].launches[0][0] == [0, 1]
    assert shards[1].launches[0][0] == [1]
    assert shards[2].launches[0][0] == [0]
    assert srv.pending() == 4
    shards[0].launches[0][1].done = True
    shards[1].launches[0][1].done = True
    srv.poll()
    assert srv.pending() == 4                  # the third context has not finished
    shards[2].launches[0][1].done = True
    srv.poll()
    assert srv.pending() == 0 and all(r.status == "done" for r in reqs)
    # a refused frame-set: rig 2 (the 4-camera rig, context 1, local 0)
    FakeShard.made = []
    sb = ShardedBackend(rigs, None, max_cams=5, shard_cls=FakeShard, refuse=(4,))
    srv = Server(sb, mem_budget=10_000, clock=clock)
    bad = srv.submit(2, ["f"] * 4)
    good = srv.submit(0, ["f"] * 3)
    srv.poll()
    assert bad.status == "failed" and "rig 2: bad frames" in bad.error
    assert [len(s.launches) for s in FakeShard.made] == [1, 0, 0]
    FakeShard.made[0].launches[0][1].done = True
    srv.poll()
    assert good.status == "done"
    with pytest.raises(ValueError, match="more than a context takes"):
        ShardedBackend([["cam"] * 3, ["cam"] * 9], None, max_cams=8, shard_cls=FakeShard)
    sb.close()
