"""Host logic of the serving loop with a stand-in batch (no GPU).

The stand-in keeps the batch's contract (admit refuses with None when the arena
is full, a step advances every QP in flight, finished tickets are collected
once), so the server's FIFO admission, memory waits, timeline and latency
accounting are checked without the library.
"""
import numpy as np
import pytest

from paper_2104_12916_amd import serve


class Info:
    def __init__(self, status=0):
        self.status = status
        self.rel_kkt = 0.0


class FakeBatch:
    """Each QP needs `work` ticks (its n / 100); footprint = n * 1000 bytes."""

    def __init__(self, capacity):
        self.capacity = capacity
        self.used = 0
        self.live = {}      # ticket -> [ticks left, bytes, n]
        self.done = []
        self.next = 1
        self.admits = []

    def footprint(self, n, m1, m2):
        return n * 1000 if n > 0 and 0 < m1 <= n and m2 > 0 else 0

    def query(self):
        return {"in_flight": len(self.live), "finished": len(self.done), "bytes_used": self.used,
                "bytes_capacity": self.capacity, "rounds": 0}

    def admit(self, H, c, A, b, C, d):
        fp = self.footprint(H.shape[0], A.shape[0], C.shape[0])
        if self.used + fp > self.capacity:
            return None
        t = self.next
        self.next += 1
        self.used += fp
        self.live[t] = [max(1, H.shape[0] // 100), fp, H.shape[0]]
        self.admits.append(H.shape[0])
        return t

    def step(self, rounds=1):
        for t in list(self.live):
            self.live[t][0] -= 1
            if self.live[t][0] == 0:
                self.used -= self.live[t][1]
                self.done.append((t, self.live.pop(t)[2]))
        return len(self.done)

    def finished(self):
        return [t for t, _ in self.done]

    def collect(self, t, accept=(0,)):
        n = dict(self.done)[t]
        self.done = [(u, m) for u, m in self.done if u != t]
        return np.full(n, float(n)), np.zeros(1), np.zeros(1), np.zeros(1), Info()

    def close(self):
        pass


def req(n):
    return (np.zeros((n, n)), np.zeros(n), np.zeros((max(1, n // 4), n)), np.zeros(max(1, n // 4)),
            np.zeros((n // 2, n)), np.zeros(n // 2))


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3      # every clock read advances 1 ms
        return self.t


def test_fifo_admission_waits_for_memory_and_returns_in_request_order():
    fb = FakeBatch(capacity=1_000_000)                  # room for n = 1000 of QPs at once
    sizes = [400, 500, 300, 800, 200, 100]
    srv = serve.Server(batch=fb, clock=Clock(), record_timeline=True)
    res = srv.run([req(n) for n in sizes])              # all arrive at t = 0
    assert [r.rid for r in res] == list(range(6))
    assert [int(r.x[0]) for r in res] == sizes          # each result belongs to its request
    assert fb.admits == sizes                           # arrival order, never overtaken
    assert srv.stats.memory_waits > 0 and srv.stats.peak_bytes_used <= 1_000_000
    assert all(r.arrival <= r.admitted <= r.finished for r in res)
    assert max(b for _, _, b in srv.stats.timeline) <= 1_000_000


def test_oversized_request_is_refused_at_submission():
    srv = serve.Server(batch=FakeBatch(capacity=100_000), clock=Clock())
    with pytest.raises(ValueError, match="more than the arena"):
        srv.submit(*req(200))
    with pytest.raises(ValueError, match="invalid"):
        srv.submit(np.zeros((0, 0)), np.zeros(0), np.zeros((1, 0)), np.zeros(1), np.zeros((1, 0)), np.zeros(1))


def test_arrivals_in_the_future_wait_and_latency_is_from_arrival():
    fb = FakeBatch(capacity=10_000_000)
    srv = serve.Server(batch=fb, clock=Clock())
    arr = [0.0, 0.05, 0.05, 0.2]
    res = srv.run([req(100), req(200), req(300), req(100)], arrivals=arr)
    for r, a in zip(res, arr):
        assert r.arrival == a and r.admitted >= a and r.latency > 0
    s = serve.latency_summary(res, skip=1)
    assert s["count"] == 3 and s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]
    with pytest.raises(ValueError):
        srv.run([req(100), req(100)], arrivals=[0.1, 0.0])


def test_poisson_arrivals_are_seeded_and_have_the_rate():
    a = serve.poisson_arrivals(20000, rate=50.0, seed=3)
    assert np.array_equal(a, serve.poisson_arrivals(20000, rate=50.0, seed=3))
    assert np.all(np.diff(a) >= 0)
    assert abs(len(a) / a[-1] - 50.0) < 2.0
