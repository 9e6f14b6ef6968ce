"""Request loop for streams of QPs: continuous batching over one qp_batch.

QPs of different sizes arrive over time.  Each request waits in a FIFO queue
until the batch's device arena has room for it (the footprint the library
reports for its sizes: its problem data, K0 factor, P_H factor and IPM state,
all kept resident in HBM until it finishes), is then admitted between two
ticks and joins the CG steps of the QPs already in flight at the next tick
(one tick = one chunk of CG steps for every QP inside a reduced solve, then
every QP's IPM phases that need no CG).  A finished QP is collected at once and
its memory returns to the arena, which admits the next waiting request.

Latency is measured from a request's arrival (its scheduled time on the
server's clock, not the moment the loop noticed it) to the tick that finished
it; admission copies the request's data to the device, so the upload counts.
Every solve runs in the library's kernels; this module only orders calls.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import qpgpu

# statuses a finished QP can carry (anything else is a call error and raises)
QP_RESULT_STATUSES = (qpgpu.QP_OK, qpgpu.QP_E_NOCONV, qpgpu.QP_E_NOT_SPD, qpgpu.QP_E_RANK)


@dataclass
class Result:
    """Final iterate of one request and its timeline (seconds on the server clock)."""
    rid: int
    x: np.ndarray
    lam: np.ndarray
    nu: np.ndarray
    s: np.ndarray
    info: qpgpu.qp_ipm_info
    arrival: float
    admitted: float
    finished: float

    @property
    def status(self) -> int:
        return self.info.status

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class _Pending:
    rid: int
    arrays: tuple
    arrival: float
    footprint: int


@dataclass
class ServerStats:
    submitted: int = 0
    admitted: int = 0
    finished: int = 0
    ticks: int = 0
    memory_waits: int = 0          # admission attempts refused for lack of arena room
    peak_bytes_used: int = 0
    peak_in_flight: int = 0
    max_queue: int = 0
    timeline: list = field(default_factory=list)   # (time, in_flight, bytes_used) after each tick


class Server:
    """Continuous-batching server over one batch of the library.

    budget_bytes  device arena of the batch (0: 80 % of the free device memory)
    clock         time source in seconds (time.perf_counter)
    opts          qp_options fields (prec, precision, kf_form, ...)
    """

    def __init__(self, budget_bytes: int = 0, clock=time.perf_counter, record_timeline: bool = False, batch=None,
                 **opts):
        # batch: an object with the qpgpu.Batch methods (the tests' stand-in); default a new qpgpu.Batch
        self.batch = qpgpu.Batch(budget_bytes, **opts) if batch is None else batch
        self.capacity = self.batch.query()["bytes_capacity"]
        self.clock = clock
        self.t0 = clock()
        self.queue: collections.deque[_Pending] = collections.deque()
        self.owner: dict[int, tuple[int, float, float]] = {}  # ticket -> (rid, arrival, admitted)
        self.stats = ServerStats()
        self.record_timeline = record_timeline
        self._next = 0

    # -- clock ----------------------------------------------------------------
    def now(self) -> float:
        return self.clock() - self.t0

    def reset_clock(self) -> None:
        self.t0 = self.clock()

    # -- requests -------------------------------------------------------------
    def footprint(self, n: int, m1: int, m2: int) -> int:
        """Arena bytes a QP of these sizes takes (0 when the sizes are invalid)."""
        return self.batch.footprint(n, m1, m2)

    def submit(self, H, c, A, b, C, d, arrival: float | None = None) -> int:
        """Queue one QP (arrays as for qp_setup).  Returns its request id.

        Raises ValueError when the QP can never fit the arena (it would block
        the queue for good) or its sizes are invalid."""
        n, m1, m2 = H.shape[0], A.shape[0], C.shape[0]
        fp = self.footprint(n, m1, m2)
        if fp == 0:
            raise ValueError(f"invalid QP sizes n={n} m1={m1} m2={m2}")
        if fp > self.capacity:
            raise ValueError(f"QP n={n} m1={m1} m2={m2} needs {fp} bytes, more than the arena's {self.capacity}")
        rid = self._next
        self._next += 1
        self.queue.append(_Pending(rid, (H, c, A, b, C, d), self.now() if arrival is None else arrival, fp))
        self.stats.submitted += 1
        self.stats.max_queue = max(self.stats.max_queue, len(self.queue))
        return rid

    def _admit(self) -> None:
        """Admit queued requests in arrival order while the arena has room."""
        while self.queue:
            p = self.queue[0]
            t = self.batch.admit(*p.arrays)
            if t is None:  # QP_E_NOMEM: wait for a QP to finish
                self.stats.memory_waits += 1
                return
            self.queue.popleft()
            self.owner[t] = (p.rid, p.arrival, self.now())
            self.stats.admitted += 1

    def tick(self) -> list[Result]:
        """One scheduling round: admit what fits, run one tick of the batch if
        anything is in flight, collect every QP that finished."""
        self._admit()
        q = self.batch.query()
        self.stats.peak_in_flight = max(self.stats.peak_in_flight, q["in_flight"])
        self.stats.peak_bytes_used = max(self.stats.peak_bytes_used, q["bytes_used"])
        out = []
        if q["in_flight"] == 0:
            return out
        self.batch.step(1)
        self.stats.ticks += 1
        t_done = self.now()
        for t in self.batch.finished():
            rid, arrival, admitted = self.owner.pop(t)
            x, lam, nu, s, info = self.batch.collect(t, accept=QP_RESULT_STATUSES)
            out.append(Result(rid, x, lam, nu, s, info, arrival, admitted, t_done))
            self.stats.finished += 1
        if self.record_timeline:
            q = self.batch.query()
            self.stats.timeline.append((t_done, q["in_flight"], q["bytes_used"]))
        return out

    @property
    def busy(self) -> bool:
        return bool(self.queue) or bool(self.owner)

    def drain(self) -> list[Result]:
        """Run ticks until every submitted request has finished."""
        out = []
        while self.busy:
            out.extend(self.tick())
        return out

    def run(self, requests, arrivals=None, progress=None) -> list[Result]:
        """Replay a trace: request k (a tuple H, c, A, b, C, d) arrives at
        arrivals[k] seconds after the call (None: all at once).  Returns the
        results in request order.  progress(done, total) is called after each
        finished request when given."""
        m = len(requests)
        arr = np.zeros(m) if arrivals is None else np.asarray(arrivals, dtype=float)
        if np.any(np.diff(arr) < 0):
            raise ValueError("arrivals must be non-decreasing")
        self.reset_clock()
        base = self._next
        results: dict[int, Result] = {}
        i = 0
        while len(results) < m:
            now = self.now()
            while i < m and arr[i] <= now:
                self.submit(*requests[i], arrival=float(arr[i]))
                i += 1
            if not self.busy:
                if i < m:  # idle until the next arrival
                    time.sleep(max(0.0, arr[i] - self.now()))
                continue
            for r in self.tick():
                results[r.rid - base] = r
                if progress:
                    progress(len(results), m)
        return [results[k] for k in range(m)]

    def close(self) -> None:
        if self.batch is not None:
            self.batch.close()
            self.batch = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def poisson_arrivals(count: int, rate: float, seed: int = 5001) -> np.ndarray:
    """Arrival times of a Poisson stream of `rate` requests per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def latency_summary(results, skip: int = 0) -> dict:
    """Throughput and latency of results[skip:] (the first `skip` are warm-up).

    Throughput counts the measured requests over the span from the first
    measured arrival to the last measured finish."""
    meas = list(results)[skip:]
    if not meas:
        return dict(count=0)
    lat = np.array([r.latency for r in meas]) * 1e3
    span = max(r.finished for r in meas) - min(r.arrival for r in meas)
    return dict(count=len(meas), solves_per_s=len(meas) / max(span, 1e-9), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()), max_ms=float(lat.max()))
