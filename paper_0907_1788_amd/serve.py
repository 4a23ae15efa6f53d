"""Request serving with continuous batching over the fntrs C ABI.

A request is one encode (k source rows -> n codeword rows) or one decode (the
k received rows of an erasure pattern -> k source rows) of a codeword of
`lanes` 16-bit lanes.  The server:

* admits waiting requests in arrival order while the device working set
  (input + output + locator state + four-step scratch of every admitted
  request) stays under a byte cap -- memory-based admission;
* turns what it admits at one time into one batch of at most
  `max_batch_bytes` of working set (by default the cap over the number of
  batches in flight): a backlog is served as several batches in flight, not
  as one batch that takes the whole cap.  Batches of new, larger shapes make
  the runtime's allocators block, and a blocked loop builds a larger backlog.
  The locators of a batch's decode requests are fetched or built together
  (fntrs_locator_batch, cached per erasure pattern on the device) and the
  batch is enqueued with one fntrs_submit;
* keeps up to `max_inflight` batches on the device at once, on rotating
  streams of default priority, so requests that arrive while others run are
  admitted as memory and slots free up and their work overlaps on the GPU;
* retires a batch when its completion event has fired, frees its memory and
  locator references, and stamps every request's completion time.

The twiddle tables and cached locators stay resident in the context between
batches.  Latency is arrival -> observed completion on the host clock.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import fntrs

ENCODE = fntrs.FNTRS_OP_ENCODE
DECODE = fntrs.FNTRS_OP_DECODE


@dataclass
class Request:
    """One coding request.  `inp` is a device tensor [1, rows, lanes] (int32
    residues): k source rows for encode; for decode the full n-row codeword
    buffer (rows at `positions` are read) unless `compact` is set, in which
    case the k received rows in position order."""
    op: int
    n: int
    k: int
    lanes: int
    inp: object
    positions: np.ndarray | None = None
    compact: bool = False
    arrival: float = 0.0          # seconds after the start of the run
    rid: int = 0
    out: object = None            # device tensor, filled on completion
    t_admit: float = field(default=float("nan"))
    t_done: float = field(default=float("nan"))

    @property
    def payload_bytes(self) -> int:
        return 2 * self.k * self.lanes

    def device_bytes(self) -> int:
        """Working-set charge: input, output, locator state, four-step scratch.

        Transforms of 2^14 points or more (encode: K = 2^ceil(log2 k);
        decode: N = 2^ceil(log2 n)) run as four-step passes through a
        scratch of N rows (decode: N + M rows, M the low-product length) of
        `lanes` rounded up to 32, which the batch holds while it runs."""
        L = self.lanes
        L32 = (L + 31) // 32 * 32
        logn = (self.n - 1).bit_length()
        logk = (self.k - 1).bit_length()
        N = 1 << logn
        if self.op == ENCODE:
            b = 4 * L * (self.k + self.n)
            if max(1, logk) >= 14:
                b += 4 * N * L32
            return b
        rows_in = self.k if self.compact else self.n
        b = 4 * L * (rows_in + self.k)
        m = 1 << max(logk + 1, logn - 1) if self.k < N else N   # M = max(2K, N/2)
        b += 4 * (2 * self.k + 2 * N + 3 * m + 64 * 8)               # locator state
        if N >= 1 << 14:
            b += 4 * (N + m) * L32
        return b


@dataclass
class Stats:
    completed: int
    payload_bytes: int
    seconds: float
    latency_ms: dict
    batches: int
    mean_batch: float
    peak_bytes: int
    peak_inflight: int
    host_ms: dict = field(default_factory=dict)   # host time per phase of the loop

    @property
    def gbps(self) -> float:
        return self.payload_bytes / self.seconds / 1e9 if self.seconds > 0 else 0.0


class Server:
    """Continuous-batching request loop on one GPU (see the module docstring)."""

    def __init__(self, ctx: fntrs.Context, mem_cap_bytes: int = 32 << 30, max_inflight: int = 4,
                 max_batch: int = 256, max_batch_bytes: int | None = None):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.cap = mem_cap_bytes
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        self.max_batch_bytes = mem_cap_bytes // max_inflight if max_batch_bytes is None else max_batch_bytes
        self.streams = [torch.cuda.Stream() for _ in range(max_inflight)]
        self.host = collections.Counter()

    def _launch(self, batch, stream):
        torch = self.torch
        t0 = time.perf_counter()
        dec = [r for r in batch if r.op == DECODE]
        locs = self.ctx.locators([(r.n, r.k, r.positions) for r in dec], stream=stream) if dec else []
        t1 = time.perf_counter()
        jobs = []
        with torch.cuda.stream(stream):
            for r in batch:
                rows = r.n if r.op == ENCODE else r.k
                r.out = torch.empty((1, rows, r.lanes), dtype=torch.int32, device="cuda")
        t2 = time.perf_counter()
        li = iter(locs)
        for r in batch:
            if r.op == ENCODE:
                jobs.append(self.ctx.encode_job(r.inp, r.out, r.n))
            else:
                flags = fntrs.FNTRS_RECV_COMPACT if r.compact else fntrs.FNTRS_RECV_FULL
                jobs.append(self.ctx.decode_job(next(li), r.inp, r.out, flags))
        self.ctx.submit(jobs, stream=stream)
        ev = torch.cuda.Event()
        ev.record(stream)
        t3 = time.perf_counter()
        self.host["locators"] += t1 - t0
        self.host["outputs"] += t2 - t1
        self.host["submit"] += t3 - t2
        return ev, locs

    def autotune(self, requests, reps: int = 3) -> list:
        """Tunes the kernel configuration of every size class of `requests`
        (run as one encode batch and one decode batch on their own buffers,
        with scratch outputs) and keeps the fastest in the context, where
        every later batch of the server uses it.  Returns one dict per class."""
        torch = self.torch
        enc = [r for r in requests if r.op == ENCODE]
        dec = [r for r in requests if r.op == DECODE]
        out = []
        stream = self.streams[0]
        with torch.cuda.stream(stream):
            if enc:
                outs = [torch.empty((1, r.n, r.lanes), dtype=torch.int32, device="cuda") for r in enc]
                out += self.ctx.autotune_batch([self.ctx.encode_job(r.inp, o, r.n) for r, o in zip(enc, outs)],
                                               reps=reps, stream=stream)
            if dec:
                locs = self.ctx.locators([(r.n, r.k, r.positions) for r in dec], stream=stream)
                outs = [torch.empty((1, r.k, r.lanes), dtype=torch.int32, device="cuda") for r in dec]
                jobs = [self.ctx.decode_job(l, r.inp, o, fntrs.FNTRS_RECV_COMPACT if r.compact else fntrs.FNTRS_RECV_FULL)
                        for r, l, o in zip(dec, locs, outs)]
                out += self.ctx.autotune_batch(jobs, reps=reps, stream=stream)
                for l in locs:
                    l.release()
        stream.synchronize()
        return out

    def run(self, requests, keep=None, on_done=None) -> Stats:
        """Serves `requests` (arrival times in seconds from now) to completion.

        keep(r) -> bool decides whether a request keeps its output tensor
        after completion (default: all); on_done(r) is called on completion.
        """
        # inputs written on the caller's stream are complete before any batch reads them
        ready = self.torch.cuda.Event()
        ready.record(self.torch.cuda.current_stream())
        for st in self.streams:
            st.wait_event(ready)
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = collections.deque(reqs)
        queue = collections.deque()
        inflight = []              # (event, batch, locators, bytes)
        used = peak = 0
        peak_inflight = 0
        nb = 0
        slot = 0
        self.host.clear()
        t0 = time.perf_counter()
        while pending or queue or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # retire finished batches
            tr = time.perf_counter()
            still = []
            for ev, batch, locs, nbytes in inflight:
                if ev.query():
                    tdone = time.perf_counter() - t0
                    for r in batch:
                        r.t_done = tdone
                        if on_done:
                            on_done(r)
                        if keep is not None and not keep(r):
                            r.out = None
                    for loc in locs:
                        loc.release()
                    used -= nbytes
                else:
                    still.append((ev, batch, locs, nbytes))
            inflight = still
            self.host["retire"] += time.perf_counter() - tr
            # admit and launch what has arrived, as memory and slots allow
            if queue and len(inflight) < self.max_inflight:
                batch, nbytes = [], 0
                while queue and len(batch) < self.max_batch:
                    need = queue[0].device_bytes()
                    if need > self.cap:
                        raise ValueError(f"request {queue[0].rid} needs {need} bytes, above the cap {self.cap}")
                    if used + nbytes + need > self.cap:
                        break
                    if batch and nbytes + need > self.max_batch_bytes:
                        break
                    r = queue.popleft()
                    r.t_admit = now
                    batch.append(r)
                    nbytes += need
                if batch:
                    stream = self.streams[slot % len(self.streams)]
                    slot += 1
                    ev, locs = self._launch(batch, stream)
                    inflight.append((ev, batch, locs, nbytes))
                    used += nbytes
                    peak = max(peak, used)
                    peak_inflight = max(peak_inflight, len(inflight))
                    nb += 1
                    continue
            if not inflight and not queue and pending:
                # idle until the next arrival
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        lat = np.array([(r.t_done - r.arrival) * 1e3 for r in reqs]) if reqs else np.zeros(1)
        span = (max(r.t_done for r in reqs) - min(r.arrival for r in reqs)) if reqs else 0.0
        return Stats(completed=len(reqs), payload_bytes=sum(r.payload_bytes for r in reqs), seconds=span,
                     latency_ms={"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                 "mean": float(lat.mean())},
                     batches=nb, mean_batch=len(reqs) / max(1, nb), peak_bytes=peak, peak_inflight=peak_inflight,
                     host_ms={k: round(v * 1e3, 3) for k, v in self.host.items()})


def poisson_arrivals(rate_per_s: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
