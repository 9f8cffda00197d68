"""Continuous-batching request loop over the C ABI.

Requests (an integrator batch of one process: momenta and a precision) arrive
at arbitrary times.  The server keeps every process handle, and with it the
uploaded colour matrix, resident; admits a waiting request as soon as its
device memory fits under an HBM budget and a stream slot is free; runs
admitted requests concurrently on a pool of HIP streams (default priority),
so work of requests that arrive while others run overlaps on the device; and
completes each request when its own events say so.  Latency is measured from
submission (arrival) to completion.

All arithmetic is done by libheget.so; this module only moves buffers,
queues launches and watches events.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Optional

import numpy as np

from .heget import Process


@dataclasses.dataclass
class Request:
    rid: int
    spec: str
    momenta: np.ndarray            # float64 [n][n_ext][4], host
    precision: str = "mixed"
    t_submit: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    result: Optional[np.ndarray] = None
    error: Optional[str] = None
    done: threading.Event = dataclasses.field(default_factory=threading.Event)

    @property
    def n(self) -> int:
        return int(self.momenta.shape[0])

    @property
    def device_bytes(self) -> int:
        return int(self.momenta.nbytes + 8 * self.n)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


class Server:
    """Admission by HBM budget, a pool of streams, completion by events."""

    def __init__(self, specs, precisions=("mixed",), hbm_budget_bytes: int = 8 << 30,
                 n_streams: int = 4, device: str = "cuda:0", alpha_s: float = 0.118):
        import torch
        self.torch = torch
        self.alpha_s = alpha_s
        self.device = torch.device(device)
        self.budget = int(hbm_budget_bytes)
        self.in_use = 0
        self.procs = {(s, p): Process(s, p) for s in specs for p in precisions}
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.free_streams = list(range(n_streams))
        self.waiting = collections.deque()
        self.running = []            # (request, stream index, done event, device buffers)
        self.completed = []
        self.lock = threading.Lock()
        self._next_id = 0

    # -------------------------------------------------------------- client side
    def submit(self, spec: str, momenta: np.ndarray, precision: str = "mixed") -> Request:
        if (spec, precision) not in self.procs:
            raise KeyError(f"process {spec!r} / {precision} not resident in this server")
        with self.lock:
            req = Request(self._next_id, spec, np.ascontiguousarray(momenta, dtype=np.float64), precision)
            self._next_id += 1
            req.t_submit = time.perf_counter()
            if req.device_bytes > self.budget:
                req.error = "request larger than the HBM budget"
                req.t_done = req.t_submit
                req.done.set()
                self.completed.append(req)
                return req
            self.waiting.append(req)
        return req

    # -------------------------------------------------------------- server side
    def _admit(self):
        torch = self.torch
        while self.waiting and self.free_streams and self.in_use + self.waiting[0].device_bytes <= self.budget:
            req = self.waiting.popleft()
            si = self.free_streams.pop()
            st = self.streams[si]
            self.in_use += req.device_bytes
            req.t_start = time.perf_counter()
            try:
                with torch.cuda.stream(st):
                    mom = torch.from_numpy(req.momenta).pin_memory().to(self.device, non_blocking=True)
                    out = torch.empty(req.n, dtype=torch.float64, device=self.device)
                    self.procs[(req.spec, req.precision)].matrix_elements(mom, self.alpha_s, out=out, stream=st)
                    host = torch.empty(req.n, dtype=torch.float64, pin_memory=True)
                    host.copy_(out, non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(st)
            except Exception as exc:       # this request fails alone: give its slot and budget back
                req.error = f"{type(exc).__name__}: {exc}"
                req.t_done = time.perf_counter()
                self.in_use -= req.device_bytes
                self.free_streams.append(si)
                self.completed.append(req)
                req.done.set()
                continue
            self.running.append((req, si, ev, (mom, out, host)))

    def _reap(self):
        still = []
        for req, si, ev, bufs in self.running:
            if ev.query():
                req.result = bufs[2].numpy().copy()
                req.t_done = time.perf_counter()
                self.in_use -= req.device_bytes
                self.free_streams.append(si)
                self.completed.append(req)
                req.done.set()
            else:
                still.append((req, si, ev, bufs))
        self.running = still

    def step(self):
        """One scheduling pass: reap finished requests, admit waiting ones."""
        with self.lock:
            self._reap()
            self._admit()

    def idle(self) -> bool:
        with self.lock:
            return not self.waiting and not self.running

    def drain(self, poll_s: float = 1e-4):
        while not self.idle():
            self.step()
            time.sleep(poll_s)


def run_poisson(server: Server, workload, rate_hz: float, n_requests: int, seed: int = 11,
                precision: str = "mixed"):
    """Submit n_requests at Poisson arrival times while the scheduler runs.

    workload: callable rng -> (spec, momenta).  Returns the completed requests.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    items = [workload(rng) for _ in range(n_requests)]
    t0 = time.perf_counter()
    arrival = t0 + np.cumsum(gaps)
    reqs = []
    i = 0
    while i < n_requests or not server.idle():
        now = time.perf_counter()
        while i < n_requests and arrival[i] <= now:
            spec, mom = items[i]
            reqs.append(server.submit(spec, mom, precision))
            i += 1
        server.step()
        if i < n_requests:
            time.sleep(max(0.0, min(1e-4, arrival[i] - time.perf_counter())))
    return reqs, time.perf_counter() - t0


def latency_summary(reqs):
    lat = np.array([r.latency for r in reqs if r.error is None])
    ev = sum(r.n for r in reqs if r.error is None)
    span = max(r.t_done for r in reqs) - min(r.t_submit for r in reqs)
    return {"requests": len(reqs), "events": int(ev),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "events_per_s": ev / span if span > 0 else 0.0}
