"""Continuous-batching request loop for sampled TR-ALS decompositions.

A request names a tensor-ring problem (order, mode sizes, ranks, samples J per
core update, number of sweeps, seed).  Its data is a generated source: the
tensor TR(G*) + noise of the request's own true cores, formed fiber by fiber
on the GPU, so that no request ever materialises a dense tensor.

The server holds a fixed number of slots, each with its own HIP stream.  A
waiting request is admitted, in arrival order, as soon as a slot is free and
its device footprint (handle workspace plus true cores) fits in what the
running requests leave of the memory budget.  An admitted request's sweeps
are enqueued on its slot's stream without waiting, so the updates of several
decompositions run on the device at the same time; a request that arrives
while others run is admitted as soon as one of them finishes.  Cores, sampling
tables and sketch of a running request stay resident in its workspace from
admission to completion.  A request whose footprint exceeds the whole budget
is refused at once; a request whose solve fails is reported with its error
and the others go on.

Results do not depend on the mix: every kernel of a request runs on its own
workspace with a fixed launch configuration and fixed-order reductions, and
its random draws are keyed by its own seed and id.

``Scheduler`` holds the host-side logic (queue, slots, memory) and is driven
by an engine object with ``footprint``, ``start``, ``poll`` and ``finish``;
``TralsEngine`` is the GPU engine.  ``run`` replays a stream of requests with
their arrival times against the wall clock.
"""
from __future__ import annotations

import collections
import ctypes as C
import dataclasses
import time

import numpy as np

from . import _lib
from . import TRALS

__all__ = ["Result", "Scheduler", "TralsEngine", "run", "summarize"]


@dataclasses.dataclass
class Result:
    id: int
    arrival: float
    admitted: float | None
    done: float
    rows: int = 0          # sampled rows the request's updates processed (J per update)
    fit: float | None = None
    cores: list | None = None
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """Admission by free slot and memory footprint, in arrival order.

    engine.footprint(req) -> bytes; engine.start(req, slot) -> job;
    engine.poll(job) -> bool (True once finished); engine.finish(job) -> dict
    with optional "fit" and "cores"; any exception from start/poll/finish
    fails that request alone.
    """

    def __init__(self, engine, slots: int, mem_budget: int):
        if slots < 1 or mem_budget <= 0:
            raise ValueError("need at least one slot and a positive memory budget")
        self.engine = engine
        self.slots = int(slots)
        self.mem_budget = int(mem_budget)
        self.queue = collections.deque()
        self.free = list(range(self.slots - 1, -1, -1))  # pop() gives the lowest slot first
        self.running = {}  # slot -> (req, job, footprint, admitted)
        self.mem_in_use = 0
        self.peak_running = 0
        self.peak_mem = 0

    def submit(self, req, now: float):
        """Queue a request; refused at once (returned as a Result) if it can never fit."""
        fp = int(self.engine.footprint(req))
        if fp > self.mem_budget:
            return Result(req["id"], req["arrival"], None, now,
                          error=f"footprint {fp} B exceeds the memory budget {self.mem_budget} B")
        self.queue.append((req, fp))
        return None

    def busy(self) -> bool:
        return bool(self.queue or self.running)

    def tick(self, now_fn) -> list:
        """Collect finished requests, then admit waiting ones; now_fn() gives the time."""
        out = []
        for slot in sorted(self.running):
            req, job, fp, adm = self.running[slot]
            try:
                finished = self.engine.poll(job)
                info = self.engine.finish(job) if finished else None
                err = None
            except Exception as e:  # a failed request is reported; the others continue
                finished, info, err = True, None, f"{type(e).__name__}: {e}"
                self._abandon(job)
            if not finished:
                continue
            t = now_fn()
            del self.running[slot]
            self.free.append(slot)
            self.free.sort(reverse=True)
            self.mem_in_use -= fp
            info = info or {}
            out.append(Result(req["id"], req["arrival"], adm, t, rows=self._rows(req),
                              fit=info.get("fit"), cores=info.get("cores"), error=err))
        while self.queue and self.free and self.mem_in_use + self.queue[0][1] <= self.mem_budget:
            req, fp = self.queue.popleft()
            slot = self.free.pop()
            adm = now_fn()
            try:
                job = self.engine.start(req, slot)
            except Exception as e:
                self.free.append(slot)
                self.free.sort(reverse=True)
                out.append(Result(req["id"], req["arrival"], adm, now_fn(), error=f"{type(e).__name__}: {e}"))
                continue
            self.running[slot] = (req, job, fp, adm)
            self.mem_in_use += fp
            self.peak_running = max(self.peak_running, len(self.running))
            self.peak_mem = max(self.peak_mem, self.mem_in_use)
        return out

    def _abandon(self, job):
        close = getattr(self.engine, "abandon", None)
        if close is not None:
            try:
                close(job)
            except Exception:
                pass

    @staticmethod
    def _rows(req) -> int:
        return int(req["samples"]) * len(req["dims"]) * int(req["sweeps"])


def run(engine, requests, slots: int, mem_budget: int, clock=time.perf_counter, wait=None):
    """Replay requests (dicts with "arrival" in seconds from the start) against the clock.

    Returns (results sorted by id, wall seconds, scheduler).  wait(seconds) is
    called when nothing is running and the next arrival is in the future (a
    fake clock's advance in tests); by default the loop spins.
    """
    sched = Scheduler(engine, slots, mem_budget)
    reqs = sorted(requests, key=lambda r: (r["arrival"], r["id"]))
    t0 = clock()
    now = lambda: clock() - t0  # noqa: E731
    results, i = [], 0
    while i < len(reqs) or sched.busy():
        t = now()
        while i < len(reqs) and reqs[i]["arrival"] <= t:
            refused = sched.submit(reqs[i], t)
            if refused is not None:
                results.append(refused)
            i += 1
        results.extend(sched.tick(now))
        if not sched.busy() and i < len(reqs) and wait is not None:
            wait(reqs[i]["arrival"] - now())
    wall = now()
    results.sort(key=lambda r: r.id)
    return results, wall, sched


def summarize(results, wall: float) -> dict:
    """Throughput and latency percentiles of a finished run."""
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    rows = sum(r.rows for r in ok)
    return dict(
        requests=len(results), completed=len(ok), failed=len(results) - len(ok),
        wall_s=wall, req_per_s=len(ok) / wall if wall > 0 else 0.0,
        rows_per_s=rows / wall if wall > 0 else 0.0,
        p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
        mean_ms=float(lat.mean() * 1e3),
        fit_median=float(np.median([r.fit for r in ok if r.fit is not None])) if ok else None,
        errors=[(r.id, r.error) for r in results if r.error is not None][:8],
    )


class TralsEngine:
    """GPU engine: one generated-source TRALS handle per running request.

    Request fields: id, dims, ranks, samples, sweeps, seed, and optionally
    noise_rel (default the engine's) and true_cores (the data the request
    carries: host arrays of shapes (R[n-1], I[n], R[n])); without them the
    engine calls ``true_cores(req)``.  The noise is keyed (seed, id), the
    initial cores and the sampler (seed, stream id = id).  A request's work
    is enqueued without waiting (handle creation, sweeps and the error
    against the clean ring); completion is polled.
    """

    def __init__(self, true_cores, precision="f32", noise_rel=0.01, device=None, keep_cores=True,
                 slot_bytes=64 << 20):
        import torch
        self.torch = torch
        self.lib = _lib.load()
        self.true_cores = true_cores
        self.precision = precision
        self.noise_rel = float(noise_rel)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.keep_cores = keep_cores
        self.slot_bytes = int(slot_bytes)  # workspace arena per slot (no allocation per request)
        self.streams = {}
        self.arenas = {}

    def warmup(self, slots, orders=(3, 4, 5), ranks=range(3, 13), samples=2048, dim=48):
        """Run one small request per order and (uniform) rank through every slot's stream, so that
        every kernel instance the request mix can reach (contraction row tiles, draw rank
        buckets, factorisation sizes) is loaded before the first real request.

        Then everything alive (the engine, torch, the library) is moved out of the cyclic
        garbage collector's reach: its first full pass over those ~170k long-lived objects
        otherwise stalls the request loop for ~40 ms a few hundred requests in."""
        import gc

        import numpy as np
        reqs, rid = [], 0
        for N in orders:
            for R in ranks:
                dims, rk = [dim] * N, [int(R)] * N
                rng = np.random.default_rng([7, N, int(R)])
                cores = [rng.standard_normal((rk[(n - 1) % N], dims[n], rk[n])) for n in range(N)]
                reqs.append(dict(id=10 ** 9 + rid, arrival=0.0, dims=dims, ranks=rk, samples=samples, sweeps=1,
                                 seed=0, true_cores=cores))
                rid += 1
        run(self, reqs, slots=slots, mem_budget=1 << 40)
        gc.collect()
        gc.freeze()

    def _stream(self, slot):
        s = self.streams.get(slot)
        if s is None:
            s = self.torch.cuda.Stream(device=self.device)  # default priority
            self.streams[slot] = s
            with self.torch.cuda.stream(s):
                self.arenas[slot] = self.torch.empty(self.slot_bytes, dtype=self.torch.uint8, device=self.device)
        return s

    def footprint(self, req) -> int:
        desc, keep = _lib.make_desc(req["dims"], req["ranks"], req["samples"], req["seed"], req["id"],
                                    {"f64": _lib.TRALS_F64, "f32": _lib.TRALS_F32, "bf16": _lib.TRALS_BF16}
                                    [self.precision])
        src, keep2 = _lib.make_source(None, _lib.TRALS_F64, req["ranks"], req.get("noise_rel", self.noise_rel),
                                      req["seed"], req["id"])
        out = C.c_size_t(0)
        _lib.check(self.lib.trals_workspace_bytes_generated(C.byref(desc), C.byref(src), C.byref(out)),
                   "trals_workspace_bytes_generated")
        N = len(req["dims"])
        core_bytes = 8 * sum(req["ranks"][(n - 1) % N] * req["dims"][n] * req["ranks"][n] for n in range(N))
        return int(out.value) + core_bytes

    def start(self, req, slot):
        stream = self._stream(slot)
        cores = req.get("true_cores")
        if cores is None:
            cores = self.true_cores(req)
        with self.torch.cuda.stream(stream):
            h = TRALS.generated(cores, req["ranks"], req["samples"],
                                noise_rel=req.get("noise_rel", self.noise_rel), noise_seed=req["seed"],
                                noise_stream=req["id"], seed=req["seed"], stream_id=req["id"],
                                precision=self.precision, stream=stream, device=self.device,
                                workspace=self.arenas[slot])
            h.sweep_async(req["sweeps"], fit=True)
        return h

    def poll(self, job) -> bool:
        return job.query()

    def finish(self, job) -> dict:
        # the fit came back with the completion (no synchronisation); the cores need a copy
        cores = None
        if self.keep_cores:
            with self.torch.cuda.stream(job.stream):
                cores = [c.cpu().numpy() for c in job.get_cores()]
        fit = job.async_fit
        job.close()
        return dict(fit=fit, cores=cores)

    def abandon(self, job):
        job.close()
