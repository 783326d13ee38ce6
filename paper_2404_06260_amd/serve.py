"""Serving driver: replays a stream of local-reduction requests against the library's
continuous-batching engine in real time and reports latency percentiles beside throughput.

Each request asks for the local basis of one subdomain (rank, precision).  Requests are
submitted with `mor_submit` when their arrival time has passed; the loop then advances the
engine by one tick (`mor_step`: admission under the HBM budget, one chunk of block-CG iterations
over every admitted system, and the dense stage of the systems that finished) and collects
completions with `mor_poll`.  Requests that arrive while others run join the next chunk, so
their work overlaps on the device.  Latency of a request = the time its completion is seen
minus its arrival time (queueing, admission and service included).

All device work runs in the HIP library; this module only schedules calls and keeps clocks.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import mor as _mor


@dataclass
class Stream:
    """A request stream: arrival time (s), subdomain, rank and precision name per request."""
    arrivals: np.ndarray
    sds: np.ndarray
    ranks: np.ndarray
    precisions: list

    def __len__(self):
        return int(self.arrivals.size)


@dataclass
class StreamResult:
    latency: np.ndarray            # seconds per request (arrival -> completion seen)
    status: np.ndarray             # library result code per request
    finish: np.ndarray             # completion time (s from stream start)
    makespan: float                # last completion - first arrival (s)
    steps: int                     # engine ticks taken
    peak_bytes: int                # device bytes held by admitted requests, peak
    budget_bytes: int
    max_live: int                  # most requests admitted at once
    extra: dict = field(default_factory=dict)

    @property
    def throughput(self) -> float:
        return float(len(self.latency) / self.makespan) if self.makespan > 0 else float("inf")

    def percentiles(self, qs=(50, 99)) -> dict:
        ok = self.latency[np.isfinite(self.latency)]
        return {f"p{q}": float(np.percentile(ok, q)) if ok.size else float("nan") for q in qs}


def make_stream(problem, n_requests: int, rate: float, seed_arrivals: int = 7, seed_order: int = 11,
                precisions=("fp32_refine",), precision_p=None, seed_precision: int = 9) -> Stream:
    """A Poisson stream over the problem's subdomains: arrivals at `rate` per second (rate =
    inf: all at t = 0), subdomains in a seeded random order (cycling when n_requests exceeds
    the number of subdomains), each with the problem's rank for that subdomain, and a
    precision drawn from `precisions` with probabilities `precision_p`."""
    from workloads import poisson_arrivals
    n_sub = problem.subdomains.n_sub
    if np.isinf(rate):
        arr = np.zeros(n_requests)
    else:
        arr = poisson_arrivals(n_requests, rate, seed=seed_arrivals)
        arr = arr - arr[0]
    rng = np.random.default_rng(seed_order)
    order = np.concatenate([rng.permutation(n_sub) for _ in range((n_requests + n_sub - 1) // n_sub)])[:n_requests]
    ranks = np.asarray(problem.ranks)[order] if problem.ranks is not None else np.full(n_requests, problem.rank)
    prng = np.random.default_rng(seed_precision)
    pr = [precisions[i] for i in prng.choice(len(precisions), size=n_requests, p=precision_p)]
    return Stream(arrivals=arr, sds=order.astype(np.int32), ranks=ranks.astype(np.int32), precisions=pr)


def run_stream(ctx, stream: Stream, clock=time.perf_counter, sleep=time.sleep, api=None,
               max_steps: int = 10_000_000, on_done=None) -> StreamResult:
    """Replay `stream` against an engine context in real time (see the module docstring).
    `api` (default: the library binding) must provide mor_submit, mor_step, mor_poll and
    mor_engine_stats with the binding's signatures; `on_done(j, n_done, t)` is called for each
    completion."""
    api = api or _mor
    n = len(stream)
    lat = np.full(n, np.nan)
    fin = np.full(n, np.nan)
    status = np.zeros(n, dtype=np.int64)
    open_tickets = {}
    nxt = 0
    done = 0
    steps = 0
    max_live = 0
    t0 = clock()
    while done < n:
        now = clock() - t0
        while nxt < n and stream.arrivals[nxt] <= now:
            tk = api.mor_submit(ctx, int(stream.sds[nxt]), int(stream.ranks[nxt]), 0.0,
                                _mor.PRECISIONS[stream.precisions[nxt]])
            open_tickets[tk] = nxt
            nxt += 1
        if not open_tickets:
            if nxt < n:
                sleep(max(0.0, float(stream.arrivals[nxt]) - (clock() - t0)))
            continue
        api.mor_step(ctx)
        steps += 1
        if steps > max_steps:
            raise RuntimeError("serving loop exceeded its step limit")
        st = api.mor_engine_stats(ctx)
        max_live = max(max_live, int(st["live"]))
        now = clock() - t0
        for tk in list(open_tickets):
            d, s = api.mor_poll(ctx, tk)
            if d:
                j = open_tickets.pop(tk)
                lat[j] = now - float(stream.arrivals[j])
                fin[j] = now
                status[j] = s
                done += 1
                if on_done is not None:
                    on_done(j, done, now)
    st = api.mor_engine_stats(ctx)
    makespan = float(np.nanmax(fin) - stream.arrivals[0]) if n else 0.0
    return StreamResult(latency=lat, status=status, finish=fin, makespan=makespan, steps=steps,
                        peak_bytes=int(st["peak_bytes"]), budget_bytes=int(st["budget"]), max_live=max_live)


def saturation_throughput(ctx, problem, n_requests: int, **kw) -> float:
    """Requests/s when the whole stream is queued at t = 0 (the engine's capacity)."""
    s = make_stream(problem, n_requests, float("inf"), **kw)
    return run_stream(ctx, s).throughput
