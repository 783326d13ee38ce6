"""CPU tests of the serving driver's host logic (request replay, latency accounting,
percentiles) against a scripted engine: no device involved."""
import numpy as np
import pytest

from paper_2404_06260_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeEngine:
    """Admits up to `slots` requests; each needs `work[sd]` ticks once admitted; a tick costs
    `dt` seconds of the fake clock."""

    def __init__(self, clock, work, slots=2, dt=0.1, budget=100):
        self.clock, self.work, self.slots, self.dt, self.budget = clock, work, slots, dt, budget
        self.pending, self.live, self.done = [], {}, {}
        self.next, self.peak = 1, 0

    def mor_submit(self, ctx, sd, rank, tol, prec):
        tk = self.next
        self.next += 1
        self.pending.append((tk, sd))
        return tk

    def mor_step(self, ctx):
        while self.pending and len(self.live) < self.slots:
            tk, sd = self.pending.pop(0)
            self.live[tk] = self.work[sd]
        self.peak = max(self.peak, 10 * len(self.live))
        self.clock.t += self.dt
        for tk in list(self.live):
            self.live[tk] -= 1
            if self.live[tk] <= 0:
                del self.live[tk]
                self.done[tk] = 0

    def mor_poll(self, ctx, tk):
        return (1, self.done[tk]) if tk in self.done else (0, 0)

    def mor_engine_stats(self, ctx):
        return dict(live=len(self.live), pending=len(self.pending), live_bytes=10 * len(self.live),
                    peak_bytes=self.peak, budget=self.budget)


def _stream(arr, sds):
    n = len(arr)
    return serve.Stream(arrivals=np.asarray(arr, float), sds=np.asarray(sds, np.int32),
                        ranks=np.full(n, 4, np.int32), precisions=["fp32_refine"] * n)


def test_latency_is_completion_minus_arrival():
    clk = FakeClock()
    eng = FakeEngine(clk, work={0: 3, 1: 1, 2: 2}, slots=4, dt=0.1)
    res = serve.run_stream(None, _stream([0.0, 0.05, 1.0], [0, 1, 2]), clock=clk, sleep=clk.sleep, api=eng)
    # request 0: ticks at 0.1, 0.2, 0.3 -> done at 0.3; request 1 arrives at 0.05, is submitted
    # after the first tick (0.1) and finishes at 0.2; request 2 waits for its arrival at 1.0.
    np.testing.assert_allclose(res.latency, [0.3, 0.15, 0.2], atol=1e-12)
    np.testing.assert_allclose(res.finish, [0.3, 0.2, 1.2], atol=1e-12)
    assert res.makespan == pytest.approx(1.2)
    assert res.steps == 5
    assert (res.status == 0).all()


def test_admission_limit_queues_requests():
    clk = FakeClock()
    eng = FakeEngine(clk, work={i: 2 for i in range(6)}, slots=2, dt=1.0)
    res = serve.run_stream(None, _stream([0.0] * 6, range(6)), clock=clk, sleep=clk.sleep, api=eng)
    # two at a time, two ticks each: pairs finish at t = 2, 4, 6
    np.testing.assert_allclose(np.sort(res.latency), [2, 2, 4, 4, 6, 6])
    assert res.max_live == 2
    assert res.throughput == pytest.approx(1.0)
    p = res.percentiles((50, 99))
    assert p["p50"] == pytest.approx(4.0) and 5.9 < p["p99"] <= 6.0


def test_make_stream_is_seeded_and_covers_subdomains():
    class P:
        class subdomains:
            n_sub = 5
        ranks = np.array([8, 9, 10, 11, 12])
        rank = 12
    a = serve.make_stream(P, 12, 3.0, precisions=("fp32_refine", "bf16_split"), precision_p=(0.5, 0.5))
    b = serve.make_stream(P, 12, 3.0, precisions=("fp32_refine", "bf16_split"), precision_p=(0.5, 0.5))
    np.testing.assert_array_equal(a.arrivals, b.arrivals)
    np.testing.assert_array_equal(a.sds, b.sds)
    assert a.precisions == b.precisions
    assert a.arrivals[0] == 0.0 and np.all(np.diff(a.arrivals) >= 0)
    assert sorted(a.sds[:5]) == list(range(5)) and sorted(a.sds[5:10]) == list(range(5))
    np.testing.assert_array_equal(a.ranks, P.ranks[a.sds])
    # the arrival gaps of a rate-3 stream average about 1/3 s
    long = serve.make_stream(P, 4000, 3.0)
    assert abs(np.mean(np.diff(long.arrivals)) - 1 / 3) < 0.02
    inf = serve.make_stream(P, 7, float("inf"))
    assert (inf.arrivals == 0).all()
