"""The serving policy of paper_1403_6854_amd.serve on a simulated device:
admission by memory budget, first come first served, continuous batching,
one completion per request, latency accounting."""
import numpy as np
import pytest

from paper_1403_6854_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeBackend:
    """Streams that finish a batch `cost(batch)` seconds after its launch."""

    def __init__(self, clock, n_streams=2, cost=lambda b: 0.01 * len(b)):
        self.clock = clock
        self.free = list(range(n_streams))
        self.cost = cost
        self.active_bytes = 0
        self.max_active = 0
        self.launches = []

    def slots(self):
        return len(self.free)

    def launch(self, reqs):
        si = self.free.pop()
        nb = sum(r.nbytes for r in reqs)
        self.active_bytes += nb
        self.max_active = max(self.max_active, self.active_bytes)
        self.launches.append((self.clock(), [r.rid for r in reqs]))
        return (si, self.clock() + self.cost(reqs), reqs, nb)

    def done(self, h):
        return self.clock() >= h[1]

    def retire(self, h):
        self.free.append(h[0])
        self.active_bytes -= h[3]
        return [{"rid": r.rid} for r in h[2]]


def _reqs(n, rate=100.0, nbytes=10, seed=0):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    sizes = nbytes if np.isscalar(nbytes) else nbytes
    out = []
    for i in range(n):
        b = int(sizes if np.isscalar(sizes) else sizes[i])
        out.append(serve.ServeRequest(i, float(t[i]), "ihs", b, make=None))
    return out


def _run(reqs, budget=10**9, max_batch=64, n_streams=2, cost=lambda b: 0.01 * len(b),
         work_ratio=0.0):
    clk = FakeClock()
    be = FakeBackend(clk, n_streams, cost)
    srv = serve.Server(be, budget, max_batch=max_batch, clock=clk, sleep=clk.sleep, poll_s=1e-4,
                       work_ratio=work_ratio)
    done = srv.run(reqs)
    return done, be, srv


def test_every_request_completes_once_with_its_own_output():
    reqs = _reqs(300)
    done, be, srv = _run(reqs)
    assert sorted(c.rid for c in done) == list(range(300))
    for c in done:
        assert c.out == {"rid": c.rid}
        assert c.arrival_s <= c.admit_s <= c.finish_s
    assert sum(srv.batch_sizes) == 300


def test_budget_is_never_exceeded():
    rng = np.random.default_rng(4)
    sizes = rng.integers(1, 40, size=200)
    reqs = _reqs(200, rate=1000.0, nbytes=sizes)
    done, be, srv = _run(reqs, budget=100, cost=lambda b: 0.005 * len(b))
    assert len(done) == 200
    assert be.max_active <= 100
    assert srv.peak_bytes <= 100


def test_first_come_first_served():
    reqs = _reqs(150, rate=500.0)
    done, be, srv = _run(reqs, budget=35, max_batch=4)
    order = [rid for _, rids in be.launches for rid in rids]
    assert order == sorted(order)
    adm = {c.rid: c.admit_s for c in done}
    assert all(adm[i] <= adm[i + 1] for i in range(149))


def test_requests_batch_up_under_load_and_not_when_idle():
    slow = _reqs(200, rate=2000.0)
    _, _, srv = _run(slow, cost=lambda b: 0.02 + 0.001 * len(b))
    assert max(srv.batch_sizes) > 1
    idle = _reqs(50, rate=1.0)
    _, _, srv2 = _run(idle, cost=lambda b: 0.001)
    assert max(srv2.batch_sizes) == 1


def test_batches_overlap_on_several_streams():
    reqs = _reqs(100, rate=2000.0)
    _, be, _ = _run(reqs, n_streams=3, max_batch=2, cost=lambda b: 0.05)
    starts = [t for t, _ in be.launches]
    # with three streams, the second and third batch start before the first ends
    assert starts[2] < starts[0] + 0.05


def test_oversized_request_runs_alone():
    reqs = _reqs(10, rate=1000.0, nbytes=[5, 5, 500, 5, 5, 5, 5, 5, 5, 5])
    done, be, srv = _run(reqs, budget=50)
    assert len(done) == 10
    big = [rids for _, rids in be.launches if 2 in rids]
    assert big == [[2]]


def test_summary_and_back_to_back():
    reqs = _reqs(40, rate=50.0)
    clk = FakeClock()

    def run_one(r):
        clk.t += 0.03
        return {"rid": r.rid}

    seq = serve.run_back_to_back(reqs, run_one, clock=clk, sleep=clk.sleep)
    assert [c.rid for c in seq] == list(range(40))
    assert all(c.finish_s - c.admit_s == pytest.approx(0.03) for c in seq)
    s = serve.summarize(seq)
    assert s["requests"] == 40 and s["p99_ms"] >= s["p50_ms"] >= 30.0 - 1e-6


def test_request_bytes_grow_with_the_region():
    a = serve.request_bytes("ihs", 100, 0, 1000)
    b = serve.request_bytes("ihs", 5000, 0, 1000)
    c = serve.request_bytes("xpehh", 5000, 5000, 1000)
    d = serve.request_bytes("xpehh", 5000, 5000, 200000)
    assert a < b < c < d
    assert d > 5000 * 2 * 200000   # the 0/1 matrices alone


def test_work_ratio_keeps_dissimilar_requests_apart_in_arrival_order():
    rng = np.random.default_rng(5)
    reqs = _reqs(300, rate=2000.0)
    for r in reqs:
        r.work = float(rng.choice([1.0, 3.0, 100.0, 400.0]))
    done, be, srv = _run(reqs, n_streams=4, work_ratio=4.0)
    assert sorted(c.rid for c in done) == list(range(300))
    work = {r.rid: r.work for r in reqs}
    order = [rid for _, rids in be.launches for rid in rids]
    assert order == list(range(300))              # first come, first served
    for _, rids in be.launches:
        w = [work[i] for i in rids]
        assert max(w) <= 4.0 * w[0] and min(w) * 4.0 >= w[0]
    assert max(len(rids) for _, rids in be.launches) > 1   # similar ones still batch
    # without the ratio the same stream mixes them
    _, be0, _ = _run(reqs, n_streams=4)
    assert any(max(work[i] for i in rids) > 4.0 * min(work[i] for i in rids)
               for _, rids in be0.launches)
    with pytest.raises(ValueError):
        serve.Server(be, 10, work_ratio=0.5)


class FlakyBackend(FakeBackend):
    """A FakeBackend whose launch raises the first time a batch holds a
    request of `bad_launch`, and whose completion check raises for every
    batch holding a request of `poison`."""

    def __init__(self, clock, bad_launch=(), poison=(), **kw):
        super().__init__(clock, **kw)
        self.bad_launch = set(bad_launch)
        self.poison = set(poison)
        self.released = 0

    def launch(self, reqs):
        bad = [r.rid for r in reqs if r.rid in self.bad_launch]
        if bad:
            self.bad_launch -= set(bad)
            raise RuntimeError("launch failed")
        return super().launch(reqs)

    def done(self, h):
        if any(r.rid in self.poison for r in h[2]):
            raise RuntimeError("device error")
        return super().done(h)

    def release(self, h):
        self.released += 1
        self.free.append(h[0])
        self.active_bytes -= h[3]


def _run_flaky(reqs, **kw):
    clk = FakeClock()
    be = FlakyBackend(clk, n_streams=2, **kw)
    srv = serve.Server(be, 10**9, max_batch=8, clock=clk, sleep=clk.sleep, poll_s=1e-4)
    return srv.run(reqs), be, srv


def test_a_failed_launch_is_retried_and_every_request_completes():
    reqs = _reqs(120, rate=2000.0)
    done, be, srv = _run_flaky(reqs, bad_launch={7, 50})
    assert sorted(c.rid for c in done) == list(range(120))
    assert all(c.error is None and c.out == {"rid": c.rid} for c in done)
    assert 1 <= srv.failures <= 2        # 7 and 50 in one batch, or in two
    # the requests of a failed batch were retried alone
    alone = [rids for _, rids in be.launches if 7 in rids or 50 in rids]
    assert all(len(r) == 1 for r in alone)


def test_a_request_that_keeps_failing_ends_with_an_error_and_the_rest_complete():
    reqs = _reqs(80, rate=2000.0)
    done, be, srv = _run_flaky(reqs, poison={33})
    assert sorted(c.rid for c in done) == list(range(80))
    bad = [c for c in done if c.rid == 33]
    assert len(bad) == 1 and bad[0].error and bad[0].out is None
    assert all(c.error is None and c.out == {"rid": c.rid} for c in done if c.rid != 33)
    # streams and memory of dropped batches were given back
    assert be.released == srv.failures and be.active_bytes == 0 and len(be.free) == 2


class PartialBackend(FakeBackend):
    """Members of a batch complete at their own times (small requests first)."""

    def launch(self, reqs):
        h = super().launch(reqs)
        t = self.clock()
        return h + ([t + 0.001 * (1 + (r.rid % 2) * 20) for r in reqs], set())

    def partial(self, h):
        got = []
        for i, t in enumerate(h[4]):
            if i not in h[5] and self.clock() >= t:
                h[5].add(i)
                got.append((i, {"rid": h[2][i].rid}))
        return got

    def done(self, h):
        return self.clock() >= max(h[4])


def test_requests_complete_when_their_own_results_are_ready():
    clk = FakeClock()
    be = PartialBackend(clk, n_streams=1)
    srv = serve.Server(be, 10**9, max_batch=16, clock=clk, sleep=clk.sleep, poll_s=1e-4)
    reqs = _reqs(40, rate=5000.0)
    done = srv.run(reqs)
    assert sorted(c.rid for c in done) == list(range(40))
    by = {c.rid: c for c in done}
    for c in done:
        assert c.out == {"rid": c.rid}
    # in each batch the even requests (1 ms) finish before the odd ones (21 ms)
    for b in {c.batch for c in done}:
        ev = [by[r].finish_s for r in by if by[r].batch == b and r % 2 == 0]
        od = [by[r].finish_s for r in by if by[r].batch == b and r % 2 == 1]
        if ev and od:
            assert max(ev) < min(od)
