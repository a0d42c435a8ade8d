"""Admission and continuous batching of the request loop, on the CPU.

The backend is a stand-in: its set-up sleeps, and every tick advances each
request in the batch by the tick's time until the request's work (set by its
size) is done, so the scheduling rules can be checked without a GPU: slots
and the memory budget are never exceeded, requests are admitted in arrival
order and no earlier than their arrival, and a request that arrives while a
long one is in flight joins the batch and finishes without waiting for the
long one.  A backend that releases finished requests later (as the GPU
backend releases its contexts on a background thread) has every release
done when run() returns.
"""
import time

import pytest

from paper_2606_08883_amd.serving import Request, Server, make_requests, summary


class FakeBackend:
    """Set-up sleeps setup_s; a request needs unit * n / 128 seconds of
    ticks; a tick takes tick_s and advances every request in the batch."""

    def __init__(self, unit=0.02, tick_s=0.002, setup_s=0.002):
        self.unit, self.tick_s, self.setup_s = unit, tick_s, setup_s
        self.active = []

    def setup(self, req):
        time.sleep(self.setup_s)
        return {"req": req, "left": self.unit * req.n / 128, "ticks": 0}

    def add(self, h):
        self.active.append(h)

    def tick(self):
        time.sleep(self.tick_s)
        for h in self.active:
            h["left"] -= self.tick_s
            h["ticks"] += 1
        return len(self.active)

    def poll(self, h):
        if h["left"] > 1e-12:
            return None
        self.active.remove(h)
        r = h["req"]
        return dict(iterations=3 * r.nrhs, converged=True, final_relres=1e-9,
                    setup_s=self.setup_s, solve_s=h["ticks"] * self.tick_s, p=None)


def fp(req):
    return req.n * req.n * 100


def _check_log(server, results, max_active, budget):
    live, used = set(), 0
    by_id = {r.rid: r for r in results}
    for t, kind, rid in sorted(server.events, key=lambda e: (e[0], e[1] != "done")):
        if kind == "admit":
            live.add(rid)
            used += by_id[rid].footprint
        else:
            live.discard(rid)
            used -= by_id[rid].footprint
        assert len(live) <= max_active
        assert used <= budget
    for r in results:
        assert r.arrival <= r.admitted + 1e-6 <= r.done + 1e-6


def test_slots_budget_and_order():
    reqs = [Request(i, 128 * (1 + i % 3), 2.0, 0, 0, 2, 0.01 * i) for i in range(10)]
    budget = fp(reqs[2]) + fp(reqs[1])  # at most one 384^2 and one 256^2 together
    s = Server(FakeBackend(), max_active=3, mem_budget=budget, footprint=fp)
    res = s.run(reqs)
    assert [r.rid for r in res] == list(range(10))
    _check_log(s, res, 3, budget)
    admits = [rid for _, kind, rid in sorted(s.events) if kind == "admit"]
    assert admits == sorted(admits)  # arrival order
    assert s.peak_bytes <= budget


def test_late_arrival_overtakes_a_long_request():
    long_req = Request(0, 1024, 2.0, 0, 0, 1, 0.0)      # 0.16 s
    shorts = [Request(i, 128, 2.0, 0, 0, 1, 0.03 * i) for i in range(1, 4)]  # 0.02 s each
    s = Server(FakeBackend(), max_active=2, mem_budget=1 << 40, footprint=fp)
    res = s.run([long_req] + shorts)
    done0 = res[0].done
    # every short request was admitted and finished while the long one ran
    for r in res[1:]:
        assert r.admitted < done0 and r.done < done0
    assert s.peak_active == 2
    # the short requests shared ticks with the long one
    assert s.ticks < sum(round(0.02 * r.n / 128 / 0.002) for r in [long_req] + shorts)


def test_closed_loop_and_summary():
    reqs = make_requests(6, sizes=(128, 256), rate=None, nrhs=2, seed=1)
    assert all(r.arrival == 0.0 for r in reqs)
    s = Server(FakeBackend(0.005), max_active=4, footprint=fp)
    t0 = time.perf_counter()
    res = s.run(reqs, realtime=False)
    wall = time.perf_counter() - t0
    out = summary(res, wall)
    assert out["requests"] == 6 and out["solves"] == 12 and out["all_converged"]
    assert out["latency_ms"]["p99"] >= out["latency_ms"]["p50"] > 0


def test_poisson_stream_is_seeded():
    a = make_requests(20, rate=50.0, seed=7)
    b = make_requests(20, rate=50.0, seed=7)
    assert [(r.n, r.sigma, r.arrival) for r in a] == [(r.n, r.sigma, r.arrival) for r in b]
    gaps = [y.arrival - x.arrival for x, y in zip(a, a[1:])]
    assert all(g > 0 for g in gaps)
    assert {r.n for r in make_requests(200, seed=3)} == {128, 256, 512, 1024}


def test_request_larger_than_budget_is_rejected():
    s = Server(FakeBackend(), max_active=2, mem_budget=10, footprint=fp)
    with pytest.raises(ValueError):
        s.run([Request(0, 128, 2.0, 0, 0, 1, 0.0)])


class ReleasingBackend(FakeBackend):
    """FakeBackend whose finished requests are released later, as the GPU
    backend releases its contexts on a background thread: poll() only queues
    the release, flush() performs the queued ones."""

    def __init__(self):
        super().__init__()
        self.queued, self.released, self.flushes = [], [], 0

    def poll(self, h):
        out = super().poll(h)
        if out is not None:
            self.queued.append(h["req"].rid)
        return out

    def flush(self):
        self.flushes += 1
        self.released += self.queued
        self.queued = []


def test_run_waits_for_the_backends_releases():
    backend = ReleasingBackend()
    reqs = make_requests(6, sizes=(128, 256), rate=None, seed=3)
    res = Server(backend, max_active=3, footprint=fp).run(reqs, realtime=False)
    assert backend.flushes == 1
    assert backend.queued == []
    assert sorted(backend.released) == sorted(r.rid for r in reqs)
    assert all(r.converged for r in res)


def test_backend_without_flush_is_served():
    res = Server(FakeBackend(), max_active=2, footprint=fp).run(
        make_requests(3, sizes=(128,), rate=None, seed=1), realtime=False)
    assert len(res) == 3
