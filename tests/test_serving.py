"""Serving layer on the CPU: admission against the memory ledger, FIFO
order, rejection, cancellation and failure isolation, driven by a simulated
executor (a sleep proportional to the request size and a result that depends
on the request alone)."""
import threading
import time

import numpy as np
import pytest

from paper_1802_05215_amd import serving as S


class SimExecutor:
    """Simulated device: records the ledger's state at each start, sleeps a
    short time and returns a result computed from the request alone."""

    def __init__(self, ledger, scale=2e-9, fail_rids=()):
        self.ledger = ledger
        self.scale = scale
        self.fail = set(fail_rids)
        self.lock = threading.Lock()
        self.starts = []
        self.max_used = 0
        self.max_running = 0

    def __call__(self, req, t0):
        start = time.perf_counter() - t0
        with self.lock:
            self.starts.append(req.rid)
            self.max_used = max(self.max_used, self.ledger.used)
            self.max_running = max(self.max_running, self.ledger.running)
        if req.rid in self.fail:
            raise RuntimeError("simulated device error")
        time.sleep(min(0.05, self.scale * S.footprint_bytes(req) / 8))
        rng = np.random.default_rng(req.pot_seed)
        lam = np.sort(rng.random(req.target)) if req.kind == "eigs" else None
        return S.Result(req.rid, req.kind, req.arrival, start, time.perf_counter() - t0,
                        nev=0 if lam is None else len(lam), lam=lam)


def _stream(count=24, rate=200.0, seed=7, **kw):
    return S.poisson_stream(seed, count, rate, n_min=1e4, n_max=2e5, **kw)


def test_stream_is_seeded_and_follows_its_recipe():
    a = S.poisson_stream(7, 400, 2.0)
    b = S.poisson_stream(7, 400, 2.0)
    assert [(r.arrival, r.N, r.kind, r.pot_seed, r.target) for r in a] == \
        [(r.arrival, r.N, r.kind, r.pot_seed, r.target) for r in b]
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) >= 0)
    # mean inter-arrival 1/rate within a few standard errors
    assert abs(np.diff(arr).mean() - 0.5) < 4 * 0.5 / np.sqrt(399)
    for r in a:
        assert r.dim in (2, 3) and r.kind in ("dos", "eigs")
        assert 50 <= r.target <= 400 and 0.05 <= r.quantile <= 0.6
        if r.dim == 2:
            assert 100 <= r.N <= 2000
        else:
            assert 22 <= r.N <= 159
    kinds = [r.kind for r in a]
    assert 150 < kinds.count("dos") < 250


def test_footprint_grows_with_size_and_target():
    base = S.Request(0, 0.0, "eigs", 3, 40, 1, target=100)
    bigger = S.Request(0, 0.0, "eigs", 3, 60, 1, target=100)
    more = S.Request(0, 0.0, "eigs", 3, 40, 1, target=300)
    dos = S.Request(0, 0.0, "dos", 3, 40, 1)
    assert S.footprint_bytes(bigger) > S.footprint_bytes(base)
    assert S.footprint_bytes(more) > S.footprint_bytes(base)
    assert S.footprint_bytes(dos) < S.footprint_bytes(base)
    # the basis dominates: at least (capacity + m + 1) FP64 columns per slice
    m, cap = S._lan_sizes(base.nev_plan, base.n)
    assert S.footprint_parts(base)["library"] >= 8 * base.n * (cap + m + 1)
    # the precision form's FP64 polish (one slice at a time, in place): two
    # n-vectors per lock-capacity column and three 32-column row-major blocks
    assert S.footprint_parts(base)["library"] >= 8 * base.n * (cap + m + 1 + 2 * cap + 96)
    # the largest request of the recipe stays within one device's memory
    big = S.Request(0, 0.0, "eigs", 3, 159, 1, target=400)
    assert S.footprint_bytes(big) < 288e9


def test_admission_never_exceeds_budget_and_is_fifo():
    reqs = _stream()
    fps = [S.footprint_bytes(r) for r in reqs]
    budget = int(2.5 * max(fps))
    led = S.Ledger(budget, max_running=4)
    ex = SimExecutor(led)
    out = S.Server(led, ex).run(reqs)
    assert [r.rid for r in out] == [r.rid for r in reqs]
    assert all(r.status == "ok" for r in out)
    assert ex.max_used <= budget and led.high_water <= budget
    assert ex.max_running <= 4
    assert led.used == 0 and led.running == 0
    # admission is in arrival order
    order = sorted(reqs, key=lambda r: (r.arrival, r.rid))
    led2 = S.Ledger(budget, 4)
    srv = S.Server(led2, SimExecutor(led2))
    srv.run(reqs)
    assert srv.admission_order == [r.rid for r in order]
    assert sorted(ex.starts) == sorted(r.rid for r in reqs)


def test_tight_budget_serialises_requests():
    # equal-size requests and a budget that holds one of them but not two
    reqs = [S.Request(i, 0.001 * i, "eigs", 3, 30, 10 + i, target=80) for i in range(6)]
    fp = S.footprint_bytes(reqs[0])
    led = S.Ledger(int(1.5 * fp), max_running=8)
    ex = SimExecutor(led, scale=1e-8)
    out = S.Server(led, ex).run(reqs)
    assert all(r.status == "ok" for r in out)
    assert led.high_water == fp and ex.max_running == 1
    spans = sorted((r.start, r.end) for r in out)
    for (s0, e0), (s1, e1) in zip(spans, spans[1:]):
        assert s1 >= e0


def test_over_budget_request_is_rejected_and_others_proceed():
    reqs = _stream(count=6)
    small = min(S.footprint_bytes(r) for r in reqs)
    big = S.Request(99, 0.0, "eigs", 3, 150, 5, target=400)
    budget = max(S.footprint_bytes(r) for r in reqs)
    assert S.footprint_bytes(big) > budget >= small
    led = S.Ledger(budget, 2)
    out = S.Server(led, SimExecutor(led)).run([big] + reqs)
    assert out[0].status == "rejected" and "exceeds" in out[0].error
    assert all(r.status == "ok" for r in out[1:])


def test_cancel_before_admission():
    reqs = _stream(count=6, rate=0.0)  # all arrive at once
    budget = max(S.footprint_bytes(r) for r in reqs)
    led = S.Ledger(budget, 1)
    ex = SimExecutor(led, scale=1e-7)
    srv = S.Server(led, ex)
    srv.cancel(reqs[3].rid)
    out = srv.run(reqs)
    assert out[3].status == "cancelled"
    assert reqs[3].rid not in ex.starts
    assert [r.status for i, r in enumerate(out) if i != 3] == ["ok"] * 5


def test_failed_request_is_reported_and_ledger_released():
    reqs = _stream(count=6)
    budget = int(3 * max(S.footprint_bytes(r) for r in reqs))
    led = S.Ledger(budget, 3)
    out = S.Server(led, SimExecutor(led, fail_rids={2})).run(reqs)
    assert out[2].status == "failed" and "simulated" in out[2].error
    assert all(r.status == "ok" for i, r in enumerate(out) if i != 2)
    assert led.used == 0 and led.running == 0


def test_results_in_a_mix_equal_solo_results():
    reqs = _stream(count=10)
    big = S.Ledger(10 ** 15, 6)
    mix = S.Server(big, SimExecutor(big)).run(reqs)
    for r, m in zip(reqs, mix):
        one = S.Ledger(10 ** 15, 1)
        solo = S.Server(one, SimExecutor(one)).run([S.Request(**{**r.__dict__, "arrival": 0.0})])
        if r.kind == "eigs":
            assert np.array_equal(solo[0].lam, m.lam)


def test_summary_percentiles():
    led = S.Ledger(10 ** 15, 2)
    res = [S.Result(i, "eigs", 0.0, 0.0, float(i + 1), nev=10) for i in range(100)]
    summ = S.summarize(res, 50.0, led)
    assert summ["eigenpairs"] == 1000 and summ["completed"] == 100
    assert summ["latency_p50_s"] == pytest.approx(50.5)
    assert summ["latency_p99_s"] == pytest.approx(99.01)


def test_bounded_bypass_lets_small_requests_pass_a_waiting_head():
    """A large request at the head that does not fit next to a running one is
    passed over by later small requests that fit, at most max_bypass times;
    then the later requests wait until the head has started."""
    big_run = S.Request(0, 0.0, "eigs", 3, 60, 1, target=300)
    head = S.Request(1, 0.001, "eigs", 3, 60, 2, target=300)
    small = [S.Request(2 + i, 0.002 + 0.0001 * i, "dos", 2, 100, 3 + i) for i in range(6)]
    fb = S.footprint_bytes(big_run)
    budget = int(1.5 * fb)
    assert S.footprint_bytes(head) + fb > budget
    assert S.footprint_bytes(small[0]) + fb <= budget
    for max_bypass in (0, 3):
        led = S.Ledger(budget, max_running=8)
        ex = SimExecutor(led, scale=3e-10)
        srv = S.Server(led, ex, max_bypass=max_bypass)
        out = srv.run([big_run, head] + small)
        assert all(r.status == "ok" for r in out)
        assert led.high_water <= budget and led.used == 0
        order = srv.admission_order
        assert order[0] == 0
        passed = order.index(1) - 1   # requests admitted between the first and the head
        assert passed <= max_bypass
        assert srv.bypassed.get(1, 0) == passed
        if max_bypass == 0:
            assert order == [0, 1] + [r.rid for r in small]
        else:
            assert passed >= 1


def test_partial_requests_are_not_counted_as_served():
    led = S.Ledger(10 ** 15, 2)
    res = [S.Result(0, "eigs", 0.0, 0.0, 1.0, nev=10),
           S.Result(1, "eigs", 0.0, 0.0, 2.0, status="partial", nev=7)]
    summ = S.summarize(res, 10.0, led)
    assert summ["eigenpairs"] == 10 and summ["completed"] == 1 and summ["partial"] == 1
