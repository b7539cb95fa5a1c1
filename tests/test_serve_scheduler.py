"""The serving scheduler's logic on the CPU, with a simulated executor and a
virtual clock: strict FIFO admission, the HBM budget is never exceeded, every
request completes, latency accounting."""
import numpy as np
import pytest

from paper_2011_10214_amd.serve import Request, priority_weights, serve


class VClock:
    def __init__(self):
        self.t = 0.0

    def clock(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeBatch:
    """Simulated batch: each run advances every admitted request by M steps;
    a run costs dt_step * M * max(sum of the running requests' sizes, floor)
    seconds (a device that small runs cannot fill costs its floor)."""

    def __init__(self, vc, max_slots, budget, M=8, dt_step=1e-4, floor=0):
        self.vc, self.max_slots, self.budget, self.M, self.dt = vc, max_slots, budget, M, dt_step
        self.floor = floor
        self.running = {}
        self.used = 0
        self.peak = 0
        self.admitted = []

    def footprint(self, req):
        return req.cfg["bytes"]

    def fits(self, req):
        return len(self.running) < self.max_slots and self.used + req.footprint <= self.budget

    def admit(self, req):
        assert self.fits(req)
        self.running[req.rid] = [req, req.steps]
        self.used += req.footprint
        self.peak = max(self.peak, self.used)
        self.admitted.append(req.rid)

    def busy(self):
        return bool(self.running)

    def run(self):
        size = sum(r.cfg["size"] for r, _ in self.running.values())
        self.vc.t += self.dt * self.M * max(size, self.floor)
        done = []
        for rid in list(self.running):
            r, left = self.running[rid]
            left -= self.M
            if left <= 0:
                del self.running[rid]
                self.used -= r.footprint
                done.append(r)
            else:
                self.running[rid][1] = left
        return done


def _requests(n, seed, rate, sizes=(1, 8)):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    reqs = []
    for i in range(n):
        size = int(rng.integers(*sizes))
        reqs.append(Request(rid=i, arrival=float(t[i]), steps=int(rng.integers(10, 100)),
                            cfg={"bytes": size * 100, "size": size}, particles=size))
    return reqs


@pytest.mark.parametrize("slots,budget", [(4, 1000), (16, 2500), (1, 10 ** 9)])
def test_fifo_budget_and_completion(slots, budget):
    vc = VClock()
    ex = FakeBatch(vc, slots, budget)
    reqs = _requests(200, 1, rate=20.0)
    st = serve(reqs, ex, clock=vc.clock, sleep=vc.sleep)
    assert st["requests"] == len(reqs)
    assert ex.admitted == sorted(ex.admitted)          # admitted in arrival order
    assert ex.peak <= budget                           # never over budget
    for r in reqs:
        assert r.arrival <= r.t_admit <= r.t_done
        assert r.latency == r.t_done - r.arrival
    lat = np.array([r.latency for r in reqs])
    assert st["latency_p50_s"] == pytest.approx(np.percentile(lat, 50))
    assert st["latency_p99_s"] == pytest.approx(np.percentile(lat, 99))


def test_batching_beats_one_at_a_time_under_load():
    # small runs that cannot fill the device alone: one run costs as much as a
    # batch of up to `floor` units of work
    reqs_a = _requests(100, 2, rate=10.0)
    reqs_b = _requests(100, 2, rate=10.0)
    vc = VClock()
    one = serve(reqs_a, FakeBatch(vc, 1, 10 ** 9, floor=16), clock=vc.clock, sleep=vc.sleep)
    vc = VClock()
    many = serve(reqs_b, FakeBatch(vc, 16, 10 ** 9, floor=16), clock=vc.clock, sleep=vc.sleep)
    assert many["latency_p99_s"] < one["latency_p99_s"]
    assert many["wall_s"] <= one["wall_s"]


def test_request_larger_than_budget_is_reported():
    vc = VClock()
    ex = FakeBatch(vc, 4, 100)
    reqs = [Request(rid=0, arrival=0.0, steps=10, cfg={"bytes": 1000, "size": 1})]
    with pytest.raises(RuntimeError):
        serve(reqs, ex, clock=vc.clock, sleep=vc.sleep)


def test_head_of_line_waits_for_memory():
    # a big request blocks later small ones until memory frees up (strict FIFO)
    vc = VClock()
    ex = FakeBatch(vc, 8, 1000)
    reqs = [Request(rid=0, arrival=0.0, steps=80, cfg={"bytes": 600, "size": 6}),
            Request(rid=1, arrival=0.1, steps=80, cfg={"bytes": 600, "size": 6}),
            Request(rid=2, arrival=0.2, steps=8, cfg={"bytes": 100, "size": 1})]
    serve(reqs, ex, clock=vc.clock, sleep=vc.sleep)
    assert ex.admitted == [0, 1, 2]
    assert reqs[2].t_admit >= reqs[1].t_admit >= reqs[0].t_done


class FakeAsyncBatch(FakeBatch):
    """FakeBatch split into launch / wait: requests admitted between the two
    join the next run (as with pic_batch_launch / pic_batch_wait)."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.in_flight = None
        self.admitted_in_flight = 0

    def admit(self, req):
        if self.in_flight is not None:
            self.admitted_in_flight += 1
        super().admit(req)

    def launch(self):
        assert self.in_flight is None
        self.in_flight = set(self.running)

    def wait(self):
        ids = self.in_flight
        self.in_flight = None
        size = sum(self.running[i][0].cfg["size"] for i in ids)
        self.vc.t += self.dt * self.M * max(size, self.floor)
        done = []
        for rid in ids:
            r, left = self.running[rid]
            left -= self.M
            if left <= 0:
                del self.running[rid]
                self.used -= r.footprint
                done.append(r)
            else:
                self.running[rid][1] = left
        return done

    def run(self):
        raise AssertionError("the overlapped loop calls launch / wait")


def test_overlapped_admission_keeps_fifo_and_budget():
    vc = VClock()
    ex = FakeAsyncBatch(vc, 8, 2500)

    # admission itself costs time (creating and loading a context), so
    # requests arrive while a run is in flight
    def on_admit(r, e):
        vc.t += 1e-3

    reqs = _requests(200, 5, rate=40.0)
    st = serve(reqs, ex, clock=vc.clock, sleep=vc.sleep, on_admit=on_admit)
    assert st["requests"] == len(reqs)
    assert ex.admitted == sorted(ex.admitted)
    assert ex.peak <= 2500
    assert ex.admitted_in_flight > 0
    for r in reqs:
        assert r.arrival <= r.t_admit <= r.t_done


def _req(rid, arrival, particles):
    return Request(rid=rid, arrival=arrival, steps=10, cfg=None, particles=particles)


def quotas(w, running, P, M):
    """The step quotas pic_batch computes from the weights (share of P
    particle-steps by weight over the particles, rounded down, 1..M)."""
    tot = sum(w.values())
    return {k: (0 if wk == 0 else min(M, max(1, int(P * (wk / tot) / running[k].particles))))
            for k, wk in w.items()}


def test_priority_weights_run_the_oldest_and_backfill_small_ones():
    running = {3: _req(7, 0.5, 100_000_000), 0: _req(4, 0.1, 80_000_000),
               1: _req(9, 0.7, 2_000_000), 2: _req(10, 0.8, 5_000_000),
               5: _req(12, 0.9, 3_000_000)}
    left = {3: 900, 0: 500, 1: 1000, 2: 50, 5: 300}
    P, M = 10 ** 9, 256
    w = priority_weights(running, left, M, P, backfill=0.1, saturation=20_000_000)
    # slot 0 is the oldest; the room beside it is 8 M particles: slot 3
    # (100 M) waits, slots 1 (2 M) and 2 (5 M) run, slot 5 (3 M) no longer fits
    assert w[3] == w[5] == 0.0 and min(w[0], w[1], w[2]) > 0
    q = quotas(w, running, P, M)
    # beside the head at most a tenth of P: 256 and 50 steps scaled to 33 and 6
    assert q[1] == 33 and q[2] == 6
    assert q[1] * 2_000_000 + q[2] * 5_000_000 <= 0.1 * P
    # the head takes the rest: (1e9 - 96e6) // 80e6 = 11 steps
    assert q[0] == 11
    # without backfill a head above saturation runs alone
    w0 = priority_weights(running, left, M, P, saturation=20_000_000)
    assert [k for k in w0 if w0[k] > 0] == [0]
    assert quotas(w0, running, P, M)[0] == 12


def test_priority_weights_leave_a_small_head_the_rest_of_the_gpu():
    running = {0: _req(0, 0.0, 1_000_000), 1: _req(1, 0.1, 15_000_000),
               2: _req(2, 0.2, 10_000_000)}
    left = {0: 1000, 1: 1000, 2: 1000}
    P, M = 3 * 10 ** 9, 256
    w = priority_weights(running, left, M, P, saturation=20_000_000)
    # room: 20 M - 1 M = 19 M: 15 M runs, then 10 M does not fit
    assert w[2] == 0.0 and w[0] > 0 and w[1] > 0
    q = quotas(w, running, P, M)
    # the head keeps M steps; the other takes what is left of P
    assert q[0] == M
    assert q[1] == (P - M * 1_000_000) * M // (M * 15_000_000)
    assert q[0] * 1_000_000 + q[1] * 15_000_000 <= P
    # a request near its end asks for no more than its remaining steps
    w = priority_weights(running, {0: 7, 1: 3, 2: 1000}, M, P, saturation=20_000_000)
    q = quotas(w, running, P, M)
    assert q[0] >= 7 and q[1] >= 3 and q[2] == 0
    # P = 0: every running request takes M steps (equal weights)
    assert priority_weights(running, left, M, 0, saturation=20_000_000) == {0: 1.0, 1: 1.0, 2: 0.0}
    assert priority_weights({}, {}, M, P) == {}
    w = priority_weights({4: _req(0, 0.0, 0)}, {4: 10}, M, P)
    assert list(w) == [4] and w[4] > 0


def test_priority_weights_without_saturation_room():
    # saturation 0: only the backfill share runs beside the head
    running = {0: _req(0, 0.0, 1000), 1: _req(1, 0.1, 50), 2: _req(2, 0.2, 200)}
    left = {0: 40, 1: 40, 2: 40}
    w = priority_weights(running, left, 8, 4000, backfill=0.1, saturation=0)
    assert w[0] > 0 and w[1] > 0 and w[2] == 0.0
    q = quotas(w, running, 4000, 8)
    assert q[1] * 50 <= 0.1 * 4000 and q[0] * 1000 + q[1] * 50 <= 4000
    w = priority_weights(running, left, 8, 4000, saturation=0)
    assert [k for k in w if w[k] > 0] == [0]


def test_priority_weights_within_head_backfill_only_what_ends_first():
    # EASY-style: beside the head only requests with no more steps left
    running = {0: _req(0, 0.0, 1_000_000), 1: _req(1, 0.1, 2_000_000),
               2: _req(2, 0.2, 3_000_000), 3: _req(3, 0.3, 4_000_000)}
    left = {0: 300, 1: 500, 2: 300, 3: 100}
    P, M = 10 ** 10, 256
    w = priority_weights(running, left, M, P, saturation=20_000_000, within_head=True)
    assert w[1] == 0.0 and w[0] > 0 and w[2] > 0 and w[3] > 0
    # without the rule all three fit in the room beside the 1 M head
    w = priority_weights(running, left, M, P, saturation=20_000_000)
    assert min(w.values()) > 0
    # the room still applies to the ones that end first
    w = priority_weights(running, left, M, P, saturation=5_000_000, within_head=True)
    assert w[2] > 0 and w[3] == 0.0 and w[1] == 0.0


def test_priority_serving_keeps_every_request_moving_to_completion():
    # a simulated executor with the priority weights: paused requests take no
    # steps; every request completes and the oldest is never paused
    vc = VClock()

    class Prio(FakeBatch):
        def run(self):
            w = priority_weights({k: r for k, (r, _) in self.running.items()},
                                 {k: left for k, (_, left) in self.running.items()},
                                 self.M, 0, backfill=0.1, saturation=5)
            oldest = min(self.running, key=lambda k: (self.running[k][0].arrival, k))
            assert w[oldest] > 0
            active = [k for k in self.running if w[k] > 0]
            size = sum(self.running[k][0].cfg["size"] for k in active)
            self.vc.t += self.dt * self.M * max(size, self.floor)
            done = []
            for rid in active:
                r, left = self.running[rid]
                left -= self.M
                if left <= 0:
                    del self.running[rid]
                    self.used -= r.footprint
                    done.append(r)
                else:
                    self.running[rid][1] = left
            return done

    reqs = _requests(150, 3, rate=30.0)
    st = serve(reqs, Prio(vc, 8, 10 ** 9), clock=vc.clock, sleep=vc.sleep)
    assert st["requests"] == len(reqs)


def test_prefetch_limits_the_requests_admitted_to_wait():
    # the executor's admission test alone (no device): with prefetch 1 a
    # second request that would wait paused is not admitted; one that runs
    # (weight > 0 in the last launch) does not count
    from paper_2011_10214_amd.serve import BatchExecutor

    class FakeBatch:
        max_slots, used_bytes, budget = 8, 0, 1 << 40

    ex = object.__new__(BatchExecutor)
    ex.batch, ex.retired, ex.policy, ex.prefetch = FakeBatch(), [], "priority", 1
    ex.slots, ex.last_w, ex.prefetch_particles, ex.prefetch_large = {}, {}, None, None
    r = _req(5, 1.0, 1000)
    r.footprint = 1
    assert ex.fits(r)                         # nothing waits yet
    ex.slots = {0: (None, None), 1: (None, None)}
    ex.last_w = {0: 3.0}                      # slot 1: admitted since the launch
    assert not ex.fits(r)
    ex.last_w = {0: 3.0, 1: 2.0}              # both run
    assert ex.fits(r)
    ex.last_w = {0: 3.0, 1: 0.0}              # slot 1 waits paused
    assert not ex.fits(r)
    ex.prefetch = None
    assert ex.fits(r)
    ex.policy, ex.prefetch, ex.last_w = "fair", 1, {}
    assert ex.fits(r)                         # only the priority policy pauses


def test_prefetch_particles_bounds_the_loading_moved_ahead():
    from paper_2011_10214_amd.serve import BatchExecutor

    class FakeBatch:
        max_slots, used_bytes, budget = 8, 0, 1 << 40

    ex = object.__new__(BatchExecutor)
    ex.batch, ex.retired, ex.policy, ex.prefetch = FakeBatch(), [], "priority", None
    ex.prefetch_particles, ex.prefetch_large = 5000, None
    big, small = _req(1, 0.1, 4000), _req(2, 0.2, 800)
    ex.slots = {0: (_req(0, 0.0, 9000), None), 1: (big, None)}
    ex.last_w = {0: 9000.0, 1: 0.0}           # the large request waits
    r = _req(3, 0.3, 1500)
    r.footprint = small.footprint = 1
    assert not ex.fits(r)                     # 4000 + 1500 > 5000
    assert ex.fits(small)                     # 4000 + 800
    ex.last_w = {0: 9000.0, 1: 4000.0}        # nothing waits: any request
    assert ex.fits(_req(4, 0.4, 10 ** 9))


def test_prefetch_large_counts_only_requests_that_cannot_run_beside_a_head():
    from paper_2011_10214_amd.serve import BatchExecutor

    class FakeBatch:
        max_slots, used_bytes, budget = 8, 0, 1 << 40

    ex = object.__new__(BatchExecutor)
    ex.batch, ex.retired, ex.policy = FakeBatch(), [], "priority"
    ex.prefetch, ex.prefetch_particles, ex.prefetch_large, ex.saturation = None, None, 1, 1000
    ex.slots = {0: (_req(0, 0.0, 5000), None), 1: (_req(1, 0.1, 3000), None),
                2: (_req(2, 0.2, 50), None)}
    ex.last_w = {0: 5000.0, 1: 0.0, 2: 0.0}    # a large and a small one wait
    large, small = _req(3, 0.3, 2000), _req(4, 0.4, 60)
    large.footprint = small.footprint = 1
    assert not ex.fits(large)                  # one large request waits already
    assert ex.fits(small)                      # small ones are not counted
    ex.last_w = {0: 5000.0, 1: 3000.0, 2: 0.0}
    assert ex.fits(large)
