"""Serving many independent charging runs on one GPU.

A request is one run: a context configuration (mesh, object, species), a loader
that fills a freshly created context with its particles and node field, and a
number of steps. The server admits requests in arrival order (strict FIFO) as
soon as a batch slot is free and the request's device footprint fits the HBM
budget, and keeps the admitted runs stepping together (continuous batching:
requests that arrive while others run join as slots and memory free up). The
per-request latency is completion time minus arrival time.

Executors:
  BatchExecutor      -- all admitted runs advance together through pic_batch
                        (batched step kernels replayed from a captured graph;
                        new requests are loaded while a run executes)
  SequentialExecutor -- one run at a time through pic_step (the reference)
Any object with the same methods (footprint, fits, admit, busy, run; optionally
launch + wait for overlapped admission) can stand in (the scheduler logic is
tested on the CPU with a simulated executor).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass
from typing import Any, Callable, Optional

import numpy as np

from . import pic


@dataclass
class Request:
    rid: int
    arrival: float                      # seconds after the start of serving
    steps: int
    cfg: Any                            # pic.Config (or an executor-specific description)
    loader: Optional[Callable] = None   # loader(ctx): loads particles and node field
    particles: int = 0                  # particles at the start (for throughput)
    footprint: int = 0                  # device bytes (filled by the executor)
    t_admit: float = float("nan")
    t_done: float = float("nan")
    result: Any = None
    collect: Optional[Callable] = None  # collect(ctx) -> result, before the context is freed

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


def priority_weights(running: dict, remaining: dict, steps_per_run: int,
                     particle_steps_per_run: int, backfill: float = 0.0,
                     saturation: int = 20_000_000, within_head: bool = False) -> dict:
    """Weights of the "priority" policy for the running requests (slot ->
    Request; `remaining`: slot -> steps left), in the units of pic_batch's
    share of a run (the particle-steps each request should take; 0 pauses it).

    The oldest request (the head) always runs. Younger ones run beside it, in
    age order, while their particles add up to at most
    max(backfill * head particles, saturation - head particles): with the
    default backfill 0 only in the room a head below `saturation` particles
    leaves on the GPU, so no request waits for one that arrived after it
    while it could use the whole GPU. The others are paused. A request beside
    the head takes min(M, its remaining) steps per run, all of them together
    at most that fraction of the run's P particle-steps and never more than
    the head leaves of P at M steps (scaled down evenly beyond it); the head
    takes the rest of P (at most M steps). With P = 0 every running request
    takes M steps. With ``within_head`` a younger request runs beside the
    head only if it has no more steps left than the head (it ends no later,
    so it never runs beside the next head: the rule of EASY backfilling,
    in runs of M steps)."""
    if not running:
        return {}
    M, P = int(steps_per_run), int(particle_steps_per_run)
    order = sorted(running, key=lambda k: (running[k].arrival, running[k].rid))
    n = {k: max(int(running[k].particles), 1) for k in order}
    left = {k: max(int(remaining.get(k, M)), 1) for k in order}
    head = order[0]
    nh = n[head]
    room = max(backfill * nh, saturation - nh)
    side = []
    for k in order[1:]:
        if within_head and left[k] > left[head]:
            continue
        if n[k] <= room:
            side.append(k)
            room -= n[k]
    w = {k: 0.0 for k in order}
    if P <= 0:
        for k in [head] + side:
            w[k] = 1.0
        return w
    q = {k: min(M, left[k]) for k in side}
    work = sum(q[k] * n[k] for k in side)
    # the share of the run beside the head: the GPU room a small head leaves
    # (or the backfill fraction), and never what the head itself can use
    free = (saturation - nh) / saturation if saturation > 0 else 0.0
    cap = P * min(1.0, max(backfill, free))
    cap = min(cap, max(backfill * P, P - min(M, left[head]) * nh))
    if work > cap:
        scale = cap / work
        q = {k: max(1, int(q[k] * scale)) for k in side}
        work = sum(q[k] * n[k] for k in side)
    q[head] = min(M, left[head], max(1, (P - work) // nh))
    # pic_batch gives slot k the quota P * w_k / sum(w) / n_k steps (rounded
    # down); a quarter step more in each weight keeps the rounding from
    # losing a step when the run is exactly full
    for k, qk in q.items():
        w[k] = (qk + 0.25) * n[k]
    return w


class BatchExecutor:
    """Continuous batching on one GPU through pic_batch.

    With ``particle_steps_per_run`` > 0 every run shares that many particle-
    steps among the running requests by weight; ``policy`` sets the weights:
      "fair"     -- all equal (each request gets about the same GPU time)
      "head"     -- the oldest running request gets the fraction ``head_share``
                    of a run, the others share the rest equally
      "priority" -- the oldest running request runs as if alone; younger
                    ones run beside it only in the room a small head leaves
                    on a GPU of ``saturation`` particles (plus ``backfill``
                    times the head's particles, 0 by default), with up to M
                    steps per run each; the others wait paused on the device
                    (priority_weights), at most ``prefetch`` of them (or
                    ``prefetch_particles`` of their particles, or
                    ``prefetch_large`` of those with at least ``saturation``
                    particles) admitted ahead (None: as many as slots and
                    memory allow); with ``within_head`` only requests that
                    end no later than the head run beside it.
    """

    def __init__(self, max_slots: int, repr: str, deposit: str, steps_per_run: int,
                 hbm_budget_bytes: int, stream: int = 0, particle_steps_per_run: int = 0,
                 policy: str = "fair", head_share: float = 0.5, backfill: float = 0.0,
                 saturation: int = 20_000_000, prefetch: Optional[int] = None,
                 prefetch_particles: Optional[int] = None, prefetch_large: Optional[int] = None,
                 within_head: bool = False):
        if policy not in ("fair", "head", "priority"):
            raise ValueError(f"unknown policy {policy!r}")
        if prefetch is not None and prefetch < 1:
            raise ValueError("prefetch must be >= 1 (or None)")
        if not 0.0 < head_share < 1.0:
            raise ValueError("head_share must be in (0, 1)")
        if not backfill >= 0.0:
            raise ValueError("backfill must be >= 0")
        self.head_share = head_share
        self.steps_per_run = int(steps_per_run)
        self.particle_steps_per_run = int(particle_steps_per_run)
        self.backfill = backfill
        self.saturation = int(saturation)
        self.batch = pic.Batch(max_slots, repr, deposit, steps_per_run, hbm_budget_bytes, stream,
                               particle_steps_per_run)
        self.stream = stream
        self.policy = policy
        self.slots = {}   # slot -> (request, context)
        # at most this many admitted requests wait paused (None: no limit):
        # creating and loading a request that will not run for a while puts
        # its GPU work in front of the requests ahead of it
        self.prefetch = prefetch
        # the same bound on their particles (their loading work): a request is
        # admitted while the waiting ones and it hold at most this many, or
        # when none waits
        self.prefetch_particles = prefetch_particles
        # the same count for the large requests only (at least `saturation`
        # particles: they can never run beside a head, and their loading is
        # the expensive one); small ones keep flowing
        self.prefetch_large = prefetch_large
        # younger requests beside the head only if they end no later than it
        self.within_head = bool(within_head)
        self.last_w = {}  # slot -> weight of the last launch
        self.retired = []  # finished (context, bytes), freed once the next run is launched

    def footprint(self, req: Request) -> int:
        return pic.footprint_bytes(req.cfg)

    def fits(self, req: Request) -> bool:
        held = sum(b for _, b in self.retired)  # detached, not yet freed
        if self.policy == "priority":
            # slots admitted since the last launch count as waiting
            waiting = [k for k in self.slots if self.last_w.get(k, 0.0) <= 0.0]
            if self.prefetch is not None and len(waiting) >= self.prefetch:
                return False
            if self.prefetch_particles is not None and waiting:
                held_n = sum(self.slots[k][0].particles for k in waiting)
                if held_n + req.particles > self.prefetch_particles:
                    return False
            if self.prefetch_large is not None and req.particles >= self.saturation:
                large = sum(1 for k in waiting if self.slots[k][0].particles >= self.saturation)
                if large >= self.prefetch_large:
                    return False
        return (len(self.slots) < self.batch.max_slots and
                self.batch.used_bytes + held + req.footprint <= self.batch.budget)

    def admit(self, req: Request) -> None:
        cfg = req.cfg
        if self.stream and not cfg.stream:
            cfg.stream = self.stream
        ctx = pic.Context(cfg)
        try:
            req.loader(ctx)
            slot = self.batch.attach(ctx, req.steps)
        except Exception:
            ctx.close()
            raise
        self.slots[slot] = (req, ctx)

    def busy(self) -> bool:
        return bool(self.slots)

    def run(self) -> list:
        self.launch()
        return self.wait()

    def launch(self) -> None:
        """Enqueues one run; admissions may proceed until wait()."""
        if self.policy == "priority":
            w = priority_weights({k: v[0] for k, v in self.slots.items()},
                                 {k: self.batch.remaining(k) for k in self.slots},
                                 self.steps_per_run, self.particle_steps_per_run,
                                 self.backfill, self.saturation, self.within_head)
            for k, wk in w.items():
                self.batch.set_weight(k, wk)
            self.last_w = w
        elif self.policy == "head" and len(self.slots) > 1:
            head = min(self.slots, key=lambda k: (self.slots[k][0].arrival, self.slots[k][0].rid))
            others = len(self.slots) - 1
            wh = self.head_share / (1.0 - self.head_share) * others
            for k in self.slots:
                self.batch.set_weight(k, wh if k == head else 1.0)
        self.batch.launch()
        self._free_retired()

    def wait(self) -> list:
        done = []
        for slot in self.batch.wait():
            req, ctx = self.slots.pop(slot)
            self.batch.detach(slot)
            if req.collect:
                req.result = req.collect(ctx)
            self.retired.append((ctx, req.footprint))
            done.append(req)
        if not self.slots:
            self._free_retired()
        return done

    def _free_retired(self):
        for ctx, _ in self.retired:
            ctx.close()
        self.retired.clear()

    def close(self):
        self._free_retired()
        for slot, (_, ctx) in list(self.slots.items()):
            self.batch.detach(slot)
            ctx.close()
        self.slots.clear()
        self.batch.close()


class SequentialExecutor:
    """One run at a time, each through pic_step (the unbatched reference)."""

    def __init__(self, hbm_budget_bytes: int, stream: int = 0):
        self.budget = int(hbm_budget_bytes)
        self.stream = stream
        self.current = None

    def footprint(self, req: Request) -> int:
        return pic.footprint_bytes(req.cfg)

    def fits(self, req: Request) -> bool:
        return self.current is None and req.footprint <= self.budget

    def admit(self, req: Request) -> None:
        cfg = req.cfg
        if self.stream and not cfg.stream:
            cfg.stream = self.stream
        ctx = pic.Context(cfg)
        try:
            req.loader(ctx)
        except Exception:
            ctx.close()
            raise
        self.current = (req, ctx)

    def busy(self) -> bool:
        return self.current is not None

    def run(self) -> list:
        req, ctx = self.current
        ctx.step(req.steps)
        ctx.synchronize()
        if req.collect:
            req.result = req.collect(ctx)
        ctx.close()
        self.current = None
        return [req]

    def close(self):
        if self.current:
            self.current[1].close()
            self.current = None


def serve(requests: list, executor, clock: Callable[[], float] = time.perf_counter,
          sleep: Callable[[float], None] = time.sleep, on_admit=None) -> dict:
    """Serves `requests` (any order; arrival times relative to the start) with
    strict FIFO admission. Returns latency and throughput statistics."""
    queue = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
    for r in queue:
        r.footprint = executor.footprint(r)
    finished = []
    t0 = clock()
    overlap = hasattr(executor, "launch") and hasattr(executor, "wait")

    def admit_arrived():
        now = clock() - t0
        while queue and queue[0].arrival <= now and executor.fits(queue[0]):
            r = queue.popleft()
            r.t_admit = clock() - t0
            executor.admit(r)
            if on_admit:
                on_admit(r, executor)

    while queue or executor.busy():
        # with runs in progress the next run is launched first, so that the
        # GPU does not wait while new requests are created and loaded
        if not (overlap and executor.busy()):
            admit_arrived()
        now = clock() - t0
        if executor.busy():
            if overlap:
                # requests that arrive during a run are created, loaded and
                # attached while it executes; they join the next run
                executor.launch()
                admit_arrived()
                done = executor.wait()
            else:
                done = executor.run()
            for r in done:
                r.t_done = clock() - t0
                finished.append(r)
        elif queue:
            if queue[0].arrival > now:
                sleep(queue[0].arrival - now)
            elif not executor.fits(queue[0]):
                raise RuntimeError(f"request {queue[0].rid} can never be admitted "
                                   f"(footprint {queue[0].footprint} B)")
    return summarize(finished, clock() - t0)


def summarize(finished: list, wall: float) -> dict:
    lat = np.array([r.latency for r in finished]) if finished else np.zeros(0)
    ps = sum(r.particles * r.steps for r in finished)
    return {
        "requests": len(finished),
        "wall_s": wall,
        "throughput_req_per_s": len(finished) / wall if wall > 0 else 0.0,
        "throughput_particle_steps_per_s": ps / wall if wall > 0 else 0.0,
        "latency_p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "latency_p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "latency_mean_s": float(lat.mean()) if len(lat) else None,
    }
