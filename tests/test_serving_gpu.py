"""Batched serving on the GPU: each request's result is the same in the batch
(continuous batching through pic_batch, steps replayed from captured graphs)
as when run alone through pic_step -- bit for bit with the fixed-point
deposit."""
import numpy as np
import pytest

import paper_2011_10214_amd as pam
import synth
from paper_2011_10214_amd.serve import BatchExecutor, Request, SequentialExecutor, serve

pytestmark = pytest.mark.gpu


def _loader(w):
    def load(ctx):
        for s in range(len(w.species)):
            c = synth.particles(w, s)
            ctx.load_particles(s, np.stack(c[:3], 1), np.stack(c[3:], 1))
        ctx.set_node_E([e.astype(np.float64) for e in synth.node_E(w)])
    return load


def _collect(ctx):
    rho, rf = ctx.get_rho()
    charge, counts = ctx.get_surface_charge()
    alive, absorbed, escaped = ctx.get_counters()
    xs = []
    for s in range(ctx.ns):
        x, v, _ = ctx.get_particles(s, with_ids=False)
        key = np.lexsort(np.concatenate([x, v], 1).T[::-1])
        xs.append((x[key], v[key]))
    return dict(rho_fixed=rf, counts=counts, alive=alive, escaped=escaped, particles=xs)


def _requests(repr_, arrivals):
    stream = synth.serving_stream(n_requests=len(arrivals), seed=11, n_min=12, n_max=28,
                                  ppc_min=2, ppc_max=6, steps_min=9, steps_max=45)
    reqs = []
    for i, ((w, steps), t) in enumerate(zip(stream, arrivals)):
        cfg = pam.config_from_workload(w, repr=repr_, deposit="fixed64")
        reqs.append(Request(rid=i, arrival=t, steps=steps, cfg=cfg, loader=_loader(w),
                            particles=w.n_particles, collect=_collect))
    return reqs


def _same(a, b):
    assert np.array_equal(a["rho_fixed"], b["rho_fixed"])
    assert np.array_equal(a["counts"], b["counts"])
    assert np.array_equal(a["alive"], b["alive"]) and np.array_equal(a["escaped"], b["escaped"])
    for (xa, va), (xb, vb) in zip(a["particles"], b["particles"]):
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)


@pytest.mark.parametrize("repr_,ps_per_run,policy", [("fp32_cell", 0, "fair"), ("fp64", 0, "fair"),
                                                     ("fp32_cell", 150_000, "fair"),
                                                     ("fp64", 150_000, "fair"),
                                                     ("fp32_cell", 150_000, "head"),
                                                     ("fp32_cell", 150_000, "priority"),
                                                     ("fp64", 0, "priority"),
                                                     ("fp32_cell", 150_000, "priority_within")])
def test_alone_and_in_the_mix_are_identical(repr_, ps_per_run, policy):
    # ps_per_run > 0: unequal step quotas per run (fair share), so contexts of
    # one run leave the persistent launches at different steps; priority with
    # no saturation room: requests above a tenth of the oldest's size wait
    # paused between runs; priority_within: the default of the serving bench
    # (room for all of these small requests beside the head, but only those
    # with no more steps left than it, at most one large one waiting)
    arrivals = [0.0, 0.0, 0.0, 0.05, 0.1, 0.1, 0.3]
    mix = _requests(repr_, arrivals)
    kw = dict(policy=policy, saturation=0, backfill=0.1)
    if policy == "priority_within":
        kw = dict(policy="priority", within_head=True, prefetch_large=1)
    ex = BatchExecutor(max_slots=3, repr=repr_, deposit="fixed64", steps_per_run=4,
                       hbm_budget_bytes=64 << 30, particle_steps_per_run=ps_per_run, **kw)
    try:
        st = serve(mix, ex)
    finally:
        ex.close()
    assert st["requests"] == len(mix)
    alone = _requests(repr_, [0.0] * len(arrivals))
    st1 = serve(alone, SequentialExecutor(hbm_budget_bytes=64 << 30))
    assert st1["requests"] == len(alone)
    for a, b in zip(sorted(mix, key=lambda r: r.rid), sorted(alone, key=lambda r: r.rid)):
        _same(a.result, b.result)


def test_batch_admission_respects_budget_and_slots():
    reqs = _requests("fp32_cell", [0.0] * 5)
    fps = [pam.footprint_bytes(r.cfg) for r in reqs]
    budget = sum(sorted(fps)[:2]) + 1  # room for about two at a time
    peak = []

    def on_admit(r, ex):
        peak.append(ex.batch.used_bytes)

    ex = BatchExecutor(max_slots=4, repr="fp32_cell", deposit="fixed64", steps_per_run=8,
                       hbm_budget_bytes=max(budget, max(fps)))
    try:
        st = serve(reqs, ex, on_admit=on_admit)
    finally:
        ex.close()
    assert st["requests"] == 5
    assert max(peak) <= max(budget, max(fps))
    with pytest.raises(pam.PicError):
        b = pam.Batch(2, "fp32_cell", "fixed64", 4, 1)  # a budget nothing fits in
        ctx = pam.Context(reqs[0].cfg)
        reqs[0].loader(ctx)
        try:
            b.attach(ctx, 5)
        finally:
            ctx.close()
            b.close()


def test_launch_wait_protocol():
    reqs = _requests("fp32_cell", [0.0] * 3)
    b = pam.Batch(4, "fp32_cell", "fixed64", 4, 64 << 30, particle_steps_per_run=100_000)
    ctxs = []
    try:
        for r in reqs[:2]:
            c = pam.Context(r.cfg)
            r.loader(c)
            ctxs.append((c, b.attach(c, r.steps)))
        assert b.wait() == []                     # nothing in flight
        with pytest.raises(pam.PicError):
            b.set_weight(ctxs[0][1], -1.0)        # weights must be >= 0
        with pytest.raises(pam.PicError):
            b.set_weight(3, 1.0)                  # no context in slot 3
        b.set_weight(ctxs[0][1], 4.0)
        b.launch()
        with pytest.raises(pam.PicError):
            b.launch()                            # one run at a time
        with pytest.raises(pam.PicError):
            b.detach(ctxs[0][1])                  # not while in flight
        c = pam.Context(reqs[2].cfg)              # attach while in flight
        reqs[2].loader(c)
        ctxs.append((c, b.attach(c, reqs[2].steps)))
        finished = set(b.wait())
        for _ in range(1000):
            if len(finished) == len(ctxs):
                break
            b.launch()
            finished |= set(b.wait())
        assert finished == {slot for _, slot in ctxs}
        for c, slot in ctxs:
            b.detach(slot)
            alive, _, _ = c.get_counters()
            assert alive.sum() > 0
    finally:
        for c, _ in ctxs:
            c.close()
        b.close()


def test_a_paused_slot_takes_no_steps():
    # weight 0 pauses a context: a run advances the others only; its state and
    # remaining steps stay; with every context paused, all of them run
    reqs = _requests("fp32_cell", [0.0] * 2)
    b = pam.Batch(2, "fp32_cell", "fixed64", 3, 64 << 30)
    ctxs = []
    try:
        for r in reqs:
            c = pam.Context(r.cfg)
            r.loader(c)
            ctxs.append((c, b.attach(c, 6)))
        (ca, sa), (cb, sb) = ctxs
        b.set_weight(sb, 0.0)
        assert b.remaining(sa) == b.remaining(sb) == 6
        b.launch()
        assert b.remaining(sa) == 6               # counted when the run is waited for
        assert b.wait() == []
        assert b.remaining(sa) == 3 and b.remaining(sb) == 6
        b.detach(sb)
        assert b.remaining(sb) == -1 and b.remaining(99) == -1
        before = _collect(cb)
        sb = b.attach(cb, 6)
        b.set_weight(sb, 0.0)
        b.launch()
        assert b.wait() == [sa]                   # 3 + 3 steps of a
        b.detach(sa)
        b.detach(sb)
        _same(_collect(cb), before)               # b did not move
        sb = b.attach(cb, 6)
        b.set_weight(sb, 0.0)                     # paused, but the only one
        b.launch()
        assert b.wait() == []
        b.launch()
        assert b.wait() == [sb]
        b.detach(sb)
        after = _collect(cb)
    finally:
        for c, _ in ctxs:
            c.close()
        b.close()
    # b took 6 steps in all: the same as 6 steps alone
    alone = _requests("fp32_cell", [0.0] * 2)
    for r in alone:
        r.steps = 6
    serve(alone, SequentialExecutor(hbm_budget_bytes=64 << 30))
    _same(after, alone[1].result)
