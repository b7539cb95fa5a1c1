"""Failure detection and checkpoint / resume on the GPU: a non-finite node
field is refused and the field in force stays (host and device loads); a
particle that runs away is reported as a range error at the next sync;
particles beyond a species' capacity are reported as lost; and a run that is
exported after half its steps and loaded into a fresh context ends bit for
bit where the uninterrupted run ends (positions, velocities, rho; tallies and
escapes add up)."""
import numpy as np
import pytest
import torch

import paper_2011_10214_amd as pam
import synth

from gpu_util import inputs

pytestmark = pytest.mark.gpu


def loaded(w, form="fp32_cell", capacity=None, E=None):
    sp, x, v, E0 = inputs(w)
    cfg = pam.config_from_workload(
        w, repr=form, capacity=capacity or [int((sp == s).sum()) for s in range(len(w.species))])
    ctx = pam.Context(cfg)
    ids = np.arange(len(sp), dtype=np.int64)
    for s in range(len(w.species)):
        m = sp == s
        ctx.load_particles(s, x[m], v[m], ids[m])
    ctx.set_node_E([np.asarray(e, np.float64) for e in (E0 if E is None else E)])
    return ctx, E0


def state(ctx, ns):
    parts = [ctx.get_particles(s) for s in range(ns)]
    x = np.concatenate([p[0] for p in parts])
    v = np.concatenate([p[1] for p in parts])
    i = np.concatenate([p[2] for p in parts])
    o = np.argsort(i)
    return x[o], v[o], i[o]


@pytest.mark.parametrize("device", [False, True])
def test_non_finite_field_is_refused_and_the_old_one_stays(device):
    w = synth.sphere_16()
    ctx, E = loaded(w)
    with ctx:
        bad = [np.array(e, np.float64) for e in E]
        bad[1][17] = np.nan
        bad[2][3] = np.inf
        if device:
            bad = [torch.tensor(e, dtype=torch.float32, device="cuda") for e in bad]
        with pytest.raises(pam.PicError) as ei:
            ctx.set_node_E(bad)
        assert ei.value.status == pam.pic.E_INVALID
        ctx.step(5)
        got = state(ctx, 2)
        rho = ctx.get_rho()[1]
    ref, _ = loaded(w)
    with ref:
        ref.step(5)
        want = state(ref, 2)
        rho_ref = ref.get_rho()[1]
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    assert np.array_equal(rho, rho_ref)


def test_runaway_particle_is_a_range_error():
    w = synth.sphere_16()
    sp, x, v, E = inputs(w)
    huge = [np.full(w.nodes, 1e37), np.zeros(w.nodes), np.zeros(w.nodes)]
    ctx, _ = loaded(w, E=huge)
    with ctx:
        ctx.step(1)
        with pytest.raises(pam.PicError) as ei:
            ctx.get_counters()
        assert ei.value.status == pam.pic.E_RANGE


def test_particles_beyond_capacity_are_reported_lost():
    w = synth.sphere_16()
    sp, x, v, E = inputs(w)
    n = [int((sp == s).sum()) for s in range(2)]
    ctx, _ = loaded(w, capacity=n)  # no room for injected particles
    with ctx:
        vol = w.nx * w.ny * w.nz
        ctx.set_injection(63, 1, [100.0 * s.count / vol for s in w.species],
                          [s.vth for s in w.species], [(0.0, 0.0, 0.0)] * 2)
        ctx.step(3)
        with pytest.raises(pam.PicError) as ei:
            ctx.synchronize()
        assert ei.value.status == pam.pic.E_NOMEM


@pytest.mark.parametrize("form", ["fp64", "fp32_abs", "fp32_cell"])
def test_export_and_resume_is_bit_exact(form):
    w = synth.scaled(synth.crater_160(), 32, 32, 16, 4.0, steps=50)
    ns = len(w.species)
    full, E = loaded(w, form)
    with full:
        full.step(50)
        want = state(full, ns)
        rho_want = full.get_rho()[1]
        _, counts_want = full.get_surface_charge()
        _, _, esc_want = full.get_counters()
    first, _ = loaded(w, form)
    with first:
        first.step(25)
        parts = [first.get_particles(s) for s in range(ns)]
        _, counts_a = first.get_surface_charge()
        _, _, esc_a = first.get_counters()
    cfg = pam.config_from_workload(w, repr=form, capacity=[max(1, len(p[0])) for p in parts])
    with pam.Context(cfg) as second:
        for s, (px, pv, pid) in enumerate(parts):
            second.load_particles(s, px, pv, pid)
        second.set_node_E([np.asarray(e, np.float64) for e in E])
        second.step(25)
        got = state(second, ns)
        rho_got = second.get_rho()[1]
        _, counts_b = second.get_surface_charge()
        _, _, esc_b = second.get_counters()
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    assert np.array_equal(rho_got, rho_want)
    assert np.array_equal(counts_a + counts_b, counts_want) and counts_want.sum() > 0
    assert np.array_equal(esc_a + esc_b, esc_want)
