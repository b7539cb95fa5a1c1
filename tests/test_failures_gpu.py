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


@pytest.mark.parametrize("form", ["fp64", "fp32_abs", "fp32_cell"])
def test_resume_continues_the_injection_and_photoemission_draws(form):
    # the lunar loop (symmetry plane, ambient injection, photoemission): a run
    # exported after 5 steps and loaded into a fresh context set to step
    # index 5 ends where one 10-step run of the oracle ends, bit for bit
    from oracle import oracle

    from helpers import problem_of
    from test_boundaries_gpu import LUNAR, ambient
    from test_photo_gpu import PHOTO, SUN, lunar_with_photoelectrons

    w = lunar_with_photoelectrons()
    half, ns = 5, 3
    sp, x, v, E = inputs(w)
    dens, vth, drift = ambient(w)
    dens[2] = 0.0
    prob = problem_of(w, form)
    prob.reflect, prob.inj_faces, prob.inj_seed = LUNAR["reflect"], LUNAR["faces"], 11
    prob.inj_density, prob.inj_vth, prob.inj_drift = dens, vth, drift
    prob.pe_species, prob.pe_seed, prob.pe_sun, prob.pe_flux, prob.pe_vth = 2, 21, SUN, 30.0, PHOTO.vth
    r = oracle.run(prob, sp, x, v, E, 2 * half)
    extra = prob.injection_bound(2 * half)
    cap = [int((sp == s).sum()) + extra for s in range(ns)]

    def boundaries(ctx):
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.set_injection(LUNAR["faces"], 11, dens, vth, drift)
        ctx.set_photoemission(2, 21, SUN, 30.0, PHOTO.vth)

    cfg = pam.config_from_workload(w, repr=form, deposit="fixed64", capacity=cap)
    cfg.reflect = LUNAR["reflect"]
    ids = np.arange(len(sp), dtype=np.int64)
    with pam.Context(cfg) as first:
        for s in range(ns):
            m = sp == s
            first.load_particles(s, x[m], v[m], ids[m])
        boundaries(first)
        first.step(half)
        parts = [first.get_particles(s) for s in range(ns)]
        counts_a = first.get_surface_charge()[1]
        esc_a = first.get_counters()[2]
        inj_a = first.get_injected()
    with pam.Context(cfg) as second:
        for s, (px, pv, pid) in enumerate(parts):
            second.load_particles(s, px, pv, pid)
        boundaries(second)
        second.set_step_index(half)
        second.step(half)
        rho_fixed = second.get_rho()[1]
        counts_b = second.get_surface_charge()[1]
        esc_b = second.get_counters()[2]
        inj_b = second.get_injected()
        got = [second.get_particles(s) for s in range(ns)]
    assert r.injected[2] > 100
    assert np.array_equal(rho_fixed, r.rho_fixed)
    assert np.array_equal(counts_a + counts_b, r.tally)
    assert np.array_equal(esc_a + esc_b, r.escaped)
    # the second context counts as injected only its own steps' particles
    assert np.array_equal(inj_a + inj_b, r.injected)
    n = len(sp)
    for s in range(ns):
        gx, gv, gid = got[s]
        keep = gid >= 0
        o = np.argsort(gid[keep])
        want = np.nonzero((r.fate[:n] == 0) & (sp == s))[0]
        assert np.array_equal(gid[keep][o], want)
        assert np.array_equal(gx[keep][o], r.x[want]) and np.array_equal(gv[keep][o], r.v[want])
        # injected and emitted particles (id -1) as a set
        m = (r.fate == 0) & (r.species == s)
        m[:n] = False
        gi = np.concatenate([gx[~keep], gv[~keep]], 1)
        ri = np.concatenate([r.x[m], r.v[m]], 1)
        assert len(gi) == len(ri)
        assert np.array_equal(gi[np.lexsort(gi.T[::-1])], ri[np.lexsort(ri.T[::-1])])


def test_step_index_is_checked():
    w = synth.sphere_16()
    ctx, _ = loaded(w)
    with ctx:
        for bad in (-1, 2 ** 31):
            with pytest.raises(pam.PicError) as ei:
                ctx.set_step_index(bad)
            assert ei.value.status == pam.pic.E_INVALID
        ctx.set_step_index(7)
