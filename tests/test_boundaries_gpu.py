"""Global boundaries on the GPU against the oracle: reflecting faces and the
injection of ambient particles (the particle setups of §3.1.3 and §5.2.2),
bit for bit in every representation with the fixed-point deposit: loaded
particles by id, injected particles as a set, rho, tallies, escapes and
injected counts."""
import numpy as np
import pytest

import paper_2011_10214_amd as pam
import synth
from oracle import oracle

from gpu_util import inputs
from helpers import problem_of

pytestmark = pytest.mark.gpu

FORMS = ["fp64", "fp32_abs", "fp32_cell"]
# OML setup: the min faces are symmetry planes, the max faces inject
OML = dict(reflect=1 | 4 | 16, faces=2 | 8 | 32)
# lunar setup: inject at x-, x+, y+, z+, reflect at y-
LUNAR = dict(reflect=4, faces=1 | 2 | 8 | 32)


def ambient(w):
    """Ambient plasma of the workload: the loaded density and thermal speeds."""
    vol = w.nx * w.ny * w.nz * w.h ** 3
    return ([s.count / vol for s in w.species], [s.vth for s in w.species],
            [tuple(s.drift) for s in w.species])


def run_pair(w, form, reflect, faces, nsteps, seed=11, split=None, patches=0):
    sp, x, v, E = inputs(w)
    dens, vth, drift = ambient(w)
    prob = problem_of(w, form)
    prob.reflect, prob.inj_faces, prob.inj_seed = reflect, faces, seed
    prob.sphere_patches = patches
    prob.inj_density, prob.inj_vth, prob.inj_drift = dens, vth, drift
    r = oracle.run(prob, sp, x, v, E, nsteps)

    ns = len(w.species)
    extra = prob.injection_bound(nsteps)
    cfg = pam.config_from_workload(w, repr=form, deposit="fixed64",
                                   capacity=[int((sp == s).sum()) + extra for s in range(ns)])
    cfg.reflect = reflect
    cfg.patches = patches
    n = len(sp)
    ids = np.arange(n, dtype=np.int64)
    with pam.Context(cfg) as ctx:
        for s in range(ns):
            m = sp == s
            ctx.load_particles(s, x[m], v[m], ids[m])
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.set_injection(faces, seed, dens, vth, drift)
        for k in (split or [nsteps]):
            ctx.step(k)
        g = dict(rho=ctx.get_rho(), counts=ctx.get_surface_charge()[1], counters=ctx.get_counters(),
                 injected=ctx.get_injected(),
                 parts=[ctx.get_particles(s) for s in range(ns)])
    return sp, r, g


def assert_same(w, sp, r, g):
    n = len(sp)
    ns = len(w.species)
    rho, rho_fixed = g["rho"]
    assert np.array_equal(rho_fixed, r.rho_fixed)
    assert np.array_equal(g["injected"], r.injected)
    alive, absorbed, escaped = g["counters"]
    assert np.array_equal(escaped, r.escaped)
    assert np.array_equal(absorbed, r.tally.sum(0))
    assert np.array_equal(g["counts"], r.tally)
    for s in range(ns):
        x, v, pid = g["parts"][s]
        assert alive[s] == int(((r.fate == 0) & (r.species == s)).sum())
        # loaded particles by id
        keep = pid >= 0
        o = np.argsort(pid[keep])
        want = np.nonzero((r.fate[:n] == 0) & (sp == s))[0]
        assert np.array_equal(pid[keep][o], want)
        assert np.array_equal(x[keep][o], r.x[want])
        assert np.array_equal(v[keep][o], r.v[want])
        # injected particles (id -1) as a set
        inj = np.nonzero((r.fate == 0) & (np.arange(len(r.fate)) >= n) & (r.species == s))[0]
        gi = np.concatenate([x[~keep], v[~keep]], 1)
        ri = np.concatenate([r.x[inj], r.v[inj]], 1)
        assert len(gi) == len(ri)
        gi = gi[np.lexsort(gi.T[::-1])]
        ri = ri[np.lexsort(ri.T[::-1])]
        assert np.array_equal(gi, ri)


@pytest.mark.parametrize("form", FORMS)
def test_oml_setup_reflect_and_inject_bit_exact(form):
    w = synth.sphere_16()
    sp, r, g = run_pair(w, form, OML["reflect"], OML["faces"], 12)
    assert r.injected.sum() > 1000
    assert_same(w, sp, r, g)


@pytest.mark.parametrize("form", FORMS)
def test_oml_setup_with_surface_patches_bit_exact(form):
    w = synth.sphere_16()
    sp, r, g = run_pair(w, form, OML["reflect"], OML["faces"], 12, patches=3)
    assert r.tally.shape[0] == 54 and r.injected.sum() > 1000
    assert_same(w, sp, r, g)


@pytest.mark.parametrize("form", ["fp64", "fp32_cell"])
def test_lunar_setup_on_a_crater_bit_exact(form):
    w = synth.scaled(synth.crater_160(), 32, 32, 16, 3.0, steps=10)
    sp, r, g = run_pair(w, form, LUNAR["reflect"], LUNAR["faces"], 10)
    assert r.injected.sum() > 1000 and r.tally.sum() > 0
    assert_same(w, sp, r, g)


def test_reflection_alone_bit_exact():
    w = synth.sphere_16()
    sp, r, g = run_pair(w, "fp32_cell", 63, 0, 15)
    assert r.escaped.sum() == 0
    assert_same(w, sp, r, g)


def test_injection_is_the_same_in_any_step_split():
    w = synth.sphere_16()
    sp, r, g = run_pair(w, "fp32_cell", OML["reflect"], OML["faces"], 9, split=[2, 3, 4])
    assert_same(w, sp, r, g)


def test_injection_settings_are_validated_on_the_context():
    w = synth.scaled(synth.crater_160(), 16, 16, 8, 1.0)
    cfg = pam.config_from_workload(w, capacity=[100, 100])
    cfg.reflect = 4
    with pam.Context(cfg) as ctx:
        for faces in (16, 4, 64):  # terrain face, a reflecting face, no such face
            with pytest.raises(pam.PicError):
                ctx.set_injection(faces, 0, [1.0, 1.0], [1.0, 1.0], [(0, 0, 0)] * 2)
        with pytest.raises(pam.PicError):
            ctx.set_injection(2, 0, [-1.0, 1.0], [1.0, 1.0], [(0, 0, 0)] * 2)
        ctx.set_injection(2, 0, [1.0, 1.0], [1.0, 1.0], [(0, 0, 0)] * 2)
        ctx.set_node_E([np.zeros(w.nodes)] * 3)
        b = pam.Batch(2, "fp32_cell", "fixed64", 4, 1 << 36)
        try:
            with pytest.raises(pam.PicError):
                b.attach(ctx, 3)  # injecting contexts run alone
        finally:
            b.close()
