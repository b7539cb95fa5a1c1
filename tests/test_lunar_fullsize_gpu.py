"""The lunar boundary setup on the full crater_160 grid (160 x 160 x 80 cells,
32,000 tiles, the overflow list over 32 workgroups), in the launch
configuration of the closed loop's particle half: the step kernel with the
code of reflecting faces (y- reflects) and the injection of the ambient
plasma at x-, x+, y+ and z+ with the density and thermal speeds of the full
520 M-particle workload, so that the injection runs over all of its ghost
slots (about 3.2 M per step); with photoemission too, from the sunlit
terrain at the flux of the closed loop's photoelectrons (Sun 10 degrees above
the ground), over all 25,600 surface columns. The loaded particles are a
seeded sample of the workload's (particles are independent of each other
under a fixed node field), so that the oracle finishes in seconds; the
injected and emitted ones are all there are. Bit for bit against the oracle:
loaded particles by id, injected and emitted particles as a set, rho,
tallies, escapes and injected counts."""
import math
import os
from dataclasses import replace

import numpy as np
import pytest

import paper_2011_10214_amd as pam
import synth
from oracle import oracle

from helpers import problem_of
from test_boundaries_gpu import LUNAR, ambient, assert_same

pytestmark = pytest.mark.gpu

STEPS = 3
SAMPLE = 1 << 16


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _photoelectrons(w):
    """The photoelectron species and emission settings of the closed loop:
    n_pe / n_sw = 64 / 8.7 and vth_pe / vth_e = 622 / 1453 (the paper's
    plasma parameters), the flux of a half-Maxwellian of that density at
    normal incidence, the Sun 10 degrees above the ground along +x."""
    e = w.species[0]
    above = w.nx * w.ny * (w.nz - w.z_flat) * w.h ** 3
    vth = e.vth * 622.0 / 1453.0
    flux = (64.0 / 8.7) * (e.count / above) * vth * math.sqrt(2.0 / math.pi)
    elev = math.radians(10.0)
    spec = synth.SpeciesSpec("photoelectron", q=-1.0, m=e.m, vth=vth, count=0, w=e.w)
    return spec, dict(seed=23, sun=(math.cos(elev), 0.0, math.sin(elev)), flux=flux, vth=vth)


@pytest.mark.parametrize("photo", [False, True])
def test_lunar_setup_on_the_full_grid_bit_exact(photo):
    w = synth.crater_160()
    assert (w.nx, w.ny, w.nz) == (160, 160, 80)
    pe = None
    if photo:
        spec, pe = _photoelectrons(w)
        w = replace(w, species=list(w.species) + [spec])
    rng = np.random.default_rng(1600)
    idx = [np.sort(rng.choice(s.count, SAMPLE, replace=False)) if s.count else
           np.zeros(0, np.int64) for s in w.species]
    sp = np.concatenate([np.full(len(i), s, np.int32) for s, i in enumerate(idx)])
    parts = [synth.particles(w, s, idx=i) for s, i in enumerate(idx) if len(i)]
    x = np.concatenate([np.stack(p[:3], 1) for p in parts]).astype(np.float64)
    v = np.concatenate([np.stack(p[3:], 1) for p in parts]).astype(np.float64)
    E = [np.asarray(e, np.float64) for e in synth.node_E(w)]
    dens, vth, drift = ambient(w)
    if photo:
        dens[2] = 0.0  # photoelectrons only come from the ground
    reflect, faces, seed = LUNAR["reflect"], LUNAR["faces"], 21

    prob = problem_of(w, "fp32_cell")
    prob.threads = _threads()
    prob.reflect, prob.inj_faces, prob.inj_seed = reflect, faces, seed
    prob.inj_density, prob.inj_vth, prob.inj_drift = dens, vth, drift
    if photo:
        prob.pe_species, prob.pe_seed, prob.pe_sun = 2, pe["seed"], pe["sun"]
        prob.pe_flux, prob.pe_vth = pe["flux"], pe["vth"]
    r = oracle.run(prob, sp, x, v, E, STEPS)
    print(f"oracle: {r.injected.tolist()} injected or emitted in {STEPS} steps, "
          f"{int(r.tally.sum())} collected, {int(r.escaped.sum())} escaped", flush=True)

    ns = len(w.species)
    extra = prob.injection_bound(STEPS)
    cfg = pam.config_from_workload(w, repr="fp32_cell", deposit="fixed64",
                                   capacity=[int((sp == s).sum()) + extra for s in range(ns)])
    cfg.reflect = reflect
    ids = np.arange(len(sp), dtype=np.int64)
    with pam.Context(cfg) as ctx:
        for s in range(ns):
            m = sp == s
            ctx.load_particles(s, x[m], v[m], ids[m])
        ctx.set_node_E(E)
        ctx.set_injection(faces, seed, dens, vth, drift)
        if photo:
            ctx.set_photoemission(2, **pe)
        ctx.step(STEPS)
        g = dict(rho=ctx.get_rho(), counts=ctx.get_surface_charge()[1],
                 counters=ctx.get_counters(), injected=ctx.get_injected(),
                 parts=[ctx.get_particles(s) for s in range(ns)])
    assert r.injected[:2].sum() > 100_000 and r.tally.sum() > 0
    if photo:
        assert r.injected[2] > 10_000 and r.tally[:, 2].sum() > 0
    assert r.escaped[2].sum() == 0  # y- reflects: nothing leaves there
    assert_same(w, sp, r, g)
