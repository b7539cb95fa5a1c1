"""Photoemission from the sunlit crater terrain on the GPU against the oracle
(the lunar setup of §5.2.2 with its photoelectrons): bit for bit in every
representation with the fixed-point deposit, together with the ambient
injection and the symmetry plane: loaded particles by id, injected and
emitted particles as a set, rho, tallies, escapes and injected counts; the
same in any step split; settings checks."""
import math
from dataclasses import replace

import numpy as np
import pytest

import paper_2011_10214_amd as pam
import synth
from oracle import oracle

from gpu_util import inputs
from helpers import problem_of
from test_boundaries_gpu import LUNAR, ambient, assert_same

pytestmark = pytest.mark.gpu

ELEV = math.radians(10.0)
SUN = (math.cos(ELEV), 0.0, math.sin(ELEV))
PHOTO = synth.SpeciesSpec("photoelectron", q=-1.0, m=1.0, vth=0.43, count=0)


def lunar_with_photoelectrons():
    w = synth.scaled(synth.crater_160(), 32, 32, 16, 2.0, steps=8)
    return replace(w, species=list(w.species) + [PHOTO])


def run_pair(w, form, nsteps, split=None, flux=30.0, seed=21):
    sp, x, v, E = inputs(w)
    dens, vth, drift = ambient(w)
    dens[2] = 0.0  # photoelectrons only come from the ground
    prob = problem_of(w, form)
    prob.reflect, prob.inj_faces, prob.inj_seed = LUNAR["reflect"], LUNAR["faces"], 11
    prob.inj_density, prob.inj_vth, prob.inj_drift = dens, vth, drift
    prob.pe_species, prob.pe_seed, prob.pe_sun, prob.pe_flux, prob.pe_vth = 2, seed, SUN, flux, PHOTO.vth
    r = oracle.run(prob, sp, x, v, E, nsteps)

    extra = prob.injection_bound(nsteps)
    cfg = pam.config_from_workload(w, repr=form, deposit="fixed64",
                                   capacity=[int((sp == s).sum()) + extra for s in range(3)])
    cfg.reflect = LUNAR["reflect"]
    ids = np.arange(len(sp), dtype=np.int64)
    with pam.Context(cfg) as ctx:
        for s in range(3):  # no photoelectrons are loaded: an empty load gives them ids
            m = sp == s
            ctx.load_particles(s, x[m], v[m], ids[m])
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.set_injection(LUNAR["faces"], 11, dens, vth, drift)
        ctx.set_photoemission(2, seed, SUN, flux, PHOTO.vth)
        for k in (split or [nsteps]):
            ctx.step(k)
        g = dict(rho=ctx.get_rho(), counts=ctx.get_surface_charge()[1], counters=ctx.get_counters(),
                 injected=ctx.get_injected(), parts=[ctx.get_particles(s) for s in range(3)])
    return sp, r, g


@pytest.mark.parametrize("form", ["fp64", "fp32_abs", "fp32_cell"])
def test_photoemission_bit_exact(form):
    w = lunar_with_photoelectrons()
    sp, r, g = run_pair(w, form, 8)
    assert r.injected[2] > 1000 and r.tally[:, 2].sum() > 0
    assert_same(w, sp, r, g)


def test_photoemission_is_the_same_in_any_step_split():
    w = lunar_with_photoelectrons()
    sp, r, g = run_pair(w, "fp32_cell", 7, split=[2, 1, 4])
    assert_same(w, sp, r, g)


def test_photoemission_settings_are_checked():
    w = lunar_with_photoelectrons()
    cfg = pam.config_from_workload(w, capacity=[10, 10, 10])
    with pam.Context(cfg) as ctx:
        for kw in (dict(species=3), dict(species=2, sun=(1.0, 0.0, 0.0)),
                   dict(species=2, flux=-1.0), dict(species=2, vth=float("inf"))):
            with pytest.raises(pam.PicError):
                ctx.set_photoemission(**kw)
        ctx.set_photoemission(2, 0, SUN, 1.0, 1.0)
        ctx.set_photoemission(None)
    s = synth.sphere_16()
    with pam.Context(pam.config_from_workload(s, capacity=[10, 10])) as ctx:
        with pytest.raises(pam.PicError):
            ctx.set_photoemission(0, 0, SUN, 1.0, 1.0)  # no terrain
