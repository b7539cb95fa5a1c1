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


def test_closed_lunar_loop_follows_the_oracle():
    # the benchmarked loop at a small size: ambient injection, the symmetry
    # plane and photoemission, then after every step a field solve with the
    # terrain as an interface and the collected charge as its surface source.
    # The oracle runs step by step (each run continued from its step index)
    # with its own field solve; the two solves agree to rounding, so positions
    # are compared within 1e-9 and the counts exactly
    w = lunar_with_photoelectrons()
    nsteps, mask, tol, eps_in = 4, 32, 1e-12, 4.0
    sp, x, v, _ = inputs(w)
    dens, vth, drift = ambient(w)
    dens[2] = 0.0
    prob = problem_of(w, "fp64")
    prob.reflect, prob.inj_faces, prob.inj_seed = LUNAR["reflect"], LUNAR["faces"], 11
    prob.inj_density, prob.inj_vth, prob.inj_drift = dens, vth, drift
    prob.pe_species, prob.pe_seed, prob.pe_sun, prob.pe_flux, prob.pe_vth = 2, 21, SUN, 30.0, PHOTO.vth
    obj = oracle.field_object_of(prob, eps_in)
    E = np.zeros((3, w.nodes))
    ox, ov, osp, oid = x.copy(), v.copy(), sp.copy(), np.arange(len(sp))
    tally = np.zeros((prob.nbins, 3), np.int64)
    injected = np.zeros(3, np.int64)
    for k in range(nsteps):
        prob.first_step = k
        r = oracle.run(prob, osp, ox, ov, E, 1)
        tally += r.tally
        injected += r.injected
        ids = np.concatenate([oid, np.full(len(r.x) - len(oid), -1)])
        alive = r.fate == 0
        ox, ov, osp, oid = r.x[alive], r.v[alive], r.species[alive], ids[alive]
        rho = (r.rho_fixed + oracle.surface_rho(prob, tally)) * 2.0 ** -32
        phi, _, _ = oracle.field_solve(w.nx, w.ny, w.nz, rho, mask, tol=tol, max_iter=5000, obj=obj)
        E = oracle.field_E(w.nx, w.ny, w.nz, phi, mask)
    assert injected[2] > 100 and tally.sum() > 0

    prob.first_step = 0
    cfg = pam.config_from_workload(w, repr="fp64", deposit="fixed64",
                                   capacity=[int((sp == s).sum()) + prob.injection_bound(nsteps)
                                             for s in range(3)])
    cfg.reflect = LUNAR["reflect"]
    with pam.Context(cfg) as ctx:
        for s in range(3):
            m = sp == s
            ctx.load_particles(s, x[m], v[m], np.arange(len(sp), dtype=np.int64)[m])
        ctx.set_node_E([np.zeros(w.nodes)] * 3)
        ctx.set_injection(LUNAR["faces"], 11, dens, vth, drift)
        ctx.set_photoemission(2, 21, SUN, 30.0, PHOTO.vth)
        for _ in range(nsteps):
            ctx.step(1)
            ctx.solve_field(mask, tol=tol, max_iter=5000, eps_object=eps_in, surface_charge=True)
        gphi = ctx.get_phi()
        counts = ctx.get_surface_charge()[1]
        g_injected = ctx.get_injected()
        parts = [ctx.get_particles(s) for s in range(3)]
    assert np.array_equal(counts, tally)
    assert np.array_equal(g_injected, injected)
    for s in range(3):
        gx, gv, gid = parts[s]
        m = osp == s
        assert len(gid) == int(m.sum())
        # loaded particles by id
        keep = gid >= 0
        o = np.argsort(gid[keep])
        want = np.nonzero(m & (oid >= 0))[0]
        want = want[np.argsort(oid[want])]
        assert np.array_equal(gid[keep][o], oid[want])
        assert np.abs(gx[keep][o] - ox[want]).max(initial=0.0) < 1e-9
        assert np.abs(gv[keep][o] - ov[want]).max(initial=0.0) < 1e-9
        # injected and emitted particles as a set
        gi = np.concatenate([gx[~keep], gv[~keep]], 1)
        ri = np.concatenate([ox[m & (oid < 0)], ov[m & (oid < 0)]], 1)
        assert len(gi) == len(ri)
        gi, ri = gi[np.lexsort(gi.T[::-1])], ri[np.lexsort(ri.T[::-1])]
        assert np.abs(gi - ri).max(initial=0.0) < 1e-9
    assert np.abs(gphi - phi).max() < 1e-8 * np.abs(phi).max()
