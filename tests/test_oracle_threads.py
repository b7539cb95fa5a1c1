"""The oracle on several threads (the particle updates in parallel, the
fixed-point deposit in one int64 array per thread added in thread order)
gives the same bits as on one thread: positions, velocities, fates, tallies,
escapes, injected counts and rho, in every representation, with the sphere
and the crater, reflection, injection and photoemission; and a runaway
particle is still a range error."""
import math
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import oracle

from helpers import problem_of

FORMS = ["fp64", "fp32_abs", "fp32_cell"]


def same(a, b):
    assert np.array_equal(a.fate, b.fate) and np.array_equal(a.where, b.where)
    assert np.array_equal(a.when, b.when)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    assert np.array_equal(a.rho_fixed, b.rho_fixed) and np.array_equal(a.rho, b.rho)
    assert np.array_equal(a.tally, b.tally) and np.array_equal(a.escaped, b.escaped)
    assert np.array_equal(a.injected, b.injected)


@pytest.mark.parametrize("form", FORMS)
def test_sphere_runs_the_same_on_any_number_of_threads(form):
    w = synth.sphere_16()
    sp, x, v = synth.all_particles(w)
    E = synth.node_E(w)
    prob = problem_of(w, form)
    prob.sphere_patches = 2
    one = oracle.run(prob, sp, x, v, E, 6)
    assert one.tally.sum() > 0 and one.escaped.sum() > 0
    for t in (2, 5):
        same(one, oracle.run(replace(prob, threads=t), sp, x, v, E, 6))


@pytest.mark.parametrize("form", FORMS)
def test_lunar_boundaries_run_the_same_on_any_number_of_threads(form):
    w = synth.scaled(synth.crater_160(), 24, 24, 12, 2.0, steps=4)
    w = replace(w, species=list(w.species) + [synth.SpeciesSpec(
        "photoelectron", q=-1.0, m=1.0, vth=0.43, count=0)])
    sp, x, v = synth.all_particles(w)
    E = synth.node_E(w)
    vol = w.nx * w.ny * w.nz
    prob = problem_of(w, form)
    prob.reflect, prob.inj_faces, prob.inj_seed = 4, 1 | 2 | 8 | 32, 3
    prob.inj_density = [s.count / vol for s in w.species]
    prob.inj_vth = [s.vth for s in w.species]
    prob.inj_drift = [tuple(s.drift) for s in w.species]
    el = math.radians(10.0)
    prob.pe_species, prob.pe_seed, prob.pe_sun = 2, 5, (math.cos(el), 0.0, math.sin(el))
    prob.pe_flux, prob.pe_vth = 30.0, 0.43
    one = oracle.run(prob, sp, x, v, E, 4)
    assert one.injected[2] > 0 and one.tally.sum() > 0
    same(one, oracle.run(replace(prob, threads=4), sp, x, v, E, 4))


def test_summing_deposits_stay_on_one_thread():
    # the FP32 / FP64 summing deposits depend on the order: the threaded run
    # keeps them sequential, so they too are unchanged
    w = synth.sphere_16()
    sp, x, v = synth.all_particles(w)
    E = synth.node_E(w)
    for dep in ("fp32", "fp64"):
        prob = problem_of(w, "fp32_cell", deposit=dep)
        a = oracle.run(prob, sp, x, v, E, 3)
        b = oracle.run(replace(prob, threads=3), sp, x, v, E, 3)
        assert np.array_equal(a.rho, b.rho) and np.array_equal(a.x, b.x)


@pytest.mark.parametrize("form", FORMS)
def test_runaway_particle_is_a_range_error_on_threads(form):
    w = synth.sphere_16()
    sp, x, v = synth.all_particles(w)
    # the cell form moves more than 2^20 cells; the absolute forms turn NaN
    big = 1e37 if form == "fp32_cell" else np.nan
    E = [np.full(w.nodes, big), np.zeros(w.nodes), np.zeros(w.nodes)]
    with pytest.raises(oracle.OracleError, match="-5"):
        oracle.run(replace(problem_of(w, form), threads=3), sp, x, v, E, 1)
