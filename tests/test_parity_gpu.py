"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Same arithmetic -> bit-exact: the FP64 form against the FP64 oracle and the two
FP32 forms against the oracle's FP32 mirrors, for every output (positions,
velocities, the alive set, collected and escaped counts, fixed-point rho).
Across precisions (FP32 GPU vs FP64 oracle): positions and velocities within
1e-5 relative after 100 steps, and fates differ only for particles within 1e-4
cells of a deciding surface.
"""
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import oracle

from gpu_util import inputs, run_gpu
from helpers import check_mismatches_near_surface, problem_of

pytestmark = pytest.mark.gpu

FORMS = ["fp64", "fp32_abs", "fp32_cell"]


def assert_bit_exact(w, sp, r, g, deposit="fixed64"):
    alive = np.nonzero(r.fate == 0)[0]
    assert np.array_equal(g.alive_ids, alive), (len(g.alive_ids), len(alive))
    assert np.array_equal(g.x, r.x[alive])
    assert np.array_equal(g.v, r.v[alive])
    assert np.array_equal(g.escaped, r.escaped)
    assert np.array_equal(g.absorbed, r.tally.sum(0))
    if r.tally.shape[0]:
        assert np.array_equal(g.counts, r.tally)
    ns = len(w.species)
    assert np.array_equal(g.alive, np.array([((r.fate == 0) & (sp == s)).sum() for s in range(ns)]))
    if deposit == "fixed64":
        assert np.array_equal(g.rho_fixed, r.rho_fixed)
        assert np.array_equal(g.rho, r.rho)


@pytest.mark.parametrize("form", FORMS)
def test_sphere16_bit_exact(form):
    w = synth.sphere_16()
    sp, x, v, E = inputs(w)
    r = oracle.run(problem_of(w, form), sp, x, v, E, w.steps)
    g = run_gpu(w, sp, x, v, E, w.steps, repr=form)
    assert_bit_exact(w, sp, r, g)
    assert np.array_equal(g.charge, r.charge(problem_of(w, form)))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("m", [1, 4])
def test_sphere_surface_patches_bit_exact(form, m):
    # 6 m^2 tally bins on the sphere: per-patch counts and charges as the oracle's
    w = synth.sphere_16()
    sp, x, v, E = inputs(w)
    prob = problem_of(w, form)
    prob.sphere_patches = m
    r = oracle.run(prob, sp, x, v, E, w.steps)
    g = run_gpu(w, sp, x, v, E, w.steps, repr=form, patches=m)
    assert r.tally.shape[0] == 6 * m * m and (r.tally.sum(1) > 0).sum() > min(6 * m * m // 2, 6)
    assert_bit_exact(w, sp, r, g)
    assert np.array_equal(g.charge, r.charge(prob))


@pytest.mark.parametrize("form", FORMS)
def test_deposit_only_bit_exact(form):
    w = synth.sphere_16()
    sp, x, v, E = inputs(w)
    r = oracle.run(problem_of(w, form), sp, x, v, E, 0)
    g = run_gpu(w, sp, x, v, E, 0, repr=form)
    assert np.array_equal(g.rho_fixed, r.rho_fixed)


@pytest.mark.parametrize("form", FORMS)
def test_sphere_ragged_multi_tile_bit_exact(form):
    # 29 x 22 x 19 cells: partial tiles on every upper face; sphere off-centre
    w = synth.scaled(synth.sphere_64(), 29, 22, 19, ppc=7, steps=30, name="sphere_ragged")
    w = replace(w, center=(13.3, 10.9, 9.2), radius=4.1)
    sp, x, v, E = inputs(w)
    r = oracle.run(problem_of(w, form), sp, x, v, E, w.steps)
    g = run_gpu(w, sp, x, v, E, w.steps, repr=form)
    assert_bit_exact(w, sp, r, g)


@pytest.mark.parametrize("form", FORMS)
def test_crater_bit_exact(form):
    w = synth.scaled(synth.crater_160(), 40, 40, 20, ppc=6, steps=25, name="crater_40")
    sp, x, v, E = inputs(w)
    r = oracle.run(problem_of(w, form), sp, x, v, E, w.steps)
    g = run_gpu(w, sp, x, v, E, w.steps, repr=form)
    assert r.tally.sum() > 0
    assert_bit_exact(w, sp, r, g)
    assert np.array_equal(g.charge, r.charge(problem_of(w, form)))


def test_device_load_path_matches_host_load_path():
    w = synth.scaled(synth.crater_160(), 24, 24, 12, ppc=5, steps=12, name="crater_24")
    sp, x, v, E = inputs(w)
    a = run_gpu(w, sp, x, v, E, w.steps, repr="fp32_cell")
    b = run_gpu(w, sp, x, v, E, w.steps, repr="fp32_cell", device_load=True)
    assert np.array_equal(a.alive_ids, b.alive_ids)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    assert np.array_equal(a.rho_fixed, b.rho_fixed)


@pytest.mark.parametrize("form", ["fp64", "fp32_cell"])
def test_invariance_to_sort_interval_order_and_step_split(form):
    w = synth.scaled(synth.sphere_64(), 20, 20, 20, ppc=6, steps=24, name="sphere_20")
    sp, x, v, E = inputs(w)
    base = run_gpu(w, sp, x, v, E, w.steps, repr=form, sort_interval=4)
    perm = np.random.default_rng(7).permutation(len(sp))
    for kw in (dict(sort_interval=1), dict(sort_interval=7), dict(sort_interval=1000),
               dict(order=perm), dict(split_steps=[5, 0, 11, 8])):
        g = run_gpu(w, sp, x, v, E, w.steps, repr=form, **{"sort_interval": 4, **kw})
        assert np.array_equal(g.alive_ids, base.alive_ids), kw
        assert np.array_equal(g.x, base.x) and np.array_equal(g.v, base.v), kw
        assert np.array_equal(g.rho_fixed, base.rho_fixed), kw
        assert np.array_equal(g.escaped, base.escaped), kw


def test_reruns_are_bit_identical():
    w = synth.scaled(synth.sphere_64(), 16, 16, 16, ppc=10, steps=20, name="sphere_16b")
    sp, x, v, E = inputs(w)
    runs = [run_gpu(w, sp, x, v, E, w.steps, repr="fp32_cell") for _ in range(3)]
    for g in runs[1:]:
        assert np.array_equal(g.rho_fixed, runs[0].rho_fixed)
        assert np.array_equal(g.x, runs[0].x)


@pytest.mark.parametrize("deposit", ["fp64", "fp32"])
def test_atomic_deposits_within_rounding_of_the_oracle(deposit):
    w = synth.sphere_16()
    sp, x, v, E = inputs(w)
    for form in ("fp64", "fp32_cell"):
        r = oracle.run(problem_of(w, form, deposit=deposit), sp, x, v, E, w.steps)
        g = run_gpu(w, sp, x, v, E, w.steps, repr=form, deposit=deposit)
        alive = np.nonzero(r.fate == 0)[0]
        assert np.array_equal(g.alive_ids, alive)
        assert np.array_equal(g.x, r.x[alive])
        # order-dependent rounding: |drho| <= (contributions per node) * eps * |partial sums|
        eps = 2.0 ** -52 if deposit == "fp64" else 2.0 ** -23
        scale = 8 * 64 * eps * max(1.0, np.abs(r.rho).max())
        assert np.abs(g.rho - r.rho).max() <= scale
        assert abs(g.rho.sum() - r.rho.sum()) <= len(alive) * 8 * eps * 4


def test_fp32_forms_within_tolerance_of_fp64_oracle():
    w = synth.scaled(synth.sphere_64(), 24, 24, 24, ppc=6, steps=100, name="sphere_24")
    sp, x, v, E = inputs(w)
    r64 = oracle.run(problem_of(w, "fp64"), sp, x, v, E, w.steps)
    g = run_gpu(w, sp, x, v, E, w.steps, repr="fp32_cell")
    alive64 = set(np.nonzero(r64.fate == 0)[0].tolist())
    both = np.array(sorted(alive64 & set(g.alive_ids.tolist())))
    gi = np.searchsorted(g.alive_ids, both)
    vth = np.where(sp[both] == 0, 1.0, 0.1)
    dx = np.abs(g.x[gi] - r64.x[both]).max(axis=1)
    dv = np.abs(g.v[gi] - r64.v[both]).max(axis=1)
    assert np.all(dx <= 1e-5 * np.maximum(np.abs(r64.x[both]).max(axis=1), 1.0))
    assert np.all(dv <= 1e-5 * np.maximum(np.abs(r64.v[both]).max(axis=1), vth))
    # particles alive in one run only: near a deciding surface in the FP64 run
    only = sorted(alive64 ^ set(g.alive_ids.tolist()))
    assert len(only) <= 1e-3 * len(sp)
    r32 = oracle.run(problem_of(w, "fp32_cell"), sp, x, v, E, w.steps)
    dist = check_mismatches_near_surface(w, sp, x, v, E, only, r64.when, r64.fate, r32.when,
                                         r32.fate)
    assert np.all(dist <= 1e-4)
