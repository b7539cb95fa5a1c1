"""The overflow list at the full lunar-crater grid size, bit for bit against
the oracle: on 160 x 160 x 80 cells (32,000 tiles) the step kernel splits the
list over 32 workgroups, each a contiguous part of it. Dense clusters that
drift across tile faces overflow the arrival zones of the tiles they enter
every step; in a batched run nothing is re-planned between the steps of a
run, so the later steps of each run push the particles held in the list
through those workgroups, and through pic_step the queued steps do the same
until the host sees the re-planning request."""
import numpy as np
import pytest

import paper_2011_10214_amd as pam
import synth
from oracle import oracle

from gpu_util import run_gpu
from helpers import problem_of
from test_parity_gpu import assert_bit_exact

pytestmark = pytest.mark.gpu

FORMS = ["fp64", "fp32_abs", "fp32_cell"]


def workload():
    sp = [synth.SpeciesSpec("electron", q=-1.0, m=1.0, vth=1.0, count=0),
          synth.SpeciesSpec("ion", q=1.0, m=100.0, vth=0.1, count=0)]
    return synth.Workload(name="overflow_160x160x80", nx=160, ny=160, nz=80, species=sp,
                          dt=0.05)


def clusters(seed):
    """Three electron clusters of 12,000 in one tile each, drifting at about
    half a cell per step along +x, -y and +z (each step an eighth of a
    cluster enters a tile planned for 64 arrivals), and 3,000 slow ions over
    the whole box."""
    w = workload()
    rng = np.random.default_rng(seed)
    xs, vs = [], []
    for lo, drift in (((40.0, 40.0, 20.0), (10.0, 0.0, 0.0)),
                      ((100.0, 120.0, 40.0), (0.0, -10.0, 0.0)),
                      ((20.0, 140.0, 8.0), (0.0, 0.0, 10.0))):
        n = 12000
        xs.append(np.asarray(lo) + rng.uniform(0.0, 4.0, size=(n, 3)))
        vs.append(np.asarray(drift) + rng.normal(0.0, 0.5, size=(n, 3)))
    ne = sum(len(a) for a in xs)
    ni = 3000
    xs.append(rng.uniform(0.0, 1.0, size=(ni, 3)) * [w.nx, w.ny, w.nz])
    vs.append(rng.normal(0.0, 0.1, size=(ni, 3)))
    sp = np.concatenate([np.zeros(ne, np.int32), np.ones(ni, np.int32)])
    E = rng.uniform(-0.1, 0.1, size=(3, w.nodes))
    return w, sp, np.vstack(xs), np.vstack(vs), E


def test_the_grid_splits_the_overflow_list_over_32_workgroups():
    # the split under test: one overflow workgroup per 1000 tiles, at most 32
    w = workload()
    tiles = -(-w.nx // 4) * -(-w.ny // 4) * -(-w.nz // 4)
    assert tiles == 32000 and min(32, max(1, tiles // 1000)) == 32


@pytest.mark.parametrize("form", FORMS)
def test_overflow_list_over_many_workgroups_through_a_batch(form):
    w, sp, x, v, E = clusters(41)
    nsteps = 16
    r = oracle.run(problem_of(w, form), sp, x, v, E, nsteps)
    g = run_gpu(w, sp, x, v, E, nsteps, repr=form, spare=40.0, profile=True,
                batch_steps_per_run=4)
    assert_bit_exact(w, sp, r, g)
    # the load's re-planning, then the clusters' requests between runs
    assert g.profile.sort_launches >= 3


@pytest.mark.parametrize("form", FORMS)
def test_overflow_list_over_many_workgroups_through_pic_step(form):
    w, sp, x, v, E = clusters(43)
    nsteps = 16
    r = oracle.run(problem_of(w, form), sp, x, v, E, nsteps)
    # all steps queued at once: the requests reach the host late and the
    # overflow workgroups push the listed particles meanwhile
    g = run_gpu(w, sp, x, v, E, nsteps, repr=form, spare=40.0)
    assert_bit_exact(w, sp, r, g)
    # every step re-planned as soon as it asks: the same results
    g2 = run_gpu(w, sp, x, v, E, nsteps, repr=form, spare=40.0, sync_steps=True)
    assert_bit_exact(w, sp, r, g2)


def test_overflowing_clusters_fill_the_list_each_step():
    # the premise of the tests above, on the CPU side of the contract: each
    # cluster sends far more particles into a neighbouring tile per step than
    # the 64 arrivals a tile planned empty has room for
    w, sp, x, v, E = clusters(41)
    r = oracle.run(problem_of(w, "fp64"), sp, x, v, E, 1)
    tile = (np.floor(r.x / 4.0)).astype(int)
    tile0 = (np.floor(x / 4.0)).astype(int)
    moved = (r.fate == 0) & (sp == 0) & (tile != tile0).any(axis=1)
    assert moved.sum() > 3 * 64 * 4
