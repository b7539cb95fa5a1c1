"""Edge cases of the hot path on the GPU, bit for bit against the oracle in
every representation: empty species and a single particle; the smallest and
ragged meshes (partial tiles on every face); the largest cell count per axis;
particles exactly on nodes, cell faces and just below the upper box faces;
fast particles that cross several cells per step (their deposit falls
outside the tile's staged region and takes the global path) and leave
through every face; a sphere that touches the box."""
import numpy as np
import pytest

import synth
from oracle import oracle

from gpu_util import run_gpu
from helpers import problem_of
from test_parity_gpu import assert_bit_exact

pytestmark = pytest.mark.gpu

FORMS = ["fp64", "fp32_abs", "fp32_cell"]


def workload(nx, ny, nz, counts=(1, 1), obj="none", center=(0.0, 0.0, 0.0), radius=0.0, dt=0.05):
    sp = [synth.SpeciesSpec("electron", q=-1.0, m=1.0, vth=1.0, count=counts[0]),
          synth.SpeciesSpec("ion", q=1.0, m=100.0, vth=0.1, count=counts[1])]
    return synth.Workload(name=f"edge_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, species=sp, obj=obj,
                          center=center, radius=radius, dt=dt)


def field(w, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=(3, w.nodes))


def check(w, sp, x, v, E, nsteps, form):
    r = oracle.run(problem_of(w, form), sp, x, v, E, nsteps)
    g = run_gpu(w, sp, x, v, E, nsteps, repr=form)
    assert_bit_exact(w, sp, r, g)
    return r


@pytest.mark.parametrize("form", FORMS)
def test_empty_species_and_a_single_particle(form):
    w = workload(8, 8, 8)
    sp = np.array([1], np.int32)  # no electrons, one ion
    x = np.array([[3.25, 4.5, 5.75]])
    v = np.array([[0.3, -0.2, 0.1]])
    r = check(w, sp, x, v, field(w, 1), 7, form)
    assert (r.fate == 0).sum() == 1
    w0 = workload(4, 4, 4)
    check(w0, np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros((0, 3)), field(w0, 2), 3, form)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n", [(1, 1, 1), (3, 2, 5), (5, 9, 7)])
def test_smallest_and_ragged_meshes(form, n):
    w = workload(*n)
    rng = np.random.default_rng(sum(n))
    m = 300
    sp = rng.integers(0, 2, m).astype(np.int32)
    x = rng.uniform(0, 1, (m, 3)) * np.array(n)
    v = rng.normal(0, 0.5, (m, 3))
    check(w, sp, x, v, field(w, 3, 0.5), 12, form)


@pytest.mark.parametrize("form", FORMS)
def test_largest_cell_count_per_axis(form):
    w = workload(1023, 2, 1)
    rng = np.random.default_rng(4)
    m = 4000
    sp = rng.integers(0, 2, m).astype(np.int32)
    x = rng.uniform(0, 1, (m, 3)) * np.array([1023, 2, 1])
    v = rng.normal(0, 2.0, (m, 3))
    check(w, sp, x, v, field(w, 5), 8, form)


@pytest.mark.parametrize("form", FORMS)
def test_particles_on_nodes_faces_and_just_below_the_upper_faces(form):
    n = (6, 5, 4)
    w = workload(*n)
    pts = []
    for i in range(n[0]):
        for j in range(n[1]):
            pts.append((i, j, 2.0))            # on nodes
            pts.append((i + 0.5, j, 1.5))      # on a face of the y grid
    # the largest FP32 value below each upper face (exact in every form)
    top = np.nextafter(np.array(n, np.float32), np.float32(0)).astype(float)
    pts += [tuple(top), (top[0], 0.0, 0.0), (0.0, top[1], 2.5), (1.5, 2.5, top[2])]
    x = np.array(pts, float)
    m = len(x)
    sp = (np.arange(m) % 2).astype(np.int32)
    v = np.zeros((m, 3))
    check(w, sp, x, v, np.zeros((3, w.nodes)), 0, form)   # deposit only
    rng = np.random.default_rng(6)
    check(w, sp, x, rng.normal(0, 0.3, (m, 3)), field(w, 7, 0.2), 5, form)


@pytest.mark.parametrize("form", FORMS)
def test_fast_particles_deposit_outside_their_tile_and_leave_through_every_face(form):
    # up to ~6 cells per step: moves far beyond the staged tile halo
    w = workload(16, 12, 10, dt=0.5)
    rng = np.random.default_rng(8)
    m = 3000
    sp = rng.integers(0, 2, m).astype(np.int32)
    x = rng.uniform(0, 1, (m, 3)) * np.array([16, 12, 10])
    v = rng.normal(0, 4.0, (m, 3)) * np.where(sp[:, None] == 0, 1.0, 10.0)
    r = check(w, sp, x, v, field(w, 9, 2.0), 6, form)
    assert np.all(r.escaped.sum(1) > 0)  # every face saw an escape


@pytest.mark.parametrize("form", FORMS)
def test_sphere_touching_the_box(form):
    w = workload(12, 12, 12, obj="sphere", center=(3.0, 6.0, 6.0), radius=3.0)
    rng = np.random.default_rng(10)
    m = 5000
    sp = rng.integers(0, 2, m).astype(np.int32)
    x = rng.uniform(0, 12, (m, 3))
    keep = np.sum((x - np.array(w.center)) ** 2, 1) > 9.0
    sp, x = sp[keep], x[keep]
    v = rng.normal(0, 1.0, (len(x), 3))
    r = check(w, sp, x, v, field(w, 11), 10, form)
    assert r.tally.sum() > 0 and r.escaped[0].sum() > 0


@pytest.mark.parametrize("device", [False, True])
def test_position_that_rounds_up_onto_the_upper_face_is_refused(device):
    # x = 8 with the origin 1e-8 lies 1e-8 below the upper face of an 8-cell
    # box: inside in FP64, but its FP32 coordinate rounds up to 8 (the face);
    # the FP32 forms refuse it (absolute: rounded onto the face; cell-relative:
    # the offset rounds up to 1 and the particle into cell 8), the FP64 form
    # takes it
    import torch

    import paper_2011_10214_amd as pam

    w = workload(8, 8, 8)
    x = np.array([[8.0, 3.5, 3.5], [2.0, 8.0, 3.5], [2.0, 2.0, 8.0]])
    v = np.zeros_like(x)
    for form in FORMS:
        cfg = pam.config_from_workload(w, repr=form, capacity=[4, 4])
        cfg.origin = (1e-8, 1e-8, 1e-8)
        with pam.Context(cfg) as ctx:
            for k in range(3):
                xs = x[k:k + 1]
                if device:
                    xs = torch.tensor(xs, dtype=torch.float32, device="cuda")
                    vs = torch.zeros_like(xs)
                else:
                    vs = v[k:k + 1]
                if form == "fp64":
                    ctx.load_particles(0, xs, vs)
                    continue
                with pytest.raises(pam.PicError) as ei:
                    ctx.load_particles(0, xs, vs)
                assert ei.value.status == pam.pic.E_INVALID
