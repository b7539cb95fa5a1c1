"""Pins of the sphere's surface patches (where on the sphere the collected
charge sits: the surface charge distribution behind the flux jump of eq.
(2.5)): each patch centre falls in its own patch, mirror images fall in the
mirrored patch, ties go to the lower axis, uniformly spread directions fill
the six cube faces evenly, and in a whole run the patches only split the
one-bin tally (the same particles collected at the same steps) in all three
representations."""
import numpy as np
import pytest

import synth
from oracle import oracle
from oracle.oracle import OracleError, Problem

from gpu_util import inputs
from helpers import problem_of

FORMS = ["fp64", "fp32_abs", "fp32_cell"]


def sphere_problem(m, repr_="fp64", R=3.0, n=8):
    return Problem(nx=n, ny=n, nz=n, dt=0.05, q=[-1.0], m=[1.0], obj="sphere",
                   center=(n / 2 + 0.25, n / 2 - 0.125, n / 2), radius=R, repr=repr_,
                   sphere_patches=m)


def patch_centre(face, iu, iv, m):
    """Unit direction through the centre of patch (face, iu, iv): on the cube
    face the direction leaves through (axis face // 2, positive for odd
    faces), the two other axes in increasing order at the middle of the
    iu-th and iv-th of m equal intervals of [-1, 1]."""
    ax = face // 2
    u, v = [a for a in range(3) if a != ax]
    d = np.zeros(3)
    d[ax] = 1.0 if face % 2 else -1.0
    d[u] = -1.0 + (2 * iu + 1) / m
    d[v] = -1.0 + (2 * iv + 1) / m
    return d / np.linalg.norm(d)


def patch_of(prob, d, r):
    c = np.asarray(prob.center)
    return oracle.object_hit(prob, *(c + r * prob.radius * d))


@pytest.mark.parametrize("repr_", FORMS)
@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_each_patch_centre_is_in_its_own_patch(repr_, m):
    prob = sphere_problem(m, repr_)
    assert prob.nbins == 6 * m * m
    seen = set()
    for face in range(6):
        for iv in range(m):
            for iu in range(m):
                for r in (0.3, 0.97):
                    b = patch_of(prob, patch_centre(face, iu, iv, m), r)
                    assert b == (face * m + iv) * m + iu
                    seen.add(b)
    assert seen == set(range(6 * m * m))


@pytest.mark.parametrize("repr_", FORMS)
def test_mirror_images_fall_in_mirrored_patches(repr_):
    m = 4
    prob = sphere_problem(m, repr_)
    rng = np.random.default_rng(1)
    checked = 0
    for d in rng.normal(size=(400, 3)):
        d /= np.linalg.norm(d)
        a = np.abs(d)
        ax = int(np.argmax(a))
        rest = sorted(a[[k for k in range(3) if k != ax]])
        t = np.array([d[k] / a[ax] for k in range(3) if k != ax])
        # stay clear of patch edges and of face changes
        if a[ax] - rest[-1] < 1e-3 or np.min(np.abs((t + 1) * m / 2 - np.round((t + 1) * m / 2))) < 1e-3:
            continue
        b = patch_of(prob, d, 0.8)
        face, iv, iu = b // (m * m), (b // m) % m, b % m
        u, v = [k for k in range(3) if k != ax]
        for k in range(3):
            e = d.copy()
            e[k] = -e[k]
            want = {ax: (face ^ 1, iu, iv), u: (face, m - 1 - iu, iv), v: (face, iu, m - 1 - iv)}[k]
            assert patch_of(prob, e, 0.8) == (want[0] * m + want[2]) * m + want[1]
        checked += 1
    assert checked > 300


def test_ties_go_to_the_lower_axis_and_outside_is_no_patch():
    m = 2
    prob = sphere_problem(m)
    c = np.asarray(prob.center)
    # |dx| = |dy| > |dz|: the x face; |dy| = |dz| > |dx|: the y face
    assert oracle.object_hit(prob, *(c + [1.0, 1.0, 0.5])) // (m * m) == 1
    assert oracle.object_hit(prob, *(c + [0.25, -1.0, 1.0])) // (m * m) == 2
    assert oracle.object_hit(prob, *(c + [-1.5, -1.5, -1.5])) // (m * m) == 0
    # the centre itself: face x+, middle patch
    assert oracle.object_hit(prob, *c) == (1 * m + 1) * m + 1
    assert oracle.object_hit(prob, *(c + [0.0, 0.0, 3.01])) == -1


def test_uniform_directions_fill_the_faces_evenly():
    m = 3
    prob = sphere_problem(m)
    rng = np.random.default_rng(2)
    d = rng.normal(size=(6000, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    counts = np.bincount([patch_of(prob, x, 0.9) // (m * m) for x in d], minlength=6)
    assert np.all(np.abs(counts / len(d) - 1 / 6) < 0.02)


@pytest.mark.parametrize("repr_", FORMS)
def test_patches_split_the_one_bin_tally(repr_):
    w = synth.scaled(synth.sphere_16(), 16, 16, 16, 4.0, steps=12)
    sp, x, v, E = inputs(w)
    one = problem_of(w, repr_)
    many = problem_of(w, repr_)
    many.sphere_patches = 4
    r1 = oracle.run(one, sp, x, v, E, w.steps)
    r6 = oracle.run(many, sp, x, v, E, w.steps)
    assert r6.tally.shape == (96, 2)
    assert np.array_equal(r6.tally.sum(0), r1.tally[0]) and r1.tally.sum() > 80
    assert np.array_equal(r1.fate, r6.fate) and np.array_equal(r1.when, r6.when)
    assert np.array_equal(r1.rho_fixed, r6.rho_fixed) and np.array_equal(r1.x, r6.x)
    got = r6.where[r6.fate == 2]
    assert np.all((got >= 0) & (got < 96)) and len(np.unique(got)) > 20
    # the recorded patch is the patch of the position where it was collected
    for p in np.nonzero(r6.fate == 2)[0][:50]:
        assert oracle.object_hit(many, *r6.x[p]) == r6.where[p]


def test_patch_settings_are_validated():
    sp = np.zeros(1, np.int32)
    x = np.array([[1.0, 1.0, 1.0]])
    v = np.zeros((1, 3))
    E = np.zeros((3, 9 ** 3))
    for m in (-1, 65):
        with pytest.raises(OracleError):
            oracle.run(sphere_problem(m), sp, x, v, E, 1)
    crater = Problem(nx=8, ny=8, nz=8, dt=0.05, q=[-1.0], m=[1.0], obj="crater", center=(4, 4, 0),
                     z_flat=3.0, rim_radius=2.0, depth=1.0, sphere_patches=2)
    with pytest.raises(OracleError):
        oracle.run(crater, sp, x, v, E, 1)
