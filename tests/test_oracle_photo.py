"""Pins of the oracle's photoemission (photoelectrons generated at the sunlit
terrain according to the local sunlight index, none in shadow; §5.2.2):
per-column counts are the floor or ceiling of the stated mean, velocities are
a half-Maxwellian about the terrain normal, emission starts on the ground and
moves a fraction of the step, normals and ground heights agree with the
terrain the particles are collected by, the shadow agrees with a ray march
against that terrain, unlit columns emit nothing, and the bookkeeping is
exact."""
import math

import numpy as np
import pytest

from oracle import oracle
from oracle.oracle import OracleError, Problem

ELEV = math.radians(10.0)
SUN = (math.cos(ELEV), 0.0, math.sin(ELEV))  # 10 degrees above the ground in the X-Z plane


def photo_problem(n=(16, 16, 12), far=False, mean=2.3, vth=0.01, sun=SUN, repr_="fp64", seed=3,
                  dt=0.05, rim=6.0, depth=4.0, z_flat=5.0):
    nx, ny, nz = n
    centre = (-1000.0, -1000.0, 0.0) if far else (nx / 2, ny / 2, 0.0)
    s = np.asarray(sun) / np.linalg.norm(sun)
    flux = mean / (dt * s[2]) if far else mean / dt
    return Problem(nx=nx, ny=ny, nz=nz, dt=dt, q=[-1.0, 1.0, -1.0], m=[1.0, 100.0, 1.0],
                   obj="crater", center=centre, z_flat=z_flat, rim_radius=rim, depth=depth,
                   repr=repr_, pe_species=2, pe_seed=seed, pe_sun=sun, pe_flux=flux, pe_vth=vth)


def emit(prob, nsteps=1):
    n = 0
    E = np.zeros((3, prob.nodes))
    return oracle.run(prob, np.zeros(n, np.int32), np.zeros((n, 3)), np.zeros((n, 3)), E, nsteps)


def test_flat_ground_counts_are_floor_or_ceiling_of_the_mean():
    prob = photo_problem(far=True, mean=2.3)
    col = oracle.photo_column(prob, 3, 4)
    assert col["lit"] and np.allclose(col["n"], [0, 0, 1])
    assert abs(col["index"] - math.sin(ELEV)) < 1e-15 and abs(col["mean"] - 2.3) < 1e-12
    r = emit(prob)
    x = r.x[r.fate != 1]
    cols = np.floor(x[:, 0]).astype(int) + prob.nx * np.floor(x[:, 1]).astype(int)
    counts = np.bincount(cols, minlength=prob.nx * prob.ny)
    assert set(np.unique(counts)) <= {2, 3}
    assert abs(counts.mean() - 2.3) < 0.1
    assert r.injected[2] == len(r.fate) and r.injected[:2].sum() == 0


def test_half_maxwellian_about_the_normal():
    vth = 0.5
    prob = photo_problem(far=True, mean=25.0, vth=vth)
    r = emit(prob)
    v = r.v[r.fate == 0]
    assert len(v) > 5000
    assert np.all(v[:, 2] > 0)
    assert abs(v[:, 2].mean() / (vth * math.sqrt(2 / math.pi)) - 1) < 0.03
    assert abs((v[:, 2] ** 2).mean() / vth ** 2 - 1) < 0.05
    for a in (0, 1):
        assert abs(v[:, a].mean()) < 4 * vth / math.sqrt(len(v))
        assert abs(v[:, a].std() / vth - 1) < 0.03


def test_emission_starts_on_the_ground_and_moves_a_fraction_of_the_step():
    prob = photo_problem(far=True, mean=8.0, vth=0.2)
    r = emit(prob)
    alive = r.fate == 0
    x, v = r.x[alive], r.v[alive]
    tau = (x[:, 2] - prob.z_flat) / v[:, 2]
    assert np.all(tau >= -1e-12) and np.all(tau < prob.dt)
    assert 0.4 * prob.dt < tau.mean() < 0.6 * prob.dt
    # the footprint: back along the velocity by the same fraction lands in [0, n)
    x0 = x[:, :2] - v[:, :2] * tau[:, None]
    assert np.all((x0 >= -1e-9) & (x0 < np.array([prob.nx, prob.ny]) + 1e-9))


def ground_of(prob, x, y):
    """Terrain height from the collection predicate: bisection on z."""
    lo, hi = -1.0, float(prob.nz)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if oracle.object_hit(prob, x, y, mid) >= 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_normals_and_ground_match_the_collecting_terrain():
    prob = photo_problem()
    for i, j in ((8, 8), (5, 9), (10, 6), (3, 3), (12, 8)):
        c = oracle.photo_column(prob, i, j)
        x, y = i + 0.5, j + 0.5
        assert abs(c["ground"] - ground_of(prob, x, y)) < 1e-9
        e = 1e-4
        gx = (ground_of(prob, x + e, y) - ground_of(prob, x - e, y)) / (2 * e)
        gy = (ground_of(prob, x, y + e) - ground_of(prob, x, y - e)) / (2 * e)
        nn = np.array([-gx, -gy, 1.0]) / math.sqrt(gx * gx + gy * gy + 1)
        assert np.abs(c["n"] - nn).max() < 1e-5
        s = np.asarray(SUN) / np.linalg.norm(SUN)
        assert abs(c["index"] - s @ c["n"]) < 1e-12


@pytest.mark.parametrize("elev", [10.0, 35.0])
def test_shadow_agrees_with_a_ray_march(elev):
    a = math.radians(elev)
    sun = (math.cos(a), 0.3 * math.cos(a), math.sin(a))
    prob = photo_problem(sun=sun)
    s = np.asarray(sun) / np.linalg.norm(sun)
    lit_count = shadow_count = 0
    for j in range(prob.ny):
        for i in range(prob.nx):
            c = oracle.photo_column(prob, i, j)
            p = np.array([i + 0.5, j + 0.5, c["ground"]])
            if c["index"] <= 0:
                assert not c["lit"]
                continue
            hit = False
            for t in np.arange(0.02, 40.0, 0.02):
                q = p + t * s
                if q[2] > prob.z_flat + 0.1:
                    break
                if oracle.object_hit(prob, *q) >= 0:
                    hit = True
                    break
            assert c["lit"] == (not hit), (i, j)
            lit_count += c["lit"]
            shadow_count += not c["lit"]
    assert lit_count > 0 and (shadow_count > 0 or elev > 30)


def test_unlit_columns_emit_nothing_and_bookkeeping_is_exact():
    prob = photo_problem(mean=3.0, vth=0.01)
    r = emit(prob, nsteps=2)
    lit = np.array([[oracle.photo_column(prob, i, j)["lit"] for i in range(prob.nx)]
                    for j in range(prob.ny)])
    assert 0 < lit.sum() < lit.size
    x = r.x[r.fate == 0]
    ii, jj = np.floor(x[:, 0]).astype(int), np.floor(x[:, 1]).astype(int)
    assert np.all(lit[jj, ii])
    alive = (r.fate == 0).sum()
    assert alive + r.tally.sum() + r.escaped.sum() == r.injected.sum() == len(r.fate)
    # the photoelectrons' charge is on the mesh
    assert r.rho_fixed.sum() == -alive * 2 ** 32


def test_emission_is_deterministic_and_keyed_by_seed():
    a = emit(photo_problem(seed=5))
    b = emit(photo_problem(seed=5))
    c = emit(photo_problem(seed=6))
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    assert len(c.x) != len(a.x) or not np.array_equal(c.x, a.x)


def test_fp32_forms_emit_the_fp64_particles_rounded():
    r64 = emit(photo_problem(mean=4.0, vth=0.3))
    for form in ("fp32_abs", "fp32_cell"):
        r32 = emit(photo_problem(mean=4.0, vth=0.3, repr_=form))
        assert len(r32.x) == len(r64.x)
        assert np.array_equal(r32.v, r64.v.astype(np.float32).astype(np.float64))
        assert np.abs(r32.x - r64.x).max() < 1e-5


def test_photoemission_settings_are_validated():
    E = np.zeros((3, 17 * 17 * 13))
    none = (np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros((0, 3)))
    for kw in (dict(sun=(1.0, 0.0, 0.0)), dict(sun=(1.0, 0.0, -0.2)), dict(vth=-1.0)):
        with pytest.raises(OracleError):
            oracle.run(photo_problem(**kw), *none, E, 1)
    p = photo_problem()
    p.pe_species = 3
    with pytest.raises(OracleError):
        oracle.run(p, *none, E, 1)
    s = Problem(nx=16, ny=16, nz=12, dt=0.05, q=[-1.0], m=[1.0], obj="sphere", center=(8, 8, 6),
                radius=2.0, pe_species=0, pe_flux=1.0, pe_vth=1.0)
    with pytest.raises(OracleError):
        oracle.run(s, *none, E, 1)


def test_a_run_continued_from_step_k_is_the_long_run():
    # injection and photoemission draw by step index: 6 steps at once equal
    # 3 steps and then 3 more from step 3 (the first run's survivors loaded),
    # as a set of particles, in rho, tallies, escapes and injected counts
    prob = photo_problem(mean=1.7, vth=0.4)
    prob.inj_faces, prob.inj_seed = 1 | 2 | 32, 9
    prob.inj_density, prob.inj_vth = [3.0, 3.0, 0.0], [1.0, 0.1, 0.0]
    prob.inj_drift = [(0.0, 0.0, 0.0), (0.0, 0.0, -0.3), (0.0, 0.0, 0.0)]
    rng = np.random.default_rng(5)
    n = 500
    x = rng.uniform(0.0, 1.0, size=(n, 3)) * [prob.nx, prob.ny, prob.nz]
    x[:, 2] = prob.z_flat + 0.5 + x[:, 2] * (prob.nz - prob.z_flat - 1.0) / prob.nz
    v = rng.normal(0.0, 1.0, size=(n, 3))
    sp = rng.integers(0, 2, n).astype(np.int32)
    E = np.zeros((3, prob.nodes))
    whole = oracle.run(prob, sp, x, v, E, 6)
    a = oracle.run(prob, sp, x, v, E, 3)
    keep = a.fate == 0
    prob.first_step = 3
    b = oracle.run(prob, a.species[keep], a.x[keep], a.v[keep], E, 3)

    def alive(r):
        m = r.fate == 0
        rows = np.column_stack([r.species[m], r.x[m], r.v[m]])
        return rows[np.lexsort(rows.T[::-1])]

    assert whole.injected[2] > 0 and whole.injected[0] > 0
    assert np.array_equal(alive(whole), alive(b))
    assert np.array_equal(whole.rho_fixed, b.rho_fixed)
    assert np.array_equal(whole.tally, a.tally + b.tally)
    assert np.array_equal(whole.escaped, a.escaped + b.escaped)
    assert np.array_equal(whole.injected, a.injected + b.injected)
    # not a tautology: the same continuation from step 0 draws differently
    prob.first_step = 0
    c = oracle.run(prob, a.species[keep], a.x[keep], a.v[keep], E, 3)
    assert not np.array_equal(alive(whole), alive(c))
