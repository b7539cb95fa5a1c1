"""Pins of the oracle's global boundaries (reflection and injection of ambient
particles, the particle setups of §3.1.3 and §5.2.2) against what the
mathematics fixes: the published SplitMix64 sequence, libm's logarithm, the
normal distribution, exact mirror positions, the one-sided flux of a drifting
Maxwellian through a face, a uniform plasma staying uniform, and exact
particle / charge bookkeeping.
"""
import math

import numpy as np
import pytest

from oracle import oracle
from oracle.oracle import OracleError, Problem

rng = np.random.default_rng(777)

FACE_XM, FACE_XP, FACE_YM, FACE_YP, FACE_ZM, FACE_ZP = 1, 2, 4, 8, 16, 32


def zero_field(prob):
    return np.zeros((3, prob.nodes))


def uniform_plasma(prob, ppc, vth, drift=(0.0, 0.0, 0.0), seed=0):
    g = np.random.default_rng(seed)
    n = int(ppc * prob.nx * prob.ny * prob.nz)
    x = g.random((n, 3)) * np.array([prob.nx, prob.ny, prob.nz])
    v = g.normal(0.0, vth, (n, 3)) + np.array(drift)
    return x, v


def one_sided_flux(n0, vth, un):
    """Particles per unit area and time crossing a face inward, for a drifting
    Maxwellian of density n0 with drift un along the inward normal."""
    a = un / (math.sqrt(2.0) * vth)
    return n0 * (vth / math.sqrt(2.0 * math.pi) * math.exp(-a * a) + 0.5 * un * (1.0 + math.erf(a)))


# --------------------------------------------------------------------------- random numbers


def test_splitmix64_published_sequence():
    # SplitMix64 started from state 0: the first outputs of the reference generator
    assert oracle.splitmix_draw(0, 0) == 0xE220A8397B1DCDAF
    assert oracle.splitmix_draw(0, 1) == 0x6E789E6AA1B965F4
    assert oracle.splitmix_draw(0, 2) == 0x06C45D188009454F


def test_uniforms_on_the_2_53_grid_and_keyed():
    vals = [oracle.inj_uniform(9, 3, 1, 2, c, j, d) for c in range(5) for j in range(4) for d in range(3)]
    for u in vals:
        assert 0.0 <= u < 1.0
        assert u * 2 ** 53 == int(u * 2 ** 53)
    assert len(set(vals)) == len(vals)
    assert oracle.inj_uniform(9, 3, 1, 2, 4, 3, 2) == oracle.inj_uniform(9, 3, 1, 2, 4, 3, 2)
    assert oracle.inj_uniform(9, 3, 1, 2, 4, 3, 2) != oracle.inj_uniform(10, 3, 1, 2, 4, 3, 2)


def test_ln_against_libm():
    xs = np.concatenate([rng.random(20000), [1.0, 0.5, 2.0 ** -30, 1e-300, 0.7071067811865476,
                                             0.7071067811865475, 1.0 - 2 ** -53, 2 ** -53]])
    for x in xs:
        if x <= 0.0:
            continue
        ref = math.log(x)
        got = oracle.ln(x)
        assert abs(got - ref) <= 4 * np.finfo(float).eps * max(1.0, abs(ref)), (x, got, ref)
    assert oracle.ln(1.0) == 0.0


def test_normals_are_standard_normal():
    z = np.array([oracle.normals3(k) for k in range(12000)]).ravel()
    n = z.size
    assert abs(z.mean()) < 4 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 4 * math.sqrt(2.0 / n)
    # Kolmogorov-Smirnov distance to the normal CDF (0.1% critical value 1.95/sqrt(n))
    zs = np.sort(z)
    cdf = 0.5 * (1.0 + np.array([math.erf(t / math.sqrt(2.0)) for t in zs]))
    ks = max(np.max(np.arange(1, n + 1) / n - cdf), np.max(cdf - np.arange(n) / n))
    assert ks < 1.95 / math.sqrt(n)


# --------------------------------------------------------------------------- reflection


@pytest.mark.parametrize("repr_", ["fp64", "fp32_abs", "fp32_cell"])
def test_reflection_at_a_min_face_is_the_mirror(repr_):
    # dyadic numbers: every position is exact in all forms
    prob = Problem(nx=4, ny=4, nz=4, dt=0.125, q=[-1.0], m=[1.0], reflect=FACE_XM, repr=repr_)
    x = np.array([[0.25, 2.0, 2.0]])
    v = np.array([[-1.0, 0.0, 0.0]])
    expect = [0.125, 0.0, 0.125, 0.25, 0.375]  # crosses 0 at the third step: -0.125 -> 0.125
    vx = [-1.0, -1.0, 1.0, 1.0, 1.0]
    for k, (xe, ve) in enumerate(zip(expect, vx)):
        r = oracle.run(prob, [0], x, v, zero_field(prob), k + 1)
        assert r.fate[0] == 0
        assert r.x[0, 0] == xe and r.v[0, 0] == ve


@pytest.mark.parametrize("repr_", ["fp64", "fp32_abs", "fp32_cell"])
def test_reflection_at_a_max_face(repr_):
    prob = Problem(nx=4, ny=4, nz=4, dt=0.125, q=[-1.0], m=[1.0], reflect=FACE_YP, repr=repr_)
    x = np.array([[2.0, 3.75, 2.0]])
    v = np.array([[0.0, 2.0, 0.0]])
    r = oracle.run(prob, [0], x, v, zero_field(prob), 1)   # 3.75 + 0.25 = 4 -> on the face
    # exactly on the face: mirrored onto itself, then placed just inside
    below = {"fp64": np.nextafter(4.0, 0.0),
             "fp32_abs": float(np.nextafter(np.float32(4.0), np.float32(0.0))),
             "fp32_cell": 3.0 + float(np.nextafter(np.float32(1.0), np.float32(0.0)))}[repr_]
    assert r.fate[0] == 0 and r.x[0, 1] == below and r.v[0, 1] == -2.0
    r = oracle.run(prob, [0], np.array([[2.0, 3.875, 2.0]]), v, zero_field(prob), 1)  # 4.125 -> 3.875
    assert r.fate[0] == 0 and r.x[0, 1] == 3.875 and r.v[0, 1] == -2.0


@pytest.mark.parametrize("repr_", ["fp64", "fp32_cell"])
def test_closed_box_keeps_every_particle_and_its_charge(repr_):
    prob = Problem(nx=6, ny=5, nz=7, dt=0.2, q=[-1.0, 1.0], m=[1.0, 4.0], reflect=63, repr=repr_)
    x, v = uniform_plasma(prob, 3, 1.5, seed=3)
    sp = rng.integers(0, 2, len(x))
    E = rng.normal(0.0, 0.3, (3, prob.nodes))
    r = oracle.run(prob, sp, x, v, E, 40)
    assert np.all(r.fate == 0)
    assert r.escaped.sum() == 0
    total = sum(round(prob.q[s] * 2 ** 32) * int((sp == s).sum()) for s in range(2))
    assert int(r.rho_fixed.sum()) == total


def test_reflecting_faces_never_count_escapes():
    prob = Problem(nx=5, ny=5, nz=5, dt=0.3, q=[-1.0], m=[1.0], reflect=FACE_XM | FACE_YP | FACE_ZM)
    x, v = uniform_plasma(prob, 4, 2.0, seed=4)
    r = oracle.run(prob, np.zeros(len(x), int), x, v, zero_field(prob), 30)
    assert r.escaped[[0, 3, 4]].sum() == 0
    assert r.escaped[[1, 2, 5]].sum() > 0


def test_boundary_settings_are_validated():
    x = np.array([[1.0, 1.0, 1.0]])
    v = np.zeros((1, 3))
    bad = [Problem(nx=4, ny=4, nz=4, dt=0.1, q=[1.0], m=[1.0], reflect=FACE_XM, inj_faces=FACE_XM,
                   inj_density=[1.0], inj_vth=[1.0], inj_drift=[(0, 0, 0)]),
           Problem(nx=4, ny=4, nz=4, dt=0.1, q=[1.0], m=[1.0], reflect=64),
           Problem(nx=4, ny=4, nz=8, dt=0.1, q=[1.0], m=[1.0], obj="crater", center=(2, 2, 0),
                   z_flat=2.0, rim_radius=1.0, depth=0.5, reflect=FACE_ZM)]
    for p in bad:
        with pytest.raises(OracleError):
            oracle.run(p, [0], x, v, zero_field(p), 1)


# --------------------------------------------------------------------------- injection


def injection_problem(faces, n0, vth, drift, dt=0.1, n=(6, 6, 6), repr_="fp64", seed=5, **kw):
    return Problem(nx=n[0], ny=n[1], nz=n[2], dt=dt, q=[-1.0], m=[1.0], repr=repr_,
                   inj_faces=faces, inj_seed=seed, inj_density=[n0], inj_vth=[vth],
                   inj_drift=[drift], **kw)


@pytest.mark.parametrize("face,drift", [(FACE_XM, (0.0, 0.0, 0.0)), (FACE_XM, (0.7, 0.3, 0.0)),
                                        (FACE_XM, (-0.5, 0.0, 0.0)), (FACE_ZP, (0.0, 0.0, -1.2)),
                                        (FACE_YP, (0.0, 0.4, 0.0))])
def test_injected_count_is_the_one_sided_flux(face, drift):
    n0, vth, dt, steps = 30.0, 1.0, 0.1, 25
    prob = injection_problem(face, n0, vth, drift, dt=dt)
    r = oracle.run(prob, np.zeros(0, int), np.zeros((0, 3)), np.zeros((0, 3)), zero_field(prob), steps)
    f = int(math.log2(face))
    axis = f // 2
    un = -drift[axis] if f & 1 else drift[axis]
    area = 36.0
    expect = one_sided_flux(n0, vth, un) * area * dt * steps
    got = int(r.injected[0])
    assert abs(got - expect) < 4.5 * math.sqrt(expect) + 1, (got, expect)


def test_injected_velocities_are_flux_weighted():
    n0, vth, dt = 400.0, 1.0, 0.1
    prob = injection_problem(FACE_XM, n0, vth, (0.0, 0.0, 0.0), dt=dt, n=(8, 8, 8))
    r = oracle.run(prob, np.zeros(0, int), np.zeros((0, 3)), np.zeros((0, 3)), zero_field(prob), 1)
    v = r.v
    x = r.x
    assert len(v) > 500
    # normal component: Rayleigh, mean vth sqrt(pi/2); tangential: N(0, vth^2)
    k = len(v)
    assert np.all(v[:, 0] > 0)
    assert abs(v[:, 0].mean() - vth * math.sqrt(math.pi / 2)) < 4 * vth * math.sqrt((2 - math.pi / 2) / k)
    for d in (1, 2):
        assert abs(v[:, d].mean()) < 4 * vth / math.sqrt(k)
        assert abs(v[:, d].var() - vth ** 2) < 5 * vth ** 2 * math.sqrt(2 / k)
    # entered during the step: 0 <= x < v_x dt; tangential positions fill the face
    assert np.all(x[:, 0] >= 0) and np.all(x[:, 0] <= v[:, 0] * dt + 1e-12)
    frac = x[:, 1:] - np.floor(x[:, 1:])
    assert np.all(np.abs(frac.mean(axis=0) - 0.5) < 4 * math.sqrt(1 / 12 / k))


@pytest.mark.parametrize("drift", [(0.0, 0.0, 0.0), (0.6, -0.3, 0.2)])
def test_open_box_with_injection_keeps_a_uniform_plasma_uniform(drift):
    # ambient plasma of density n0 everywhere outside: the population of the
    # box stays at n0 * volume (absorbing faces + injection = open boundary)
    n0, vth, dt, steps = 12.0, 1.0, 0.1, 40
    prob = injection_problem(63, n0, vth, drift, dt=dt, n=(7, 6, 5))
    x, v = uniform_plasma(prob, n0, vth, drift, seed=6)
    N0 = len(x)
    r = oracle.run(prob, np.zeros(N0, int), x, v, zero_field(prob), steps)
    alive = int((r.fate == 0).sum())
    # loaded + injected = alive + escaped (exact); alive within Poisson noise of N0
    assert N0 + int(r.injected[0]) == alive + int(r.escaped.sum())
    assert abs(alive - N0) < 5 * math.sqrt(N0)
    # the density stays flat: the inner half of the box holds its share
    xa = r.x[r.fate == 0]
    inner = np.all((xa > np.array([1.75, 1.5, 1.25])) & (xa < np.array([5.25, 4.5, 3.75])), axis=1)
    share = inner.sum() / alive
    assert abs(share - (3.5 * 3 * 2.5) / (7 * 6 * 5)) < 0.03


def test_injection_bookkeeping_and_charge_are_exact():
    prob = injection_problem(FACE_XM | FACE_YP | FACE_ZP, 15.0, 1.0, (0.3, 0.0, -0.2), dt=0.15,
                             n=(8, 6, 7), obj="sphere", center=(4.0, 3.0, 3.5), radius=1.5)
    prob.q = [-1.0]
    x, v = uniform_plasma(prob, 5, 1.0, seed=8)
    keep = np.sum((x - np.array([4.0, 3.0, 3.5])) ** 2, axis=1) > 1.5 ** 2
    x, v = x[keep], v[keep]
    E = rng.normal(0.0, 0.2, (3, prob.nodes))
    r = oracle.run(prob, np.zeros(len(x), int), x, v, E, 20)
    n_loaded, n_inj = len(x), int(r.injected[0])
    assert len(r.fate) == n_loaded + n_inj
    assert int((r.fate == 0).sum()) + int(r.tally.sum()) + int(r.escaped.sum()) == n_loaded + n_inj
    assert int(r.rho_fixed.sum()) == round(-1.0 * 2 ** 32) * int((r.fate == 0).sum())


def test_injection_is_deterministic_and_keyed_by_seed():
    prob = injection_problem(FACE_XM | FACE_XP, 20.0, 1.0, (0.0, 0.0, 0.0))
    e = (np.zeros(0, int), np.zeros((0, 3)), np.zeros((0, 3)))
    a = oracle.run(prob, *e, zero_field(prob), 5)
    b = oracle.run(prob, *e, zero_field(prob), 5)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    prob.inj_seed = 6
    c = oracle.run(prob, *e, zero_field(prob), 5)
    assert not (len(c.x) == len(a.x) and np.array_equal(c.x, a.x))


def test_fp32_forms_inject_the_fp64_particles_rounded():
    # min faces only: a particle that entered stays inside after rounding
    base = dict(faces=FACE_XM | FACE_YM, n0=25.0, vth=1.0, drift=(0.2, 0.1, -0.4), dt=0.1)
    e = (np.zeros(0, int), np.zeros((0, 3)), np.zeros((0, 3)))
    p64 = injection_problem(**base)
    r64 = oracle.run(p64, *e, zero_field(p64), 1)
    for rep in ("fp32_abs", "fp32_cell"):
        p = injection_problem(**base, repr_=rep)
        r = oracle.run(p, *e, zero_field(p), 1)
        assert len(r.x) == len(r64.x)
        assert np.allclose(r.x, r64.x, rtol=0, atol=6e-7 * 6)
        assert np.allclose(r.v, r64.v, rtol=1e-7, atol=1e-7)
