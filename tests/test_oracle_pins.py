"""Pins of the CPU oracle against what the mathematics fixes, independently of
the oracle's own code: closed forms, invariants, special cases and brute force
(exact rational arithmetic in Python) on tiny inputs.

The oracle follows the PIC loop of §2.1 (scatter, gather, push), the outer
boundary removal of §3.1.3 and the collection at objects of §5.2.2, with
trilinear weighting and a leapfrog push (the paper names neither).
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import synth
from oracle import oracle
from oracle.oracle import Problem

from helpers import check_mismatches_near_surface, fate_mismatches, problem_of

rng = np.random.default_rng(12345)


def hat(t):
    """1-D linear hat function of width 1 (exact for Fractions)."""
    a = abs(t)
    return 1 - a if a < 1 else 0


def bruteforce_interp(nodes_val, nx, ny, nz, g):
    """Field at point g as the sum over ALL nodes of value * product of hats."""
    acc = F(0)
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                w = hat(F(g[0]) - i) * hat(F(g[1]) - j) * hat(F(g[2]) - k)
                if w:
                    acc += w * F(nodes_val[i + (nx + 1) * (j + (ny + 1) * k)])
    return acc


def node_index(nx, ny, i, j, k):
    return i + (nx + 1) * (j + (ny + 1) * k)


# --------------------------------------------------------------------------- weights


def test_weights_sum_to_one_fp64_and_fp32():
    for _ in range(2000):
        f = rng.random(3)
        W = oracle.weights(f)
        assert abs(W.sum() - 1.0) <= 4 * np.finfo(np.float64).eps
        assert np.all(W >= 0)
        W32 = oracle.weights(f.astype(np.float32), np.float32)
        assert abs(float(W32.astype(np.float64).sum()) - 1.0) <= 8 * np.finfo(np.float32).eps


def test_weights_exact_for_dyadic_offsets():
    for _ in range(500):
        f = rng.integers(0, 256, 3) / 256.0
        W = oracle.weights(f)
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    ex = ((1 - F(f[0])) if a == 0 else F(f[0])) * \
                         ((1 - F(f[1])) if b == 0 else F(f[1])) * \
                         ((1 - F(f[2])) if c == 0 else F(f[2]))
                    assert F(W[a + 2 * b + 4 * c]) == ex
        assert sum(F(x) for x in W) == 1


def test_particle_on_node_puts_everything_on_that_node():
    W = oracle.weights([0.0, 0.0, 0.0])
    assert W[0] == 1.0 and np.all(W[1:] == 0.0)
    C = oracle.fixed_contrib(-1.0, W)
    assert C[0] == -(2 ** 32) and np.all(C[1:] == 0)


def test_fixed_point_contributions_round_half_even_and_conserve():
    for trial in range(2000):
        chg = float(rng.choice([-1.0, 1.0, 0.5, -3.0, 1.0 / 3.0]))
        f = rng.random(3)
        W = oracle.weights(f)
        C = oracle.fixed_contrib(chg, W)
        for n in range(7):
            exact = F(float(chg * W[n])) * 2 ** 32  # the product is rounded in FP64 first
            assert C[n] == round(exact)  # Python rounds Fractions half to even
        assert int(C.sum()) == round(F(chg) * 2 ** 32)
        # float32 mirror: contributions of the float product, same remainder rule
        W32 = oracle.weights(f.astype(np.float32), np.float32)
        C32 = oracle.fixed_contrib(np.float32(chg), W32, np.float32)
        for n in range(7):
            assert C32[n] == round(F(float(np.float32(chg) * W32[n])) * 2 ** 32)
        assert int(C32.sum()) == round(F(float(np.float32(chg))) * 2 ** 32)


def test_fixed_point_half_way_cases_go_to_even():
    # chg * W * 2^32 = k + 1/2 exactly: chg = 2^-33 * (2k+1), W[n] = 1 on node 0
    W = oracle.weights([0.0, 0.0, 0.0])
    for k in (0, 1, 2, 3, 10, 11):
        chg = (2 * k + 1) * 2.0 ** -33
        C = oracle.fixed_contrib(chg, W)
        assert C[0] == (k if k % 2 == 0 else k + 1)


# --------------------------------------------------------------------------- gather


def _poly_field(nx, ny, nz, coef):
    """Node values of p = c0 + c1 x + c2 y + c3 z + c4 xy + c5 yz + c6 zx + c7 xyz
    (the span that trilinear interpolation reproduces exactly)."""
    vals = np.empty((nx + 1) * (ny + 1) * (nz + 1))
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                vals[node_index(nx, ny, i, j, k)] = float(_poly(coef, i, j, k))
    return vals


def _poly(c, x, y, z):
    x, y, z = F(x), F(y), F(z)
    return (F(c[0]) + F(c[1]) * x + F(c[2]) * y + F(c[3]) * z + F(c[4]) * x * y
            + F(c[5]) * y * z + F(c[6]) * z * x + F(c[7]) * x * y * z)


def test_gather_reproduces_trilinear_span_exactly():
    nx, ny, nz = 3, 4, 2
    for _ in range(20):
        coefs = [rng.integers(-8, 9, 8) / 8.0 for _ in range(3)]
        E = [_poly_field(nx, ny, nz, c) for c in coefs]
        for _ in range(20):
            i = [int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))]
            f = rng.integers(0, 64, 3) / 64.0
            out = oracle.gather(nx, ny, nz, E, i, f)
            g = [i[d] + f[d] for d in range(3)]
            for d in range(3):
                assert F(out[d]) == _poly(coefs[d], *g)


def test_gather_matches_bruteforce_hat_sum():
    nx, ny, nz = 3, 3, 2
    E = [rng.standard_normal((nx + 1) * (ny + 1) * (nz + 1)) for _ in range(3)]
    for _ in range(40):
        g = rng.random(3) * np.array([nx, ny, nz])
        i = np.floor(g).astype(int)
        f = g - i
        out = oracle.gather(nx, ny, nz, E, i, f)
        for d in range(3):
            ex = float(bruteforce_interp(E[d], nx, ny, nz, g))
            assert abs(out[d] - ex) <= 1e-14 * max(1.0, abs(ex))


def test_gather_continuous_across_cell_faces():
    nx, ny, nz = 4, 4, 4
    E = [rng.standard_normal((nx + 1) ** 3) for _ in range(3)]
    for _ in range(50):
        f = rng.random(3)
        a = oracle.gather(nx, ny, nz, E, [1, 2, 1], [1.0, f[1], f[2]])  # right face of cell 1
        b = oracle.gather(nx, ny, nz, E, [2, 2, 1], [0.0, f[1], f[2]])  # left face of cell 2
        assert np.allclose(a, b, rtol=0, atol=1e-14)


# --------------------------------------------------------------------------- push


def _uniform_field(prob, e):
    return [np.full(prob.nodes, e[d]) for d in range(3)]


@pytest.mark.parametrize("form", ["fp64", "fp32_abs", "fp32_cell"])
def test_push_uniform_field_closed_form(form):
    # dyadic dt, E, x0, v0 so that every intermediate is exact in both FP64 and FP32
    dt = 2.0 ** -4
    prob = Problem(nx=64, ny=64, nz=64, dt=dt, q=[-1.0, 1.0], m=[1.0, 4.0], repr=form)
    e = (0.25, -0.5, 0.125)
    E = _uniform_field(prob, e)
    x0 = np.array([[20.5, 30.25, 40.0], [10.0, 50.5, 33.75]])
    v0 = np.array([[0.5, -0.25, 1.0], [-0.5, 0.0, 0.25]])
    sp = np.array([0, 1])
    N = 24
    r = oracle.run(prob, sp, x0, v0, E, N)
    for p in range(2):
        qm = F(prob.q[sp[p]]) / F(prob.m[sp[p]])
        for d in range(3):
            a = qm * F(e[d])
            xN = F(x0[p, d]) + N * F(v0[p, d]) * F(dt) + a * F(dt) ** 2 * F(N * (N + 1), 2)
            vN = F(v0[p, d]) + N * a * F(dt)
            assert F(r.x[p, d]) == xN, (form, p, d)
            assert F(r.v[p, d]) == vN, (form, p, d)
    assert np.all(r.fate == 0)


def test_push_zero_field_is_ballistic():
    prob = Problem(nx=32, ny=32, nz=32, dt=0.05, q=[-1.0], m=[1.0])
    E = _uniform_field(prob, (0.0, 0.0, 0.0))
    x0 = rng.random((100, 3)) * 10 + 11
    v0 = rng.standard_normal((100, 3))
    r = oracle.run(prob, np.zeros(100, int), x0, v0, E, 50)
    assert np.array_equal(r.v, v0)
    # fma-accumulated drift: |x - (x0 + 50 v dt)| within 50 roundings
    assert np.allclose(r.x, x0 + 50 * v0 * 0.05, rtol=0, atol=1e-12)


def test_push_harmonic_field_matches_discrete_leapfrog_solution():
    # E_x = k (x - xc) on an electron (q = -1, m = 1): acceleration -k (x - xc),
    # omega^2 = k. Leapfrog's exact discrete solution is A cos(n th) + B sin(n th)
    # with sin(th / 2) = omega dt / 2.
    n = 32
    xc, k, dt = 16.0, 1.0, 0.05
    prob = Problem(nx=n, ny=n, nz=n, dt=dt, q=[-1.0], m=[1.0])
    Ex = np.empty(prob.nodes)
    for kk in range(n + 1):
        for j in range(n + 1):
            for i in range(n + 1):
                Ex[node_index(n, n, i, j, kk)] = k * (i - xc)
    E = [Ex, np.zeros(prob.nodes), np.zeros(prob.nodes)]
    y0, u0 = 5.0, 0.3
    N = 1000
    r = oracle.run(prob, np.array([0]), np.array([[xc + y0, 7.5, 9.25]]),
                   np.array([[u0, 0.0, 0.0]]), E, N)
    w = math.sqrt(k)
    th = 2 * math.asin(w * dt / 2)
    u_half = u0 - k * y0 * dt
    y1 = y0 + u_half * dt
    A = y0
    B = (y1 - y0 * math.cos(th)) / math.sin(th)
    yN = A * math.cos(N * th) + B * math.sin(N * th)
    assert abs((r.x[0, 0] - xc) - yN) <= 1e-11 * math.hypot(A, B)
    # the velocity at N - 1/2 is (y_N - y_{N-1}) / dt
    yNm1 = A * math.cos((N - 1) * th) + B * math.sin((N - 1) * th)
    assert abs(r.v[0, 0] - (yN - yNm1) / dt) <= 1e-9
    assert r.x[0, 1] == 7.5 and r.x[0, 2] == 9.25


def test_ion_mass_enters_kick():
    prob = Problem(nx=16, ny=16, nz=16, dt=0.0625, q=[1.0], m=[100.0])
    E = _uniform_field(prob, (2.0, 0.0, 0.0))
    r = oracle.run(prob, np.array([0]), np.array([[8.0, 8.0, 8.0]]),
                   np.array([[0.0, 0.0, 0.0]]), E, 1)
    assert r.v[0, 0] == 1.0 / 100.0 * 0.0625 * 2.0
    assert r.x[0, 0] == 8.0 + r.v[0, 0] * 0.0625


# --------------------------------------------------------------------------- boundaries


def test_radial_ballistic_particle_absorbed_at_predicted_step():
    dt = 1.0 / 16
    prob = Problem(nx=16, ny=16, nz=16, dt=dt, q=[-1.0], m=[1.0], obj="sphere",
                   center=(8.0, 8.0, 8.0), radius=3.0)
    E = _uniform_field(prob, (0.0, 0.0, 0.0))
    # x after step s (0-based) = 13.5 - (s + 1)/16; on the surface (|x - c| = 3) at s = 39
    r = oracle.run(prob, np.array([0]), np.array([[13.5, 8.0, 8.0]]),
                   np.array([[-1.0, 0.0, 0.0]]), E, 60)
    assert r.fate[0] == 2 and r.when[0] == 39 and r.where[0] == 0
    assert r.tally[0, 0] == 1
    # the same particle one step short of the surface survives
    r = oracle.run(prob, np.array([0]), np.array([[13.5, 8.0, 8.0]]),
                   np.array([[-1.0, 0.0, 0.0]]), E, 39)
    assert r.fate[0] == 0 and r.x[0, 0] == 11.0 + 1.0 / 16


@pytest.mark.parametrize("form", ["fp64", "fp32_abs", "fp32_cell"])
def test_box_exit_faces(form):
    dt = 0.5
    prob = Problem(nx=8, ny=8, nz=8, dt=dt, q=[-1.0], m=[1.0], repr=form)
    E = _uniform_field(prob, (0.0, 0.0, 0.0))
    x0 = np.array([[0.25, 4, 4], [7.75, 4, 4], [4, 0.25, 4], [4, 7.75, 4], [4, 4, 0.25],
                   [4, 4, 7.75], [0.25, 7.75, 4], [4, 4, 4]], float)
    v0 = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1],
                   [-1, 1, 0], [0.5, 0.5, 0.5]], float)
    r = oracle.run(prob, np.zeros(8, int), x0, v0, E, 1)
    assert list(r.fate) == [1, 1, 1, 1, 1, 1, 1, 0]
    # first offending axis (x before y), lower before upper
    assert list(r.where[:7]) == [0, 1, 2, 3, 4, 5, 0]
    assert r.escaped[:, 0].tolist() == [2, 1, 1, 1, 1, 1]
    # a particle landing exactly on the upper face has left the half-open box
    r = oracle.run(prob, np.array([0]), np.array([[7.5, 4, 4]]), np.array([[1.0, 0, 0]]), E, 1)
    assert r.fate[0] == 1 and r.where[0] == 1
    # ... and exactly on the lower face it is still inside
    r = oracle.run(prob, np.array([0]), np.array([[0.5, 4, 4]]), np.array([[-1.0, 0, 0]]), E, 1)
    assert r.fate[0] == 0 and r.x[0, 0] == 0.0


def _crater_problem(form="fp64"):
    return Problem(nx=160, ny=160, nz=80, dt=0.05, q=[-1.0], m=[1.0], obj="crater",
                   center=(80.0, 80.0, 0.0), z_flat=10.0, rim_radius=40.0, depth=15.0, repr=form)


def crater_height(x, y, xc=80.0, yc=80.0, zf=10.0, a=40.0, d=15.0):
    """Terrain height of a flat plane with a spherical-bowl crater (closed form)."""
    r2 = (x - xc) ** 2 + (y - yc) ** 2
    if r2 >= a * a:
        return zf
    Rc = (a * a + d * d) / (2 * d)
    return zf - d + Rc - math.sqrt(Rc * Rc - r2)


@pytest.mark.parametrize("form", ["fp64", "fp32_abs", "fp32_cell"])
def test_crater_predicate(form):
    prob = _crater_problem(form)
    assert crater_height(80, 80) == pytest.approx(-5.0)
    assert crater_height(120, 80) == pytest.approx(10.0)
    # below z = 0 is ground (the bowl bottom lies below the mesh)
    assert oracle.object_hit(prob, 80.0, 80.0, 0.5) == -1
    assert oracle.object_hit(prob, 80.0, 80.0, -0.01) == 80 + 160 * 80
    # flat ground: on or below the plane absorbs
    assert oracle.object_hit(prob, 10.5, 20.5, 10.0) == 10 + 160 * 20
    assert oracle.object_hit(prob, 10.5, 20.5, 9.5) == 10 + 160 * 20
    assert oracle.object_hit(prob, 10.5, 20.5, 10.01) == -1
    # inside the bowl, just above / below the closed-form surface
    for (x, y) in [(110.25, 80.0), (80.0, 50.5), (100.0, 100.0), (55.0, 60.0)]:
        zs = crater_height(x, y)
        assert zs > 0
        assert oracle.object_hit(prob, x, y, zs + 1e-3) == -1
        assert oracle.object_hit(prob, x, y, zs - 1e-3) == int(x) + 160 * int(y)


def test_crater_floor_where_bowl_is_below_mesh():
    # for r < ~24.15 the bowl lies below z = 0 and the mesh floor absorbs
    prob = _crater_problem()
    assert crater_height(62.5, 71.0) < 0
    assert oracle.object_hit(prob, 62.5, 71.0, 0.001) == -1
    assert oracle.object_hit(prob, 62.5, 71.0, -0.001) == 62 + 160 * 71


def test_crater_z_below_mesh_is_absorbed_not_escaped():
    prob = _crater_problem()
    E = _uniform_field(prob, (0.0, 0.0, 0.0))
    r = oracle.run(prob, np.array([0, 0]), np.array([[20.5, 30.5, 10.25], [150.5, 3.5, 10.5]]),
                   np.array([[0.0, 0.0, -10.0], [0.0, 0.0, 1.0]]), E, 1)
    assert r.fate.tolist() == [2, 0]
    assert r.where[0] == 20 + 160 * 30
    assert r.tally[20 + 160 * 30, 0] == 1 and r.escaped.sum() == 0


def test_wrap_edge_rule_keeps_offset_in_unit_interval():
    # o = 0 and a drift of -2^-26 gives o' = -2^-26, floor -1, and o' + 1 rounds
    # to 1.0 in float: the rule moves it back to offset 0 of the same cell, the
    # float position nearest to the exact 5 - 2^-26.
    dt = 1.0 / 16
    prob = Problem(nx=8, ny=8, nz=8, dt=dt, q=[-1.0], m=[1.0], repr="fp32_cell")
    E = _uniform_field(prob, (0.0, 0.0, 0.0))
    r = oracle.run(prob, np.array([0]), np.array([[5.0, 4.0, 4.0]]),
                   np.array([[-(2.0 ** -22), 0.0, 0.0]]), E, 3)
    assert r.x[0, 0] == 5.0 and r.fate[0] == 0
    # a drift of -2^-20 is representable below the face: cell 4, offset 1 - 2^-24
    r = oracle.run(prob, np.array([0]), np.array([[5.0, 4.0, 4.0]]),
                   np.array([[-(2.0 ** -20), 0.0, 0.0]]), E, 1)
    assert r.x[0, 0] == 5.0 - 2.0 ** -24


# --------------------------------------------------------------------------- deposit


@pytest.mark.parametrize("mode", ["fixed64", "fp64", "fp32"])
@pytest.mark.parametrize("nlat", [2, 4])
def test_lattice_loading_deposit(mode, nlat):
    # n^3 particles per cell at offsets (2m+1)/(2n): every interior node gets
    # exactly chg * n^3, face / edge / corner nodes 1/2, 1/4, 1/8 of it.
    nx, ny, nz = 3, 4, 2
    prob = Problem(nx=nx, ny=ny, nz=nz, dt=0.05, q=[-1.0], m=[1.0], deposit=mode)
    offs = [(2 * m + 1) / (2 * nlat) for m in range(nlat)]
    pts = [(i + a, j + b, k + c) for k in range(nz) for j in range(ny) for i in range(nx)
           for a in offs for b in offs for c in offs]
    x = np.array(pts)
    r = oracle.run(prob, np.zeros(len(x), int), x, np.zeros_like(x),
                   _uniform_field(prob, (0.0, 0.0, 0.0)), 0)
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                nb = sum(1 for (t, n) in ((i, nx), (j, ny), (k, nz)) if t == 0 or t == n)
                ex = -(nlat ** 3) / 2 ** nb
                assert r.rho[node_index(nx, ny, i, j, k)] == ex
    if mode == "fixed64":
        assert int(r.rho_fixed.sum()) == -len(x) * 2 ** 32


def test_deposit_matches_bruteforce_hat_sum():
    nx, ny, nz = 3, 2, 2
    n = 60
    x = rng.random((n, 3)) * np.array([nx, ny, nz])
    sp = rng.integers(0, 2, n)
    for mode in ("fp64", "fixed64"):
        prob = Problem(nx=nx, ny=ny, nz=nz, dt=0.05, q=[-1.0, 1.0], m=[1.0, 100.0], w=[1.0, 0.5],
                       deposit=mode)
        r = oracle.run(prob, sp, x, np.zeros_like(x), _uniform_field(prob, (0, 0, 0)), 0)
        chg = [F(-1.0), F(0.5)]
        for k in range(nz + 1):
            for j in range(ny + 1):
                for i in range(nx + 1):
                    ex = sum(chg[sp[p]] * hat(F(x[p, 0]) - i) * hat(F(x[p, 1]) - j)
                             * hat(F(x[p, 2]) - k) for p in range(n))
                    got = r.rho[node_index(nx, ny, i, j, k)]
                    if mode == "fp64":
                        assert abs(F(got) - ex) <= F(1, 10 ** 13)
                    else:
                        # each contribution is rounded to 2^-32 (corner 7 carries at
                        # most 8 half-units of rounding)
                        assert abs(F(int(r.rho_fixed[node_index(nx, ny, i, j, k)])) - ex * 2 ** 32) <= 4 * n
        if mode == "fixed64":
            assert int(r.rho_fixed.sum()) == round(sum(chg[s] for s in sp) * 2 ** 32)


def test_deposit_uses_positions_after_the_push():
    nx, ny, nz = 4, 3, 3
    n = 40
    dt = 1.0 / 16
    x = 0.5 + rng.random((n, 3)) * (np.array([nx, ny, nz]) - 1.0)
    v = rng.standard_normal((n, 3)) * 2
    prob = Problem(nx=nx, ny=ny, nz=nz, dt=dt, q=[1.0], m=[1.0], deposit="fp64")
    r = oracle.run(prob, np.zeros(n, int), x, v, _uniform_field(prob, (0, 0, 0)), 1)
    assert np.all(r.fate == 0)
    xn = r.x  # after one ballistic step
    assert np.allclose(xn, x + v * dt, rtol=0, atol=1e-14)
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                ex = sum(hat(F(xn[p, 0]) - i) * hat(F(xn[p, 1]) - j) * hat(F(xn[p, 2]) - k)
                         for p in range(n))
                assert abs(F(r.rho[node_index(nx, ny, i, j, k)]) - ex) <= F(1, 10 ** 13)


# --------------------------------------------------------------------------- whole step


@pytest.mark.parametrize("form", ["fp64", "fp32_abs", "fp32_cell"])
def test_sphere16_conservation(form):
    w = synth.sphere_16()
    sp, x, v = synth.all_particles(w)
    E = synth.node_E(w)
    prob = Problem(nx=16, ny=16, nz=16, dt=w.dt, q=[-1.0, 1.0], m=[1.0, 100.0], obj="sphere",
                   center=w.center, radius=w.radius, repr=form)
    r = oracle.run(prob, sp, x, v, E, w.steps)
    for s in range(2):
        loaded = int((sp == s).sum())
        alive = int(((r.fate == 0) & (sp == s)).sum())
        assert alive + int(r.tally[:, s].sum()) + int(r.escaped[:, s].sum()) == loaded
    # volume + collected + escaped charge = initial charge, exactly
    q = np.array([-1, 1])
    alive_q = int(q[sp[r.fate == 0]].sum())
    assert int(r.rho_fixed.sum()) == alive_q * 2 ** 32
    assert alive_q + int((r.tally @ q).sum()) + int((r.escaped @ q).sum()) == int(q[sp].sum())
    assert r.charge(prob)[0] == float((r.tally @ q).sum())
    # fates are consistent with the counters
    assert np.array_equal(np.bincount(r.where[r.fate == 1] * 2 + sp[r.fate == 1], minlength=12),
                          r.escaped.reshape(-1))


@pytest.mark.parametrize("form", ["fp32_abs", "fp32_cell"])
def test_fp32_mirrors_within_tolerance_of_fp64(form):
    w = synth.scaled(synth.sphere_64(), 24, 24, 24, ppc=6, steps=100)
    sp, x, v = synth.all_particles(w)
    E = synth.node_E(w)
    r64 = oracle.run(problem_of(w, "fp64"), sp, x, v, E, w.steps)
    r32 = oracle.run(problem_of(w, form), sp, x, v, E, w.steps)
    both = (r64.fate == 0) & (r32.fate == 0)
    vth = np.where(sp == 0, 1.0, 0.1)[both]
    dx = np.abs(r32.x[both] - r64.x[both]).max(axis=1)
    dv = np.abs(r32.v[both] - r64.v[both]).max(axis=1)
    assert np.all(dx <= 1e-5 * np.maximum(np.abs(r64.x[both]).max(axis=1), 1.0))
    assert np.all(dv <= 1e-5 * np.maximum(np.abs(r64.v[both]).max(axis=1), vth))
    # fates differ only for particles within 1e-4 cells of a deciding surface
    # at the step where the two runs part
    diff = fate_mismatches(r64.fate, r64.where, r64.when, r32.fate, r32.where, r32.when)
    assert len(diff) <= 1e-3 * len(sp)
    dist = check_mismatches_near_surface(w, sp, x, v, E, diff, r64.when, r64.fate, r32.when,
                                         r32.fate)
    assert np.all(dist <= 1e-4), dist


def test_invalid_inputs_are_rejected():
    prob = Problem(nx=4, ny=4, nz=4, dt=0.05, q=[-1.0], m=[1.0])
    E = _uniform_field(prob, (0, 0, 0))
    with pytest.raises(oracle.OracleError):
        oracle.run(prob, np.array([0]), np.array([[4.0, 1.0, 1.0]]), np.zeros((1, 3)), E, 1)
    with pytest.raises(oracle.OracleError):
        oracle.run(prob, np.array([1]), np.array([[1.0, 1.0, 1.0]]), np.zeros((1, 3)), E, 1)
    Enan = _uniform_field(prob, (float("nan"), 0, 0))
    with pytest.raises(oracle.OracleError):
        oracle.run(prob, np.array([0]), np.array([[1.0, 1.0, 1.0]]), np.zeros((1, 3)), Enan, 1)
