"""Pins of the oracle's field solve with the object as an interface (eq.
(2.2)-(2.5): permittivity eps_in inside the object, the collected surface
charge as the flux-jump source): a two-layer capacitor and a charged sheet,
both solved exactly at the nodes (1-D closed forms); Gauss's law (the flux
through the Dirichlet faces equals the total charge); the interior field of a
dielectric sphere in a uniform field against its closed form; reduction to
the uniform operator; reciprocity; multigrid iteration counts with jumps; the
level sets and the surface charge deposit."""
import math

import numpy as np
import pytest

from oracle import oracle
from oracle.oracle import FieldObject, OracleError, Problem

XM, XP, YM, YP, ZM, ZP = 1, 2, 4, 8, 16, 32


def grid(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    return i.ravel().astype(float), j.ravel().astype(float), k.ravel().astype(float)


def flat_ground(z_flat, eps_in):
    # a crater whose bowl lies far outside the mesh: flat terrain at z_flat
    return FieldObject(kind="crater", eps_in=eps_in, center=(-1000.0, -1000.0, 0.0),
                       z_flat=z_flat, rim_radius=1.0, depth=0.5)


def w_boundary(a, n):
    return np.where((a == 0) | (a == n), 0.5, 1.0)


@pytest.mark.parametrize("n,levels", [((6, 5, 12), 0), ((16, 12, 24), 2)])
@pytest.mark.parametrize("z_flat", [3.0, 3.37, 7.9])
@pytest.mark.parametrize("eps_in", [4.0, 0.3])
def test_two_layer_capacitor_is_exact(n, levels, z_flat, eps_in):
    nx, ny, nz = n
    i, j, k = grid(nx, ny, nz)
    V0, L = 2.0, float(nz)
    info = {}
    phi, it, rr = oracle.field_solve(nx, ny, nz, np.zeros_like(i), ZM | ZP,
                                     values=[0, 0, 0, 0, V0, 0], tol=1e-14, info=info,
                                     obj=flat_ground(z_flat, eps_in))
    assert info["levels"] == levels
    D = V0 / (z_flat / eps_in + (L - z_flat) / 1.0)  # the flux eps E, the same in both layers
    want = np.where(k <= z_flat, V0 - D * k / eps_in, D * (L - k))
    assert np.max(np.abs(phi - want)) < 1e-12


@pytest.mark.parametrize("z_flat", [3.0, 4.25])
def test_charged_sheet_on_the_terrain_is_exact(z_flat):
    # uniform eps; every surface column collected 3 electrons and 1 ion:
    # a sheet of -2 per unit area at z_flat between two grounded plates
    nx, ny, nz = 8, 6, 10
    prob = Problem(nx=nx, ny=ny, nz=nz, dt=0.05, q=[-1.0, 1.0], m=[1.0, 100.0], obj="crater",
                   center=(-1000.0, -1000.0, 0.0), z_flat=z_flat, rim_radius=1.0, depth=0.5)
    tally = np.tile([3, 1], (nx * ny, 1))
    rho_fixed = oracle.surface_rho(prob, tally)
    assert rho_fixed.sum() == -2 * nx * ny * 2 ** 32
    rho = rho_fixed * 2.0 ** -32
    i, j, k = grid(nx, ny, nz)
    phi, it, rr = oracle.field_solve(nx, ny, nz, rho, ZM | ZP, tol=1e-14)
    sigma, L = -2.0, float(nz)
    want = np.where(k <= z_flat, sigma * (L - z_flat) * k / L, sigma * z_flat * (L - k) / L)
    assert np.max(np.abs(phi - want)) < 1e-11


def sphere_setup(m=3, counts_seed=0):
    n = 24
    prob = Problem(nx=n, ny=n, nz=n, dt=0.05, q=[-1.0, 1.0], m=[1.0, 100.0], obj="sphere",
                   center=(11.7, 12.2, 12.05), radius=5.3, sphere_patches=m)
    rng = np.random.default_rng(counts_seed)
    tally = rng.integers(0, 20, size=(prob.nbins, 2))
    return prob, tally


@pytest.mark.parametrize("eps_in", [1.0, 4.0, 10.0])
def test_gauss_law_flux_through_the_faces_is_the_total_charge(eps_in):
    prob, tally = sphere_setup()
    n = prob.nx
    rho = oracle.surface_rho(prob, tally) * 2.0 ** -32
    Q = float((tally @ np.array([-1.0, 1.0])).sum())
    assert abs(rho.sum() - Q) < 1e-9
    obj = oracle.field_object_of(prob, eps_in)
    phi, it, rr = oracle.field_solve(n, n, n, rho, 63, tol=1e-14, obj=obj)
    P = phi.reshape(n + 1, n + 1, n + 1)  # [k, j, i]
    a = np.arange(n + 1)
    wt = w_boundary(a, n)
    W2 = np.outer(wt, wt)
    # links from the first interior layer to each face (plasma side: eps = 1)
    flux = 0.0
    for sl_in, sl_out in ((np.s_[1, :, :], np.s_[0, :, :]), (np.s_[n - 1, :, :], np.s_[n, :, :])):
        for t in range(3):
            Pt = np.moveaxis(P, t, 0)
            flux += (W2[1:-1, 1:-1] * (Pt[sl_in] - Pt[sl_out])[1:-1, 1:-1]).sum()
    assert abs(flux - Q) < 1e-9 * max(1.0, abs(Q))


@pytest.mark.parametrize("eps_in,ratio", [(4.0, 0.5), (0.25, 3.0 / 2.25)])
def test_dielectric_sphere_in_a_uniform_field(eps_in, ratio):
    # E inside = 3 eps / (eps_in + 2 eps) E0 for an isolated sphere; the mesh
    # (R = 6 cells) and the box walls (R / L = 3/16) hold it to a few percent
    n, V = 32, 1.0
    obj = FieldObject(kind="sphere", eps_in=eps_in, center=(16.0, 16.0, 16.0), radius=6.0)
    phi, it, rr = oracle.field_solve(n, n, n, np.zeros((n + 1) ** 3), XM | XP,
                                     values=[V, -V, 0, 0, 0, 0], tol=1e-12, obj=obj)
    P = phi.reshape(n + 1, n + 1, n + 1)
    E0 = 2 * V / n
    Ein = -(P[16, 16, 18] - P[16, 16, 14]) / 4.0
    assert abs(Ein / E0 - ratio) < 0.05 * ratio
    assert abs(Ein / E0 - 1.0) > 0.3  # far from the field without the sphere


def test_equal_permittivities_give_the_uniform_operator():
    n = 16
    rng = np.random.default_rng(3)
    rho = rng.normal(size=(n + 1) ** 3)
    ref, _, _ = oracle.field_solve(n, n, n, rho, ZP, tol=1e-13)
    for obj in (FieldObject(kind="sphere", eps_in=1.0, center=(7.5, 8.2, 8.0), radius=4.0),
                FieldObject(kind="crater", eps_in=1.0, center=(8.0, 8.0, 0.0), z_flat=5.0,
                            rim_radius=5.0, depth=2.0)):
        phi, _, _ = oracle.field_solve(n, n, n, rho, ZP, tol=1e-13, obj=obj)
        assert np.max(np.abs(phi - ref)) < 1e-10 * np.max(np.abs(ref))


def test_reciprocity_with_an_interface():
    n = 12
    nodes = (n + 1) ** 3
    obj = FieldObject(kind="crater", eps_in=4.0, center=(6.0, 6.0, 0.0), z_flat=4.5,
                      rim_radius=4.0, depth=2.0)
    rng = np.random.default_rng(5)
    for mask in (ZP, 63):
        a, b = rng.choice(nodes, 2, replace=False)
        ea = np.zeros(nodes); ea[a] = 1.0
        eb = np.zeros(nodes); eb[b] = 1.0
        pa, _, _ = oracle.field_solve(n, n, n, ea, mask, tol=1e-14, obj=obj)
        pb, _, _ = oracle.field_solve(n, n, n, eb, mask, tol=1e-14, obj=obj)
        assert abs(pa[b] - pb[a]) < 1e-11 * max(1.0, abs(pa[b]))


@pytest.mark.parametrize("eps_in", [4.0, 10.0])
def test_multigrid_with_jumps_stays_fast_and_symmetric(eps_in):
    n = 32
    rng = np.random.default_rng(6)
    rho = rng.normal(size=(n + 1) * (n + 1) * (n // 2 + 1))
    obj = FieldObject(kind="crater", eps_in=eps_in, center=(16.0, 16.0, 0.0), z_flat=6.3,
                      rim_radius=10.0, depth=4.0)
    info = {}
    _, it, rr = oracle.field_solve(n, n, n // 2, rho, ZP, tol=1e-8, info=info, obj=obj)
    _, itj, _ = oracle.field_solve(n, n, n // 2, rho, ZP, tol=1e-8, precond="jacobi", obj=obj)
    assert info["levels"] == 3 and rr <= 1e-8 and it <= 15 and itj > 5 * it
    a, b = rng.normal(size=rho.size), rng.normal(size=rho.size)
    za, _ = oracle.field_vcycle(n, n, n // 2, a, ZP, obj=obj)
    zb, _ = oracle.field_vcycle(n, n, n // 2, b, ZP, obj=obj)
    assert abs(za @ b - zb @ a) < 1e-12 * np.sqrt((za @ za) * (b @ b)) and za @ a > 0


def test_level_sets():
    s = FieldObject(kind="sphere", eps_in=2.0, center=(1.0, 2.0, 3.0), radius=2.0)
    assert oracle.object_psi(s, 1.0, 2.0, 3.0) == -2.0
    assert oracle.object_psi(s, 1.0, 2.0, 7.0) == 2.0
    c = FieldObject(kind="crater", eps_in=2.0, center=(10.0, 10.0, 0.0), z_flat=5.0,
                    rim_radius=4.0, depth=2.0)
    assert oracle.object_psi(c, 30.0, 10.0, 5.0) == 0.0      # flat ground
    assert oracle.object_psi(c, 30.0, 10.0, 2.5) == -2.5
    assert abs(oracle.object_psi(c, 10.0, 10.0, 3.0)) < 1e-15  # bowl bottom at z_flat - depth
    assert abs(oracle.object_psi(c, 14.0, 10.0, 5.0)) < 1e-14  # rim
    Rc = (16 + 4) / 4.0
    assert abs(oracle.object_psi(c, 12.0, 10.0, 3.0) - (3.0 - (3.0 + Rc - math.sqrt(Rc * Rc - 4)))) < 1e-14


def test_surface_charge_points_and_settings():
    prob, tally = sphere_setup(m=2)
    rho = oracle.surface_rho(prob, tally)
    assert rho.sum() == int((tally @ np.array([-1, 1])).sum()) * 2 ** 32
    # the charge sits within one cell of the sphere surface
    i, j, k = grid(prob.nx, prob.ny, prob.nz)
    r = np.sqrt((i - 11.7) ** 2 + (j - 12.2) ** 2 + (k - 12.05) ** 2)
    assert np.all(np.abs(r[rho != 0] - 5.3) < math.sqrt(3))
    one = Problem(nx=8, ny=8, nz=8, dt=0.05, q=[-1.0], m=[1.0], obj="sphere", center=(4, 4, 4),
                  radius=2.0)
    with pytest.raises(OracleError):
        oracle.surface_rho(one, np.zeros((1, 1), np.int64))  # no patches: no surface points
    with pytest.raises(OracleError):
        oracle.field_solve(8, 8, 8, np.zeros(729), ZP,
                           obj=FieldObject(kind="sphere", eps_in=0.0, center=(4, 4, 4), radius=2))
