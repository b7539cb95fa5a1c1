"""Pins of the oracle's field solve (the boundary value problem of §2.1 with a
uniform permittivity, node-centred finite volumes, Jacobi-preconditioned CG)
and of E = -grad phi: exact discrete eigenfunctions, exactly reproduced
linear and quadratic potentials, the symmetry of the Green's function, warm
starts and argument checks."""
import math

import numpy as np
import pytest

from oracle import oracle
from oracle.oracle import OracleError

XM, XP, YM, YP, ZM, ZP = 1, 2, 4, 8, 16, 32


def grid(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    return i.ravel().astype(float), j.ravel().astype(float), k.ravel().astype(float)


def vol_fraction(nx, ny, nz):
    i, j, k = grid(nx, ny, nz)
    f = np.ones_like(i)
    for a, n in ((i, nx), (j, ny), (k, nz)):
        f = f * np.where((a == 0) | (a == n), 0.5, 1.0)
    return f


@pytest.mark.parametrize("n,h,eps", [((6, 5, 4), 1.0, 1.0), ((9, 7, 8), 0.5, 2.5)])
def test_dirichlet_sine_mode_is_an_eigenvector(n, h, eps):
    nx, ny, nz = n
    i, j, k = grid(nx, ny, nz)
    phi = np.sin(math.pi * i / nx) * np.sin(math.pi * j / ny) * np.sin(math.pi * k / nz)
    lam = sum(2.0 - 2.0 * math.cos(math.pi / m) for m in n)
    rho = eps / h ** 2 * lam * phi
    got, it, rr = oracle.field_solve(nx, ny, nz, rho, 63, h=h, eps=eps, tol=1e-13)
    assert rr <= 1e-13
    assert np.max(np.abs(got - phi)) < 1e-11


def test_neumann_min_faces_cosine_mode():
    # zero-Neumann at the min faces, phi = 0 at the max faces (the OML field setup)
    nx, ny, nz = 7, 6, 5
    i, j, k = grid(nx, ny, nz)
    th = [math.pi / (2 * m) for m in (nx, ny, nz)]
    phi = np.cos(th[0] * i) * np.cos(th[1] * j) * np.cos(th[2] * k)
    lam = sum(2.0 - 2.0 * math.cos(t) for t in th)
    # the deposited density of a node counts only the part of its cloud in the box
    rho = lam * phi * vol_fraction(nx, ny, nz)
    got, it, rr = oracle.field_solve(nx, ny, nz, rho, XP | YP | ZP, tol=1e-13)
    assert np.max(np.abs(got - phi)) < 1e-11


def test_linear_potential_and_its_field():
    nx, ny, nz, h = 8, 5, 6, 0.25
    i, j, k = grid(nx, ny, nz)
    rho = np.zeros_like(i)
    phi, it, rr = oracle.field_solve(nx, ny, nz, rho, XM | XP, values=[2.0, -1.0, 0, 0, 0, 0], h=h,
                                     tol=1e-14)
    want = 2.0 - 3.0 * i / nx
    assert np.max(np.abs(phi - want)) < 1e-12
    E = oracle.field_E(nx, ny, nz, phi, XM | XP, h=h)
    assert np.max(np.abs(E[0] - 3.0 / (nx * h))) < 1e-10
    assert np.max(np.abs(E[1])) < 1e-10 and np.max(np.abs(E[2])) < 1e-10


def test_uniform_charge_between_two_plates_is_the_parabola():
    nx, ny, nz, h, rho0 = 10, 4, 3, 0.5, 3.0
    i, j, k = grid(nx, ny, nz)
    x = i * h
    L = nx * h
    rho = rho0 * vol_fraction(nx, ny, nz)
    phi, it, rr = oracle.field_solve(nx, ny, nz, rho, XM | XP, h=h, tol=1e-14)
    # with phi = 0 on the plates the boundary rows carry only their half volume;
    # rho on the plates does not enter the system
    want = rho0 * x * (L - x) / 2.0
    assert np.max(np.abs(phi - want)) < 1e-10
    E = oracle.field_E(nx, ny, nz, phi, XM | XP, h=h)
    assert np.max(np.abs(E[0] + rho0 * (L - 2 * x) / 2.0)) < 1e-9


def test_green_function_is_symmetric():
    nx, ny, nz = 5, 4, 6
    nodes = (nx + 1) * (ny + 1) * (nz + 1)
    rng = np.random.default_rng(3)
    for mask in (ZP, XM | YP, 63):
        a, b = rng.choice(nodes, 2, replace=False)
        ea = np.zeros(nodes); ea[a] = 1.0
        eb = np.zeros(nodes); eb[b] = 1.0
        pa, _, _ = oracle.field_solve(nx, ny, nz, ea, mask, tol=1e-14)
        pb, _, _ = oracle.field_solve(nx, ny, nz, eb, mask, tol=1e-14)
        assert abs(pa[b] - pb[a]) < 1e-11 * max(1.0, abs(pa[b]))


def test_warm_start_needs_no_iteration_and_tolerance_is_met():
    nx, ny, nz = 8, 8, 8
    rng = np.random.default_rng(4)
    rho = rng.normal(size=(nx + 1) ** 3)
    phi, it, rr = oracle.field_solve(nx, ny, nz, rho, ZP, tol=1e-8)
    assert 0 < it < 500 and rr <= 1e-8
    phi2, it2, rr2 = oracle.field_solve(nx, ny, nz, rho, ZP, phi0=phi, tol=1e-8)
    assert it2 == 0 and np.array_equal(phi, phi2)


def test_field_arguments_are_checked():
    rho = np.zeros(27)
    for mask in (0, 64):
        with pytest.raises(OracleError):
            oracle.field_solve(2, 2, 2, rho, mask)
    with pytest.raises(OracleError):
        oracle.field_solve(2, 2, 2, rho, 1, tol=0.0)
