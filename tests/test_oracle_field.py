"""Pins of the oracle's field solve (the boundary value problem of §2.1 with a
uniform permittivity, node-centred finite volumes, preconditioned CG with the
Jacobi or the multigrid V-cycle preconditioner) and of E = -grad phi: exact
discrete eigenfunctions, exactly reproduced linear and quadratic potentials,
the symmetry of the Green's function, warm starts, argument checks; for the
V-cycle: its symmetry and definiteness, its equality with the two-grid
operator assembled as matrices, and iteration counts that do not grow with
the grid."""
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


def solve(nx, ny, nz, rho, mask, precond, levels, **kw):
    """The oracle's solve with the given preconditioner; checks which one ran
    (levels: the multigrid level count expected, 0 for Jacobi)."""
    info = {}
    out = oracle.field_solve(nx, ny, nz, rho, mask, precond=precond, info=info, **kw)
    assert info["levels"] == levels
    return out


# (grid, preconditioner, multigrid levels): grids of at most 1024 nodes, or
# with an odd cell count, keep Jacobi
SINE_CASES = [((6, 5, 4), 1.0, 1.0, "multigrid", 0), ((9, 7, 8), 0.5, 2.5, "multigrid", 0),
              ((16, 12, 8), 0.5, 2.5, "multigrid", 2), ((32, 16, 16), 1.0, 1.0, "multigrid", 3),
              ((32, 16, 16), 1.0, 1.0, "jacobi", 0)]


@pytest.mark.parametrize("n,h,eps,precond,levels", SINE_CASES)
def test_dirichlet_sine_mode_is_an_eigenvector(n, h, eps, precond, levels):
    nx, ny, nz = n
    i, j, k = grid(nx, ny, nz)
    phi = np.sin(math.pi * i / nx) * np.sin(math.pi * j / ny) * np.sin(math.pi * k / nz)
    lam = sum(2.0 - 2.0 * math.cos(math.pi / m) for m in n)
    rho = eps / h ** 2 * lam * phi
    got, it, rr = solve(nx, ny, nz, rho, 63, precond, levels, h=h, eps=eps, tol=1e-13)
    assert rr <= 1e-13
    assert np.max(np.abs(got - phi)) < 1e-11


@pytest.mark.parametrize("n,levels", [((7, 6, 5), 0), ((16, 12, 10), 2)])
def test_neumann_min_faces_cosine_mode(n, levels):
    # zero-Neumann at the min faces, phi = 0 at the max faces (the OML field setup)
    nx, ny, nz = n
    i, j, k = grid(nx, ny, nz)
    th = [math.pi / (2 * m) for m in (nx, ny, nz)]
    phi = np.cos(th[0] * i) * np.cos(th[1] * j) * np.cos(th[2] * k)
    lam = sum(2.0 - 2.0 * math.cos(t) for t in th)
    # the deposited density of a node counts only the part of its cloud in the box
    rho = lam * phi * vol_fraction(nx, ny, nz)
    got, it, rr = solve(nx, ny, nz, rho, XP | YP | ZP, "multigrid", levels, tol=1e-13)
    assert np.max(np.abs(got - phi)) < 1e-11


@pytest.mark.parametrize("n,levels", [((8, 5, 6), 0), ((16, 10, 12), 2)])
def test_linear_potential_and_its_field(n, levels):
    (nx, ny, nz), h = n, 0.25
    i, j, k = grid(nx, ny, nz)
    rho = np.zeros_like(i)
    phi, it, rr = solve(nx, ny, nz, rho, XM | XP, "multigrid", levels,
                        values=[2.0, -1.0, 0, 0, 0, 0], h=h, tol=1e-14)
    want = 2.0 - 3.0 * i / nx
    assert np.max(np.abs(phi - want)) < 1e-12
    E = oracle.field_E(nx, ny, nz, phi, XM | XP, h=h)
    assert np.max(np.abs(E[0] - 3.0 / (nx * h))) < 1e-10
    assert np.max(np.abs(E[1])) < 1e-10 and np.max(np.abs(E[2])) < 1e-10


@pytest.mark.parametrize("n,levels", [((10, 4, 3), 0), ((20, 8, 6), 2)])
def test_uniform_charge_between_two_plates_is_the_parabola(n, levels):
    (nx, ny, nz), h, rho0 = n, 0.5, 3.0
    i, j, k = grid(nx, ny, nz)
    x = i * h
    L = nx * h
    rho = rho0 * vol_fraction(nx, ny, nz)
    phi, it, rr = solve(nx, ny, nz, rho, XM | XP, "multigrid", levels, h=h, tol=1e-14)
    # with phi = 0 on the plates the boundary rows carry only their half volume;
    # rho on the plates does not enter the system
    want = rho0 * x * (L - x) / 2.0
    assert np.max(np.abs(phi - want)) < 1e-10
    E = oracle.field_E(nx, ny, nz, phi, XM | XP, h=h)
    assert np.max(np.abs(E[0] + rho0 * (L - 2 * x) / 2.0)) < 1e-9


@pytest.mark.parametrize("n,levels", [((5, 4, 6), 0), ((10, 8, 12), 2)])
def test_green_function_is_symmetric(n, levels):
    nx, ny, nz = n
    nodes = (nx + 1) * (ny + 1) * (nz + 1)
    rng = np.random.default_rng(3)
    for mask in (ZP, XM | YP, 63):
        a, b = rng.choice(nodes, 2, replace=False)
        ea = np.zeros(nodes); ea[a] = 1.0
        eb = np.zeros(nodes); eb[b] = 1.0
        pa, _, _ = solve(nx, ny, nz, ea, mask, "multigrid", levels, tol=1e-14)
        pb, _, _ = solve(nx, ny, nz, eb, mask, "multigrid", levels, tol=1e-14)
        assert abs(pa[b] - pb[a]) < 1e-11 * max(1.0, abs(pa[b]))


@pytest.mark.parametrize("n,precond", [((8, 8, 8), "multigrid"), ((16, 16, 16), "multigrid"),
                                       ((16, 16, 16), "jacobi")])
def test_warm_start_needs_no_iteration_and_tolerance_is_met(n, precond):
    nx, ny, nz = n
    rng = np.random.default_rng(4)
    rho = rng.normal(size=(nx + 1) * (ny + 1) * (nz + 1))
    phi, it, rr = oracle.field_solve(nx, ny, nz, rho, ZP, tol=1e-8, precond=precond)
    assert 0 < it < 500 and rr <= 1e-8
    phi2, it2, rr2 = oracle.field_solve(nx, ny, nz, rho, ZP, phi0=phi, tol=1e-8, precond=precond)
    assert it2 == 0 and np.array_equal(phi, phi2)


def test_field_arguments_are_checked():
    rho = np.zeros(27)
    for mask in (0, 64):
        with pytest.raises(OracleError):
            oracle.field_solve(2, 2, 2, rho, mask)
    with pytest.raises(OracleError):
        oracle.field_solve(2, 2, 2, rho, 1, tol=0.0)
    with pytest.raises(KeyError):
        oracle.field_solve(2, 2, 2, rho, 1, precond="ilu")


# ---- the multigrid V-cycle -------------------------------------------------------

def fv_matrix(nx, ny, nz, h, eps, mask):
    """The finite-volume operator assembled from its definition: for each pair
    of neighbouring nodes, -eps/h^2 times the product of the two tangential
    half-width factors (1/2 on a boundary index); Dirichlet rows and columns
    removed. Returns (A, unknown mask)."""
    i, j, k = grid(nx, ny, nz)
    n = (nx, ny, nz)
    N = i.size
    c = [np.where((a == 0) | (a == m), 0.5, 1.0) for a, m in zip((i, j, k), n)]
    A = np.zeros((N, N))
    idx = np.arange(N)
    step = (1, nx + 1, (nx + 1) * (ny + 1))
    coord = (i, j, k)
    for d in range(3):
        t = [c[e] for e in range(3) if e != d]
        has = coord[d] < n[d]
        p = idx[has]
        q = p + step[d]
        w = eps / h ** 2 * (t[0] * t[1])[has]
        A[p, q] -= w
        A[q, p] -= w
        A[p, p] += w
        A[q, q] += w
    dirn = np.zeros(N, bool)
    for f, (a, val) in enumerate(((i, 0), (i, nx), (j, 0), (j, ny), (k, 0), (k, nz))):
        if (mask >> f) & 1:
            dirn |= a == val
    u = ~dirn
    return A[np.ix_(u, u)], u


def hat_interpolation(nx, ny, nz):
    """Trilinear interpolation from the grid with half the cells to the fine
    grid, as tensor products of 1-D hat functions of width two fine cells."""
    def one(n):
        x = np.arange(n + 1)[:, None]
        X = 2 * np.arange(n // 2 + 1)[None, :]
        return np.maximum(0.0, 1.0 - np.abs(x - X) / 2.0)
    Px, Py, Pz = one(nx), one(ny), one(nz)
    return np.kron(Pz, np.kron(Py, Px))


def test_two_grid_vcycle_equals_the_assembled_operator():
    nx, ny, nz, h, eps, omega = 12, 10, 8, 0.5, 1.5, 6.0 / 7.0
    for mask in (63, ZP, XP | YP | ZP):
        A, u = fv_matrix(nx, ny, nz, h, eps, mask)
        Ac, uc = fv_matrix(nx // 2, ny // 2, nz // 2, 2 * h, eps, mask)
        P = hat_interpolation(nx, ny, nz)[np.ix_(u, uc)]
        Dinv = np.diag(1.0 / np.diag(A))
        I = np.eye(A.shape[0])
        S = np.zeros_like(A)           # two damped-Jacobi sweeps from zero, as a matrix
        for _ in range(2):
            S = S + omega * Dinv @ (I - A @ S)
        B = S + P @ np.linalg.solve(Ac, P.T / 8.0 @ (I - A @ S))
        for _ in range(2):
            B = B + omega * Dinv @ (I - A @ B)
        assert np.max(np.abs(B - B.T)) < 1e-12 * np.max(np.abs(B))
        rng = np.random.default_rng(mask)
        for _ in range(3):
            r = np.zeros(u.size)
            r[u] = rng.normal(size=u.sum())
            z, levels = oracle.field_vcycle(nx, ny, nz, r, mask, h=h, eps=eps)
            assert levels == 2
            want = B @ r[u]
            assert np.max(np.abs(z[u] - want)) < 1e-12 * np.max(np.abs(want))
            assert np.all(z[~u] == 0.0)


@pytest.mark.parametrize("mask", [63, ZP, XP | YP | ZP])
def test_vcycle_is_symmetric_positive_definite(mask):
    nx, ny, nz = 32, 16, 16
    nodes = 33 * 17 * 17
    rng = np.random.default_rng(7)
    a, b = rng.normal(size=nodes), rng.normal(size=nodes)
    za, levels = oracle.field_vcycle(nx, ny, nz, a, mask)
    zb, _ = oracle.field_vcycle(nx, ny, nz, b, mask)
    assert levels == 3
    assert abs(za @ b - zb @ a) < 1e-12 * np.sqrt((za @ za) * (b @ b))
    # on the unknown nodes (the Dirichlet nodes are not in the operator)
    assert za @ a > 0 and zb @ b > 0
    # values on the Dirichlet nodes are not part of the residual
    _, u = fv_matrix(nx, ny, nz, 1.0, 1.0, mask)
    z0, _ = oracle.field_vcycle(nx, ny, nz, np.where(u, 0.0, 1.0), mask)
    assert np.all(z0 == 0.0)
    # a grid of at most 1024 nodes is not coarsened
    assert oracle.field_vcycle(8, 8, 8, np.ones(729), mask) == (None, 0)


def test_multigrid_iterations_do_not_grow_with_the_grid():
    counts = []
    for n in (16, 32, 64):
        rng = np.random.default_rng(n)
        rho = rng.normal(size=(n + 1) ** 3)
        info = {}
        _, it, rr = oracle.field_solve(n, n, n, rho, 63, tol=1e-8, info=info)
        assert rr <= 1e-8 and info["levels"] >= 2
        counts.append(it)
    assert max(counts) <= 10 and max(counts) - min(counts) <= 2
    rho = np.random.default_rng(5).normal(size=33 ** 3)
    _, itj, _ = oracle.field_solve(32, 32, 32, rho, 63, tol=1e-8, precond="jacobi")
    assert itj > 8 * max(counts)
