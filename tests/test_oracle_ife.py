"""Pins of the oracle's immersed finite elements (the paper's discretisation of
the interface on the PIC mesh cut into five tetrahedra per cell, §2.3 and
§3.1.1), each against what the mathematics fixes: the five tetrahedra fill
every cube and neighbouring cubes share their face diagonals; an uncut
element is the linear finite element (gradients of the barycentric
coordinates computed here independently); a cut element's basis functions
take their vertex values, are continuous across the interface plane and
carry a continuous flux eps dphi/dn, and reproduce every piecewise-linear
function with that flux condition; the inside volume against a Monte Carlo
estimate and its complement; the element matrix against the basis;
linear potentials are discrete-harmonic (patch test); the assembled
operator is symmetric; a two-layer capacitor with a mesh-aligned interface
is solved exactly and with a fractional interface converges under
refinement; Gauss's law holds exactly; a dielectric sphere in a uniform
field has the closed-form interior field; equal permittivities give the
plain elements; the multigrid V-cycle stays symmetric and preconditions it."""
import numpy as np
import pytest

from oracle import oracle

CORNERS = [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]


def barycentric_gradients(X):
    """Independent of the oracle: rows of inv([X 1]) are the coefficients of
    the barycentric coordinates."""
    M = np.hstack([X, np.ones((4, 1))])
    C = np.linalg.inv(M)
    return C[:3, :].T, abs(np.linalg.det(M)) / 6.0


def random_cut(rng):
    while True:
        T = oracle.cube_tets(*rng.integers(0, 5, 3))[rng.integers(5)].astype(np.float64)
        psi = rng.normal(size=4)
        if rng.random() < 0.25:
            psi[rng.integers(4)] = 0.0
        if (psi < 0).any() and (psi >= 0).any():
            return T, psi


@pytest.mark.parametrize("cube", [(0, 0, 0), (1, 0, 0), (3, 4, 6)])
def test_five_tetrahedra_fill_the_cube(cube):
    T = oracle.cube_tets(*cube).astype(np.float64)
    vols = [barycentric_gradients(t)[1] for t in T]
    assert np.isclose(sum(vols), 1.0, rtol=0, atol=1e-15)
    assert np.isclose(vols[0], 1 / 3) and np.allclose(vols[1:], 1 / 6)
    # every point of the cube lies in exactly one tetrahedron
    pts = np.random.default_rng(1).uniform(0, 1, size=(4000, 3))
    inside = np.zeros((len(pts), 5), bool)
    for t in range(5):
        M = np.hstack([T[t], np.ones((4, 1))])
        lam = np.linalg.solve(M.T, np.hstack([pts, np.ones((len(pts), 1))]).T).T
        inside[:, t] = (lam > 1e-12).all(axis=1)
    assert (inside.sum(axis=1) == 1).all()


def edges_on_face(cube, axis, side):
    """Mesh edges of a cube lying on one of its faces (global node triples)."""
    out = set()
    for t in oracle.cube_tets(*cube):
        g = [tuple(int(v) for v in np.asarray(cube) + c) for c in t]
        for a in range(4):
            for b in range(a + 1, 4):
                if g[a][axis] == g[b][axis] == cube[axis] + side:
                    out.add(frozenset((g[a], g[b])))
    return out


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_neighbouring_cubes_share_their_face_diagonals(axis):
    c0 = (2, 3, 4)
    c1 = tuple(c0[d] + (1 if d == axis else 0) for d in range(3))
    assert edges_on_face(c0, axis, 1) == edges_on_face(c1, axis, 0)


def test_uncut_element_is_the_linear_finite_element():
    rng = np.random.default_rng(2)
    for _ in range(20):
        T = oracle.cube_tets(*rng.integers(0, 5, 3))[rng.integers(5)].astype(np.float64) * 0.7
        G, V = barycentric_gradients(T)
        for psi, eps in ((np.full(4, 1.0), 2.5), (np.full(4, -1.0), 7.0), (np.zeros(4), 2.5)):
            K = oracle.ife_element(T, psi, 7.0, 2.5)
            assert np.allclose(K, eps * V * G @ G.T, rtol=1e-13, atol=1e-15)


def test_cut_basis_takes_its_vertex_values_and_the_interface_conditions():
    rng = np.random.default_rng(3)
    for _ in range(300):
        T, psi = random_cut(rng)
        ein, eout = 10 ** rng.uniform(-2, 2), 10 ** rng.uniform(-2, 2)
        B = oracle.ife_basis(T, psi, ein, eout)
        G, V = barycentric_gradients(T)
        assert B["cut"] and np.isclose(B["vol"], V)
        g = psi @ G
        assert np.allclose(B["g"], g, rtol=1e-12, atol=1e-14)
        d = np.where(psi < 0, 0.0, psi)
        for i in range(4):
            # phi- = sum_j c_ij lambda_j; phi+ = phi- + t psi_h: vertex values
            vals = B["c"][i] + B["t"][i] * d
            assert np.allclose(vals, np.eye(4)[i], atol=1e-12)
            assert np.allclose(B["a"][i], B["c"][i] @ G, rtol=1e-12, atol=1e-12)
            # flux continuity across the interface plane (normal g)
            fin = ein * B["a"][i] @ g
            fout = eout * (B["a"][i] + B["t"][i] * g) @ g
            assert np.isclose(fin, fout, rtol=1e-11, atol=1e-12 * (abs(fin) + 1))


def test_cut_element_reproduces_piecewise_linear_solutions():
    # u- = alpha . x + beta inside, u+ = u- + tau psi_h with the flux condition:
    # its interpolant through the basis is u itself
    rng = np.random.default_rng(4)
    for _ in range(200):
        T, psi = random_cut(rng)
        ein, eout = 10 ** rng.uniform(-2, 2), 10 ** rng.uniform(-2, 2)
        G, _ = barycentric_gradients(T)
        g = psi @ G
        alpha, beta = rng.normal(size=3), rng.normal()
        tau = (ein - eout) / (eout * (g @ g)) * (alpha @ g)
        u = T @ alpha + beta + tau * np.where(psi < 0, 0.0, psi)
        B = oracle.ife_basis(T, psi, ein, eout)
        assert np.allclose(u @ B["a"], alpha, rtol=1e-10, atol=1e-10)
        assert np.isclose(u @ B["t"], tau, rtol=1e-10, atol=1e-10)


def test_inside_volume():
    rng = np.random.default_rng(5)
    T = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float64)
    # one vertex alone inside, the plane through the edge midpoints: 1/8 of it
    B = oracle.ife_basis(T, np.array([-1.0, 1.0, 1.0, 1.0]), 4.0, 1.0)
    assert np.isclose(B["vin"], B["vol"] / 8, rtol=1e-15)
    for _ in range(30):
        T, psi = random_cut(rng)
        psi = np.where(psi == 0.0, 0.3, psi)
        a = oracle.ife_basis(T, psi, 2.0, 1.0)
        b = oracle.ife_basis(T, -psi, 2.0, 1.0)
        assert np.isclose(a["vin"] + b["vin"], a["vol"], rtol=1e-13)
        # Monte Carlo: points uniform in the tetrahedron (Dirichlet weights)
        lam = rng.dirichlet(np.ones(4), 200000)
        frac = ((lam @ psi) < 0).mean()
        want = a["vin"] / a["vol"]
        sd = np.sqrt(max(want * (1 - want), 1.0 / len(lam)) / len(lam))
        assert abs(frac - want) < 5 * sd


def test_element_matrix_from_the_basis():
    rng = np.random.default_rng(6)
    for _ in range(200):
        T, psi = random_cut(rng)
        ein, eout = 10 ** rng.uniform(-2, 2), 10 ** rng.uniform(-2, 2)
        B = oracle.ife_basis(T, psi, ein, eout)
        K = oracle.ife_element(T, psi, ein, eout)
        b = B["a"] + B["t"][:, None] * B["g"][None, :]
        want = ein * B["vin"] * B["a"] @ B["a"].T + eout * (B["vol"] - B["vin"]) * b @ b.T
        assert np.allclose(K, want, rtol=1e-12, atol=1e-14 * np.abs(want).max())
        assert np.array_equal(K, K.T)
        scale = np.abs(K).max()
        assert np.abs(K.sum(axis=1)).max() <= 1e-10 * scale
        assert np.linalg.eigvalsh(K).min() >= -1e-10 * scale


def node_coords(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(np.float64)


def apply_links(links, phi, nx, ny, nz):
    """(A phi)_p = sum_q c_pq (phi_p - phi_q) over the in-box neighbours."""
    X = node_coords(nx, ny, nz).astype(int)
    out = np.zeros(len(phi))
    for l, (di, dj, dk) in enumerate(oracle.IFE_LINKS):
        q = X + [di, dj, dk]
        ok = (q >= 0).all(1) & (q[:, 0] <= nx) & (q[:, 1] <= ny) & (q[:, 2] <= nz)
        qi = q[ok, 0] + (nx + 1) * (q[ok, 1] + (ny + 1) * q[ok, 2])
        out[ok] += links[ok, l] * (phi[ok] - phi[qi])
    return out


SPHERE = oracle.FieldObject(kind="sphere", eps_in=4.0, center=(6.3, 5.6, 6.1), radius=3.4)
CRATER = oracle.FieldObject(kind="crater", eps_in=10.0, center=(6.0, 5.0, 0.0), z_flat=6.5,
                            rim_radius=4.0, depth=2.5)


@pytest.mark.parametrize("obj", [None, SPHERE])
def test_linear_potentials_are_discrete_harmonic(obj):
    nx, ny, nz = 12, 11, 13
    links = oracle.ife_links(nx, ny, nz, h=0.5, eps=2.0, obj=obj)
    X = node_coords(nx, ny, nz)
    phi = X @ [0.7, -1.3, 0.4] + 2.0
    r = apply_links(links, phi, nx, ny, nz)
    interior = ((X > 0) & (X < [nx, ny, nz])).all(axis=1)
    if obj is not None:  # away from the elements that the interface cuts
        far = np.abs(np.linalg.norm(X - obj.center, axis=1) - obj.radius) > 2.0
        interior &= far
    assert np.abs(r[interior]).max() < 1e-12


@pytest.mark.parametrize("obj", [SPHERE, CRATER])
def test_assembled_operator_is_symmetric_with_zero_row_sums(obj):
    nx, ny, nz = 12, 11, 13
    links = oracle.ife_links(nx, ny, nz, obj=obj)
    X = node_coords(nx, ny, nz).astype(int)
    for l, off in enumerate(oracle.IFE_LINKS):
        back = oracle.IFE_LINKS.index(tuple(-o for o in off))
        q = X + off
        ok = (q >= 0).all(1) & (q[:, 0] <= nx) & (q[:, 1] <= ny) & (q[:, 2] <= nz)
        qi = q[ok, 0] + (nx + 1) * (q[ok, 1] + (ny + 1) * q[ok, 2])
        assert np.array_equal(links[ok, l], links[qi, back])
        assert not links[~ok, l].any()  # no link leaves the box
    # the constant is in the kernel: A 1 = 0 (rows sum to zero) up to rounding
    r = apply_links(links, np.ones(len(X)), nx, ny, nz)
    assert np.abs(r).max() == 0.0


def test_equal_permittivities_give_the_plain_elements():
    nx, ny, nz = 12, 11, 13
    same = oracle.FieldObject(kind="sphere", eps_in=2.0, center=SPHERE.center, radius=SPHERE.radius)
    a = oracle.ife_links(nx, ny, nz, eps=2.0, obj=same)
    b = oracle.ife_links(nx, ny, nz, eps=2.0)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-15)


def capacitor(nz_cells, h, z0, ein, precond="multigrid", tol=1e-13):
    """Plates phi = 0 at z = 0 and 1 at the top, ground below z0 (eps_in)."""
    nx = ny = 8
    nz = nz_cells
    obj = oracle.FieldObject(kind="crater", eps_in=ein, center=(1e3, 1e3, 0.0),
                             z_flat=z0 / h, rim_radius=1.0, depth=1.0)
    rho = np.zeros((nx + 1) * (ny + 1) * (nz + 1))
    info = {}
    phi, it, rr = oracle.field_solve(nx, ny, nz, rho, 16 | 32, values=[0, 0, 0, 0, 0.0, 1.0],
                                     h=h, obj=obj, op="ife", tol=tol, precond=precond, info=info)
    L = nz * h
    D = 1.0 / (z0 / ein + (L - z0))
    z = np.arange(nz + 1) * h
    exact = np.where(z < z0, D * z / ein, D * z0 / ein + D * (z - z0))
    return np.abs(phi.reshape(nz + 1, ny + 1, nx + 1) - exact[:, None, None]).max(), it, info


@pytest.mark.parametrize("ein", [4.0, 0.3])
@pytest.mark.parametrize("precond", ["multigrid", "jacobi"])
def test_two_layer_capacitor_with_a_mesh_aligned_interface_is_exact(ein, precond):
    err, it, info = capacitor(16, 1.0, 5.0, ein, precond)
    assert err < 1e-11
    assert (info["levels"] >= 2) == (precond == "multigrid")


def test_two_layer_capacitor_with_a_fractional_interface_converges():
    # the interface at 3.3 of a height of 8: the linear IFE is not exact there
    # (its basis functions do not match across element faces); the nodal
    # error falls under refinement
    errs = [capacitor(8 * m, 1.0 / m, 3.3, 4.0)[0] for m in (1, 2, 4, 8)]
    assert errs[0] < 0.01
    assert errs[-1] < errs[0] / 3
    assert all(b < a for a, b in zip(errs, errs[1:]))


@pytest.mark.parametrize("obj", [SPHERE, CRATER])
def test_gauss_law_is_exact(obj):
    # grounded box: the flux leaving through the Dirichlet nodes equals the
    # charge inside (the operator is symmetric with zero row sums)
    nx, ny, nz = 12, 11, 13
    rng = np.random.default_rng(9)
    rho = np.zeros((nx + 1) * (ny + 1) * (nz + 1))
    X = node_coords(nx, ny, nz)
    interior = np.nonzero(((X > 0) & (X < [nx, ny, nz])).all(axis=1))[0]
    rho[rng.choice(interior, 40, replace=False)] = rng.normal(size=40)
    phi, _, _ = oracle.field_solve(nx, ny, nz, rho, 63, obj=obj, op="ife", tol=1e-14)
    links = oracle.ife_links(nx, ny, nz, obj=obj)
    Aphi = apply_links(links, phi, nx, ny, nz)
    boundary = ~((X > 0) & (X < [nx, ny, nz])).all(axis=1)
    assert np.isclose(-Aphi[boundary].sum(), rho.sum(), rtol=1e-9)
    assert np.abs(Aphi[interior] - rho[interior]).max() < 1e-10 * np.abs(rho).max()


@pytest.mark.parametrize("ein", [4.0, 0.25])
def test_dielectric_sphere_in_a_uniform_field(ein):
    # closed form: inside a dielectric sphere in a uniform field E0 the field
    # is uniform, 3 eps / (eps_in + 2 eps) E0; walls at +-L/2 with fixed
    # potentials, zero-Neumann sides
    n = 32
    R = 6.0
    c = (n / 2, n / 2, n / 2)
    obj = oracle.FieldObject(kind="sphere", eps_in=ein, center=c, radius=R)
    E0 = 1.0
    rho = np.zeros((n + 1) ** 3)
    phi, it, _ = oracle.field_solve(n, n, n, rho, 1 | 2, values=[E0 * n / 2, -E0 * n / 2, 0, 0, 0, 0],
                                    obj=obj, op="ife", tol=1e-10)
    E = oracle.field_E(n, n, n, phi, 1 | 2)
    X = node_coords(n, n, n)
    core = np.linalg.norm(X - c, axis=1) < R - 2.0
    want = 3.0 / (ein + 2.0) * E0
    assert abs(E[0][core].mean() - want) < 0.05 * want
    assert np.abs(E[1][core]).max() < 0.05 * want and np.abs(E[2][core]).max() < 0.05 * want


def test_ife_and_finite_volumes_solve_the_same_problem():
    n = 24
    obj = oracle.FieldObject(kind="sphere", eps_in=4.0, center=(12.2, 11.7, 12.4), radius=5.3)
    rng = np.random.default_rng(10)
    rho = rng.normal(size=(n + 1) ** 3) * 0.1 + 0.05
    a, _, _ = oracle.field_solve(n, n, n, rho, 63, obj=obj, op="ife", tol=1e-10)
    b, _, _ = oracle.field_solve(n, n, n, rho, 63, obj=obj, op="fv", tol=1e-10)
    assert np.abs(a - b).max() < 0.05 * np.abs(b).max()


@pytest.mark.parametrize("obj", [SPHERE, CRATER])
def test_multigrid_preconditions_the_ife_operator(obj):
    n = 32
    big = oracle.FieldObject(**{**obj.__dict__, "center": tuple(2.5 * v for v in obj.center),
                                "radius": 2.5 * obj.radius,
                                "z_flat": 2.5 * obj.z_flat, "rim_radius": 2.5 * obj.rim_radius,
                                "depth": 2.5 * obj.depth})
    rng = np.random.default_rng(11)
    rho = rng.normal(size=(n + 1) ** 3)
    info = {}
    _, it_mg, rr = oracle.field_solve(n, n, n, rho, 32, obj=big, op="ife", tol=1e-8, info=info)
    _, it_j, _ = oracle.field_solve(n, n, n, rho, 32, obj=big, op="ife", tol=1e-8,
                                    precond="jacobi")
    assert info["levels"] >= 3 and rr <= 1e-8
    assert it_mg <= 30 and it_mg * 4 < it_j
    # one V-cycle with the IFE operator on the finest level is symmetric
    r1, r2 = rng.normal(size=(2, (n + 1) ** 3))
    m = node_coords(n, n, n)[:, 2] == n
    r1[m] = r2[m] = 0.0
    z1, _ = oracle.field_vcycle(n, n, n, r1, 32, obj=big, op="ife")
    z2, _ = oracle.field_vcycle(n, n, n, r2, 32, obj=big, op="ife")
    assert np.isclose(r1 @ z2, r2 @ z1, rtol=1e-11)
    assert r1 @ z1 > 0 and r2 @ z2 > 0
