"""The field solve by immersed finite elements on the GPU (pic_field.op =
PIC_FIELD_IFE) against the oracle's: the two-layer capacitor with a
mesh-aligned interface is exact; with a fractional one both give the same
(approximate) solution; a sphere with surface patches and the crater terrain
with the collected charge as the surface source, multigrid and Jacobi; the
plain linear elements without an object; switching the operator on one
context (the IFE rows and diagonal do not disturb the finite volumes'
cached operator). Both sides solve to a relative residual of 1e-13, so the
potentials agree to rounding; at the paper's tolerance the GPU runs as many
iterations as the oracle did and the two iterates agree to rounding."""
import numpy as np
import pytest

import paper_2011_10214_amd as pam
import synth
from oracle import oracle

from gpu_util import inputs
from helpers import problem_of

pytestmark = pytest.mark.gpu

XM, XP, YM, YP, ZM, ZP = 1, 2, 4, 8, 16, 32
OML = XP | YP | ZP


def empty_crater_context(n, z_flat, repr="fp64"):
    nx, ny, nz = n
    cfg = pam.Config(nx=nx, ny=ny, nz=nz, dt=0.05, species=[(-1.0, 1.0, 1.0)], capacity=[1],
                     obj="crater", center=(-1000.0, -1000.0, 0.0), z_flat=z_flat, rim_radius=1.0,
                     depth=0.5, repr=repr)
    ctx = pam.Context(cfg)
    ctx.set_node_E([np.zeros(cfg.nodes)] * 3)
    ctx.step(0)
    return ctx


@pytest.mark.parametrize("precond", ["multigrid", "jacobi"])
def test_ife_capacitor_with_a_mesh_aligned_interface_is_exact(precond):
    nx, ny, nz = 16, 12, 24
    V0, eps_in, z_flat = 2.0, 4.0, 3.0
    with empty_crater_context((nx, ny, nz), z_flat) as ctx:
        ctx.solve_field(ZM | ZP, values=[0, 0, 0, 0, V0, 0], tol=1e-14, max_iter=3000,
                        precond=precond, eps_object=eps_in, op="ife")
        assert ctx.get_field_levels() == (2 if precond == "multigrid" else 0)
        phi = ctx.get_phi()
    k = np.repeat(np.arange(nz + 1), (nx + 1) * (ny + 1)).astype(float)
    D = V0 / (z_flat / eps_in + (nz - z_flat))
    want = np.where(k <= z_flat, V0 - D * k / eps_in, D * (nz - k))
    assert np.max(np.abs(phi - want)) < 1e-11


@pytest.mark.parametrize("precond", ["multigrid", "jacobi"])
def test_ife_capacitor_with_a_fractional_interface_matches_the_oracle(precond):
    nx, ny, nz = 16, 12, 24
    V0, eps_in, z_flat = 2.0, 4.0, 7.37
    with empty_crater_context((nx, ny, nz), z_flat) as ctx:
        ctx.solve_field(ZM | ZP, values=[0, 0, 0, 0, V0, 0], tol=1e-13, max_iter=3000,
                        precond=precond, eps_object=eps_in, op="ife")
        phi = ctx.get_phi()
    obj = oracle.FieldObject(kind="crater", eps_in=eps_in, center=(-1000.0, -1000.0, 0.0),
                             z_flat=z_flat, rim_radius=1.0, depth=0.5)
    ref, _, _ = oracle.field_solve(nx, ny, nz, np.zeros((nx + 1) * (ny + 1) * (nz + 1)), ZM | ZP,
                                   values=[0, 0, 0, 0, V0, 0], tol=1e-13, obj=obj, op="ife")
    assert np.abs(phi - ref).max() < 1e-10 * V0
    # not the finite volumes' solution (which is exact here)
    k = np.repeat(np.arange(nz + 1), (nx + 1) * (ny + 1)).astype(float)
    D = V0 / (z_flat / eps_in + (nz - z_flat))
    exact = np.where(k <= z_flat, V0 - D * k / eps_in, D * (nz - k))
    assert 1e-5 < np.abs(phi - exact).max() < 0.01 * V0


@pytest.mark.parametrize("dims", [(15, 12, 24), (16, 13, 8), (15, 15, 15)])
def test_ife_on_odd_cell_counts_matches_the_oracle(dims):
    # an even number of nodes along x (odd cell count) gives the enumeration
    # of the finest level by node parity a padding slot in every row; odd
    # cell counts elsewhere keep the grid from coarsening (Jacobi-PCG)
    nx, ny, nz = dims
    V0, eps_in, z_flat = 1.5, 4.0, 0.37 * nz
    with empty_crater_context(dims, z_flat) as ctx:
        ctx.solve_field(ZM | ZP, values=[0, 0, 0, 0, V0, 0], tol=1e-13, max_iter=5000,
                        eps_object=eps_in, op="ife")
        phi = ctx.get_phi()
    obj = oracle.FieldObject(kind="crater", eps_in=eps_in, center=(-1000.0, -1000.0, 0.0),
                             z_flat=z_flat, rim_radius=1.0, depth=0.5)
    ref, _, _ = oracle.field_solve(nx, ny, nz, np.zeros((nx + 1) * (ny + 1) * (nz + 1)), ZM | ZP,
                                   values=[0, 0, 0, 0, V0, 0], tol=1e-13, max_iter=5000, obj=obj,
                                   op="ife")
    assert np.abs(phi - ref).max() < 1e-10 * V0


def run_and_solve(w, form, patches, nsteps, mask, eps_in, tol, max_iter, precond="multigrid",
                  surface=True):
    sp, x, v, E = inputs(w)
    prob = problem_of(w, form)
    prob.sphere_patches = patches
    r = oracle.run(prob, sp, x, v, E, nsteps)
    rho = r.rho_fixed.copy()
    if surface:
        rho += oracle.surface_rho(prob, r.tally)
    info = {}
    obj = oracle.field_object_of(prob, eps_in) if eps_in > 0 else None
    ref, it_ref, rr_ref = oracle.field_solve(w.nx, w.ny, w.nz, rho * 2.0 ** -32 / w.h ** 3, mask,
                                             h=w.h, tol=tol, max_iter=max_iter, info=info,
                                             obj=obj, precond=precond, op="ife")
    cfg = pam.config_from_workload(w, repr=form,
                                   capacity=[int((sp == s).sum()) for s in range(len(w.species))])
    cfg.patches = patches
    ids = np.arange(len(sp), dtype=np.int64)
    with pam.Context(cfg) as ctx:
        for s in range(len(w.species)):
            m = sp == s
            ctx.load_particles(s, x[m], v[m], ids[m])
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.step(nsteps)
        it, rr = ctx.solve_field(mask, tol=tol, max_iter=max_iter, precond=precond,
                                 eps_object=eps_in, surface_charge=surface, op="ife")
        levels = ctx.get_field_levels()
        phi = ctx.get_phi()
        E_gpu = ctx.get_node_E()
    return (phi, it, rr, levels, E_gpu), (ref, it_ref, rr_ref, info["levels"]), r


@pytest.mark.parametrize("form", ["fp64", "fp32_cell"])
@pytest.mark.parametrize("precond", ["multigrid", "jacobi"])
def test_ife_sphere_with_surface_charge_matches_the_oracle(form, precond):
    w = synth.sphere_16()
    (phi, it, rr, lv, Eg), (ref, it_ref, rr_ref, lv_ref), r = run_and_solve(
        w, form, 3, 10, OML, 4.0, 1e-13, 3000, precond)
    assert r.tally.sum() > 0 and lv == lv_ref == (2 if precond == "multigrid" else 0)
    assert rr <= 1e-13 and rr_ref <= 1e-13
    assert np.abs(phi - ref).max() <= 1e-9 * np.abs(ref).max()
    # the node field is -grad phi of the solution (stored in the form's type)
    Er = oracle.field_E(w.nx, w.ny, w.nz, ref, OML)
    tol = 1e-8 if form == "fp64" else 2e-6
    assert np.abs(Eg - Er).max() <= tol * np.abs(Er).max()


def test_ife_crater_with_surface_charge_matches_the_oracle():
    w = synth.scaled(synth.crater_160(), 32, 32, 16, 3.0, steps=10)
    (phi, it, rr, lv, _), (ref, it_ref, rr_ref, lv_ref), r = run_and_solve(
        w, "fp32_cell", 0, 10, ZP, 4.0, 1e-13, 500)
    assert r.tally.sum() > 100 and lv == lv_ref == 3
    assert rr <= 1e-13 and rr_ref <= 1e-13 and it <= 60
    assert np.abs(phi - ref).max() <= 1e-9 * np.abs(ref).max()


def test_ife_crater_on_a_grid_of_2048_dot_product_workgroups():
    # 128 x 128 x 32 cells (549 K nodes, 5 levels): the IFE kernels and the
    # dot products at their full 2048 workgroups, as in the crater_160 solve
    w = synth.scaled(synth.crater_160(), 128, 128, 32, 1.0, steps=2)
    (phi, it, rr, lv, _), (ref, it_ref, rr_ref, lv_ref), r = run_and_solve(
        w, "fp32_cell", 0, 2, ZP, 4.0, 1e-11, 300)
    assert r.tally.sum() > 100 and lv == lv_ref == 5
    assert rr <= 1e-11 and rr_ref <= 1e-11 and abs(it - it_ref) <= 1
    assert np.abs(phi - ref).max() <= 1e-9 * np.abs(ref).max()


def test_ife_crater_at_the_papers_tolerance_follows_the_oracles_iterates():
    # tol 1e-6 (the paper's): both converge within an iteration of each other;
    # then both run exactly the oracle's iteration count (a tolerance neither
    # can meet) and hold the same preconditioned-CG iterate up to rounding
    w = synth.scaled(synth.crater_160(), 32, 32, 16, 3.0, steps=10)
    (phi, it, rr, lv, _), (ref, it_ref, rr_ref, _), _ = run_and_solve(
        w, "fp32_cell", 0, 10, ZP, 4.0, 1e-6, 150)
    assert rr <= 1e-6 and rr_ref <= 1e-6 and it <= 20 and abs(it - it_ref) <= 1
    (phi, it, rr, lv, _), (ref, it_n, rr_ref, _), _ = run_and_solve(
        w, "fp32_cell", 0, 10, ZP, 4.0, 1e-300, it_ref)
    assert it == it_n == it_ref
    assert abs(rr - rr_ref) <= 1e-6 * rr_ref
    assert np.abs(phi - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("mask", [ZP, XM | XP | YM | YP | ZM | ZP])
def test_plain_linear_elements_without_an_object(mask):
    w = synth.scaled(synth.sphere_16(), 24, 20, 16, 2.0, steps=5)
    sp, x, v, E = inputs(w)
    r = oracle.run(problem_of(w, "fp64"), sp, x, v, E, 5)
    ref, _, _ = oracle.field_solve(w.nx, w.ny, w.nz, r.rho_fixed * 2.0 ** -32, mask, tol=1e-13,
                                   values=[0.5, -0.25, 0, 0, 1.0, 0.3], op="ife")
    cfg = pam.config_from_workload(w, repr="fp64",
                                   capacity=[int((sp == s).sum()) for s in range(2)])
    with pam.Context(cfg) as ctx:
        for s in range(2):
            ctx.load_particles(s, x[sp == s], v[sp == s])
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.step(5)
        ctx.solve_field(mask, values=[0.5, -0.25, 0, 0, 1.0, 0.3], tol=1e-13, max_iter=3000,
                        op="ife")
        phi = ctx.get_phi()
    assert np.abs(phi - ref).max() <= 1e-9 * np.abs(ref).max()


def test_switching_the_operator_on_one_context():
    # finite volumes, then IFE, then finite volumes again, each with the
    # interface: every solve equals the oracle's with its operator
    w = synth.scaled(synth.crater_160(), 32, 32, 16, 3.0, steps=4)
    sp, x, v, E = inputs(w)
    prob = problem_of(w, "fp32_cell")
    r = oracle.run(prob, sp, x, v, E, 4)
    rho = (r.rho_fixed + oracle.surface_rho(prob, r.tally)) * 2.0 ** -32
    obj = oracle.field_object_of(prob, 4.0)
    refs = {op: oracle.field_solve(w.nx, w.ny, w.nz, rho, ZP, tol=1e-13, obj=obj, op=op)[0]
            for op in ("fv", "ife")}
    assert np.abs(refs["fv"] - refs["ife"]).max() > 1e-6 * np.abs(refs["fv"]).max()
    cfg = pam.config_from_workload(w, capacity=[int((sp == s).sum()) for s in range(2)])
    with pam.Context(cfg) as ctx:
        for s in range(2):
            ctx.load_particles(s, x[sp == s], v[sp == s])
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.step(4)
        for op in ("fv", "ife", "fv", "ife"):
            # each solve starts from the previous solution: a few iterations
            ctx.solve_field(ZP, tol=1e-13, max_iter=500, eps_object=4.0, surface_charge=True,
                            op=op)
            phi = ctx.get_phi()
            assert np.abs(phi - refs[op]).max() <= 1e-9 * np.abs(refs[op]).max(), op


def test_operator_setting_is_checked():
    with empty_crater_context((8, 8, 8), 3.0) as ctx:
        with pytest.raises(ValueError):
            ctx.solve_field(ZP, op="spectral")
        f = pam.pic._Field()
        f.dirichlet, f.eps, f.tol, f.max_iter, f.op = ZP, 1.0, 1e-6, 10, 7
        assert pam.lib().pic_solve_field(ctx._h, f, None, None) == pam.pic.E_INVALID
