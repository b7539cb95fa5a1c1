"""The field solve with the object as an interface on the GPU (pic_field
eps_object, surface_charge) against the oracle: the exact two-layer
capacitor; sphere (with surface patches) and crater terrain with the
collected charge as the surface source, at tight and at the paper's
tolerance, multigrid and Jacobi; re-solving with other permittivities
(cached level sets, diagonals and coarsest inverse); the closed PIC loop with
the interface; and the settings checks. The oracle's inputs come from the
oracle's own particle run."""
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


def empty_crater_context(n, z_flat):
    nx, ny, nz = n
    cfg = pam.Config(nx=nx, ny=ny, nz=nz, dt=0.05, species=[(-1.0, 1.0, 1.0)], capacity=[1],
                     obj="crater", center=(-1000.0, -1000.0, 0.0), z_flat=z_flat, rim_radius=1.0,
                     depth=0.5, repr="fp64")
    ctx = pam.Context(cfg)
    ctx.set_node_E([np.zeros(cfg.nodes)] * 3)
    ctx.step(0)
    return ctx


@pytest.mark.parametrize("precond", ["multigrid", "jacobi"])
@pytest.mark.parametrize("z_flat", [3.0, 7.37])
def test_two_layer_capacitor_is_exact_on_the_gpu(precond, z_flat):
    nx, ny, nz = 16, 12, 24
    V0, eps_in = 2.0, 4.0
    with empty_crater_context((nx, ny, nz), z_flat) as ctx:
        it, rr = ctx.solve_field(ZM | ZP, values=[0, 0, 0, 0, V0, 0], tol=1e-14, max_iter=3000,
                                 precond=precond, eps_object=eps_in)
        assert ctx.get_field_levels() == (2 if precond == "multigrid" else 0)
        phi = ctx.get_phi()
    k = np.repeat(np.arange(nz + 1), (nx + 1) * (ny + 1)).astype(float)
    D = V0 / (z_flat / eps_in + (nz - z_flat))
    want = np.where(k <= z_flat, V0 - D * k / eps_in, D * (nz - k))
    assert np.max(np.abs(phi - want)) < 1e-11


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
                                             obj=obj, precond=precond)
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
                                 eps_object=eps_in, surface_charge=surface)
        levels = ctx.get_field_levels()
        phi = ctx.get_phi()
    return (phi, it, rr, levels), (ref, it_ref, rr_ref, info["levels"]), r


@pytest.mark.parametrize("form", ["fp64", "fp32_cell"])
@pytest.mark.parametrize("precond", ["multigrid", "jacobi"])
def test_sphere_interface_with_surface_charge_matches_the_oracle(form, precond):
    w = synth.sphere_16()
    (phi, it, rr, lv), (ref, it_ref, rr_ref, lv_ref), r = run_and_solve(
        w, form, 3, 10, OML, 4.0, 1e-11, 3000, precond)
    assert r.tally.sum() > 0 and lv == lv_ref == (2 if precond == "multigrid" else 0)
    assert rr <= 1e-11 and rr_ref <= 1e-11 and abs(it - it_ref) <= (1 if lv else 2)
    assert np.abs(phi - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("tol,max_iter", [(1e-12, 300), (1e-6, 150)])
def test_crater_interface_with_surface_charge_matches_the_oracle(tol, max_iter):
    w = synth.scaled(synth.crater_160(), 32, 32, 16, 3.0, steps=10)
    (phi, it, rr, lv), (ref, it_ref, rr_ref, lv_ref), r = run_and_solve(
        w, "fp32_cell", 0, 10, ZP, 4.0, tol, max_iter)
    assert r.tally.sum() > 100 and lv == lv_ref == 3
    assert rr <= tol and rr_ref <= tol and it <= 20 and abs(it - it_ref) <= 1
    scale = np.abs(ref).max()
    if it == it_ref:  # the same iterate: rounding only
        assert np.abs(phi - ref).max() <= 1e-9 * scale
    # the iterates themselves: both sides run exactly the oracle's iteration
    # count (a tolerance neither can meet) and agree to rounding
    (phi_n, it_n, _, _), (ref_n, it_rn, _, _), _ = run_and_solve(
        w, "fp32_cell", 0, 10, ZP, 4.0, 1e-300, it_ref)
    assert it_n == it_rn == it_ref
    assert np.abs(phi_n - ref_n).max() <= 1e-9 * np.abs(ref_n).max()


def test_crater_interface_on_a_grid_of_2048_dot_product_workgroups():
    # 128 x 128 x 32 cells (549 K nodes, 5 levels): the dot-product kernels
    # run their full 2048 workgroups, so the consumers add their partials
    # eight at a time (the path of the crater_160 solve)
    w = synth.scaled(synth.crater_160(), 128, 128, 32, 1.0, steps=2)
    (phi, it, rr, lv), (ref, it_ref, rr_ref, lv_ref), r = run_and_solve(
        w, "fp32_cell", 0, 2, ZP, 4.0, 1e-11, 300)
    assert (w.nx + 1) * (w.ny + 1) * (w.nz + 1) >= 2048 * 256
    assert r.tally.sum() > 100 and lv == lv_ref == 5
    assert rr <= 1e-11 and rr_ref <= 1e-11 and abs(it - it_ref) <= 1
    assert np.abs(phi - ref).max() <= 1e-9 * np.abs(ref).max()


def test_permittivity_changes_refresh_the_cached_operator():
    w = synth.scaled(synth.crater_160(), 32, 32, 16, 3.0, steps=10)
    sp, x, v, E = inputs(w)
    cfg = pam.config_from_workload(w, capacity=[int((sp == s).sum()) for s in range(2)])
    ids = np.arange(len(sp), dtype=np.int64)

    def fresh():
        ctx = pam.Context(cfg)
        for s in range(2):
            m = sp == s
            ctx.load_particles(s, x[m], v[m], ids[m])
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.step(3)
        return ctx

    def solve(ctx, e):
        ctx.solve_field(ZP, tol=1e-12, max_iter=300, eps_object=e, surface_charge=e > 0)
        return ctx.get_phi()

    want = {}
    for e in (4.0, 10.0, 0.0):
        with fresh() as ctx:
            want[e] = solve(ctx, e)
    with fresh() as ctx:
        for e in (4.0, 10.0, 0.0, 4.0):
            got = solve(ctx, e)
            assert np.abs(got - want[e]).max() <= 1e-9 * np.abs(want[e]).max(), e
    assert np.abs(want[4.0] - want[10.0]).max() > 1e-3 * np.abs(want[4.0]).max()


def test_closed_loop_with_the_interface_follows_the_oracle():
    w = synth.scaled(synth.sphere_16(), 16, 16, 16, 4.0, steps=5)
    mask, tol, eps_in, m = OML, 1e-12, 4.0, 2
    sp, x, v, _ = inputs(w)
    prob = problem_of(w, "fp64")
    prob.sphere_patches = m
    obj = oracle.field_object_of(prob, eps_in)
    ids = np.arange(len(sp))
    E = np.zeros((3, w.nodes))
    ox, ov, osp, oid = x.copy(), v.copy(), sp.copy(), ids.copy()
    tally = np.zeros((prob.nbins, 2), np.int64)
    for _ in range(w.steps):
        r = oracle.run(prob, osp, ox, ov, E, 1)
        tally += r.tally
        alive = r.fate == 0
        ox, ov, osp, oid = r.x[alive], r.v[alive], osp[alive], oid[alive]
        rho = (r.rho_fixed + oracle.surface_rho(prob, tally)) * 2.0 ** -32
        phi, _, _ = oracle.field_solve(w.nx, w.ny, w.nz, rho, mask, tol=tol, max_iter=5000, obj=obj)
        E = oracle.field_E(w.nx, w.ny, w.nz, phi, mask)
    assert tally.sum() > 0
    cfg = pam.config_from_workload(w, repr="fp64",
                                   capacity=[int((sp == s).sum()) for s in range(len(w.species))])
    cfg.patches = m
    with pam.Context(cfg) as ctx:
        for s in range(len(w.species)):
            msk = sp == s
            ctx.load_particles(s, x[msk], v[msk], ids[msk])
        ctx.set_node_E([np.zeros(w.nodes)] * 3)
        for _ in range(w.steps):
            ctx.step(1)
            ctx.solve_field(mask, tol=tol, max_iter=5000, eps_object=eps_in, surface_charge=True)
        parts = [ctx.get_particles(s) for s in range(len(w.species))]
        gphi = ctx.get_phi()
        counts = ctx.get_surface_charge()[1]
    assert np.array_equal(counts, tally)
    gx = np.concatenate([p[0] for p in parts])
    gid = np.concatenate([p[2] for p in parts])
    o, q = np.argsort(gid), np.argsort(oid)
    assert np.array_equal(gid[o], oid[q])
    assert np.abs(gx[o] - ox[q]).max() < 1e-9
    assert np.abs(gphi - phi).max() < 1e-8 * np.abs(phi).max()


def test_interface_settings_are_checked():
    w = synth.sphere_16()
    cfg = pam.config_from_workload(w, repr="fp64", capacity=[1, 1])
    with pam.Context(cfg) as ctx:
        ctx.set_node_E([np.zeros(w.nodes)] * 3)
        ctx.step(0)
        for kw in (dict(eps_object=-1.0), dict(eps_object=float("nan")),
                   dict(surface_charge=True)):  # a sphere without patches
            with pytest.raises(pam.PicError):
                ctx.solve_field(OML, **kw)
        f = pam.pic._Field()
        f.dirichlet, f.eps, f.tol, f.max_iter, f.surface_charge = OML, 1.0, 1e-6, 10, 2
        import ctypes
        assert pam.pic.lib().pic_solve_field(ctx._h, ctypes.byref(f), None, None) == -1
    cfg = pam.Config(nx=8, ny=8, nz=8, dt=0.05, species=[(-1.0, 1.0, 1.0)], capacity=[1])
    with pam.Context(cfg) as ctx:
        ctx.set_node_E([np.zeros(cfg.nodes)] * 3)
        ctx.step(0)
        with pytest.raises(pam.PicError):
            ctx.solve_field(ZP, eps_object=4.0)  # no object
