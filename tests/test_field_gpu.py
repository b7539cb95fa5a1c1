"""The field solve on the GPU (pic_solve_field) against the oracle's solve,
with the multigrid and the Jacobi preconditioner: the same preconditioner
choice and level count, the same iteration count (within one: the two runs
differ only in the order of their sums), the same potential and node field
within the solver tolerance, exact discrete solutions, a deterministic
result, and the closed PIC loop (deposit -> solve -> gather / push)
following the oracle's loop."""
import ctypes

import numpy as np
import pytest

import paper_2011_10214_amd as pam
import synth
from oracle import oracle

from gpu_util import inputs
from helpers import problem_of

pytestmark = pytest.mark.gpu

OML_DIRICHLET = 2 | 8 | 32      # phi = 0 at the max faces, zero-Neumann at the min faces
LUNAR_DIRICHLET = 32            # phi = 0 at z+, zero-Neumann elsewhere


def loaded_context(w, form="fp64", deposit="fixed64"):
    sp, x, v, E = inputs(w)
    cfg = pam.config_from_workload(w, repr=form, deposit=deposit,
                                   capacity=[int((sp == s).sum()) for s in range(len(w.species))])
    ctx = pam.Context(cfg)
    ids = np.arange(len(sp), dtype=np.int64)
    for s in range(len(w.species)):
        m = sp == s
        ctx.load_particles(s, x[m], v[m], ids[m])
    return ctx, sp, x, v


def crater_32():
    # 32 x 32 x 16 cells: three multigrid levels (33^2 x 17, 17^2 x 9, 9^2 x 5 nodes)
    return synth.scaled(synth.crater_160(), 32, 32, 16, 3.0)


@pytest.mark.parametrize("form,mask,precond", [("fp64", OML_DIRICHLET, "multigrid"),
                                               ("fp32_cell", OML_DIRICHLET, "multigrid"),
                                               ("fp64", LUNAR_DIRICHLET, "multigrid"),
                                               ("fp64", OML_DIRICHLET, "jacobi"),
                                               ("fp64", LUNAR_DIRICHLET, "jacobi")])
def test_potential_and_field_match_the_oracle(form, mask, precond):
    w = synth.sphere_16()
    ctx, sp, x, v = loaded_context(w, form)
    with ctx:
        ctx.step(0)  # deposit only
        rho, _ = ctx.get_rho()
        it, rr = ctx.solve_field(mask, tol=1e-11, max_iter=2000, precond=precond)
        levels = ctx.get_field_levels()
        phi = ctx.get_phi()
        E = ctx.get_node_E()
    info = {}
    ref, it_ref, rr_ref = oracle.field_solve(w.nx, w.ny, w.nz, rho, mask, tol=1e-11, max_iter=2000,
                                             precond=precond, info=info)
    assert levels == info["levels"] == (2 if precond == "multigrid" else 0)
    assert rr <= 1e-11 and rr_ref <= 1e-11
    assert abs(it - it_ref) <= (1 if precond == "multigrid" else 2)
    scale = np.abs(ref).max()
    assert np.abs(phi - ref).max() <= 1e-9 * scale
    Eref = oracle.field_E(w.nx, w.ny, w.nz, ref, mask)
    tol = 1e-8 * np.abs(Eref).max() if form == "fp64" else 1e-6 * np.abs(Eref).max()
    assert np.abs(E - Eref).max() <= tol


@pytest.mark.parametrize("mask", [LUNAR_DIRICHLET, OML_DIRICHLET, 63])
@pytest.mark.parametrize("tol,max_iter", [(1e-12, 200), (1e-6, 150)])
def test_three_level_multigrid_matches_the_oracle(mask, tol, max_iter):
    w = crater_32()
    ctx, sp, x, v = loaded_context(w, "fp32_cell")
    with ctx:
        ctx.step(0)
        rho, _ = ctx.get_rho()
        it, rr = ctx.solve_field(mask, tol=tol, max_iter=max_iter)
        levels = ctx.get_field_levels()
        phi = ctx.get_phi()
    info = {}
    ref, it_ref, rr_ref = oracle.field_solve(w.nx, w.ny, w.nz, rho, mask, tol=tol,
                                             max_iter=max_iter, info=info)
    assert levels == info["levels"] == 3
    assert rr <= tol and rr_ref <= tol and it <= 15
    assert abs(it - it_ref) <= 1
    scale = np.abs(ref).max()
    if it == it_ref:  # the same iterate: rounding only
        assert np.abs(phi - ref).max() <= 1e-9 * scale
    # the iterates themselves: both sides run exactly the oracle's iteration
    # count from zero (a tolerance neither can meet) and agree to rounding
    ctx, sp, x, v = loaded_context(w, "fp32_cell")
    with ctx:
        ctx.step(0)
        ctx.solve_field(mask, tol=1e-300, max_iter=it_ref)
        phi_n = ctx.get_phi()
    ref_n, it_n, _ = oracle.field_solve(w.nx, w.ny, w.nz, rho, mask, tol=1e-300, max_iter=it_ref)
    assert it_n == it_ref
    assert np.abs(phi_n - ref_n).max() <= 1e-9 * np.abs(ref_n).max()


@pytest.mark.parametrize("mask", [LUNAR_DIRICHLET, 1 | 2])
def test_multigrid_with_one_cell_along_an_axis_matches_the_oracle(mask):
    # 32 x 32 x 2 cells: the coarse level is 16 x 16 x 1, one cell along z,
    # so that a node there has no z link on one side and its stand-in link
    # (weight 0) is the node on the other side, a Dirichlet one with the
    # lunar mask and a zero-Neumann one with phi fixed on the x faces
    w = synth.scaled(synth.sphere_16(), 32, 32, 2, 4.0, name="thin_32x32x2")
    ctx, sp, x, v = loaded_context(w, "fp64")
    with ctx:
        ctx.step(0)
        rho, _ = ctx.get_rho()
        it, rr = ctx.solve_field(mask, tol=1e-11, max_iter=2000)
        levels = ctx.get_field_levels()
        phi = ctx.get_phi()
    info = {}
    ref, it_ref, rr_ref = oracle.field_solve(w.nx, w.ny, w.nz, rho, mask, tol=1e-11, max_iter=2000,
                                             info=info)
    assert levels == info["levels"] == 2
    assert rr <= 1e-11 and rr_ref <= 1e-11
    assert abs(it - it_ref) <= 1
    assert np.abs(phi - ref).max() <= 1e-9 * np.abs(ref).max()


def test_paper_settings_converge_and_the_oracle_agrees_on_the_residual():
    # the PCG of the paper's runs: tolerance 1e-6 within 150 iterations, on a
    # 64 x 64 x 32 crater-shaped mesh (4 levels), cold and warm started
    w = synth.scaled(synth.crater_160(), 64, 64, 32, 2.0)
    ctx, sp, x, v = loaded_context(w, "fp32_cell")
    with ctx:
        ctx.step(0)
        rho, _ = ctx.get_rho()
        it, rr = ctx.solve_field(LUNAR_DIRICHLET, tol=1e-6, max_iter=150)
        assert ctx.get_field_levels() == 4
        assert rr <= 1e-6 and it <= 12
        phi = ctx.get_phi()
        ctx.step(1)
        rho1, _ = ctx.get_rho()
        it1, rr1 = ctx.solve_field(LUNAR_DIRICHLET, tol=1e-6, max_iter=150)
        phi1 = ctx.get_phi()
        assert rr1 <= 1e-6 and it1 <= it
    # the oracle, warm-started from each GPU potential, finds the residual
    # bound already met (its own sums, a hair of slack for their order)
    for r_, p_ in ((rho, phi), (rho1, phi1)):
        _, it0, rr0 = oracle.field_solve(w.nx, w.ny, w.nz, r_, LUNAR_DIRICHLET, phi0=p_,
                                         tol=1.001e-6, max_iter=0)
        assert it0 == 0 and rr0 <= 1.001e-6


def test_linear_potential_between_two_plates_on_the_gpu():
    w = synth.sphere_16()
    cfg = pam.config_from_workload(w, repr="fp64", capacity=[1, 1])
    with pam.Context(cfg) as ctx:
        ctx.set_node_E([np.zeros(w.nodes)] * 3)
        ctx.step(0)  # no particles: rho = 0
        it, rr = ctx.solve_field(1 | 2, values=[3.0, -1.0, 0, 0, 0, 0], tol=1e-14, max_iter=1000)
        phi = ctx.get_phi()
        E = ctx.get_node_E()
    i = np.tile(np.arange(w.nx + 1), (w.ny + 1) * (w.nz + 1))
    assert np.abs(phi - (3.0 - 4.0 * i / w.nx)).max() < 1e-11
    assert np.abs(E[0] - 4.0 / w.nx).max() < 1e-10
    assert np.abs(E[1:]).max() < 1e-10


def test_solve_is_deterministic_and_warm_started():
    w = synth.sphere_16()
    ctx, sp, x, v = loaded_context(w, "fp32_cell")
    with ctx:
        ctx.step(0)
        it1, _ = ctx.solve_field(OML_DIRICHLET, tol=1e-8, max_iter=1000)
        phi1 = ctx.get_phi()
        it2, rr2 = ctx.solve_field(OML_DIRICHLET, tol=1e-8, max_iter=1000)  # warm start
        phi2 = ctx.get_phi()
    assert it1 > 3 and it2 == 0 and np.array_equal(phi1, phi2)
    ctx, sp, x, v = loaded_context(w, "fp32_cell")
    with ctx:
        ctx.step(0)
        it3, _ = ctx.solve_field(OML_DIRICHLET, tol=1e-8, max_iter=1000)
        phi3 = ctx.get_phi()
    assert it3 == it1 and np.array_equal(phi1, phi3)


def test_closed_pic_loop_follows_the_oracle():
    # deposit -> field solve -> gather / push, a few steps, FP64 form
    w = synth.scaled(synth.sphere_16(), 12, 12, 12, 6.0, steps=6)
    mask, tol = OML_DIRICHLET, 1e-12
    sp, x, v, _ = inputs(w)
    prob = problem_of(w, "fp64")
    ids = np.arange(len(sp))
    E = np.zeros((3, w.nodes))
    ox, ov, osp, oid = x.copy(), v.copy(), sp.copy(), ids.copy()
    for _ in range(w.steps):
        r = oracle.run(prob, osp, ox, ov, E, 1)
        alive = r.fate == 0
        ox, ov, osp, oid = r.x[alive], r.v[alive], osp[alive], oid[alive]
        phi, _, _ = oracle.field_solve(w.nx, w.ny, w.nz, r.rho, mask, tol=tol, max_iter=5000)
        E = oracle.field_E(w.nx, w.ny, w.nz, phi, mask)
    cfg = pam.config_from_workload(w, repr="fp64",
                                   capacity=[int((sp == s).sum()) for s in range(len(w.species))])
    with pam.Context(cfg) as ctx:
        for s in range(len(w.species)):
            m = sp == s
            ctx.load_particles(s, x[m], v[m], ids[m])
        ctx.set_node_E([np.zeros(w.nodes)] * 3)
        for _ in range(w.steps):
            ctx.step(1)
            ctx.solve_field(mask, tol=tol, max_iter=5000)
        parts = [ctx.get_particles(s) for s in range(len(w.species))]
        gphi = ctx.get_phi()
    gx = np.concatenate([p[0] for p in parts])
    gv = np.concatenate([p[1] for p in parts])
    gid = np.concatenate([p[2] for p in parts])
    o = np.argsort(gid)
    gx, gv, gid = gx[o], gv[o], gid[o]
    q = np.argsort(oid)
    assert np.array_equal(gid, oid[q])
    assert np.abs(gx - ox[q]).max() < 1e-9
    assert np.abs(gv - ov[q]).max() < 1e-9
    assert np.abs(gphi - phi).max() < 1e-8 * np.abs(phi).max()


def test_field_settings_are_checked():
    w = synth.sphere_16()
    cfg = pam.config_from_workload(w, repr="fp64", capacity=[1, 1])
    with pam.Context(cfg) as ctx:
        with pytest.raises(pam.PicError):
            ctx.solve_field(32)  # no deposit yet
        ctx.set_node_E([np.zeros(w.nodes)] * 3)
        ctx.step(0)
        for kw in (dict(dirichlet=0), dict(dirichlet=64), dict(dirichlet=1, eps=0.0),
                   dict(dirichlet=1, tol=0.0), dict(dirichlet=1, max_iter=-1)):
            with pytest.raises(pam.PicError):
                ctx.solve_field(**kw)
        f = pam.pic._Field()
        f.dirichlet, f.eps, f.tol, f.max_iter, f.preconditioner = 1, 1.0, 1e-6, 10, 2
        assert pam.pic.lib().pic_solve_field(ctx._h, ctypes.byref(f), None, None) == -1
        with pytest.raises(pam.PicError):
            pam.Context(cfg).get_phi()
