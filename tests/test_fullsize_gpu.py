"""Full-size runs in the launch configuration the benchmark times (FP32 cell
form, int64 fixed-point deposit), checked against the oracle on sampled
particles (particles are independent under a fixed node field, so the oracle
can run the sample alone): bit for bit against its FP32 cell-form mirror, and
within the cross-precision bounds against its FP64 form (positions and
velocities within 1e-5 relative; fates differ only within 1e-4 cells of a
deciding surface, their number printed); and against properties that hold at
any size."""
import os

import numpy as np
import pytest

import paper_2011_10214_amd as pam
import synth
from oracle import oracle

from helpers import check_mismatches_near_surface, fate_mismatches, problem_of

pytestmark = pytest.mark.gpu

SAMPLE = 2048


def _load_full(ctx, w):
    import torch

    for s, spec in enumerate(w.species):
        cols = synth.particles(w, s)
        dev = [torch.from_numpy(c).to("cuda") for c in cols]
        del cols
        ids = torch.arange(spec.count, dtype=torch.int64, device="cuda")
        ctx.load_particles_cols(s, dev, ids)
        del dev, ids
        torch.cuda.empty_cache()


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# sampled particles per species: 1/64 of sphere_64 (the subsample of the
# FP32 vs FP64 comparison at 64^3 over 100 steps), 2^18 of crater_160
SAMPLED = {"sphere_64": lambda count: np.arange(0, count, 64),
           "crater_160": None}


@pytest.mark.parametrize("name", ["sphere_64", "crater_160"])
def test_full_size_sampled_parity(name):
    import torch

    w = synth.WORKLOADS[name]()
    print(f"[{name}] {w.n_particles} particles, {w.steps} steps", flush=True)
    E = synth.node_E(w)
    cfg = pam.config_from_workload(w, repr="fp32_cell", deposit="fixed64")
    rng = np.random.default_rng(2011)
    if SAMPLED[name] is not None:
        samples = [SAMPLED[name](s.count) for s in w.species]
    else:
        samples = [np.sort(rng.choice(s.count, 1 << 18, replace=False)) for s in w.species]
    with pam.Context(cfg) as ctx:
        _load_full(ctx, w)
        ctx.set_node_E([torch.from_numpy(e).to("cuda") for e in E])
        ctx.step(w.steps)
        rho, rho_fixed = ctx.get_rho()
        alive, absorbed, escaped = ctx.get_counters()
        charge, counts = ctx.get_surface_charge()
        got = [ctx.get_particles_by_id(s, samples[s]) for s in range(len(w.species))]
    # properties at full size: conservation of the deposited charge against the
    # removal counters, and the charge/count consistency of the tallies
    chg = np.array([s.q * s.w for s in w.species])
    assert int(rho_fixed.sum()) == int(round(float((alive * chg).sum()))) * 2 ** 32
    assert np.array_equal(counts.sum(0), absorbed)
    assert np.allclose(charge, counts @ chg, rtol=0, atol=0)
    assert np.all(alive > 0) and absorbed.sum() > 0

    # the sample through the FP32 cell-form mirror of the oracle: bit for bit
    sp = np.concatenate([np.full(len(samples[s]), s, np.int32) for s in range(len(w.species))])
    parts = [synth.particles(w, s, idx=samples[s]) for s in range(len(w.species))]
    x = np.concatenate([np.stack(p[:3], 1) for p in parts]).astype(np.float64)
    v = np.concatenate([np.stack(p[3:], 1) for p in parts]).astype(np.float64)
    thr = _threads()
    mirror = problem_of(w, "fp32_cell")
    mirror.threads = thr
    r = oracle.run(mirror, sp, x, v, E, w.steps)
    gx_all, gv_all, found_all = [], [], []
    for s in range(len(w.species)):
        found, gx, gv = got[s]
        sel = sp == s
        assert np.array_equal(found, r.fate[sel] == 0)
        assert np.array_equal(gx[found], r.x[sel][found])
        assert np.array_equal(gv[found], r.v[sel][found])
        gx_all.append(gx)
        gv_all.append(gv)
        found_all.append(found)
    print(f"[{name}] sampled {len(sp)} particles bit-exact against the FP32 mirror; "
          f"alive {alive.tolist()}", flush=True)

    # across precisions (R19): the FP32 GPU path against the FP64 oracle on the
    # same sample. Positions within 1e-5 max(|x|, 1), velocities within
    # 1e-5 max(|v|, vth) over particles alive in both; a particle whose fate
    # differs must lie within 1e-4 cells of the deciding surface in the FP64
    # run (the GPU's fates are the mirror's, equal by the check above)
    ref = problem_of(w, "fp64")
    ref.threads = thr
    r64 = oracle.run(ref, sp, x, v, E, w.steps)
    gx, gv, found = np.concatenate(gx_all), np.concatenate(gv_all), np.concatenate(found_all)
    both = found & (r64.fate == 0)
    vth = np.array([w.species[s].vth for s in sp])
    dx = np.abs(gx[both] - r64.x[both])
    dv = np.abs(gv[both] - r64.v[both])
    xrel = (dx / np.maximum(np.abs(r64.x[both]), 1.0)).max()
    vrel = (dv / np.maximum(np.abs(r64.v[both]), vth[both][:, None])).max()
    mism = fate_mismatches(r.fate, r.where, r.when, r64.fate, r64.where, r64.when)
    dist = check_mismatches_near_surface(w, sp, x, v, E, mism, r.when, r.fate, r64.when,
                                         r64.fate)
    print(f"[{name}] FP32 GPU vs FP64 oracle on {len(sp)} sampled particles, {w.steps} steps: "
          f"max rel. error x {xrel:.2e}, v {vrel:.2e}; {len(mism)} fate differences "
          f"(FP64 distance to the deciding surface at most "
          f"{dist.max() if len(dist) else 0.0:.2e} cells)", flush=True)
    assert xrel <= 1e-5 and vrel <= 1e-5
    assert np.all(dist <= 1e-4)

    # rho of a small sample alone, same launch configuration
    small = [samples[s][:: max(1, len(samples[s]) // SAMPLE)][:SAMPLE]
             for s in range(len(w.species))]
    sp = np.concatenate([np.full(len(small[s]), s, np.int32) for s in range(len(w.species))])
    parts = [synth.particles(w, s, idx=small[s]) for s in range(len(w.species))]
    x = np.concatenate([np.stack(p[:3], 1) for p in parts]).astype(np.float64)
    v = np.concatenate([np.stack(p[3:], 1) for p in parts]).astype(np.float64)
    r = oracle.run(mirror, sp, x, v, E, w.steps)
    cfg_s = pam.config_from_workload(w, repr="fp32_cell", deposit="fixed64",
                                     capacity=[len(a) for a in small])
    with pam.Context(cfg_s) as ctx:
        for s in range(len(w.species)):
            ctx.load_particles(s, x[sp == s], v[sp == s])
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.step(w.steps)
        _, rf = ctx.get_rho()
        _, cnt = ctx.get_surface_charge()
    assert np.array_equal(rf, r.rho_fixed)
    assert np.array_equal(cnt, r.tally)
