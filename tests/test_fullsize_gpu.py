"""Full-size runs in the launch configuration the benchmark times (FP32 cell
form, int64 fixed-point deposit, re-bucketing every 4 steps), checked against
the oracle on sampled particles (particles are independent under a fixed node
field, so the oracle can run the sample alone) and against properties that hold
at any size."""
import numpy as np
import pytest

import paper_2011_10214_amd as pam
import synth
from oracle import oracle

from helpers import problem_of

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


@pytest.mark.parametrize("name", ["sphere_64", "crater_160"])
def test_full_size_sampled_parity(name):
    import torch

    w = synth.WORKLOADS[name]()
    print(f"[{name}] {w.n_particles} particles, {w.steps} steps", flush=True)
    E = synth.node_E(w)
    cfg = pam.config_from_workload(w, repr="fp32_cell", deposit="fixed64", sort_interval=4)
    rng = np.random.default_rng(2011)
    samples = [np.sort(rng.choice(s.count, SAMPLE, replace=False)) for s in w.species]
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

    # the sample through the FP32 cell-form mirror of the oracle
    sp = np.concatenate([np.full(SAMPLE, s, np.int32) for s in range(len(w.species))])
    parts = [synth.particles(w, s, idx=samples[s]) for s in range(len(w.species))]
    x = np.concatenate([np.stack(p[:3], 1) for p in parts]).astype(np.float64)
    v = np.concatenate([np.stack(p[3:], 1) for p in parts]).astype(np.float64)
    r = oracle.run(problem_of(w, "fp32_cell"), sp, x, v, E, w.steps)
    for s in range(len(w.species)):
        found, gx, gv = got[s]
        sel = sp == s
        assert np.array_equal(found, r.fate[sel] == 0)
        assert np.array_equal(gx[found], r.x[sel][found])
        assert np.array_equal(gv[found], r.v[sel][found])
    print(f"[{name}] sampled {len(sp)} particles bit-exact; alive {alive.tolist()}", flush=True)

    # rho of the sample alone, same launch configuration
    cfg_s = pam.config_from_workload(w, repr="fp32_cell", deposit="fixed64", sort_interval=4,
                                     capacity=[SAMPLE] * len(w.species))
    with pam.Context(cfg_s) as ctx:
        for s in range(len(w.species)):
            ctx.load_particles(s, x[sp == s], v[sp == s])
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.step(w.steps)
        _, rf = ctx.get_rho()
        _, cnt = ctx.get_surface_charge()
    assert np.array_equal(rf, r.rho_fixed)
    assert np.array_equal(cnt, r.tally)
