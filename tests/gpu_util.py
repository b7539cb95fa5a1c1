"""Helpers of the GPU tests: run a workload through the C-ABI and gather the
results by particle id."""
import numpy as np

import paper_2011_10214_amd as pam
import synth


class GpuRun:
    def __init__(self, x, v, alive_ids, rho, rho_fixed, charge, counts, alive, absorbed, escaped,
                 profile=None):
        self.x, self.v, self.alive_ids = x, v, alive_ids
        self.rho, self.rho_fixed = rho, rho_fixed
        self.charge, self.counts = charge, counts
        self.alive, self.absorbed, self.escaped = alive, absorbed, escaped
        self.profile = profile


def run_gpu(w, sp, x, v, E, nsteps, repr="fp64", deposit="fixed64", sort_interval=0,
            order=None, device_load=False, split_steps=None, patches=0, spare=1.0,
            profile=False, sync_steps=False, batch_steps_per_run=None):
    """Runs nsteps on the GPU; particle ids are the indices into (sp, x, v).
    Returns state of alive particles ordered by id (and the launch profile if
    profile). spare scales every species' capacity; sync_steps waits for each
    step before the next, so the host sees each step's re-planning request;
    batch_steps_per_run runs the steps through a one-slot batch instead, in
    runs of that many steps."""
    import torch

    n = len(sp)
    ids = np.arange(n, dtype=np.int64)
    if order is not None:
        sp, x, v, ids = sp[order], x[order], v[order], ids[order]
    cap = [max(1, int(spare * (sp == s).sum())) for s in range(len(w.species))]
    cfg = pam.config_from_workload(w, repr=repr, deposit=deposit, sort_interval=sort_interval,
                                   capacity=cap)
    cfg.patches = patches
    with pam.Context(cfg) as ctx:
        if profile:
            ctx.profile_enable(True)
        for s in range(len(w.species)):
            m = sp == s
            if device_load:
                xt = torch.tensor(x[m], dtype=torch.float32, device="cuda")
                vt = torch.tensor(v[m], dtype=torch.float32, device="cuda")
                it = torch.tensor(ids[m], dtype=torch.int64, device="cuda")
                ctx.load_particles(s, xt, vt, it)
            else:
                ctx.load_particles(s, x[m], v[m], ids[m])
        if device_load:
            ctx.set_node_E([torch.tensor(e, dtype=torch.float32, device="cuda") for e in E])
        else:
            ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        if batch_steps_per_run:
            b = pam.Batch(1, repr, deposit, batch_steps_per_run, 64 << 30)
            try:
                slot = b.attach(ctx, nsteps)
                done = []
                for _ in range(nsteps + 1):
                    b.launch()
                    done += b.wait()
                    if slot in done:
                        break
                assert slot in done
                b.detach(slot)
            finally:
                b.close()
        elif sync_steps:
            for _ in range(nsteps):
                ctx.step(1)
                ctx.synchronize()
        elif split_steps:
            for k in split_steps:
                ctx.step(k)
        else:
            ctx.step(nsteps)
        rho, rho_fixed = ctx.get_rho()
        charge, counts = ctx.get_surface_charge()
        alive, absorbed, escaped = ctx.get_counters()
        prof = ctx.profile_read() if profile else None
        xs, vs, is_ = [], [], []
        for s in range(len(w.species)):
            px, pv, pid = ctx.get_particles(s)
            xs.append(px)
            vs.append(pv)
            is_.append(pid)
    pid = np.concatenate(is_)
    o = np.argsort(pid)
    return GpuRun(np.concatenate(xs)[o], np.concatenate(vs)[o], pid[o], rho, rho_fixed, charge,
                  counts, alive, absorbed, escaped, prof)


def inputs(w):
    sp, x, v = synth.all_particles(w)
    E = synth.node_E(w)
    return sp, x, v, E
