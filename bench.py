#!/usr/bin/env python3
"""Throughput of the particle-mesh hot path (gather + leapfrog push + collection
+ trilinear deposit, with the periodic tile re-bucketing) on one MI355X.

Default workload: the lunar-crater shape, one subdomain on one GPU:
160 x 160 x 80 cells (2.05M), 2 x 260,000,000 particles, FP32 cell-relative
state with int64 fixed-point deposition; particles are re-bucketed by tile
inside every step (full re-planning of the tile regions only on demand).

A step is one pass of the whole hot path over all particles; particle-steps
count the particles alive at the start of each step. Inputs are generated on
the host, loaded into HBM, and are resident before the timed region starts.

Prints one JSON line (the last line of stdout). Progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time
from dataclasses import replace

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (gather+push+deposit), % HBM roofline; p50/p99 req latency"
HBM_PEAK_GBS = 8000.0
# state read + written per particle-step: FP32 cell form 24 B (offsets that
# carry the cell within the tile + velocities), FP32 absolute 24 B, FP64 48 B
BYTES_PER_PARTICLE_STEP = {"fp32_cell": 48, "fp32_abs": 48, "fp64": 96}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2011_10214_amd", "csrc", "pic_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_kernel_crater_160.json")


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def host_info():
    model = platform.processor()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem = round(int(line.split()[1]) / 2 ** 20, 1)
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"cpu": model, "logical_cpus": cores, "ram_gib": mem}


def kernel_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_for(workload, repr_, deposit, particles_per_launch):
    """HBM bytes per launch of the step kernel from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE counters (calibrated against a plain copy of known size), scaled
    to this run's particles per launch -- only if the stored measurement was
    taken on the current kernel source, else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_source_sha256") != kernel_hash() or t.get("workload") != workload
            or t.get("repr") != repr_ or t.get("deposit") != deposit):
        return None
    return t["hbm_bytes_per_particle_step"] * particles_per_launch


def copy_ceiling(nbytes=4 << 30, reps=5):
    """Measured HBM ceiling, read + write of nbytes each, best of reps, in
    GB/s, by two streams: the runtime's device-to-device copy and a plain
    streaming kernel (an out-of-place elementwise multiply, which streams
    faster than the copy on these boxes). Returns (ceiling, by_kind)."""
    import torch

    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    kinds = {"device_copy": lambda: y.copy_(x),
             "streaming_kernel": lambda: torch.mul(x, 1.0000001, out=y)}
    by_kind = {}
    for name, fn in kinds.items():
        fn()
        best = 0.0
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            best = max(best, 2 * nbytes / (a.elapsed_time(b) * 1e-3) / 1e9)
        by_kind[name] = best
    del x, y
    torch.cuda.empty_cache()
    return max(by_kind.values()), by_kind


def cpu_baseline(w, target_s):
    """The FP64 oracle on a bounded sample of the workload, timed twice: on one
    thread, and on every host core (OpenMP: the particle updates in parallel,
    the fixed-point rho per thread, summed in thread order; the same bits as
    one thread). `value` and `cores` are the all-cores run's."""
    import numpy as np

    import synth
    from oracle import oracle

    E = synth.node_E(w)
    prob = oracle.Problem(nx=w.nx, ny=w.ny, nz=w.nz, dt=w.dt, q=[s.q for s in w.species],
                          m=[s.m for s in w.species], w=[s.w for s in w.species], obj=w.obj,
                          center=w.center, radius=w.radius, z_flat=w.z_flat,
                          rim_radius=w.rim_radius, depth=w.depth, repr="fp64", deposit="fixed64")

    def sample(per):
        sp, xs, vs = [], [], []
        for s in range(len(w.species)):
            if w.species[s].count == 0:
                continue
            a = synth.particles(w, s, 0, per)
            sp.append(np.full(per, s, np.int32))
            xs.append(np.stack(a[:3], 1).astype(np.float64))
            vs.append(np.stack(a[3:], 1).astype(np.float64))
        return np.concatenate(sp), np.concatenate(xs), np.concatenate(vs)

    def timed(per, threads):
        sp, x, v = sample(per)
        pr = replace(prob, threads=threads)
        t0 = time.perf_counter()
        oracle.run(pr, sp, x, v, E, 1)
        one = time.perf_counter() - t0
        steps = int(max(1, min(w.steps, target_s / max(one, 1e-3))))
        t0 = time.perf_counter()
        r = oracle.run(pr, sp, x, v, E, steps)
        dt = time.perf_counter() - t0
        ps = int(np.where(r.fate == 0, steps, r.when + 1).sum())
        return ps / dt, steps, dt

    cores = host_info()["logical_cpus"] or 1
    v1, st1, t1 = timed(1 << 19, 1)
    log(f"cpu baseline, one thread: {v1:.3e} particle-steps/s ({st1} steps, {t1:.1f} s)")
    per_n = 1 << 19 if cores <= 1 else 1 << 21
    vn, stn, tn = timed(per_n, cores)
    log(f"cpu baseline, {cores} threads: {vn:.3e} particle-steps/s ({stn} steps, {tn:.1f} s)")
    return {"value": vn, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": (f"first {per_n} particles of each species of {w.name}, {stn} steps, FP64 "
                       f"oracle with fixed-point deposit on {cores} threads, {tn:.1f} s; one "
                       f"thread: first {1 << 19} per species, {st1} steps, {t1:.1f} s"),
            "single_thread": {"value": v1, "cores": 1},
            "host": host_info()}


def serving_run(args):
    """Serving benchmark: a stream of independent sphere-charging requests
    (grids 16^3..96^3, 8-64 particles per cell per species, 100-1000 steps)
    served with continuous batching (pic_batch: persistent step kernels
    replayed from captured graphs, admission by HBM footprint, loading
    overlapped with the running batch; two share policies) and, as the
    reference, one at a time through pic_step, with the same Poisson arrivals
    at a load of `--load` times the one-at-a-time service rate."""
    import numpy as np

    import paper_2011_10214_amd as pam
    import synth
    from paper_2011_10214_amd.serve import (BatchExecutor, Request, SequentialExecutor,
                                            serve)

    stream_w = synth.serving_stream(n_requests=args.requests, seed=4)
    budget = int(args.budget_gb * (1 << 30))

    def requests(arrivals):
        out = []
        for i, ((w, steps), t) in enumerate(zip(stream_w, arrivals)):
            def loader(ctx, w=w):
                for s in range(len(w.species)):
                    ctx.load_particles_cols(s, synth.particles_dev(w, s))
                ctx.set_node_E([e.astype(np.float64) for e in synth.node_E(w)])

            def collect(ctx):
                return ctx.get_counters()[0].sum()
            out.append(Request(rid=i, arrival=float(t), steps=steps,
                               cfg=pam.config_from_workload(w, repr="fp32_cell", deposit="fixed64"),
                               loader=loader, particles=w.n_particles, collect=collect))
        return out

    log(f"serving: {len(stream_w)} requests, "
        f"{sum(w.n_particles * s for w, s in stream_w) / 1e12:.2f}e12 particle-steps")
    # one-at-a-time service rate with every request waiting at t = 0
    seq0 = serve(requests([0.0] * len(stream_w)), SequentialExecutor(budget))
    mu = seq0["throughput_req_per_s"]
    log(f"one at a time, all queued: {seq0['wall_s']:.1f} s, {mu:.2f} req/s")
    # the same exponential draws for every load, scaled by 1 / rate
    gaps = np.random.default_rng(4).exponential(1.0, len(stream_w))

    def arrivals_at(rate):
        a = np.cumsum(gaps / rate)
        return a - a[0]

    rate = args.load * mu
    arrivals = arrivals_at(rate)
    seq = serve(requests(arrivals), SequentialExecutor(budget))
    log(f"one at a time, Poisson {rate:.2f} req/s: p50 {seq['latency_p50_s']:.2f} s, "
        f"p99 {seq['latency_p99_s']:.2f} s, mean {seq['latency_mean_s']:.2f} s")
    batched = {}
    # priority (the default here): the oldest request runs, younger ones
    # beside it only in the room a small one leaves on the GPU and only if
    # they end no later than it (EASY-style backfill), at most one large
    # request admitted to wait; priority_any_side: any younger request that
    # fits the room, no admission bound; prefetch 2: at most two admitted to
    # wait; fifo: nothing beside the head (strict arrival order); head half:
    # the oldest running request gets half of a run's particle-steps, the
    # others share the rest; fair share: equal shares
    M, P = args.steps_per_run, int(args.ps_per_run)
    base = dict(policy="priority", backfill=args.backfill, saturation=int(args.saturation))
    prio = dict(base, within_head=True, prefetch_large=1)
    variants = [("priority", prio),
                ("priority_within_head_sat_10M", dict(base, within_head=True,
                                                      saturation=10_000_000)),
                ("priority_within_head", dict(base, within_head=True)),
                ("priority_any_side", base),
                ("priority_prefetch_2", dict(base, prefetch=2)),
                ("priority_prefetch_large_1", dict(base, prefetch_large=1)),
                ("priority_prefetch_large_2", dict(base, prefetch_large=2)),
                ("priority_sat_10M", dict(base, saturation=10_000_000)),
                ("priority_sat_5M", dict(base, saturation=5_000_000)),
                ("priority_fifo", dict(base, saturation=0)),
                ("head_half", dict(policy="head")),
                ("fair_share", dict(policy="fair"))]
    if args.serve_variants:
        keep = [v.strip() for v in args.serve_variants.split(",") if v.strip()]
        unknown = set(keep) - {n for n, _ in variants}
        if unknown:
            raise SystemExit(f"unknown serving variants: {sorted(unknown)}")
        variants = [(n, kw) for n, kw in variants if n in keep]
    for name, kw in variants:
        ex = BatchExecutor(max_slots=args.slots, repr="fp32_cell", deposit="fixed64",
                           steps_per_run=M, hbm_budget_bytes=budget, particle_steps_per_run=P,
                           **kw)
        try:
            st = serve(requests(arrivals), ex)
        finally:
            ex.close()
        st.update(steps_per_run=M, particle_steps_per_run=P,
                  **{k: v for k, v in kw.items() if k != "policy"})
        batched[name] = st
        log(f"batched ({name}), Poisson {rate:.2f} req/s: p50 {st['latency_p50_s']:.2f} s, "
            f"p99 {st['latency_p99_s']:.2f} s, mean {st['latency_mean_s']:.2f} s")
    # other loads: one at a time and the default batched policy
    sweep = {}
    for load in [float(x) for x in args.sweep.split(",") if x.strip()]:
        r = load * mu
        a = arrivals_at(r)
        sq = serve(requests(a), SequentialExecutor(budget))
        ex = BatchExecutor(max_slots=args.slots, repr="fp32_cell", deposit="fixed64",
                           steps_per_run=M, hbm_budget_bytes=budget, particle_steps_per_run=P,
                           **prio)
        try:
            bt = serve(requests(a), ex)
        finally:
            ex.close()
        sweep[str(load)] = {"arrival_rate_req_per_s": r, "one_at_a_time": sq, "batched_priority": bt}
        for name, st in (("one at a time", sq), ("batched (priority)", bt)):
            log(f"load {load}: {name}, Poisson {r:.2f} req/s: p50 {st['latency_p50_s']:.2f} s, "
                f"p99 {st['latency_p99_s']:.2f} s, mean {st['latency_mean_s']:.2f} s, "
                f"wall {st['wall_s']:.1f} s")
    return {"requests": len(stream_w), "arrival_rate_req_per_s": rate, "load": args.load,
            "service_rate_one_at_a_time_req_per_s": mu, "slots": args.slots,
            "hbm_budget_bytes": budget, "batched": batched, "one_at_a_time": seq,
            "load_sweep": sweep}


PRECISION_FORMS = [("fp64", "fixed64"), ("fp64", "fp64"), ("fp32_abs", "fixed64"),
                   ("fp32_abs", "fp32"), ("fp32_cell", "fixed64"), ("fp32_cell", "fp32")]


def precision_study(args):
    """Precision of every representation x deposit form on the crater shape
    (seed 3) after `steps` steps: error of rho, sampled positions/velocities and
    surface charge against the FP64 path (FP64 oracle on the sampled particles;
    for the mesh quantities the FP64 GPU path with fixed-point deposit, which
    reproduces the FP64 oracle bit for bit), and determinism over reruns."""
    import hashlib as hl

    import numpy as np
    import torch

    import paper_2011_10214_amd as pam
    import synth
    from oracle import oracle

    w = synth.crater_160_precision()
    if args.scale != 1.0:  # fewer particles, same mesh and geometry (quick runs)
        w = w.with_counts([int(s.count * args.scale) for s in w.species])
    steps = args.steps
    rng = np.random.default_rng(3)
    samples = [np.sort(rng.choice(s.count, args.sample, replace=False)) for s in w.species]
    log(f"precision study: {w.name}, {w.n_particles} particles, {steps} steps, "
        f"{args.reruns} reruns, sample {args.sample} per species")
    host = [synth.particles(w, s) for s in range(len(w.species))]
    E = synth.node_E(w)
    stream = torch.cuda.Stream()

    def one_run(repr_, dep):
        cfg = pam.config_from_workload(w, repr=repr_, deposit=dep, stream=stream.cuda_stream)
        with pam.Context(cfg) as ctx:
            for s, spec in enumerate(w.species):
                dev = [torch.from_numpy(c).to("cuda") for c in host[s]]
                ids = torch.arange(spec.count, dtype=torch.int64, device="cuda")
                ctx.load_particles_cols(s, dev, ids)
                del dev, ids
            ctx.set_node_E([torch.from_numpy(e).to("cuda") for e in E])
            t0 = time.perf_counter()
            ctx.step(steps)
            ctx.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            rho, _ = ctx.get_rho()
            charge, counts = ctx.get_surface_charge()
            alive, _, _ = ctx.get_counters()
            smp = [ctx.get_particles_by_id(s, samples[s]) for s in range(len(w.species))]
        torch.cuda.empty_cache()
        h = hl.sha256(rho.tobytes() + counts.tobytes())
        for f, x, v in smp:
            h.update(f.tobytes() + np.nan_to_num(x).tobytes() + np.nan_to_num(v).tobytes())
        return dict(rho=rho, charge=charge, counts=counts, alive=alive, smp=smp, ms=ms,
                    hash=h.hexdigest())

    # the sampled particles through the FP64 oracle
    sp = np.concatenate([np.full(args.sample, s, np.int32) for s in range(len(w.species))])
    parts = [synth.particles(w, s, idx=samples[s]) for s in range(len(w.species))]
    x0 = np.concatenate([np.stack(p[:3], 1) for p in parts]).astype(np.float64)
    v0 = np.concatenate([np.stack(p[3:], 1) for p in parts]).astype(np.float64)
    prob = oracle.Problem(nx=w.nx, ny=w.ny, nz=w.nz, dt=w.dt, q=[s.q for s in w.species],
                          m=[s.m for s in w.species], w=[s.w for s in w.species], obj=w.obj,
                          center=w.center, z_flat=w.z_flat, rim_radius=w.rim_radius,
                          depth=w.depth, repr="fp64", deposit="fixed64")
    ref = oracle.run(prob, sp, x0, v0, E, steps)
    vth = np.where(sp == 0, w.species[0].vth, w.species[-1].vth)

    table = []
    base = None
    for repr_, dep in PRECISION_FORMS:
        runs = []
        for k in range(args.reruns):
            runs.append(one_run(repr_, dep))
            log(f"{repr_}/{dep} run {k}: {runs[-1]['ms']:.2f} ms/step")
        r = runs[0]
        if base is None:
            base = r
        row = {"repr": repr_, "deposit": dep,
               "ms_per_step": r["ms"],  # with ids tracked and the one-off initial re-bucketing
               "distinct_results_over_reruns": len({q["hash"] for q in runs})}
        drho = np.abs(r["rho"] - base["rho"])
        big = np.abs(base["rho"]) > 1.0
        row["rho_max_abs_err"] = float(drho.max())
        row["rho_max_rel_err_where_abs_gt_1"] = float((drho[big] / np.abs(base["rho"][big])).max()) if big.any() else None
        row["rho_rms_err"] = float(np.sqrt((drho ** 2).mean()))
        # the net rho is a difference of two nearly equal species densities, so
        # its pointwise relative error is ill-conditioned; also give the error
        # relative to the largest |rho| and the ms/step caveat
        row["rho_max_abs_err_over_max_abs_rho"] = float(drho.max() / max(np.abs(base["rho"]).max(), 1e-300))
        dq = np.abs(r["charge"] - base["charge"])
        row["surface_charge_max_abs_err_per_bin"] = float(dq.max())
        row["surface_charge_total_rel_err"] = float(abs(r["charge"].sum() - base["charge"].sum()) /
                                                    max(abs(base["charge"].sum()), 1.0))
        found = np.concatenate([f for f, _, _ in r["smp"]])
        gx = np.concatenate([x for _, x, _ in r["smp"]])
        gv = np.concatenate([v for _, _, v in r["smp"]])
        both = found & (ref.fate == 0)
        row["sample_fate_mismatches"] = int((found != (ref.fate == 0)).sum())
        dx = np.abs(gx[both] - ref.x[both]).max(axis=1)
        dv = np.abs(gv[both] - ref.v[both]).max(axis=1)
        row["x_max_abs_err"] = float(dx.max()) if both.any() else 0.0
        row["x_max_rel_err"] = float((dx / np.maximum(np.abs(ref.x[both]).max(axis=1), 1.0)).max()) if both.any() else 0.0
        row["v_max_rel_err"] = float((dv / np.maximum(np.abs(ref.v[both]).max(axis=1), vth[both])).max()) if both.any() else 0.0
        table.append(row)
        log(json.dumps(row))
    print(json.dumps({"precision_study": w.name, "steps": steps, "particles": w.n_particles,
                      "reruns": args.reruns, "sample_per_species": args.sample,
                      "reference": "FP64 oracle on the sample; FP64 GPU path with fixed-point "
                                   "deposit (bit-exact to the FP64 oracle) for rho and charge",
                      "forms": table}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="crater_160")
    ap.add_argument("--repr", default="fp32_cell", choices=sorted(BYTES_PER_PARTICLE_STEP))
    ap.add_argument("--deposit", default="fixed64", choices=["fixed64", "fp32", "fp64"])
    ap.add_argument("--sort-interval", type=int, default=0,
                    help="re-plan the tile regions every K steps (0: on demand)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--field", default="off", choices=["off", "lunar", "oml"],
                    help="close the PIC loop: a field solve after every step (lunar: phi = 0 "
                         "at z+, zero-Neumann elsewhere; oml: phi = 0 at the max faces); "
                         "PCG tolerance 1e-6 and at most 150 iterations as in the paper")
    ap.add_argument("--eps-object", type=float, default=4.0,
                    help="field modes: permittivity inside the object relative to the plasma "
                         "(the paper's regolith and OML sphere: 4; 0: no interface)")
    ap.add_argument("--field-op", default="fv", choices=["fv", "ife"],
                    help="field modes: node-centred finite volumes, or immersed finite elements "
                         "on five tetrahedra per cell (the paper's discretisation)")
    ap.add_argument("--no-surface-charge", action="store_true",
                    help="field modes: leave the collected charge out of the field source")
    ap.add_argument("--patches", type=int, default=8,
                    help="sphere workloads: surface patches per cube-face edge (tally bins)")
    ap.add_argument("--boundaries", default="open", choices=["open", "lunar", "oml"],
                    help="open: all faces remove; lunar: y- reflects and ambient plasma is "
                         "injected at x-, x+, y+, z+ every step; oml: the min faces reflect "
                         "and the max faces inject")
    ap.add_argument("--photoemission", action="store_true",
                    help="with --boundaries lunar: a photoelectron species emitted from the "
                         "sunlit terrain (Sun 10 degrees above the ground in the X-Z plane; "
                         "density and thermal speed relative to the solar-wind electrons as "
                         "in the paper's table of plasma parameters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the plain copy kernel (counter calibration)")
    ap.add_argument("--precision", action="store_true",
                    help="precision study of all forms on the crater shape (seed 3)")
    ap.add_argument("--reruns", type=int, default=5)
    ap.add_argument("--sample", type=int, default=20000)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark (continuous batching vs one at a time)")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--steps-per-run", type=int, default=256)
    ap.add_argument("--ps-per-run", type=float, default=1e10,
                    help="serving: particle-steps shared by the running requests per "
                         "batched run, about 0.12 s of GPU time (0: every request gets "
                         "--steps-per-run steps)")
    ap.add_argument("--backfill", type=float, default=0.0,
                    help="serving, priority policy: share of a large head's runs that "
                         "younger requests may take")
    ap.add_argument("--saturation", type=float, default=2e7,
                    help="serving, priority policy: particles that fill the GPU")
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--serve-variants", default="",
                    help="comma-separated batched policies to run (default: all)")
    ap.add_argument("--sweep", default="0.5,1.0",
                    help="--serve: further loads (comma-separated) run one at a time and "
                         "with the default batched policy")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: one MI355X holds the whole subdomain and the "
              "path has no multi-GPU form (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2011_10214_amd as pam
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_only:
        c, by_kind = copy_ceiling()
        print(json.dumps({"copy_ceiling_GBs": c, "by_kind": by_kind, "copy_bytes_each_way": 4 << 30}))
        return
    if args.serve:
        print(json.dumps({"serving": serving_run(args)}), flush=True)
        return
    if args.precision:
        if args.steps == 50:
            args.steps = 200
        precision_study(args)
        return
    torch.cuda.set_device(0)
    w = synth.WORKLOADS[args.workload]()
    photo = None
    if args.photoemission:
        if args.boundaries != "lunar" or w.obj != "crater":
            log("--photoemission needs --boundaries lunar on a crater workload")
            sys.exit(2)
        # photoelectrons at 90 degrees Sun: n_pe / n_sw = 64 / 8.7 and
        # vth_pe / vth_e = 622 / 1453 (the paper's plasma parameters); the
        # emitted half-Maxwellian of surface density n_pe carries the flux
        # n_pe vth_pe sqrt(2 / pi) at normal incidence
        e = w.species[0]
        above = w.nx * w.ny * (w.nz - w.z_flat) * w.h ** 3
        vth_pe = e.vth * 622.0 / 1453.0
        flux = (64.0 / 8.7) * (e.count / above) * vth_pe * math.sqrt(2.0 / math.pi)
        elev = math.radians(10.0)
        photo = dict(seed=23, sun=(math.cos(elev), 0.0, math.sin(elev)), flux=flux, vth=vth_pe)
        w = replace(w, species=list(w.species) + [synth.SpeciesSpec(
            "photoelectron", q=-1.0, m=e.m, vth=vth_pe, count=0, w=e.w)])
    # a stream of torch's own (default priority) that the library enqueues on,
    # so that the events below bracket exactly the library's work
    stream = torch.cuda.Stream()
    cap = None
    if args.boundaries != "open":  # injection: room for the population to fluctuate
        cap = [int(sp.count * 1.1) + 4096 for sp in w.species]
    if photo:  # the photoelectrons of every step stay near the ground; the tile
        # regions keep room for some 20 more steps of them between re-plannings
        per_step = photo["flux"] * math.sin(math.radians(10.0)) * w.nx * w.ny * w.dt
        cap[-1] = int(per_step * (args.warmup + args.steps + 2 + 24) * 1.2) + 65536
    cfg = pam.config_from_workload(w, repr=args.repr, deposit=args.deposit,
                                   sort_interval=args.sort_interval, stream=stream.cuda_stream,
                                   capacity=cap)
    if w.obj == "sphere" and args.field != "off":
        cfg.patches = args.patches  # where the collected charge sits
    inj = None
    if args.boundaries == "lunar":
        # the lunar setup of §5.2.2: symmetry plane y-, ambient plasma injected
        # at x-, x+, y+ and z+ with the loaded density above the flat ground
        cfg.reflect = 4
        above = w.nx * w.ny * (w.nz - w.z_flat) * w.h ** 3
        inj = dict(faces=1 | 2 | 8 | 32, seed=17, density=[sp.count / above for sp in w.species],
                   vth=[sp.vth for sp in w.species], drift=[tuple(sp.drift) for sp in w.species])
    elif args.boundaries == "oml":
        # the OML setup of §3.1.3: the min faces are symmetry planes, the max
        # faces inject the ambient plasma at the loaded density
        cfg.reflect = 1 | 4 | 16
        vol = w.nx * w.ny * w.nz * w.h ** 3
        inj = dict(faces=2 | 8 | 32, seed=17, density=[sp.count / vol for sp in w.species],
                   vth=[sp.vth for sp in w.species], drift=[tuple(sp.drift) for sp in w.species])
    log(f"workload {w.name}: {w.nx}x{w.ny}x{w.nz} cells, {w.n_particles} particles, "
        f"{args.repr}/{args.deposit}, K={args.sort_interval}, boundaries {args.boundaries}")
    ctx = pam.Context(cfg)
    if inj:  # (a photoelectron species has no loaded particles: density 0, not injected)
        ctx.set_injection(**inj)
    if photo:
        ctx.set_photoemission(len(w.species) - 1, **photo)
    t0 = time.perf_counter()
    for s in range(len(w.species)):
        cols = synth.particles(w, s)
        log(f"species {s}: generated {len(cols[0])} particles ({time.perf_counter() - t0:.1f} s)")
        dev = [torch.from_numpy(c).to("cuda") for c in cols]
        del cols
        ctx.load_particles_cols(s, dev)
        del dev
        torch.cuda.empty_cache()
        log(f"species {s}: loaded ({time.perf_counter() - t0:.1f} s)")
    E = [torch.from_numpy(e).to("cuda") for e in synth.node_E(w)]
    ctx.set_node_E(E)
    del E

    field_mask = {"off": 0, "lunar": 32, "oml": 2 | 8 | 32}[args.field]
    surface = field_mask != 0 and not args.no_surface_charge and w.obj != "none"
    field_kw = dict(eps_object=args.eps_object if w.obj != "none" else 0.0, surface_charge=surface,
                    op=args.field_op)

    def advance(k):
        if not field_mask:
            ctx.step(k)
            return
        for _ in range(k):  # deposit -> field solve -> gather / push
            ctx.step(1)
            ctx.solve_field(field_mask, tol=1e-6, max_iter=150, **field_kw)

    log(f"warmup {args.warmup} steps")
    if field_mask:
        ctx.step(0)
        it, rr = ctx.solve_field(field_mask, tol=1e-6, max_iter=2000, **field_kw)
        log(f"initial field: {it} iterations, relative residual {rr:.2e}")
    advance(args.warmup)
    ctx.synchronize()
    alive0, _, _ = ctx.get_counters()
    injected0 = ctx.get_injected()

    # the K timed steps in 5 blocks (as equal as K allows), each bracketed by
    # events on the library's stream and synchronised; value = all particle-
    # steps / the summed block times, beside the median of the block rates
    nblocks = min(5, args.steps)
    sizes = [args.steps // nblocks + (1 if b < args.steps % nblocks else 0)
             for b in range(nblocks)]
    ms = 0.0
    block_rates = []
    tot = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in sizes:
        ctx.profile_enable(True)  # (resets the totals)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        advance(k)
        e1.record(stream)
        torch.cuda.synchronize()
        bms = e0.elapsed_time(e1)
        p = ctx.profile_read()
        ms += bms
        block_rates.append(p.particle_steps / (bms / 1e3))
        if tot is None:
            tot = p
        else:
            for f in p.__dataclass_fields__:
                setattr(tot, f, getattr(tot, f) + getattr(p, f))
    wall_ms = (time.perf_counter() - t0) * 1e3
    ctx.synchronize()
    prof = tot
    alive1, absorbed, escaped = ctx.get_counters()
    injected = ctx.get_injected()
    log(f"timed {args.steps} steps: {ms:.2f} ms (host wall {wall_ms:.2f} ms); step kernel {prof.step_ms / max(1, prof.step_launches):.3f} ms avg, "
        f"sort {prof.sort_ms / max(1, prof.sort_launches):.3f} ms avg x{prof.sort_launches}")
    ctx.close()
    copy_gbs, copy_kinds = copy_ceiling()
    log(f"copy ceiling {copy_gbs:.0f} GB/s ({', '.join(f'{k} {v:.0f}' for k, v in copy_kinds.items())})")

    value = prof.particle_steps / (ms / 1e3)
    bpp = BYTES_PER_PARTICLE_STEP[args.repr]
    step_s = prof.step_ms / 1e3
    achieved = bpp * prof.particle_steps / step_s / 1e9 if step_s > 0 else 0.0
    per_launch_particles = prof.particle_steps / max(1, prof.step_launches)
    traffic = traffic_for(w.name, args.repr, args.deposit, per_launch_particles)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.repr != "fp64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} cells, {w.n_particles} particles "
                        f"({len(w.species)} species), "
                        + ("crater terrain" if w.obj == "crater" else
                           f"absorbing sphere radius {w.radius}" if w.obj == "sphere" else
                           "no object") + f", dt {w.dt}",
            "repr": args.repr,
            "deposit": args.deposit + (" (int64 at 2^-32)" if args.deposit == "fixed64" else ""),
            "sort_interval": args.sort_interval,
            "particles_alive_start": int(alive0.sum()),
            "particles_alive_end": int(alive1.sum()),
            "timed_wall_ms": wall_ms,
            "timed_blocks": sizes,
        },
        "median_of_blocks": {
            "value": float(np.median(block_rates)),
            "unit": "particle-steps/s",
            "block_values": block_rates,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "step_kernel (gather+push+collect+deposit)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_particle_step": bpp,
            "step_kernel_ms_avg": prof.step_ms / max(1, prof.step_launches),
            "particles_per_launch": per_launch_particles,
            "copy_ceiling_GBs": copy_gbs,
            "copy_ceiling_by_kind": copy_kinds,
            "frac_of_copy_ceiling": achieved / copy_gbs if copy_gbs else None,
        },
        "phases_ms_per_step": {
            "step_kernel": prof.step_ms / args.steps,
            "sort": prof.sort_ms / args.steps,
            "rho_clear": prof.clear_ms / args.steps,
            "injection": prof.inject_ms / args.steps,
            "photoemission": prof.photo_ms / args.steps,
            "field_solve": prof.field_ms / args.steps,
        },
    }
    if field_mask:
        nodes = (w.nx + 1) * (w.ny + 1) * (w.nz + 1)
        iters = prof.field_iterations / max(1, prof.field_solves)
        out["config"]["field"] = (f"{args.field}: Dirichlet faces mask {field_mask}, PCG tol 1e-6, "
                                  "max 150 iterations, warm start, multigrid preconditioner; "
                                  f"operator {'immersed finite elements' if args.field_op == 'ife' else 'finite volumes'}; "
                                  f"object permittivity {field_kw['eps_object']} (0: none), "
                                  f"surface charge {'on' if surface else 'off'}")
        out["field_solve"] = {
            "ms_per_solve": prof.field_ms / max(1, prof.field_solves),
            "iterations_per_solve": iters,
            "nodes": nodes,
        }
    if inj:
        out["config"]["boundaries"] = (
            "lunar: y- reflects; ambient plasma injected at x-, x+, y+, z+ (ghost slabs, "
            "drifting Maxwellian)" if args.boundaries == "lunar" else
            "oml: x-, y-, z- reflect; ambient plasma injected at x+, y+, z+ (ghost slabs, "
            "drifting Maxwellian)")
        ambient = slice(0, len(w.species) - 1) if photo else slice(None)
        out["injection"] = {
            "kernel_ms_avg": prof.inject_ms / max(1, prof.inject_launches),
            "injected_per_step": int((injected - injected0)[ambient].sum()) / args.steps,
            "share_of_step": prof.inject_ms / ms if ms > 0 else None,
        }
    if photo:
        out["config"]["photoemission"] = (
            "photoelectrons from the sunlit terrain: Sun 10 degrees above the ground in the X-Z "
            f"plane, flux {photo['flux']:.4g} per unit area and time at normal incidence, "
            f"vth {photo['vth']:.4g}")
        out["photoemission"] = {
            "kernel_ms_avg": prof.photo_ms / max(1, prof.photo_launches),
            "emitted_per_step": int((injected - injected0)[-1]) / args.steps,
            "share_of_step": prof.photo_ms / ms if ms > 0 else None,
        }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
