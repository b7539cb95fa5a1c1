"""Shared test helpers: oracle problems from workloads, cross-precision fate
checks. Host-only; no GPU calls."""
import math

import numpy as np

import synth
from oracle import oracle
from oracle.oracle import Problem


def problem_of(w: synth.Workload, repr="fp64", deposit="fixed64") -> Problem:
    return Problem(nx=w.nx, ny=w.ny, nz=w.nz, dt=w.dt, q=[s.q for s in w.species],
                   m=[s.m for s in w.species], w=[s.w for s in w.species], h=w.h,
                   origin=w.origin, obj=w.obj, center=w.center, radius=w.radius,
                   z_flat=w.z_flat, rim_radius=w.rim_radius, depth=w.depth, repr=repr,
                   deposit=deposit)


def surface_distance(w: synth.Workload, pos) -> float:
    """Distance of a point (cell units) to the nearest surface that can decide a
    particle's fate: a box face, the sphere, or a crater surface part."""
    pos = np.asarray(pos, dtype=np.float64)
    n = np.array([w.nx, w.ny, w.nz], dtype=np.float64)
    d = float(np.minimum(np.abs(pos), np.abs(n - pos)).min())
    if w.obj == "sphere":
        d = min(d, abs(float(np.linalg.norm(pos - np.asarray(w.center))) - w.radius))
    elif w.obj == "crater":
        a, dep = w.rim_radius, w.depth
        Rc = (a * a + dep * dep) / (2 * dep)
        zc = w.z_flat - dep + Rc
        c = np.array([w.center[0], w.center[1], zc])
        d = min(d, abs(pos[2] - w.z_flat), abs(pos[2]),
                abs(float(np.linalg.norm(pos - c)) - Rc))
    return d


def fate_mismatches(ra_fate, ra_where, ra_when, rb_fate, rb_where, rb_when):
    return np.nonzero((ra_fate != rb_fate) | (ra_where != rb_where) | (ra_when != rb_when))[0]


def deciding_step(fa, wa, fb, wb):
    """First step at which one of two runs removed the particle."""
    steps = [s for f, s in ((fa, wa), (fb, wb)) if f != 0]
    return min(steps)


def check_mismatches_near_surface(w, species, x, v, E, idx, when_a, fate_a, when_b, fate_b,
                                  delta=1e-4):
    """For each particle index in idx whose fate differs between two runs, rerun
    it alone in the FP64 oracle up to the first step at which either run removed
    it, and return the FP64 distances to the nearest deciding surface there."""
    prob = problem_of(w, "fp64")
    out = []
    for p in idx:
        s = deciding_step(fate_a[p], when_a[p], fate_b[p], when_b[p])
        r = oracle.run(prob, species[p:p + 1], x[p:p + 1], v[p:p + 1], E, s + 1)
        out.append(surface_distance(w, r.x[0]))
    return np.array(out)
