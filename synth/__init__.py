"""Seeded synthetic workloads for the particle-mesh hot path.

Inputs only (particles and node fields); nothing here performs a PIC step.
The C generator ``synth.c`` is compiled with gcc (OpenMP) into ``libsynth.so``.

Workloads (all in normalised units: unit cells h = 1, origin 0, dt = 0.05,
as §3.1.1 and §5.2.1 normalise lengths by the Debye length / the cell):

* ``sphere_16``  : 16^3 cells, absorbing sphere R = 3 at the centre, electrons
  (q = -1, m = 1, vth = 1) and ions (q = +1, m = 100, vth = 0.1), 8 particles per
  cell per species (2 x 32,768), node E of a ball of charge Q = -50, 10 steps,
  seed 0. Used in FP64.
* ``sphere_64``  : 64^3 cells, sphere R = 8, 50 particles per cell per species
  (2 x 13,107,200), Q = -50 (8/3)^2 (same surface field), node noise 1e-3,
  100 steps, seed 1. The OML-sphere shape of §3.
* ``crater_160`` : 160 x 160 x 80 cells (2.05M), flat ground at z = 10 with a
  spherical-bowl crater of radius 40 and depth 15 centred at (80, 80), electrons
  and drifting ions (drift 4 vth_i at 45 degrees to the vertical, towards the
  surface), 2 x 260,000,000 particles over the plasma region, sheath-like node E
  plus noise 1e-3, 50 steps, seed 2. The one-subdomain scale of §5 (2M cells,
  ~520M particles).
* ``crater_160_precision`` : the crater_160 shape, seed 3, 200 steps.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, replace

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "synth.c")
LIB = os.path.join(HERE, "libsynth.so")
SRC_DEV = os.path.join(HERE, "synth_dev.hip")
LIB_DEV = os.path.join(HERE, "libsynth_dev.so")


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", SRC,
                           "-o", tmp, "-lm"])
    os.replace(tmp, LIB)
    tmp = LIB_DEV + ".tmp"
    subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-fPIC",
                           "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           SRC_DEV, "-o", tmp], stderr=subprocess.DEVNULL)
    os.replace(tmp, LIB_DEV)
    return LIB


class _Species(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64), ("stream", ctypes.c_uint64),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("obj_kind", ctypes.c_int32), ("center", ctypes.c_double * 3), ("radius", ctypes.c_double),
        ("z_flat", ctypes.c_double), ("rim_radius", ctypes.c_double), ("depth", ctypes.c_double),
        ("vth", ctypes.c_double), ("drift", ctypes.c_double * 3),
    ]


_fp = ctypes.POINTER(ctypes.c_float)
_dp = ctypes.POINTER(ctypes.c_double)
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.synth_particles.argtypes = [ctypes.POINTER(_Species), ctypes.c_int64, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64)] + [_fp] * 6
        L.synth_node_E_coulomb.argtypes = [ctypes.c_int32] * 3 + [_dp, ctypes.c_double,
                                                                  ctypes.c_double, ctypes.c_double,
                                                                  ctypes.c_uint64] + [_fp] * 3
        L.synth_node_E_sheath.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double] * 4 + [
            ctypes.c_uint64] + [_fp] * 3
        L.synth_draw_u64.restype = ctypes.c_uint64
        L.synth_draw_u64.argtypes = [ctypes.c_uint64] * 4
        _lib = L
    return _lib


@dataclass
class SpeciesSpec:
    name: str
    q: float
    m: float
    vth: float
    count: int
    w: float = 1.0
    drift: tuple = (0.0, 0.0, 0.0)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    species: list
    obj: str = "none"            # "none" | "sphere" | "crater"
    center: tuple = (0.0, 0.0, 0.0)
    radius: float = 0.0
    z_flat: float = 0.0
    rim_radius: float = 0.0
    depth: float = 0.0
    field: str = "coulomb"       # "coulomb" | "sheath" | "zero"
    charge: float = 0.0          # ball charge (coulomb)
    noise: float = 0.0
    field_seed: int = 0
    sheath: tuple = (10.0, 0.2, 5.0)  # (z0, E0, L)
    dt: float = 0.05
    steps: int = 10
    seed: int = 0
    h: float = 1.0
    origin: tuple = (0.0, 0.0, 0.0)

    @property
    def nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_particles(self) -> int:
        return sum(s.count for s in self.species)

    @property
    def nbins(self) -> int:
        return self.nx * self.ny if self.obj == "crater" else 1

    def with_counts(self, counts) -> "Workload":
        sp = [replace(s, count=int(c)) for s, c in zip(self.species, counts)]
        return replace(self, species=sp)

    def _cspec(self, s: int) -> _Species:
        sp = self.species[s]
        c = _Species()
        c.seed, c.stream = self.seed, s
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.obj_kind = {"none": 0, "sphere": 1, "crater": 2}[self.obj]
        c.center[:] = list(self.center)
        c.radius = self.radius
        c.z_flat, c.rim_radius, c.depth = self.z_flat, self.rim_radius, self.depth
        c.vth = sp.vth
        c.drift[:] = list(sp.drift)
        return c


def particles(w: Workload, s: int, start: int = 0, count: int | None = None, idx=None):
    """Positions and half-step velocities (float32 arrays x, y, z, vx, vy, vz) of
    particles start..start+count-1 of species s, or of the listed indices."""
    L = lib()
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        count = len(idx)
    elif count is None:
        count = w.species[s].count - start
    out = [np.empty(count, np.float32) for _ in range(6)]
    spec = w._cspec(s)
    L.synth_particles(ctypes.byref(spec), start, count,
                      idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if idx is not None else None,
                      *[a.ctypes.data_as(_fp) for a in out])
    return out


_lib_dev = None


def particles_dev(w: Workload, s: int, stream: int = 0):
    """Particles of species s generated on the GPU into six float32 torch
    tensors (x, y, z, vx, vy, vz). Same draws as `particles`; velocities may
    differ in the last bits (device log / sin / cos)."""
    global _lib_dev
    import torch

    if _lib_dev is None:
        L = ctypes.CDLL(LIB_DEV)
        L.synth_particles_dev.restype = ctypes.c_int
        L.synth_particles_dev.argtypes = [ctypes.POINTER(_Species), ctypes.c_int64,
                                          ctypes.c_int64] + [ctypes.c_void_p] * 7
        _lib_dev = L
    n = w.species[s].count
    out = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(6)]
    spec = w._cspec(s)
    rc = _lib_dev.synth_particles_dev(ctypes.byref(spec), 0, n, *[t.data_ptr() for t in out],
                                      stream or None)
    if rc != 0:
        raise RuntimeError("device generator launch failed")
    return out


def node_E(w: Workload):
    """Node electric field (Ex, Ey, Ez), float32, (nx+1)(ny+1)(nz+1) each, x fastest."""
    L = lib()
    E = [np.zeros(w.nodes, np.float32) for _ in range(3)]
    if w.field == "coulomb":
        c = (ctypes.c_double * 3)(*w.center)
        L.synth_node_E_coulomb(w.nx, w.ny, w.nz, c, w.radius, w.charge, w.noise, w.field_seed,
                               *[e.ctypes.data_as(_fp) for e in E])
    elif w.field == "sheath":
        z0, E0, Ls = w.sheath
        L.synth_node_E_sheath(w.nx, w.ny, w.nz, z0, E0, Ls, w.noise, w.field_seed,
                              *[e.ctypes.data_as(_fp) for e in E])
    elif w.field != "zero":
        raise ValueError(w.field)
    return E


def all_particles(w: Workload):
    """Every particle of every species: (species (n,), x (n,3) f64, v (n,3) f64)."""
    sp, xs, vs = [], [], []
    for s in range(len(w.species)):
        a = particles(w, s)
        sp.append(np.full(len(a[0]), s, np.int32))
        xs.append(np.stack(a[:3], 1).astype(np.float64))
        vs.append(np.stack(a[3:], 1).astype(np.float64))
    return np.concatenate(sp), np.concatenate(xs), np.concatenate(vs)


def _electrons(count):
    return SpeciesSpec("electron", q=-1.0, m=1.0, vth=1.0, count=count)


def _ions(count, drift=(0.0, 0.0, 0.0)):
    return SpeciesSpec("ion", q=1.0, m=100.0, vth=0.1, count=count, drift=drift)


def sphere_16() -> Workload:
    n = 8 * 16 ** 3
    return Workload("sphere_16", 16, 16, 16, [_electrons(n), _ions(n)], obj="sphere",
                    center=(8.0, 8.0, 8.0), radius=3.0, field="coulomb", charge=-50.0,
                    steps=10, seed=0)


def sphere_64() -> Workload:
    n = 50 * 64 ** 3
    return Workload("sphere_64", 64, 64, 64, [_electrons(n), _ions(n)], obj="sphere",
                    center=(32.0, 32.0, 32.0), radius=8.0, field="coulomb",
                    charge=-50.0 * (8.0 / 3.0) ** 2, noise=1e-3, field_seed=1, steps=100, seed=1)


ION_DRIFT_45 = (0.4 * math.sin(math.pi / 4), 0.0, -0.4 * math.cos(math.pi / 4))


def crater_160(seed: int = 2, steps: int = 50) -> Workload:
    n = 260_000_000
    return Workload("crater_160", 160, 160, 80, [_electrons(n), _ions(n, ION_DRIFT_45)],
                    obj="crater", center=(80.0, 80.0, 0.0), z_flat=10.0, rim_radius=40.0,
                    depth=15.0, field="sheath", sheath=(10.0, 0.2, 5.0), noise=1e-3,
                    field_seed=seed, steps=steps, seed=seed)


def crater_160_precision() -> Workload:
    return replace(crater_160(seed=3, steps=200), name="crater_160_precision")


def scaled(w: Workload, nx: int, ny: int, nz: int, ppc: float, steps: int | None = None,
           name: str | None = None) -> Workload:
    """The same physics on a smaller box: geometry scaled by nx / w.nx, ppc
    particles per cell per species."""
    f = nx / w.nx
    n = int(round(ppc * nx * ny * nz))
    sp = [replace(s, count=n) for s in w.species]
    charge = w.charge * f * f
    return replace(w, name=name or f"{w.name}_scaled_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                   species=sp, center=tuple(c * f for c in w.center), radius=w.radius * f,
                   z_flat=w.z_flat * f, rim_radius=w.rim_radius * f, depth=w.depth * f,
                   charge=charge, sheath=(w.sheath[0] * f, w.sheath[1], w.sheath[2] * f),
                   steps=steps if steps is not None else w.steps)


def serving_stream(n_requests: int = 256, seed: int = 4, n_min: int = 16, n_max: int = 96,
                   ppc_min: int = 8, ppc_max: int = 64, steps_min: int = 100,
                   steps_max: int = 1000):
    """Independent sphere-charging requests: grid n^3 with n ~ U{n_min..n_max},
    sphere radius n/8 at the centre, ppc ~ U{ppc_min..ppc_max} per species,
    steps ~ U{steps_min..steps_max}; the per-request seed is drawn from the
    master seed. Returns a list of (Workload, steps)."""
    lib()
    out = []
    for r in range(n_requests):
        def draw(k):
            return synth_draw(seed, 7, r, k)
        n = n_min + draw(0) % (n_max - n_min + 1)
        ppc = ppc_min + draw(1) % (ppc_max - ppc_min + 1)
        steps = steps_min + draw(2) % (steps_max - steps_min + 1)
        rseed = draw(3) & 0x7FFFFFFF
        R = n / 8.0
        cnt = ppc * n ** 3
        w = Workload(f"request_{r}_n{n}", n, n, n, [_electrons(cnt), _ions(cnt)], obj="sphere",
                     center=(n / 2.0,) * 3, radius=R, field="coulomb",
                     charge=-50.0 * (R / 3.0) ** 2, steps=int(steps), seed=int(rseed))
        out.append((w, int(steps)))
    return out


def synth_draw(seed, stream, index, draw) -> int:
    return int(lib().synth_draw_u64(seed, stream, index, draw))


WORKLOADS = {
    "sphere_16": sphere_16,
    "sphere_64": sphere_64,
    "crater_160": crater_160,
    "crater_160_precision": crater_160_precision,
}
