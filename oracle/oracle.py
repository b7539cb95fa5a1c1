"""ctypes binding of the CPU oracle (``oracle/pic_oracle.cpp``).

Test infrastructure: only the tests, the smoke check and the CPU-baseline leg of
the benchmark import this module. It imports nothing from the GPU package.

The oracle runs the explicit PIC step of §2.1 (gather, leapfrog push, boundary
and object removal of §3.1.3 / §5.2.2, trilinear charge deposit) on the CPU in
FP64, or in one of two FP32 mirror forms with the same expression order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

REPR = {"fp64": 0, "fp32_abs": 1, "fp32_cell": 2}
DEPOSIT = {"fixed64": 0, "fp32": 1, "fp64": 2}
OBJECT = {"none": 0, "sphere": 1, "crater": 2}

# -ffp-contract=off: no multiply-add is fused unless written as fma.
# -fopenmp: the particle updates and the fixed-point deposit on several
# threads when Problem.threads > 1 (bit-identical to one thread).
CFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared"]


def build() -> str:
    """Compile the oracle shared library with g++ (always recompiles)."""
    tmp = LIB + ".tmp"
    subprocess.check_call(["g++", *CFLAGS, SRC, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("h", ctypes.c_double), ("origin", ctypes.c_double * 3), ("dt", ctypes.c_double),
        ("n_species", ctypes.c_int32),
        ("q", ctypes.c_double * 4), ("m", ctypes.c_double * 4), ("w", ctypes.c_double * 4),
        ("obj_kind", ctypes.c_int32), ("center", ctypes.c_double * 3), ("radius", ctypes.c_double),
        ("z_flat", ctypes.c_double), ("rim_radius", ctypes.c_double), ("depth", ctypes.c_double),
        ("repr", ctypes.c_int32), ("deposit", ctypes.c_int32),
        ("reflect", ctypes.c_int32), ("inj_faces", ctypes.c_int32), ("inj_seed", ctypes.c_uint64),
        ("inj_density", ctypes.c_double * 4), ("inj_vth", ctypes.c_double * 4),
        ("inj_drift", ctypes.c_double * 12),
        ("sphere_patches", ctypes.c_int32),
        ("pe_species", ctypes.c_int32), ("pe_seed", ctypes.c_uint64),
        ("pe_sun", ctypes.c_double * 3), ("pe_flux", ctypes.c_double), ("pe_vth", ctypes.c_double),
        ("first_step", ctypes.c_int32),
        ("threads", ctypes.c_int32),
    ]


class _FieldObj(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("center", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("z_flat", ctypes.c_double),
                ("rim_radius", ctypes.c_double), ("depth", ctypes.c_double),
                ("eps_in", ctypes.c_double)]


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


class _Out(ctypes.Structure):
    _fields_ = [
        ("x", _dp), ("y", _dp), ("z", _dp), ("vx", _dp), ("vy", _dp), ("vz", _dp),
        ("fate", _i32p), ("where", _i32p), ("when", _i32p),
        ("rho", _dp), ("rho_fixed", _i64p), ("tally", _i64p), ("escaped", _i64p),
        ("cap", ctypes.c_int64), ("n_out", ctypes.c_int64), ("species", _i32p),
        ("injected", _i64p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int64, _i32p] + [_dp] * 9 + [
            ctypes.c_int32, ctypes.POINTER(_Out)]
        L.orc_weights_f64.argtypes = [_dp, _dp]
        L.orc_weights_f32.argtypes = [_fp, _fp]
        L.orc_gather_f64.argtypes = [ctypes.c_int32] * 3 + [_dp] * 3 + [_i32p, _dp, _dp]
        L.orc_fixed_contrib_f64.argtypes = [ctypes.c_double, _dp, _i64p]
        L.orc_fixed_contrib_f32.argtypes = [ctypes.c_float, _fp, _i64p]
        L.orc_splitmix_draw.restype = ctypes.c_uint64
        L.orc_splitmix_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_inj_uniform.restype = ctypes.c_double
        L.orc_inj_uniform.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_uint64]
        L.orc_ln.restype = ctypes.c_double
        L.orc_ln.argtypes = [ctypes.c_double]
        L.orc_normals3.argtypes = [ctypes.c_uint64, _dp]
        L.orc_field_solve.restype = ctypes.c_int
        L.orc_field_solve.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double, ctypes.c_double,
                                                             ctypes.c_int32, _dp, _dp, _dp,
                                                             ctypes.c_double, ctypes.c_int32,
                                                             ctypes.c_int32,
                                                             ctypes.POINTER(_FieldObj),
                                                             ctypes.c_int32, _i32p, _dp, _i32p]
        L.orc_field_vcycle.restype = ctypes.c_int
        L.orc_field_vcycle.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double, ctypes.c_double,
                                                              ctypes.c_int32,
                                                              ctypes.POINTER(_FieldObj),
                                                              ctypes.c_int32, _dp, _dp]
        L.orc_ife_basis.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_ife_element.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_cube_tets.argtypes = [ctypes.c_int32] * 3 + [_i32p]
        L.orc_ife_links.restype = ctypes.c_int
        L.orc_ife_links.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double, ctypes.c_double,
                                                           ctypes.POINTER(_FieldObj), _dp]
        L.orc_object_psi.restype = ctypes.c_double
        L.orc_object_psi.argtypes = [ctypes.POINTER(_FieldObj), ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double]
        L.orc_photo_column.restype = ctypes.c_int
        L.orc_photo_column.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int64, ctypes.c_int64, _dp]
        L.orc_photo_max_per_step.restype = ctypes.c_int64
        L.orc_photo_max_per_step.argtypes = [ctypes.POINTER(_Cfg)]
        L.orc_surface_rho.restype = ctypes.c_int
        L.orc_surface_rho.argtypes = [ctypes.POINTER(_Cfg), _i64p, _i64p]
        L.orc_field_E.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double, ctypes.c_int32, _dp,
                                                         _dp, _dp, _dp]
        L.orc_object_hit.restype = ctypes.c_int32
        L.orc_object_hit.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double]
        _lib = L
    return _lib


@dataclass
class Problem:
    """Mesh, species, object and numerics of one run (cell units when h = 1)."""
    nx: int
    ny: int
    nz: int
    dt: float
    q: list
    m: list
    w: list = None
    h: float = 1.0
    origin: tuple = (0.0, 0.0, 0.0)
    obj: str = "none"
    center: tuple = (0.0, 0.0, 0.0)
    radius: float = 0.0
    z_flat: float = 0.0
    rim_radius: float = 0.0
    depth: float = 0.0
    repr: str = "fp64"
    deposit: str = "fixed64"
    # global boundaries: face masks (bit f: face f = x-, x+, y-, y+, z-, z+)
    reflect: int = 0
    inj_faces: int = 0
    inj_seed: int = 0
    inj_density: list = None   # per species, particles per unit volume
    inj_vth: list = None
    inj_drift: list = None     # per species, 3 components
    sphere_patches: int = 0    # sphere: 0 one bin, m > 0 6 m^2 surface patches
    # photoemission from the crater terrain (pe_species -1: none)
    pe_species: int = -1
    pe_seed: int = 0
    pe_sun: tuple = (1.0, 0.0, 1.0)
    pe_flux: float = 0.0
    pe_vth: float = 0.0
    # index of the run's first step (the injection and photoemission draws are
    # keyed by the step index): a run continued from step k
    first_step: int = 0
    # OpenMP threads of the particle updates and the fixed-point deposit (the
    # results are bit-identical to one thread's)
    threads: int = 1

    @property
    def n_species(self):
        return len(self.q)

    @property
    def nodes(self):
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def nbins(self):
        if self.obj == "crater":
            return self.nx * self.ny
        if self.obj != "sphere":
            return 0  # nothing collects particles
        return 6 * self.sphere_patches ** 2 if self.sphere_patches else 1

    def cstruct(self) -> _Cfg:
        c = _Cfg()
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.h = self.h
        c.origin[:] = list(self.origin)
        c.dt = self.dt
        c.n_species = self.n_species
        w = self.w if self.w is not None else [1.0] * self.n_species
        for s in range(self.n_species):
            c.q[s], c.m[s], c.w[s] = self.q[s], self.m[s], w[s]
        c.obj_kind = OBJECT[self.obj]
        c.center[:] = list(self.center)
        c.radius = self.radius
        c.z_flat, c.rim_radius, c.depth = self.z_flat, self.rim_radius, self.depth
        c.repr = REPR[self.repr]
        c.deposit = DEPOSIT[self.deposit]
        c.reflect = int(self.reflect)
        c.inj_faces = int(self.inj_faces)
        c.inj_seed = int(self.inj_seed) & (2 ** 64 - 1)
        c.sphere_patches = int(self.sphere_patches)
        c.pe_species = int(self.pe_species)
        c.pe_seed = int(self.pe_seed) & (2 ** 64 - 1)
        c.pe_sun[:] = [float(a) for a in self.pe_sun]
        c.pe_flux = float(self.pe_flux)
        c.pe_vth = float(self.pe_vth)
        c.first_step = int(self.first_step)
        c.threads = int(self.threads)
        for s in range(self.n_species):
            c.inj_density[s] = self.inj_density[s] if self.inj_density else 0.0
            c.inj_vth[s] = self.inj_vth[s] if self.inj_vth else 0.0
            for d in range(3):
                c.inj_drift[3 * s + d] = self.inj_drift[s][d] if self.inj_drift else 0.0
        return c

    def injection_bound(self, nsteps: int) -> int:
        """Most particles that nsteps of injection and photoemission can add
        (each face cell gets at most floor(n L) + 1 ghosts per step and
        species, each lit column floor(mean) + 1 photoelectrons)."""
        photo = int(lib().orc_photo_max_per_step(ctypes.byref(self.cstruct()))) * int(nsteps)
        if not self.inj_faces:
            return photo
        n = (self.nx, self.ny, self.nz)
        tot = 0
        for s in range(self.n_species):
            dens = self.inj_density[s] if self.inj_density else 0.0
            if dens <= 0:
                continue
            ncell = dens * (self.h * self.h * self.h)
            vth = self.inj_vth[s] / self.h
            for f in range(6):
                if not (self.inj_faces >> f) & 1:
                    continue
                ax = f // 2
                un = (self.inj_drift[s][ax] / self.h) * (-1.0 if f & 1 else 1.0)
                L = min(1.0, self.dt * (max(0.0, un) + 6.0 * vth))
                cells = n[0] * n[1] * n[2] // n[ax]
                tot += cells * (int(ncell * L) + 1)
        return tot * int(nsteps) + photo


class OracleError(RuntimeError):
    pass


@dataclass
class Result:
    x: np.ndarray
    v: np.ndarray          # (n, 3)
    fate: np.ndarray       # 0 alive, 1 escaped, 2 absorbed
    where: np.ndarray
    when: np.ndarray
    rho: np.ndarray
    rho_fixed: np.ndarray  # None unless fixed-point mode
    tally: np.ndarray      # (nbins, n_species)
    escaped: np.ndarray    # (6, n_species)
    species: np.ndarray = None   # (n_out,) species of every particle (loaded, then injected)
    injected: np.ndarray = None  # (n_species,) particles injected
    extra: dict = field(default_factory=dict)

    def charge(self, prob: Problem) -> np.ndarray:
        """Collected charge per bin: sum over species of q*w*count, in FP64."""
        w = prob.w if prob.w is not None else [1.0] * prob.n_species
        chg = np.array([prob.q[s] * w[s] for s in range(prob.n_species)], dtype=np.float64)
        return self.tally.astype(np.float64) @ chg


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def run(prob: Problem, species, x, v, E, nsteps: int) -> Result:
    """Run the oracle. x, v: (n, 3) physical positions and half-step velocities;
    E: (3, nodes) node field, x fastest; species: (n,) int."""
    L = lib()
    n = len(species)
    sp = _c(species, np.int32)
    x = _c(x, np.float64).reshape(n, 3)
    v = _c(v, np.float64).reshape(n, 3)
    cols = [_c(x[:, d], np.float64) for d in range(3)] + [_c(v[:, d], np.float64) for d in range(3)]
    E = [_c(E[d], np.float64) for d in range(3)]
    for e in E:
        if e.size != prob.nodes:
            raise ValueError("node field has the wrong size")
    cap = n + prob.injection_bound(nsteps)
    ox = [np.empty(cap) for _ in range(6)]
    fate = np.empty(cap, np.int32)
    where = np.empty(cap, np.int32)
    when = np.empty(cap, np.int32)
    spo = np.empty(cap, np.int32)
    inj = np.zeros(prob.n_species, np.int64)
    rho = np.empty(prob.nodes)
    rho_fixed = np.empty(prob.nodes, np.int64) if prob.deposit == "fixed64" else None
    tally = np.zeros((prob.nbins, prob.n_species), np.int64)
    esc = np.zeros((6, prob.n_species), np.int64)
    out = _Out()
    for name, arr in zip(("x", "y", "z", "vx", "vy", "vz"), ox):
        setattr(out, name, arr.ctypes.data_as(_dp))
    out.fate = fate.ctypes.data_as(_i32p)
    out.where = where.ctypes.data_as(_i32p)
    out.when = when.ctypes.data_as(_i32p)
    out.rho = rho.ctypes.data_as(_dp)
    out.rho_fixed = rho_fixed.ctypes.data_as(_i64p) if rho_fixed is not None else None
    out.tally = tally.ctypes.data_as(_i64p)
    out.escaped = esc.ctypes.data_as(_i64p)
    out.cap = cap
    out.species = spo.ctypes.data_as(_i32p)
    out.injected = inj.ctypes.data_as(_i64p)
    cfg = prob.cstruct()
    rc = L.orc_run(ctypes.byref(cfg), n, sp.ctypes.data_as(_i32p),
                   *[c.ctypes.data_as(_dp) for c in cols], *[e.ctypes.data_as(_dp) for e in E],
                   int(nsteps), ctypes.byref(out))
    if rc != 0:
        raise OracleError(f"oracle returned {rc}")
    k = int(out.n_out)
    return Result(x=np.stack([a[:k] for a in ox[:3]], 1), v=np.stack([a[:k] for a in ox[3:]], 1),
                  fate=fate[:k], where=where[:k], when=when[:k], rho=rho, rho_fixed=rho_fixed,
                  tally=tally, escaped=esc, species=spo[:k], injected=inj)


def weights(f, dtype=np.float64) -> np.ndarray:
    L = lib()
    f = _c(f, dtype)
    W = np.empty(8, dtype)
    if dtype == np.float64:
        L.orc_weights_f64(f.ctypes.data_as(_dp), W.ctypes.data_as(_dp))
    else:
        L.orc_weights_f32(f.ctypes.data_as(_fp), W.ctypes.data_as(_fp))
    return W


def gather(nx, ny, nz, E, i, f) -> np.ndarray:
    L = lib()
    E = [_c(E[d], np.float64) for d in range(3)]
    ii = _c(i, np.int32)
    ff = _c(f, np.float64)
    out = np.empty(3)
    L.orc_gather_f64(nx, ny, nz, *[e.ctypes.data_as(_dp) for e in E], ii.ctypes.data_as(_i32p),
                     ff.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    return out


def fixed_contrib(chg, W, dtype=np.float64) -> np.ndarray:
    L = lib()
    W = _c(W, dtype)
    C = np.empty(8, np.int64)
    if dtype == np.float64:
        L.orc_fixed_contrib_f64(float(chg), W.ctypes.data_as(_dp), C.ctypes.data_as(_i64p))
    else:
        L.orc_fixed_contrib_f32(float(chg), W.ctypes.data_as(_fp), C.ctypes.data_as(_i64p))
    return C


def object_hit(prob: Problem, x, y, z) -> int:
    cfg = prob.cstruct()
    return int(lib().orc_object_hit(ctypes.byref(cfg), float(x), float(y), float(z)))


def splitmix_draw(key: int, d: int) -> int:
    """Raw 64-bit draw d of a key (the SplitMix64 output for state key + (d+1) gamma)."""
    return int(lib().orc_splitmix_draw(key & (2 ** 64 - 1), d))


def inj_uniform(seed, step, s, f, cell, j, d) -> float:
    return float(lib().orc_inj_uniform(seed & (2 ** 64 - 1), step, s, f, cell, j, d))


def ln(x: float) -> float:
    return float(lib().orc_ln(float(x)))


def normals3(key: int) -> np.ndarray:
    z = np.empty(3)
    lib().orc_normals3(key & (2 ** 64 - 1), z.ctypes.data_as(_dp))
    return z


PRECONDITIONERS = {"multigrid": 0, "jacobi": 1}


@dataclass
class FieldObject:
    """The object as an interface of the field problem, in the field mesh's
    cell units with node 0 at the origin; eps_in inside it."""
    kind: str                   # "sphere" or "crater"
    eps_in: float
    center: tuple = (0.0, 0.0, 0.0)
    radius: float = 0.0
    z_flat: float = 0.0
    rim_radius: float = 0.0
    depth: float = 0.0

    def cstruct(self) -> _FieldObj:
        o = _FieldObj()
        o.kind = OBJECT[self.kind]
        o.center[:] = list(self.center)
        o.radius, o.z_flat, o.rim_radius, o.depth = self.radius, self.z_flat, self.rim_radius, self.depth
        o.eps_in = self.eps_in
        return o


def field_object_of(prob: "Problem", eps_in: float) -> FieldObject:
    """The run's object in cell units."""
    c = tuple((prob.center[d] - prob.origin[d]) / prob.h for d in range(3))
    return FieldObject(kind=prob.obj, eps_in=eps_in, center=c, radius=prob.radius / prob.h,
                       z_flat=(prob.z_flat - prob.origin[2]) / prob.h,
                       rim_radius=prob.rim_radius / prob.h, depth=prob.depth / prob.h)


def object_psi(obj: FieldObject, x, y, z) -> float:
    o = obj.cstruct()
    return float(lib().orc_object_psi(ctypes.byref(o), float(x), float(y), float(z)))


def photo_column(prob: "Problem", i: int, j: int) -> dict:
    """The terrain of column (i, j) as the photoemission sees it."""
    out = np.zeros(7)
    cfg = prob.cstruct()
    if lib().orc_photo_column(ctypes.byref(cfg), int(i), int(j), out.ctypes.data_as(_dp)) != 0:
        raise OracleError("no photoemission in this problem")
    return dict(n=out[:3].copy(), ground=out[3], index=out[4], lit=bool(out[5]), mean=out[6])


def surface_rho(prob: "Problem", tally) -> np.ndarray:
    """Fixed-point nodal charge (int64 at 2^32) of the collected surface
    charge placed at the bins' surface points (see the oracle source)."""
    t = _c(tally, np.int64)
    if t.shape != (prob.nbins, prob.n_species):
        raise ValueError("tally has the wrong shape")
    out = np.zeros(prob.nodes, np.int64)
    cfg = prob.cstruct()
    rc = lib().orc_surface_rho(ctypes.byref(cfg), t.ctypes.data_as(_i64p), out.ctypes.data_as(_i64p))
    if rc != 0:
        raise OracleError(f"oracle returned {rc}")
    return out


OPERATORS = {"fv": 0, "ife": 1}


def field_solve(nx, ny, nz, rho, dirichlet, values=None, h=1.0, eps=1.0, phi0=None, tol=1e-10,
                max_iter=10000, precond="multigrid", info=None, obj: FieldObject = None,
                op="fv"):
    """Solves the field problem on the nodes (see the oracle source); returns
    (phi, iterations, relative residual). precond "multigrid" uses the V-cycle
    where the grid coarsens (else Jacobi); a dict passed as info gets the
    multigrid level count used ("levels", 0 for Jacobi); obj makes the object
    an interface with permittivity obj.eps_in inside; op: "fv" node-centred
    finite volumes, "ife" immersed finite elements on five tetrahedra per
    cell."""
    nodes = (nx + 1) * (ny + 1) * (nz + 1)
    rho = _c(rho, np.float64).ravel()
    if rho.size != nodes:
        raise ValueError("rho has the wrong size")
    phi = np.zeros(nodes) if phi0 is None else _c(phi0, np.float64).ravel().copy()
    g = _c(values if values is not None else np.zeros(6), np.float64)
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    lv = ctypes.c_int32(0)
    o = ctypes.byref(obj.cstruct()) if obj is not None else None
    rc = lib().orc_field_solve(nx, ny, nz, float(h), float(eps), int(dirichlet),
                               g.ctypes.data_as(_dp), rho.ctypes.data_as(_dp),
                               phi.ctypes.data_as(_dp), float(tol), int(max_iter),
                               PRECONDITIONERS[precond], o, OPERATORS[op], ctypes.byref(it),
                               ctypes.byref(rr), ctypes.byref(lv))
    if rc != 0:
        raise OracleError(f"oracle returned {rc}")
    if info is not None:
        info["levels"] = lv.value
    return phi, it.value, rr.value


def field_vcycle(nx, ny, nz, r, dirichlet, h=1.0, eps=1.0, obj: FieldObject = None, op="fv"):
    """One multigrid V-cycle z = B r (homogeneous Dirichlet faces); returns
    (z, levels), z None when the grid does not coarsen."""
    r = _c(r, np.float64).ravel()
    if r.size != (nx + 1) * (ny + 1) * (nz + 1):
        raise ValueError("r has the wrong size")
    z = np.zeros(r.size)
    o = ctypes.byref(obj.cstruct()) if obj is not None else None
    rc = lib().orc_field_vcycle(nx, ny, nz, float(h), float(eps), int(dirichlet), o,
                                OPERATORS[op], r.ctypes.data_as(_dp), z.ctypes.data_as(_dp))
    if rc < 0:
        raise OracleError(f"oracle returned {rc}")
    return (z if rc > 0 else None), rc


def ife_basis(X, psi, eps_in, eps) -> dict:
    """The IFE basis of one tetrahedron (vertices X (4, 3), level set psi (4,)):
    a (4, 3) grad phi- per basis function, t (4,), c (4, 4) with
    phi- = sum_j c[i, j] lambda_j, g = grad psi_h, vol, vin (inside volume), cut."""
    X = _c(X, np.float64).ravel()
    p = _c(psi, np.float64)
    out = np.zeros(38)
    lib().orc_ife_basis(X.ctypes.data_as(_dp), p.ctypes.data_as(_dp), float(eps_in), float(eps),
                        out.ctypes.data_as(_dp))
    return dict(a=out[:12].reshape(4, 3), t=out[12:16].copy(), c=out[16:32].reshape(4, 4),
                g=out[32:35].copy(), vol=out[35], vin=out[36],
                cut=bool(out[37]))


def ife_element(X, psi, eps_in, eps) -> np.ndarray:
    X = _c(X, np.float64).ravel()
    p = _c(psi, np.float64)
    K = np.zeros(16)
    lib().orc_ife_element(X.ctypes.data_as(_dp), p.ctypes.data_as(_dp), float(eps_in), float(eps),
                          K.ctypes.data_as(_dp))
    return K.reshape(4, 4)


def cube_tets(i, j, k) -> np.ndarray:
    """The five tetrahedra of cube (i, j, k): (5, 4, 3) corner offsets."""
    out = np.zeros(60, np.int32)
    lib().orc_cube_tets(int(i), int(j), int(k), out.ctypes.data_as(_i32p))
    return out.reshape(5, 4, 3)


# neighbour offsets of the IFE link table, in the oracle's order
IFE_LINKS = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1),
             (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 1, 0), (-1, 0, -1), (1, 0, -1),
             (-1, 0, 1), (1, 0, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1), (0, 1, 1)]


def ife_links(nx, ny, nz, h=1.0, eps=1.0, obj: FieldObject = None) -> np.ndarray:
    """The assembled IFE link coefficients (nodes, 18), c_pq = -A_pq."""
    nodes = (nx + 1) * (ny + 1) * (nz + 1)
    c = np.zeros(nodes * 18)
    o = ctypes.byref(obj.cstruct()) if obj is not None else None
    if lib().orc_ife_links(nx, ny, nz, float(h), float(eps), o, c.ctypes.data_as(_dp)) != 0:
        raise OracleError("invalid arguments")
    return c.reshape(nodes, 18)


def field_E(nx, ny, nz, phi, dirichlet, h=1.0) -> np.ndarray:
    """E = -grad phi at the nodes, (3, nodes)."""
    phi = _c(phi, np.float64).ravel()
    E = [np.empty(phi.size) for _ in range(3)]
    lib().orc_field_E(nx, ny, nz, float(h), int(dirichlet), phi.ctypes.data_as(_dp),
                      *[e.ctypes.data_as(_dp) for e in E])
    return np.stack(E)
