"""ctypes binding of the C-ABI declared in ``include/pic.h``.

Argument marshalling only: every step of the particle-mesh path runs in the
HIP library ``libpic.so``. There is no CPU fallback; if the library is missing
the import fails loudly. PyTorch tensors (device memory) are accepted where the
C-ABI takes device pointers, and a torch stream can be passed as the context's
stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

MAX_SPECIES = 4
OK, E_INVALID, E_NOMEM, E_DEVICE, E_STATE, E_RANGE = 0, -1, -2, -3, -4, -5
REPR = {"fp64": 0, "fp32_abs": 1, "fp32_cell": 2}
DEPOSIT = {"fixed64": 0, "fp32": 1, "fp64": 2}
OBJECT = {"none": 0, "sphere": 1, "crater": 2}


class _Species(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("m", ctypes.c_double), ("weight", ctypes.c_double)]


class _Object(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("center", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("z_flat", ctypes.c_double),
                ("rim_radius", ctypes.c_double), ("depth", ctypes.c_double),
                ("patches", ctypes.c_int32)]


# pic_config.alloc / dealloc
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
DEALLOC_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double), ("origin", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("n_species", ctypes.c_int32), ("species", _Species * MAX_SPECIES),
                ("object", _Object), ("repr", ctypes.c_int32), ("deposit", ctypes.c_int32),
                ("sort_interval", ctypes.c_int32), ("reflect", ctypes.c_int32),
                ("capacity", ctypes.c_int64 * MAX_SPECIES), ("stream", ctypes.c_void_p),
                ("alloc", ALLOC_FN), ("dealloc", DEALLOC_FN), ("alloc_user", ctypes.c_void_p)]


class _Field(ctypes.Structure):
    _fields_ = [("dirichlet", ctypes.c_int32), ("value", ctypes.c_double * 6),
                ("eps", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("preconditioner", ctypes.c_int32), ("eps_object", ctypes.c_double),
                ("surface_charge", ctypes.c_int32), ("op", ctypes.c_int32)]


PRECONDITIONERS = {"multigrid": 0, "jacobi": 1}
FIELD_OPS = {"fv": 0, "ife": 1}


class _Injection(ctypes.Structure):
    _fields_ = [("faces", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("density", ctypes.c_double * MAX_SPECIES), ("vth", ctypes.c_double * MAX_SPECIES),
                ("drift", ctypes.c_double * (3 * MAX_SPECIES))]


class _Photo(ctypes.Structure):
    _fields_ = [("species", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("sun", ctypes.c_double * 3), ("flux", ctypes.c_double), ("vth", ctypes.c_double)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("repr", ctypes.c_int32),
                ("deposit", ctypes.c_int32), ("steps_per_run", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64),
                ("particle_steps_per_run", ctypes.c_int64), ("stream", ctypes.c_void_p)]


class _Profile(ctypes.Structure):
    _fields_ = [("step_launches", ctypes.c_int64), ("step_ms", ctypes.c_double),
                ("sort_launches", ctypes.c_int64), ("sort_ms", ctypes.c_double),
                ("clear_launches", ctypes.c_int64), ("clear_ms", ctypes.c_double),
                ("particle_steps", ctypes.c_int64), ("inject_launches", ctypes.c_int64),
                ("inject_ms", ctypes.c_double), ("field_solves", ctypes.c_int64),
                ("field_ms", ctypes.c_double), ("field_iterations", ctypes.c_int64),
                ("photo_launches", ctypes.c_int64), ("photo_ms", ctypes.c_double)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_st = ctypes.c_int

# name -> (restype, argtypes); one entry per declaration of include/pic.h
SIGNATURES = {
    "pic_create": (_st, [ctypes.POINTER(_Config), ctypes.POINTER(_vp)]),
    "pic_destroy": (None, [_vp]),
    "pic_load_particles": (_st, [_vp, _i32, _i64] + [_vp] * 7),
    "pic_load_particles_f32_dev": (_st, [_vp, _i32, _i64] + [_vp] * 7),
    "pic_set_node_E": (_st, [_vp, _vp, _vp, _vp]),
    "pic_set_node_E_f32_dev": (_st, [_vp, _vp, _vp, _vp]),
    "pic_step": (_st, [_vp, _i32]),
    "pic_set_injection": (_st, [_vp, ctypes.POINTER(_Injection)]),
    "pic_solve_field": (_st, [_vp, ctypes.POINTER(_Field), ctypes.POINTER(_i32),
                              ctypes.POINTER(ctypes.c_double)]),
    "pic_get_phi": (_st, [_vp, _vp]),
    "pic_get_field_levels": (_st, [_vp, ctypes.POINTER(_i32)]),
    "pic_get_node_E": (_st, [_vp, _vp, _vp, _vp]),
    "pic_get_injected": (_st, [_vp, _vp]),
    "pic_set_step_index": (_st, [_vp, _i64]),
    "pic_set_photoemission": (_st, [_vp, ctypes.POINTER(_Photo)]),
    "pic_synchronize": (_st, [_vp]),
    "pic_get_rho": (_st, [_vp, _vp, _vp]),
    "pic_num_bins": (_i64, [_vp]),
    "pic_get_surface_charge": (_st, [_vp, _i64, _vp, _vp]),
    "pic_get_counters": (_st, [_vp, _vp, _vp, _vp]),
    "pic_get_particles": (_st, [_vp, _i32, _i64, _vp] + [_vp] * 7),
    "pic_get_particles_by_id": (_st, [_vp, _i32, _i64, _vp, _vp] + [_vp] * 6),
    "pic_get_particles_by_id_noalloc": (_st, [_vp, _i32, _i64, _vp, _vp] + [_vp] * 6),
    "pic_profile_enable": (_st, [_vp, _i32]),
    "pic_profile_read": (_st, [_vp, ctypes.POINTER(_Profile)]),
    "pic_last_error": (ctypes.c_char_p, [_vp]),
    "pic_status_string": (ctypes.c_char_p, [_st]),
    "pic_footprint_bytes": (_i64, [ctypes.POINTER(_Config)]),
    "pic_batch_create": (_st, [ctypes.POINTER(_BatchConfig), ctypes.POINTER(_vp)]),
    "pic_batch_destroy": (None, [_vp]),
    "pic_batch_attach": (_st, [_vp, _vp, _i64, ctypes.POINTER(_i32)]),
    "pic_batch_run": (_st, [_vp, ctypes.POINTER(_i32), _vp]),
    "pic_batch_launch": (_st, [_vp]),
    "pic_batch_set_weight": (_st, [_vp, _i32, ctypes.c_double]),
    "pic_batch_wait": (_st, [_vp, ctypes.POINTER(_i32), _vp]),
    "pic_batch_detach": (_st, [_vp, _i32]),
    "pic_batch_used_bytes": (_i64, [_vp]),
    "pic_batch_remaining": (_i64, [_vp, _i32]),
    "pic_batch_last_error": (ctypes.c_char_p, [_vp]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no CPU fallback)")
        # PyTorch ships its own HIP runtime under the same soname as the
        # system's. Loading torch first makes the library bind to that one
        # runtime; loading the library first would bring in a second HIP/HSA
        # runtime, after which torch finds no GPU (and device pointers and
        # streams could not be shared).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class PicError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{lib().pic_status_string(status).decode()}: {message}")
        self.status = status


@dataclass
class Config:
    """Mirror of ``pic_config``."""
    nx: int
    ny: int
    nz: int
    dt: float
    species: list                       # [(q, m, weight), ...]
    capacity: list                      # max particles per species
    h: float = 1.0
    origin: tuple = (0.0, 0.0, 0.0)
    obj: str = "none"
    center: tuple = (0.0, 0.0, 0.0)
    radius: float = 0.0
    z_flat: float = 0.0
    rim_radius: float = 0.0
    depth: float = 0.0
    patches: int = 0                    # sphere: 0 one tally bin, m > 0 6 m^2 surface patches
    repr: str = "fp32_cell"
    deposit: str = "fixed64"
    sort_interval: int = 0
    reflect: int = 0                    # bit f: box face f (x-, x+, y-, y+, z-, z+) reflects
    stream: int = 0                     # hipStream_t handle (e.g. torch stream.cuda_stream)
    # device memory of the context: None -> hipMalloc; "torch" -> torch's caching
    # allocator; or an object with alloc(nbytes) -> int pointer (0 if it cannot)
    # and free(ptr)
    allocator: object = None

    @property
    def nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    def cstruct(self) -> _Config:
        c = _Config()
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.h = self.h
        c.origin[:] = list(self.origin)
        c.dt = self.dt
        c.n_species = len(self.species)
        for s, (q, m, w) in enumerate(self.species):
            c.species[s].q, c.species[s].m, c.species[s].weight = q, m, w
        c.object.kind = OBJECT[self.obj]
        c.object.center[:] = list(self.center)
        c.object.radius = self.radius
        c.object.z_flat, c.object.rim_radius, c.object.depth = (self.z_flat, self.rim_radius,
                                                                self.depth)
        c.object.patches = int(self.patches)
        c.repr = REPR[self.repr]
        c.deposit = DEPOSIT[self.deposit]
        c.reflect = int(self.reflect)
        c.sort_interval = self.sort_interval
        for s in range(len(self.species)):
            c.capacity[s] = int(self.capacity[s])
        c.stream = self.stream or None
        return c


class TorchAllocator:
    """Device memory from torch's caching allocator, on the context's stream
    (or torch's current stream), so that a context's buffers come out of the
    same pool as the framework's tensors."""

    def __init__(self, stream: int = 0):
        self.stream = stream or None

    def alloc(self, nbytes: int) -> int:
        import torch

        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), stream=self.stream))
        except (RuntimeError, MemoryError):  # torch raises when it is out of memory
            return 0

    def free(self, ptr: int):
        import torch

        torch.cuda.caching_allocator_delete(int(ptr))


def _hooks(allocator):
    """ctypes callbacks for pic_config.alloc / dealloc around an allocator
    object (kept alive by the caller for the context's lifetime)."""
    def alloc(nbytes, _user):
        try:
            p = int(allocator.alloc(int(nbytes)))
        except Exception:  # an exception must not cross into the library
            return None
        return p or None

    def dealloc(ptr, _user):
        try:
            allocator.free(int(ptr))
        except Exception:
            pass
    return ALLOC_FN(alloc), DEALLOC_FN(dealloc)


def _ptr(a):
    """Data pointer of a numpy array or a torch tensor (None passes NULL)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _is_device(a) -> bool:
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


def _check_dev(tensors, dtype, n, what):
    """Device tensors handed to the library as raw pointers: each must be a
    contiguous tensor of the expected dtype and length on the current GPU
    (the library reads exactly n elements from its data pointer)."""
    import torch

    for k, t in enumerate(tensors):
        _check_shape(t, dtype, n, f"{what} {k}")
    dev = torch.cuda.current_device()
    for k, t in enumerate(tensors):
        if t.device.index != dev:
            raise ValueError(f"{what} {k}: the tensor is on device {t.device.index}, "
                             f"not the current device {dev}")


def _check_shape(t, dtype, n, what):
    if not (hasattr(t, "is_cuda") and t.is_cuda):
        raise ValueError(f"{what}: a CUDA tensor is required")
    if t.dtype != dtype:
        raise ValueError(f"{what}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: the tensor must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{what}: {t.numel()} elements, expected {n}")


def _device_sync():
    """Device arrays handed to the library may still be in flight on torch's
    current stream: wait for that stream (not the whole device, so that work of
    other contexts keeps running)."""
    import torch

    torch.cuda.current_stream().synchronize()


@dataclass
class Profile:
    step_launches: int
    step_ms: float
    sort_launches: int
    sort_ms: float
    clear_launches: int
    clear_ms: float
    particle_steps: int
    inject_launches: int = 0
    inject_ms: float = 0.0
    field_solves: int = 0
    field_ms: float = 0.0
    field_iterations: int = 0
    photo_launches: int = 0
    photo_ms: float = 0.0


class Context:
    """One ``pic_ctx``: the particle-mesh state of one subdomain on one GPU."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self._c = cfg.cstruct()
        self._hooks = None
        if cfg.allocator is not None:
            a = TorchAllocator(cfg.stream) if cfg.allocator == "torch" else cfg.allocator
            # the callbacks live as long as the context: the library calls
            # dealloc from pic_destroy
            self._allocator = a
            self._hooks = _hooks(a)
            self._c.alloc, self._c.dealloc = self._hooks
        h = _vp()
        st = lib().pic_create(ctypes.byref(self._c), ctypes.byref(h))
        if st != OK:
            raise PicError(st, lib().pic_last_error(None).decode())
        self._h = h
        self.ns = len(cfg.species)

    # -- plumbing
    def _check(self, st):
        if st != OK:
            raise PicError(st, lib().pic_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().pic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls
    def load_particles(self, species: int, x, v, ids=None):
        """x, v: (n, 3) positions and half-step velocities. numpy (host, FP64)
        or float32 CUDA tensors (device) -- see pic_load_particles(_f32_dev)."""
        if _is_device(x):
            if x.dim() != 2 or x.shape[1] != 3 or tuple(v.shape) != tuple(x.shape):
                raise ValueError("x and v must be (n, 3) tensors of the same shape")
            cols = [x[:, d].contiguous() for d in range(3)] + [v[:, d].contiguous() for d in range(3)]
            idt = ids.contiguous() if ids is not None else None
            self.load_particles_cols(species, cols, idt)
            return
        x = _host(x, np.float64).reshape(-1, 3)
        v = _host(v, np.float64).reshape(-1, 3)
        cols = [_host(x[:, d], np.float64) for d in range(3)] + [_host(v[:, d], np.float64)
                                                                 for d in range(3)]
        idh = _host(ids, np.int64) if ids is not None else None
        self._check(lib().pic_load_particles(self._h, species, x.shape[0],
                                             *[_ptr(c) for c in cols], _ptr(idh)))

    def load_particles_cols(self, species: int, cols, ids=None):
        """cols: six float32 device tensors (x, y, z, vx, vy, vz) of equal length;
        ids: None or an int64 device tensor of that length."""
        import torch

        if len(cols) != 6:
            raise ValueError(f"{len(cols)} columns given, expected 6 (x, y, z, vx, vy, vz)")
        n = int(cols[0].numel())
        if ids is not None:
            _check_shape(ids, torch.int64, n, "ids")
        _check_dev(cols, torch.float32, n, "column")
        if ids is not None:
            _check_dev([ids], torch.int64, n, "ids")
        _device_sync()
        self._check(lib().pic_load_particles_f32_dev(self._h, species, n,
                                                     *[_ptr(c) for c in cols], _ptr(ids)))

    def set_node_E(self, E):
        """E: three arrays of (nx+1)(ny+1)(nz+1) values, x fastest: numpy (host,
        FP64) or float32 CUDA tensors."""
        if len(E) != 3:
            raise ValueError("three field components are required")
        if _is_device(E[0]):
            import torch

            Es = [e.contiguous() for e in E]
            _check_dev(Es, torch.float32, self.cfg.nodes, "E component")
            _device_sync()
            self._check(lib().pic_set_node_E_f32_dev(self._h, *[_ptr(e) for e in Es]))
            return
        Es = [_host(e, np.float64) for e in E]
        for e in Es:
            if e.size != self.cfg.nodes:
                raise ValueError("node field has the wrong size")
        self._check(lib().pic_set_node_E(self._h, *[_ptr(e) for e in Es]))

    def step(self, nsteps: int):
        self._check(lib().pic_step(self._h, int(nsteps)))

    def set_step_index(self, step: int):
        """Index of the next step (keys the injection and photoemission draws):
        a run resumed from an export after k steps continues at k."""
        self._check(lib().pic_set_step_index(self._h, int(step)))

    def set_injection(self, faces: int, seed: int = 0, density=None, vth=None, drift=None):
        """Ambient particles injected through the faces in the bit mask each
        step (``faces`` = 0 turns it off); per species density, thermal speed
        and drift (3 components), physical units."""
        if not faces:
            self._check(lib().pic_set_injection(self._h, None))
            return
        c = _Injection()
        c.faces = int(faces)
        c.seed = int(seed) & (2 ** 64 - 1)
        for s in range(self.ns):
            c.density[s] = float(density[s]) if density is not None else 0.0
            c.vth[s] = float(vth[s]) if vth is not None else 0.0
            for d in range(3):
                c.drift[3 * s + d] = float(drift[s][d]) if drift is not None else 0.0
        self._check(lib().pic_set_injection(self._h, ctypes.byref(c)))

    def set_photoemission(self, species: int = None, seed: int = 0, sun=(1.0, 0.0, 1.0),
                          flux: float = 0.0, vth: float = 0.0):
        """Photoemission of the species from the sunlit crater terrain each step
        (``species`` None turns it off); sun: direction towards the Sun; flux:
        emitted physical particles per unit area and time at normal incidence;
        vth: thermal speed of the emitted half-Maxwellian."""
        if species is None:
            self._check(lib().pic_set_photoemission(self._h, None))
            return
        c = _Photo()
        c.species = int(species)
        c.seed = int(seed) & (2 ** 64 - 1)
        c.sun[:] = [float(a) for a in sun]
        c.flux = float(flux)
        c.vth = float(vth)
        self._check(lib().pic_set_photoemission(self._h, ctypes.byref(c)))

    def solve_field(self, dirichlet: int, values=None, eps: float = 1.0, tol: float = 1e-6,
                    max_iter: int = 150, precond: str = "multigrid", eps_object: float = 0.0,
                    surface_charge: bool = False, op: str = "fv"):
        """Field solve for the last deposit (pic_solve_field); the node field
        becomes -grad phi. eps_object > 0 makes the object an interface with
        that permittivity inside; surface_charge adds the collected charge as
        its surface source; op "fv" (node-centred finite volumes) or "ife"
        (immersed finite elements). Returns (iterations, relative residual)."""
        if op not in FIELD_OPS:
            raise ValueError(f"op must be one of {sorted(FIELD_OPS)}")
        f = _Field()
        f.op = FIELD_OPS[op]
        f.dirichlet = int(dirichlet)
        f.preconditioner = PRECONDITIONERS[precond]
        f.eps_object = float(eps_object)
        f.surface_charge = 1 if surface_charge else 0
        for k in range(6):
            f.value[k] = float(values[k]) if values is not None else 0.0
        f.eps, f.tol, f.max_iter = float(eps), float(tol), int(max_iter)
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        self._check(lib().pic_solve_field(self._h, ctypes.byref(f), ctypes.byref(it),
                                          ctypes.byref(rr)))
        return it.value, rr.value

    def get_node_E(self) -> np.ndarray:
        E = [np.empty(self.cfg.nodes) for _ in range(3)]
        self._check(lib().pic_get_node_E(self._h, *[_ptr(e) for e in E]))
        return np.stack(E)

    def get_field_levels(self) -> int:
        """Multigrid levels of the last field solve (0: Jacobi ran)."""
        n = _i32(0)
        self._check(lib().pic_get_field_levels(self._h, ctypes.byref(n)))
        return n.value

    def get_phi(self) -> np.ndarray:
        phi = np.empty(self.cfg.nodes)
        self._check(lib().pic_get_phi(self._h, _ptr(phi)))
        return phi

    def get_injected(self) -> np.ndarray:
        out = np.zeros(self.ns, np.int64)
        self._check(lib().pic_get_injected(self._h, _ptr(out)))
        return out

    def synchronize(self):
        self._check(lib().pic_synchronize(self._h))

    def get_rho(self):
        rho = np.empty(self.cfg.nodes)
        fixed = np.empty(self.cfg.nodes, np.int64) if self.cfg.deposit == "fixed64" else None
        self._check(lib().pic_get_rho(self._h, _ptr(rho), _ptr(fixed)))
        return rho, fixed

    @property
    def nbins(self) -> int:
        return int(lib().pic_num_bins(self._h))

    def get_surface_charge(self):
        nb = self.nbins
        charge = np.empty(nb)
        counts = np.empty((nb, self.ns), np.int64)
        self._check(lib().pic_get_surface_charge(self._h, nb, _ptr(charge) if nb else None,
                                                 _ptr(counts) if nb else None))
        return charge, counts

    def get_counters(self):
        alive = np.empty(self.ns, np.int64)
        absorbed = np.empty(self.ns, np.int64)
        escaped = np.empty((6, self.ns), np.int64)
        self._check(lib().pic_get_counters(self._h, _ptr(alive), _ptr(absorbed), _ptr(escaped)))
        return alive, absorbed, escaped

    def get_particles(self, species: int, with_ids: bool = True):
        n_out = ctypes.c_int64(0)
        alive, _, _ = self.get_counters()
        cap = int(alive[species])
        for _ in range(2):
            cols = [np.empty(cap) for _ in range(6)]
            ids = np.empty(cap, np.int64) if with_ids else None
            st = lib().pic_get_particles(self._h, species, cap, ctypes.byref(n_out),
                                         *[_ptr(c) for c in cols], _ptr(ids))
            if st == E_INVALID and n_out.value > cap:
                cap = n_out.value
                continue
            self._check(st)
            n = n_out.value
            x = np.stack([c[:n] for c in cols[:3]], 1)
            v = np.stack([c[:n] for c in cols[3:]], 1)
            return x, v, (ids[:n] if ids is not None else None)
        raise PicError(E_INVALID, "particle count changed during read-back")

    def get_particles_by_id(self, species: int, ids):
        """State of the particles with the given ids (any order). Returns
        (found (n,) bool, x (n, 3), v (n, 3)) in the order of `ids`."""
        ids = np.asarray(ids, dtype=np.int64)
        order = np.argsort(ids, kind="stable")
        srt = np.ascontiguousarray(ids[order])
        n = len(srt)
        found = np.zeros(n, np.int32)
        cols = [np.full(n, np.nan) for _ in range(6)]
        self._check(lib().pic_get_particles_by_id(self._h, species, n, _ptr(srt), _ptr(found),
                                                  *[_ptr(c) for c in cols]))
        inv = np.empty(n, np.int64)
        inv[order] = np.arange(n)
        x = np.stack(cols[:3], 1)[inv]
        v = np.stack(cols[3:], 1)[inv]
        return found[inv].astype(bool), x, v

    def profile_enable(self, on: bool = True):
        self._check(lib().pic_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> Profile:
        p = _Profile()
        self._check(lib().pic_profile_read(self._h, ctypes.byref(p)))
        return Profile(p.step_launches, p.step_ms, p.sort_launches, p.sort_ms, p.clear_launches,
                       p.clear_ms, p.particle_steps, p.inject_launches, p.inject_ms,
                       p.field_solves, p.field_ms, p.field_iterations, p.photo_launches,
                       p.photo_ms)


def footprint_bytes(cfg: Config) -> int:
    """Device bytes pic_create allocates for cfg (without ids)."""
    v = lib().pic_footprint_bytes(ctypes.byref(cfg.cstruct()))
    if v < 0:
        raise PicError(E_INVALID, "invalid configuration")
    return int(v)


class Batch:
    """A ``pic_batch``: contexts advanced together by captured batched steps.
    ``particle_steps_per_run`` > 0 gives every context an equal share of that
    many particle-steps per run (between 1 and ``steps_per_run`` steps)."""

    def __init__(self, max_slots: int, repr: str, deposit: str, steps_per_run: int,
                 hbm_budget_bytes: int, stream: int = 0, particle_steps_per_run: int = 0):
        c = _BatchConfig()
        c.max_slots, c.repr, c.deposit = max_slots, REPR[repr], DEPOSIT[deposit]
        c.steps_per_run, c.hbm_budget_bytes = steps_per_run, int(hbm_budget_bytes)
        c.particle_steps_per_run = int(particle_steps_per_run)
        c.stream = stream or None
        h = _vp()
        st = lib().pic_batch_create(ctypes.byref(c), ctypes.byref(h))
        if st != OK:
            raise PicError(st, lib().pic_batch_last_error(None).decode())
        self._h = h
        self.max_slots = max_slots
        self.budget = int(hbm_budget_bytes)

    def _check(self, st):
        if st != OK:
            raise PicError(st, lib().pic_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().pic_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def used_bytes(self) -> int:
        return int(lib().pic_batch_used_bytes(self._h))

    def remaining(self, slot: int) -> int:
        """Steps the context in `slot` has left (-1: empty slot)."""
        return int(lib().pic_batch_remaining(self._h, slot))

    def attach(self, ctx: "Context", nsteps: int) -> int:
        slot = ctypes.c_int32(-1)
        self._check(lib().pic_batch_attach(self._h, ctx._h, int(nsteps), ctypes.byref(slot)))
        return slot.value

    def run(self) -> list:
        n = ctypes.c_int32(0)
        done = (ctypes.c_int32 * self.max_slots)()
        self._check(lib().pic_batch_run(self._h, ctypes.byref(n), done))
        return [done[i] for i in range(n.value)]

    def launch(self):
        """Enqueues a run and returns at once (attach may be called meanwhile)."""
        self._check(lib().pic_batch_launch(self._h))

    def wait(self) -> list:
        """Waits for the run in flight; returns the slots that finished."""
        n = ctypes.c_int32(0)
        done = (ctypes.c_int32 * self.max_slots)()
        self._check(lib().pic_batch_wait(self._h, ctypes.byref(n), done))
        return [done[i] for i in range(n.value)]

    def detach(self, slot: int):
        self._check(lib().pic_batch_detach(self._h, int(slot)))

    def set_weight(self, slot: int, weight: float):
        """Share weight of an attached context (default 1)."""
        self._check(lib().pic_batch_set_weight(self._h, int(slot), float(weight)))


def config_from_workload(w, repr="fp32_cell", deposit="fixed64", sort_interval=0, capacity=None,
                         stream=0) -> Config:
    """Config of a synthetic workload description (duck-typed: needs the mesh,
    object, species q/m/w and dt attributes)."""
    cap = capacity if capacity is not None else [s.count for s in w.species]
    return Config(nx=w.nx, ny=w.ny, nz=w.nz, dt=w.dt, h=w.h, origin=w.origin,
                  species=[(s.q, s.m, s.w) for s in w.species], capacity=cap, obj=w.obj,
                  center=w.center, radius=w.radius, z_flat=w.z_flat, rim_radius=w.rim_radius,
                  depth=w.depth, repr=repr, deposit=deposit, sort_interval=sort_interval,
                  stream=stream)
