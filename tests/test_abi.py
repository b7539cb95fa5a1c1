"""The C-ABI library on the host: it loads, exports every declared entry point,
and validates configurations before touching a device (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2011_10214_amd as pam
from paper_2011_10214_amd import pic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declarations_are_exported_and_bound():
    decl = declared_functions()
    assert len(decl) >= 17
    out = subprocess.run(["nm", "-D", "--defined-only", pam.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pic_\w+)", out))
    missing = [f for f in decl if f not in exported]
    assert not missing, missing
    assert sorted(pam.SIGNATURES) == decl
    L = pam.lib()
    for f in decl:
        assert getattr(L, f) is not None


def test_status_strings():
    L = pam.lib()
    assert L.pic_status_string(0) == b"PIC_OK"
    assert L.pic_status_string(-5) == b"PIC_E_RANGE"
    assert L.pic_status_string(7) == b"unknown pic_status"


def _cfg(**kw):
    base = dict(nx=8, ny=8, nz=8, dt=0.05, species=[(-1.0, 1.0, 1.0), (1.0, 100.0, 1.0)],
                capacity=[1000, 1000], obj="sphere", center=(4.0, 4.0, 4.0), radius=1.0)
    base.update(kw)
    return pam.Config(**base)


def _create(cfg):
    h = ctypes.c_void_p()
    st = pam.lib().pic_create(ctypes.byref(cfg.cstruct()), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(nz=1024), dict(dt=0.0), dict(dt=float("nan")), dict(h=-1.0),
    dict(species=[]), dict(species=[(1.0, 0.0, 1.0)], capacity=[1]),
    dict(species=[(4e6, 1.0, 1.0)], capacity=[1]), dict(capacity=[-1, 5]),
    dict(capacity=[2 ** 31, 5]), dict(repr="fp32_cell", radius=0.0),
    dict(obj="crater", rim_radius=10.0, depth=0.0), dict(sort_interval=-1),
    dict(patches=-1), dict(patches=65),
    dict(obj="crater", rim_radius=2.0, depth=1.0, z_flat=3.0, patches=2),
])
def test_invalid_config_is_rejected_before_any_device_call(bad):
    st, h = _create(_cfg(**bad))
    assert st == pic.E_INVALID
    assert not h.value
    assert pam.lib().pic_last_error(None) not in (b"", b"no error")


def test_invalid_enum_values_are_rejected():
    c = _cfg().cstruct()
    c.repr = 7
    h = ctypes.c_void_p()
    assert pam.lib().pic_create(ctypes.byref(c), ctypes.byref(h)) == pic.E_INVALID
    c = _cfg().cstruct()
    c.deposit = -2
    assert pam.lib().pic_create(ctypes.byref(c), ctypes.byref(h)) == pic.E_INVALID
    assert pam.lib().pic_create(None, ctypes.byref(h)) == pic.E_INVALID
    assert pam.lib().pic_create(ctypes.byref(c), None) == pic.E_INVALID


def test_budget_override_gives_nomem(monkeypatch):
    monkeypatch.setenv("PIC_HBM_BUDGET_BYTES", "4096")
    st, h = _create(_cfg())
    assert st == pic.E_NOMEM and not h.value
    assert b"PIC_HBM_BUDGET_BYTES" in pam.lib().pic_last_error(None)


def test_null_context_calls_are_invalid():
    L = pam.lib()
    assert L.pic_step(None, 1) == pic.E_INVALID
    assert L.pic_get_rho(None, None, None) == pic.E_INVALID
    assert L.pic_synchronize(None) == pic.E_INVALID
    assert L.pic_num_bins(None) == 0
    L.pic_destroy(None)


def test_no_device_is_reported(monkeypatch):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _create(_cfg())
    assert st == pic.E_DEVICE and not h.value


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(pic, "_lib", None)
    monkeypatch.setattr(pic, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        pic.lib()


def test_binding_shares_one_hip_runtime_with_torch():
    # the binding loaded first, torch second: one HIP runtime in the process
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2011_10214_amd import pic\n"
        "pic.lib()\n"
        "import torch\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "libs = {l.split()[-1] for l in maps if 'libamdhip64' in l}\n"
        "print(len(libs))\n" % ROOT)
    out = subprocess.run([os.sys.executable, "-c", code], capture_output=True, text=True,
                         check=True, timeout=300).stdout.strip().splitlines()[-1]
    assert out == "1"


def test_allocator_hooks_must_come_together():
    c = _cfg().cstruct()
    c.alloc = pic.ALLOC_FN(lambda n, u: None)
    h = ctypes.c_void_p()
    assert pam.lib().pic_create(ctypes.byref(c), ctypes.byref(h)) == pic.E_INVALID
    assert b"together" in pam.lib().pic_last_error(None)


class _FakeDev:
    """Stands in for a CUDA tensor on a host without a GPU: the binding's
    checks of device arguments run before anything reads the pointer."""

    def __init__(self, n, dtype, contiguous=True):
        import torch

        self.is_cuda = True
        self.dtype = dtype
        self._n = n
        self._contig = contiguous
        self.device = torch.device("cuda", 0)
        self.shape = (n,)

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._contig

    def contiguous(self):
        return self

    def data_ptr(self):
        raise AssertionError("the pointer must not be taken")


class _NoCtx(pam.Context):
    """A Context shell without a library context (argument checks only)."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.ns = len(cfg.species)
        self._h = None


@pytest.mark.parametrize("case", ["five_columns", "float64", "short", "non_contiguous",
                                  "ids_int32", "ids_short", "host_tensor"])
def test_device_columns_are_checked_before_the_call(case):
    import torch

    f32 = torch.float32
    cols = [_FakeDev(10, f32) for _ in range(6)]
    ids = None
    if case == "five_columns":
        cols = cols[:5]
    elif case == "float64":
        cols[3] = _FakeDev(10, torch.float64)
    elif case == "short":
        cols[5] = _FakeDev(9, f32)
    elif case == "non_contiguous":
        cols[1] = _FakeDev(10, f32, contiguous=False)
    elif case == "ids_int32":
        ids = _FakeDev(10, torch.int32)
    elif case == "ids_short":
        ids = _FakeDev(11, torch.int64)
    elif case == "host_tensor":
        cols[0] = torch.zeros(10, dtype=f32)
    ctx = _NoCtx(_cfg())
    with pytest.raises(ValueError):
        ctx.load_particles_cols(0, cols, ids)


@pytest.mark.parametrize("case", ["two_components", "short", "float64"])
def test_device_field_is_checked_before_the_call(case):
    import torch

    cfg = _cfg()
    E = [_FakeDev(cfg.nodes, torch.float32) for _ in range(3)]
    if case == "two_components":
        E = E[:2]
    elif case == "short":
        E[2] = _FakeDev(cfg.nodes - 1, torch.float32)
    else:
        E[0] = _FakeDev(cfg.nodes, torch.float64)
    with pytest.raises(ValueError):
        _NoCtx(cfg).set_node_E(E)
