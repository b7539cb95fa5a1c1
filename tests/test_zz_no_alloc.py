"""pic_get_particles_by_id_noalloc, the id lookup for callers that cannot
allocate: through the C-ABI it returns what pic_get_particles_by_id returns,
bit for bit (found flags, positions, velocities, and the caller's entries of
ids that are not found left as they were), on two calls in a row, the second
with fewer ids than the first (the shared scratch keeps the first call's
contents), from two contexts on the same GPU; it refuses more than
PIC_NOALLOC_MAX_IDS ids, and it allocates no device memory (a counting
allocator sees no call)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2011_10214_amd as pam
import synth

from gpu_util import inputs

pytestmark = pytest.mark.gpu

MAX_IDS = 65536


class Counting:
    def __init__(self):
        self.calls = 0

    def alloc(self, nbytes):
        self.calls += 1
        return torch.cuda.caching_allocator_alloc(nbytes)

    def free(self, ptr):
        torch.cuda.caching_allocator_delete(ptr)


def context(w, form, allocator=None):
    sp, x, v, E = inputs(w)
    cfg = pam.config_from_workload(w, repr=form, deposit="fixed64")
    cfg.allocator = allocator
    ctx = pam.Context(cfg)
    ids = np.arange(len(sp), dtype=np.int64)
    for s in range(len(w.species)):
        m = sp == s
        ctx.load_particles(s, x[m], v[m], ids[m])
    ctx.set_node_E([np.asarray(e, np.float64) for e in E])
    ctx.step(5)
    ctx.synchronize()
    return ctx, sp


def lookup(ctx, fn, species, ids):
    """Calls the C entry point fn with sentinel-filled outputs."""
    n = len(ids)
    found = np.full(n, -3, np.int32)
    cols = [np.full(n, -7.25 - d) for d in range(6)]
    srt = np.ascontiguousarray(ids, dtype=np.int64)
    st = fn(ctx._h, species, n, srt.ctypes.data, found.ctypes.data,
            *[c.ctypes.data for c in cols])
    return st, found, cols


def same(a, b):
    assert a[0] == b[0] == pam.pic.OK
    assert np.array_equal(a[1], b[1])
    for ca, cb in zip(a[2], b[2]):
        assert np.array_equal(ca, cb)


@pytest.mark.parametrize("form", ["fp64", "fp32_cell"])
def test_noalloc_lookup_equals_the_allocating_one(form):
    L = pam.lib()
    w = synth.sphere_16()
    ctx, sp = context(w, form)
    other, _ = context(w, "fp32_abs")
    with ctx, other:
        rng = np.random.default_rng(5)
        n0 = int((sp == 0).sum())
        # ids of species 0 (some removed by now) and ids it never had
        big = np.unique(np.concatenate([rng.choice(n0, 9000, replace=False),
                                        np.arange(n0 + 100, n0 + 600)]))
        small = np.sort(rng.choice(big, 300, replace=False))
        ref_big = lookup(ctx, L.pic_get_particles_by_id, 0, big)
        ref_small = lookup(ctx, L.pic_get_particles_by_id, 0, small)
        assert 0 < ref_big[1].sum() < len(big)
        same(lookup(ctx, L.pic_get_particles_by_id_noalloc, 0, big), ref_big)
        same(lookup(ctx, L.pic_get_particles_by_id_noalloc, 0, small), ref_small)
        # another context on the same GPU shares the scratch area
        other_ref = lookup(other, L.pic_get_particles_by_id, 1, small + n0)
        same(lookup(other, L.pic_get_particles_by_id_noalloc, 1, small + n0), other_ref)
        same(lookup(ctx, L.pic_get_particles_by_id_noalloc, 0, big), ref_big)


def test_noalloc_lookup_limits_and_errors():
    L = pam.lib()
    w = synth.sphere_16()
    ctx, sp = context(w, "fp32_cell")
    with ctx:
        too_many = np.arange(MAX_IDS + 1, dtype=np.int64)
        st, _, _ = lookup(ctx, L.pic_get_particles_by_id_noalloc, 0, too_many)
        assert st == pam.pic.E_INVALID
        assert b"PIC_NOALLOC_MAX_IDS" in L.pic_last_error(ctx._h)
        st, found, _ = lookup(ctx, L.pic_get_particles_by_id_noalloc, 0,
                              np.arange(MAX_IDS, dtype=np.int64))
        assert st == pam.pic.OK and found.sum() > 0
        st, _, _ = lookup(ctx, L.pic_get_particles_by_id_noalloc, 0,
                          np.array([3, 2], dtype=np.int64))
        assert st == pam.pic.E_INVALID
        st, _, _ = lookup(ctx, L.pic_get_particles_by_id_noalloc, 7, np.array([1], np.int64))
        assert st == pam.pic.E_INVALID
        st, _, _ = lookup(ctx, L.pic_get_particles_by_id_noalloc, 0, np.zeros(0, np.int64))
        assert st == pam.pic.OK


def test_noalloc_lookup_allocates_nothing():
    L = pam.lib()
    w = synth.sphere_16()
    a = Counting()
    ctx, sp = context(w, "fp32_cell", allocator=a)
    with ctx:
        ids = np.arange(0, int((sp == 0).sum()), 7, dtype=np.int64)
        before = a.calls
        r1 = lookup(ctx, L.pic_get_particles_by_id_noalloc, 0, ids)
        r2 = lookup(ctx, L.pic_get_particles_by_id_noalloc, 0, ids[:50])
        assert a.calls == before
        ref = lookup(ctx, L.pic_get_particles_by_id, 0, ids)
        assert a.calls == before + 3  # the allocating lookup's three staging buffers
        same(r1, ref)
        assert r2[0] == pam.pic.OK
