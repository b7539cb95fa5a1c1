"""The caller's device allocator (pic_config.alloc / dealloc): a context that
takes its memory from torch's caching allocator through a counting wrapper
gives every byte back by the end of pic_destroy and computes the same bits
as one on hipMalloc; an allocator that refuses makes the call fail with
PIC_E_NOMEM and leaves nothing allocated; the binding's "torch" allocator
draws the footprint from torch's pool."""
import numpy as np
import pytest
import torch

import paper_2011_10214_amd as pam
import synth

from gpu_util import inputs

pytestmark = pytest.mark.gpu


class Counting:
    """torch's caching allocator, counting live allocations; refuses every
    allocation after the first `limit`."""

    def __init__(self, limit=None):
        self.live = {}
        self.calls = 0
        self.limit = limit

    def alloc(self, nbytes):
        self.calls += 1
        if self.limit is not None and self.calls > self.limit:
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes)
        assert p % 256 == 0
        self.live[p] = nbytes
        return p

    def free(self, ptr):
        assert ptr in self.live, "dealloc of a pointer alloc did not return"
        del self.live[ptr]
        torch.cuda.caching_allocator_delete(ptr)


def run(w, allocator):
    sp, x, v, E = inputs(w)
    cfg = pam.config_from_workload(w, repr="fp32_cell", deposit="fixed64")
    cfg.allocator = allocator
    ids = np.arange(len(sp), dtype=np.int64)
    with pam.Context(cfg) as ctx:
        for s in range(len(w.species)):
            m = sp == s
            ctx.load_particles(s, x[m], v[m], ids[m])  # ids: one more allocation per species
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.step(3)
        ctx.solve_field(32, tol=1e-8)  # the field buffers
        ctx.step(2)
        found, px, _ = ctx.get_particles_by_id(0, ids[sp == 0][:100])  # staging for the call
        rho = ctx.get_rho()[1]
    return rho, found, px


def test_counting_allocator_gets_every_byte_back():
    w = synth.sphere_16()
    a = Counting()
    rho, found, px = run(w, a)
    assert a.calls > 20 and not a.live
    rho0, found0, px0 = run(w, None)
    assert np.array_equal(rho, rho0)
    assert np.array_equal(found, found0) and np.array_equal(px[found], px0[found0])


@pytest.mark.parametrize("limit", [0, 5, 27])
def test_refusing_allocator_gives_nomem_and_leaves_nothing(limit):
    w = synth.sphere_16()
    a = Counting(limit)
    cfg = pam.config_from_workload(w)
    cfg.allocator = a
    with pytest.raises(pam.PicError) as ei:
        pam.Context(cfg)
    assert ei.value.status == pam.pic.E_NOMEM
    assert not a.live


def test_refused_field_buffers_leave_the_context_usable():
    # the first field solve allocates its buffers: refused, it fails with
    # PIC_E_NOMEM and the context keeps stepping
    w = synth.sphere_16()
    sp, x, v, E = inputs(w)
    a = Counting()
    cfg = pam.config_from_workload(w)
    cfg.allocator = a
    with pam.Context(cfg) as ctx:
        for s in range(2):
            ctx.load_particles(s, x[sp == s], v[sp == s])
        ctx.set_node_E([np.asarray(e, np.float64) for e in E])
        ctx.step(1)
        a.limit = a.calls
        with pytest.raises(pam.PicError) as ei:
            ctx.solve_field(32)
        assert ei.value.status == pam.pic.E_NOMEM
        ctx.step(1)
        ctx.synchronize()
    assert not a.live


def test_torch_allocator_takes_the_footprint_from_torchs_pool():
    w = synth.sphere_16()
    cfg = pam.config_from_workload(w)
    need = pam.footprint_bytes(cfg)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    cfg.allocator = "torch"
    with pam.Context(cfg):
        during = torch.cuda.memory_allocated()
    after = torch.cuda.memory_allocated()
    assert during - before >= need
    assert after == before
