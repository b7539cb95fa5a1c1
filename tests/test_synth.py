"""The seeded generator: determinism, quantisation, placement and statistics."""
import json
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hashes_match_stored_digests():
    import sys
    sys.path.insert(0, GOLDEN)
    from make_golden import synth_hashes

    with open(os.path.join(GOLDEN, "synth_hashes.json")) as f:
        stored = json.load(f)
    assert synth_hashes() == stored


def test_same_seed_same_values_and_index_addressing():
    w = synth.sphere_16()
    a = synth.particles(w, 0, 100, 500)
    b = synth.particles(w, 0, idx=np.arange(100, 600))
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    c = synth.particles(w, 1, 100, 500)
    assert not np.array_equal(a[0], c[0])


def test_positions_are_on_the_2pow16_grid_inside_box_and_outside_object():
    for w in (synth.sphere_16(), synth.scaled(synth.crater_160(), 40, 40, 20, ppc=4)):
        for s in range(2):
            x, y, z, vx, vy, vz = synth.particles(w, s, 0, 20000)
            for a, n in ((x, w.nx), (y, w.ny), (z, w.nz)):
                assert np.all(a >= 0) and np.all(a < n)
                assert np.array_equal(a * 65536.0, np.floor(a * 65536.0))
            p = np.stack([x, y, z], 1).astype(np.float64)
            if w.obj == "sphere":
                assert np.all(np.linalg.norm(p - np.asarray(w.center), axis=1) > w.radius)
            else:
                a_, d_ = w.rim_radius, w.depth
                Rc = (a_ * a_ + d_ * d_) / (2 * d_)
                zc = w.z_flat - d_ + Rc
                below = (p[:, 2] <= w.z_flat) & (
                    np.linalg.norm(p - np.array([w.center[0], w.center[1], zc]), axis=1) >= Rc)
                assert not below.any()


def test_maxwellian_moments_and_drift():
    w = synth.scaled(synth.crater_160(), 40, 40, 20, ppc=8)
    for s, sp in enumerate(w.species):
        _, _, _, vx, vy, vz = synth.particles(w, s, 0, 200000)
        for d, a in enumerate((vx, vy, vz)):
            a = a.astype(np.float64)
            assert abs(a.mean() - sp.drift[d]) < 5 * sp.vth / np.sqrt(len(a))
            assert abs(a.std() / sp.vth - 1.0) < 0.01


def test_node_field_shapes_and_values():
    w = synth.sphere_16()
    Ex, Ey, Ez = synth.node_E(w)
    assert Ex.shape == (17 ** 3,) and Ex.dtype == np.float32
    # node (8 + 6, 8, 8): radial field of the ball charge, Q / (4 pi r^2)
    node = 14 + 17 * (8 + 17 * 8)
    assert Ex[node] == np.float32(-50.0 / (4 * np.pi * 36.0))
    assert Ey[node] == 0 and Ez[node] == 0
    # centre node: zero field (linear inside the ball)
    assert Ex[8 + 17 * (8 + 17 * 8)] == 0
    w = synth.scaled(synth.crater_160(), 40, 40, 20, ppc=1)
    Ex, Ey, Ez = synth.node_E(w)
    assert np.abs(Ex).max() <= 1e-3 and np.abs(Ey).max() <= 1e-3
    nodes_per_plane = 41 * 41
    # below the sheath edge z0 = 2.5 the field is -E0 = -0.2 within the noise
    assert np.all(np.abs(Ez[: 3 * nodes_per_plane] + 0.2) <= 1e-3 + 1e-7)
    # and it decays above it
    assert np.abs(Ez[-nodes_per_plane:]).max() <= 1e-3 + 1e-7
