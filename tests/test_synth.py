"""Seeded generators: determinism, layout and the structure each workload
description fixes (one terminal per pixel, symmetric pairs, value ranges)."""
import numpy as np

import synth


def test_grid_uniform_structure():
    a = synth.grid_uniform(64, 64, seed=3)
    b = synth.grid_uniform(64, 64, seed=3)
    for x, y in zip(a.arrays(), b.arrays()):
        assert x.dtype == np.int32 and x.shape == (4096,)
        np.testing.assert_array_equal(x, y)
    assert not np.any((a.cap_src > 0) & (a.cap_snk > 0))
    assert a.cap_src.max() <= 100 and a.cap_snk.max() <= 100
    r = a.cap_right.reshape(64, 64)
    l = a.cap_left.reshape(64, 64)
    assert np.all(r[:, -1] == 0) and np.all(l[:, 0] == 0)
    np.testing.assert_array_equal(r[:, :-1], l[:, 1:])
    d = a.cap_down.reshape(64, 64)
    u = a.cap_up.reshape(64, 64)
    assert np.all(d[-1] == 0) and np.all(u[0] == 0)
    np.testing.assert_array_equal(d[:-1], u[1:])
    assert max(r.max(), d.max()) <= 50


def test_grid_blobs_structure():
    g = synth.grid_blobs(96, 130, seed=1)
    assert g.n_pixels == 96 * 130
    assert not np.any((g.cap_src > 0) & (g.cap_snk > 0))
    assert g.cap_src.max() <= 50 and g.cap_snk.max() <= 50
    assert g.cap_right.max() <= 50
    g4 = synth.grid_blobs(64, 64, seed=1, pair_scale=200.0)
    assert g4.cap_right.max() <= 200


def test_grid_batch_sizes():
    b = synth.grid_batch(seed=0, n_small=5, include_big=False)
    assert len(b) == 5
    assert all(128 <= g.H <= 512 and 128 <= g.W <= 512 for g in b)


def test_assign_generators():
    c = synth.assign_uniform(50, seed=1)
    assert c.dtype == np.int32 and c.min() >= 0 and c.max() <= 1000
    np.testing.assert_array_equal(c, synth.assign_uniform(50, seed=1))
    p = synth.assign_points(70, seed=0, instance=3)
    assert p.shape == (70, 70) and p.min() >= 0
    pt = synth.assign_points(70, seed=0, instance=3, train=True)
    assert not np.array_equal(p, pt)
    ns = [x.shape[0] for x in synth.assign_batch(seed=0, count=6)]
    assert all(64 <= n <= 512 for n in ns)
