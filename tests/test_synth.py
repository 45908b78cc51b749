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


def _check_pairs(n, tail, head, cap):
    tail, head, cap = np.asarray(tail), np.asarray(head), np.asarray(cap)
    assert len(tail) % 2 == 0
    assert np.array_equal(tail[0::2], head[1::2]) and np.array_equal(head[0::2], tail[1::2])
    assert tail.min(initial=0) >= 0 and max(tail.max(initial=0), head.max(initial=0)) < n
    assert np.all(cap >= 0)


def test_volume_and_8_connected_generators():
    n, tail, head, cap, s, t = synth.grid3d_arcs(3, 4, 5, seed=1)
    _check_pairs(n, tail, head, cap)
    inner = 3 * 4 * 5
    # terminal pairs + (D(H)(W-1) + D(H-1)W + (D-1)HW) neighbour pairs
    assert len(tail) == 2 * (2 * inner + 3 * 4 * 4 + 3 * 3 * 5 + 2 * 4 * 5)
    assert np.array_equal(cap[4 * inner::2], cap[4 * inner + 1::2])  # symmetric
    n8, t8, h8, c8, _, _ = synth.grid8_arcs(4, 6, seed=1)
    _check_pairs(n8, t8, h8, c8)
    assert len(t8) == 2 * (2 * 24 + 4 * 5 + 3 * 6 + 2 * 3 * 5)
    assert np.array_equal(synth.grid8_arcs(4, 6, seed=1)[3], c8)    # seeded


def test_mincost_generators_are_feasible_by_construction():
    for g in (synth.mcf_random(40, 150, seed=2), synth.mcf_transport(5, 7, seed=3)):
        n, tail, head, cap, cost, supply = g
        _check_pairs(n, tail, head, cap)
        assert np.array_equal(cost[0::2], -cost[1::2])
        assert int(np.asarray(supply, np.int64).sum()) == 0
    n, tail, head, cap, cost, supply = synth.mcf_transport(5, 7, seed=3)
    assert np.all(supply[:5] > 0) and np.all(supply[5:] <= 0)


def test_sparse_assignment_generator():
    row_ptr, col, cost = synth.assign_sparse(50, 3, seed=4, parallel=0.5, lo=-9, hi=9)
    assert row_ptr[0] == 0 and row_ptr[-1] == len(col) and np.all(np.diff(row_ptr) >= 4)
    assert col.min() >= 0 and col.max() < 50 and cost.min() >= -9 and cost.max() <= 9
    rp2, c2, _ = synth.assign_sparse(50, 0, seed=4)
    assert np.array_equal(np.sort(c2), np.arange(50))  # the planted permutation
