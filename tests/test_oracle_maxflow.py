"""Pins for the max-flow oracle (CPU only).

Each pin ties the oracle to something other than itself: exhaustive min cuts
on tiny grids, scipy's independent max-flow routine, closed forms and
metamorphic relations of the max-flow / min-cut definition (Section 3).
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import maximum_flow

import oracle
import synth
from oracle import brute
from certificates import grid_cut_value

SMALL_SHAPES = [(1, 1), (1, 2), (2, 1), (1, 5), (2, 2), (2, 3), (3, 2),
                (3, 3), (1, 9), (3, 4)]


@pytest.mark.parametrize("shape", SMALL_SHAPES)
@pytest.mark.parametrize("both", [True, False])
def test_bruteforce_min_cut(shape, both):
    H, W = shape
    for seed in range(6):
        inst = synth.grid_random_small(H, W, seed, both_terminals=both,
                                       density=0.7 if seed % 2 else 1.0)
        want_val, want_side = brute.grid_min_cut_bruteforce(inst)
        for method in ("ek", "fifo"):
            val, side = oracle.grid_maxflow(inst, method)
            assert val == want_val, (method, inst.name)
            np.testing.assert_array_equal(side, want_side, err_msg=method)


def _scipy_value(inst):
    n, tail, head, cap, s, t = oracle.grid_arcs(inst)
    keep = cap > 0
    m = csr_matrix((cap[keep].astype(np.int32),
                    (tail[keep], head[keep])), shape=(n, n))
    return int(maximum_flow(m, s, t).flow_value)


@pytest.mark.parametrize("H,W", [(8, 8), (16, 24), (40, 33)])
def test_matches_scipy_random(H, W):
    for seed in range(4):
        inst = synth.grid_random_small(H, W, seed, max_cap=50, max_term=60)
        v_fifo, side = oracle.grid_maxflow(inst, "fifo")
        assert v_fifo == _scipy_value(inst)
        assert grid_cut_value(inst, side) == v_fifo
        if H * W <= 1024:
            v_ek, side_ek = oracle.grid_maxflow(inst, "ek")
            assert v_ek == v_fifo
            np.testing.assert_array_equal(side_ek, side)


@pytest.mark.parametrize("seed", range(5))
def test_uniform64_config_three_ways(seed):
    inst = synth.grid_uniform(64, 64, seed)
    v_fifo, side = oracle.grid_maxflow(inst, "fifo")
    v_ek, side_ek = oracle.grid_maxflow(inst, "ek")
    assert v_fifo == v_ek == _scipy_value(inst)
    np.testing.assert_array_equal(side, side_ek)
    assert grid_cut_value(inst, side) == v_fifo


def test_blobs_medium_matches_scipy():
    inst = synth.grid_blobs(96, 80, seed=3)
    v, side = oracle.grid_maxflow(inst, "fifo")
    assert v == _scipy_value(inst)
    assert grid_cut_value(inst, side) == v


def test_closed_form_no_pairs_one_terminal():
    """Zero neighbour capacities and one terminal per pixel: no s-t path, so
    |f| = 0, and the source arcs stay residual: S_min = {p : cap_src > 0}."""
    inst = synth.grid_uniform(12, 9, seed=1)
    z = np.zeros_like(inst.cap_right)
    inst = synth.GridInstance(12, 9, inst.cap_src, inst.cap_snk, z, z, z, z)
    for method in ("ek", "fifo"):
        v, side = oracle.grid_maxflow(inst, method)
        assert v == 0
        np.testing.assert_array_equal(side, (inst.cap_src > 0).astype(np.uint8))


def test_closed_form_no_pairs_both_terminals():
    """Isolated pixels with both terminals: each carries min(src, snk); the
    pixel is on the minimal source side iff src > snk."""
    g = np.random.default_rng(5)
    H, W = 7, 6
    src = g.integers(0, 40, H * W).astype(np.int32)
    snk = g.integers(0, 40, H * W).astype(np.int32)
    z = np.zeros(H * W, np.int32)
    inst = synth.GridInstance(H, W, src, snk, z, z, z, z)
    for method in ("ek", "fifo"):
        v, side = oracle.grid_maxflow(inst, method)
        assert v == int(np.minimum(src, snk).astype(np.int64).sum())
        np.testing.assert_array_equal(side, (src > snk).astype(np.uint8))


def test_closed_form_chain():
    """A 1xW path with the source at the left end and the sink at the right
    end carries the minimum capacity along the path."""
    g = np.random.default_rng(11)
    for _ in range(5):
        W = int(g.integers(2, 30))
        src = np.zeros(W, np.int32)
        snk = np.zeros(W, np.int32)
        src[0] = g.integers(1, 100)
        snk[-1] = g.integers(1, 100)
        right = g.integers(1, 100, W - 1)
        left = g.integers(0, 100, W - 1)
        inst = synth.grid_from_pairs(1, W, src, snk, right[None], left[None],
                                     np.zeros((0, W)), np.zeros((0, W)))
        want = min(int(src[0]), int(snk[-1]), int(right.min()))
        for method in ("ek", "fifo"):
            assert oracle.grid_maxflow(inst, method)[0] == want


def _transpose(inst):
    H, W = inst.H, inst.W
    t = lambda a: np.ascontiguousarray(a.reshape(H, W).T.reshape(-1))
    # right/left become down/up in the transposed grid
    return synth.GridInstance(W, H, t(inst.cap_src), t(inst.cap_snk),
                              t(inst.cap_down), t(inst.cap_up),
                              t(inst.cap_right), t(inst.cap_left))


def test_metamorphic_transpose_and_scale():
    for seed in range(4):
        inst = synth.grid_random_small(13, 7, seed, max_cap=30)
        v, side = oracle.grid_maxflow(inst, "fifo")
        vt, side_t = oracle.grid_maxflow(_transpose(inst), "fifo")
        assert vt == v
        np.testing.assert_array_equal(side_t.reshape(7, 13).T.reshape(-1), side)
        k = 3
        sc = synth.GridInstance(inst.H, inst.W,
                                *[(a * k).astype(np.int32) for a in inst.arrays()])
        vk, side_k = oracle.grid_maxflow(sc, "fifo")
        assert vk == k * v
        np.testing.assert_array_equal(side_k, side)


def test_metamorphic_reverse_network():
    """Swapping s and t and reversing every arc keeps |f|; the minimal source
    side of the reversed network is the complement of the maximal source side
    of the original, which must itself be a minimum cut containing S_min."""
    for seed in range(4):
        inst = synth.grid_random_small(9, 11, seed, max_cap=25)
        v, side = oracle.grid_maxflow(inst, "fifo")
        rev = synth.GridInstance(inst.H, inst.W, inst.cap_snk, inst.cap_src,
                                 _rev_right(inst), _rev_left(inst),
                                 _rev_down(inst), _rev_up(inst))
        vr, side_r = oracle.grid_maxflow(rev, "fifo")
        assert vr == v
        s_max = 1 - side_r
        assert grid_cut_value(inst, s_max) == v
        assert np.all(s_max >= side)


# reversed arcs: the capacity of p->p+1 in the reversed network is the
# original capacity of p+1->p, i.e. cap_left[p+1]; and so on.
def _shift(a, H, W, di, dj):
    g = a.reshape(H, W)
    out = np.zeros_like(g)
    src = g[max(di, 0):H + min(di, 0), max(dj, 0):W + min(dj, 0)]
    out[max(-di, 0):H + min(-di, 0), max(-dj, 0):W + min(-dj, 0)] = src
    return np.ascontiguousarray(out.reshape(-1))


def _rev_right(i):
    return _shift(i.cap_left, i.H, i.W, 0, 1)


def _rev_left(i):
    return _shift(i.cap_right, i.H, i.W, 0, -1)


def _rev_down(i):
    return _shift(i.cap_up, i.H, i.W, 1, 0)


def _rev_up(i):
    return _shift(i.cap_down, i.H, i.W, -1, 0)


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        oracle.graph_maxflow(3, [0, 1], [1, 0], [-1, 0], 0, 2)


def test_golden_file_consistent_with_oracle():
    """The stored full-size expectations were written by
    tests/golden/make_grid_golden.py from the oracle; re-derive a cheap
    subset here."""
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "grid_golden.json")
    gold = json.load(open(path))
    assert len(gold["batch_seed0"]) == 65
    insts = synth.grid_batch(seed=0, n_small=3, include_big=False)
    for inst, rec in zip(insts, gold["batch_seed0"][:3]):
        v, side = oracle.grid_maxflow(inst, "fifo")
        assert rec["name"] == inst.name and rec["flow"] == v
        assert rec["source_side_sha256"] == hashlib.sha256(side.tobytes()).hexdigest()


def _arc_min_cut_bruteforce(n, tail, head, cap, s, t):
    """Minimum s-t cut of an arc list by enumerating every source side (the
    definition of Section 3); returns (value, the minimal source side, which
    is the intersection of all minimum ones)."""
    others = [v for v in range(n) if v not in (s, t)]
    tail, head, cap = np.asarray(tail), np.asarray(head), np.asarray(cap, np.int64)
    best, sides = None, []
    for mask in range(1 << len(others)):
        side = np.zeros(n, np.uint8)
        side[s] = 1
        for k, v in enumerate(others):
            if mask >> k & 1:
                side[v] = 1
        val = int(cap[(side[tail] == 1) & (side[head] == 0)].sum())
        if best is None or val < best:
            best, sides = val, [side]
        elif val == best:
            sides.append(side)
    return best, np.minimum.reduce(sides)


@pytest.mark.parametrize("gen,args", [
    (synth.grid3d_arcs, (2, 2, 2)), (synth.grid3d_arcs, (1, 2, 5)),
    (synth.grid3d_arcs, (2, 3, 2)), (synth.grid8_arcs, (3, 3)),
    (synth.grid8_arcs, (2, 5))])
def test_volume_and_8_connected_grids_bruteforce(gen, args):
    """6-connected volumes and 8-connected grids (Section 4.3's neighbourhood
    systems beyond the 4-connected one) as arc lists: both oracle methods
    against every cut."""
    for seed in range(4):
        n, tail, head, cap, s, t = gen(*args, seed=seed, tmax=20, pmax=10)
        want, wside = _arc_min_cut_bruteforce(n, tail, head, cap, s, t)
        for method in ("ek", "fifo"):
            v, side, _ = oracle.graph_maxflow(n, tail, head, cap, s, t, method)
            assert v == want, (gen.__name__, args, seed, method)
            np.testing.assert_array_equal(side, wside)


@pytest.mark.parametrize("gen,args", [(synth.grid3d_arcs, (8, 12, 10)),
                                      (synth.grid8_arcs, (30, 40))])
def test_volume_and_8_connected_grids_match_scipy(gen, args):
    n, tail, head, cap, s, t = gen(*args, seed=1)
    keep = cap > 0
    m = csr_matrix((cap[keep].astype(np.int32), (tail[keep], head[keep])),
                   shape=(n, n))
    v, side, _ = oracle.graph_maxflow(n, tail, head, cap, s, t)
    assert v == int(maximum_flow(m, s, t).flow_value)
    assert int(cap[(side[tail] == 1) & (side[head] == 0)].sum()) == v
