"""GPU parity for max-flow on arbitrary networks (arc lists in mate pairs):
the HIP library against the CPU oracle.

The flow value and the minimal source side of a minimum cut are unique and
must equal the oracle's exactly; the cut's capacity must equal the flow value
(max-flow min-cut, a check that needs no oracle).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1110_6231_amd import lpr  # noqa: E402


def cut_capacity(tail, head, cap, side):
    tail, head = np.asarray(tail), np.asarray(head)
    crossing = (side[tail] == 1) & (side[head] == 0)
    return int(np.asarray(cap, np.int64)[crossing].sum())


def check(g, **kw):
    n, tail, head, cap, s, t = g
    print(f"[graph] n={n} m={len(tail)} s={s} t={t} {kw}", flush=True)
    v, side, st = lpr.lpr_graph_maxflow(n, tail, head, cap, s, t, **kw)
    want, wside, _ = oracle.graph_maxflow(n, tail, head, cap, s, t)
    side = side.cpu().numpy()
    assert v == want, (v, want, st)
    assert np.array_equal(side, wside)
    assert side[s] == 1 and side[t] == 0
    assert cut_capacity(tail, head, cap, side) == v
    return st


@pytest.mark.parametrize("n,edges", [(2, 1), (3, 6), (10, 40), (100, 400),
                                     (2000, 8000), (30000, 120000)])
def test_random_graphs(n, edges):
    for seed in range(3):
        check(synth.graph_random(n, edges, seed=seed))


def test_random_graphs_two_way_and_dense():
    check(synth.graph_random(300, 20000, seed=5, two_way=1.0, max_cap=10**6))
    check(synth.graph_random(64, 64 * 63, seed=6, two_way=0.0, max_cap=3))


@pytest.mark.parametrize("layers,width,degree", [(5, 20, 2), (50, 100, 3),
                                                  (400, 20, 2)])
def test_layered_graphs(layers, width, degree):
    """Long augmenting paths: the BFS runs hundreds of levels."""
    check(synth.graph_layered(layers, width, degree, seed=1))


@pytest.mark.parametrize("nx,ny,edges", [(500, 400, 3000), (3000, 3000, 12000)])
def test_bipartite_matching_networks(nx, ny, edges):
    st = check(synth.graph_bipartite(nx, ny, edges, seed=2))
    assert st["rounds"] >= 0


def test_grid_as_a_graph_matches_the_grid_solver():
    """The same network solved by form 1 on its grid layout and as an arc list."""
    inst = synth.grid_blobs(96, 80, seed=3)
    g = synth.grid_to_arcs(inst)
    st = check(g)
    caps = [torch.as_tensor(a, device="cuda") for a in inst.arrays()]
    v, side, _ = lpr.lpr_grid_maxflow(inst.H, inst.W, *caps)
    v2, side2, _ = lpr.lpr_graph_maxflow(*g)
    assert v == v2
    assert np.array_equal(side.cpu().numpy(), side2.cpu().numpy()[:inst.H * inst.W])
    assert st["pushes"] > 0


@pytest.mark.parametrize("gen,args", [(synth.grid3d_arcs, (1, 1, 1)),
                                      (synth.grid3d_arcs, (3, 4, 5)),
                                      (synth.grid3d_arcs, (16, 24, 20)),
                                      (synth.grid3d_arcs, (40, 40, 40)),
                                      (synth.grid8_arcs, (1, 7)),
                                      (synth.grid8_arcs, (64, 64)),
                                      (synth.grid8_arcs, (150, 170))])
def test_volume_and_8_connected_grids(gen, args):
    """Neighbourhood systems other than the 4-connected grid (6-connected
    volumes, 8-connected images) through the arc-list solver."""
    for seed in range(2):
        check(gen(*args, seed=seed))


def test_edge_cases():
    # no arcs
    v, side, _ = lpr.lpr_graph_maxflow(5, [], [], [], 0, 4)
    assert v == 0 and side.cpu().tolist() == [1, 0, 0, 0, 0]
    # t unreachable, s isolated from the rest
    check((4, *synth.pairs_to_arcs([1, 2], [2, 1], [5, 5], [0, 0]), 0, 3))
    # parallel arcs, self-loops and zero capacities
    u = [0, 0, 1, 1, 2, 2, 1]
    w = [1, 1, 1, 2, 3, 3, 3]
    check((4, *synth.pairs_to_arcs(u, w, [3, 4, 9, 0, 5, 1, 2], [0, 1, 0, 2, 0, 0, 0]), 0, 3))
    # capacities at the limit: a mate pair's sum is 2^31 - 1
    big = (1 << 31) - 1
    check((3, *synth.pairs_to_arcs([0, 1], [1, 2], [big, big - 5], [0, 5]), 0, 2))
    # t -> s only: nothing flows
    check((2, *synth.pairs_to_arcs([1], [0], [7], [0]), 0, 1))


def test_options():
    g = synth.graph_layered(30, 40, 3, seed=4)
    for cycle, sweeps in ((1, 1), (7, 3), (500, 1), (16, 64)):
        check(g, opts=lpr.make_graph_opts(cycle=cycle, sweeps_per_relabel=sweeps))
    with pytest.raises(lpr.LprError):
        lpr.lpr_graph_maxflow(*g, opts=lpr.make_graph_opts(max_rounds=1, cycle=1,
                                                           sweeps_per_relabel=1))
    with pytest.raises(lpr.LprError):
        lpr.lpr_graph_maxflow(*g, opts=lpr.make_graph_opts(sweeps_per_relabel=1025))


def test_invalid_inputs_are_rejected():
    tail, head, cap = synth.pairs_to_arcs([0, 1], [1, 2], [3, 4], [0, 0])
    with pytest.raises(lpr.LprError) as e:  # odd arc count
        lpr.lpr_graph_maxflow(3, tail[:3], head[:3], cap[:3], 0, 2)
    assert e.value.status == lpr.LPR_EINVAL
    bad = head.copy()
    bad[1] = 2  # arc 1 no longer reverses arc 0
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_graph_maxflow(3, tail, bad, cap, 0, 2)
    assert e.value.status == lpr.LPR_EINVAL
    with pytest.raises(lpr.LprError) as e:  # node out of range
        lpr.lpr_graph_maxflow(2, tail, head, cap, 0, 1)
    assert e.value.status == lpr.LPR_EINVAL
    neg = cap.copy()
    neg[2] = -1
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_graph_maxflow(3, tail, head, neg, 0, 2)
    assert e.value.status == lpr.LPR_ERANGE
    over = cap.copy()
    over[0], over[1] = (1 << 31) - 1, 1
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_graph_maxflow(3, tail, head, over, 0, 2)
    assert e.value.status == lpr.LPR_ERANGE
    with pytest.raises(lpr.LprError) as e:  # s == t
        lpr.lpr_graph_maxflow(3, tail, head, cap, 1, 1)
    assert e.value.status == lpr.LPR_EINVAL
