"""Pins for the min-cost flow oracle (CPU only).

The successive-shortest-path oracle is tied to scipy's independent LP solver
(a network LP has an integral optimum, so the optimal values agree exactly),
to the assignment and max-flow oracles on the special cases the min-cost
flow problem contains, and to its own optimality certificate.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
import synth


def lp_optimum(n, tail, head, cap, cost, supply):
    """The same problem as an LP over every arc (both arcs of a pair as
    variables in [0, cap]); None when infeasible."""
    m = len(tail)
    A = np.zeros((n, m))
    A[tail, np.arange(m)] += 1.0
    A[head, np.arange(m)] -= 1.0
    r = linprog(np.asarray(cost, float), A_eq=A, b_eq=np.asarray(supply, float),
                bounds=list(zip([0] * m, np.asarray(cap, float))), method="highs")
    if r.status == 2:
        return None
    assert r.status == 0
    return int(round(r.fun))


def check_flow(n, tail, head, cap, cost, supply, res, pi, total):
    tail, head = np.asarray(tail), np.asarray(head)
    cap = np.asarray(cap, np.int64)
    f = cap - res                                   # net flow along each arc
    assert np.all(f[0::2] == -f[1::2])
    assert np.all(res >= 0)
    out = np.zeros(n, np.int64)
    np.add.at(out, tail[0::2], f[0::2])
    np.add.at(out, head[0::2], -f[0::2])
    assert np.array_equal(out, np.asarray(supply, np.int64))     # conservation
    assert int((f[0::2] * np.asarray(cost, np.int64)[0::2]).sum()) == total
    red = np.asarray(cost, np.int64) + pi[tail] - pi[head]
    assert np.all(red[res > 0] >= 0)                # no negative residual arc


@pytest.mark.parametrize("n,edges", [(2, 1), (3, 4), (6, 12), (20, 60), (60, 300)])
def test_matches_linprog(n, edges):
    for seed in range(4):
        g = synth.mcf_random(n, edges, seed=seed, max_cap=9, max_cost=20)
        got = oracle.mincost_flow(*g)
        want = lp_optimum(*g)
        assert got is not None and want is not None
        assert got[0] == want
        check_flow(*g, got[1], got[2], got[0])


def test_transportation_matches_linprog():
    g = synth.mcf_transport(7, 9, seed=2, max_cost=50, max_supply=20, cap=1000)
    got = oracle.mincost_flow(*g)
    assert got[0] == lp_optimum(*g)
    check_flow(*g, got[1], got[2], got[0])


def test_infeasible_supplies():
    n, tail, head, cap, cost, _ = synth.mcf_random(12, 20, seed=3, max_cap=3)
    supply = np.zeros(n, np.int32)
    supply[0], supply[1] = 1000, -1000       # more than any cut can carry
    assert oracle.mincost_flow(n, tail, head, cap, cost, supply) is None
    assert lp_optimum(n, tail, head, cap, cost, supply) is None


def test_assignment_is_a_special_case():
    """Unit supplies on X, unit demands on Y, unit capacities: the
    assignment problem of Section 3, so the optimum is the Hungarian one."""
    for n, seed in ((5, 1), (30, 2)):
        c = synth.assign_random_small(n, seed, lo=-200, hi=200)
        u = np.repeat(np.arange(n), n)
        v = n + np.tile(np.arange(n), n)
        tail, head, cap = synth.pairs_to_arcs(u, v, np.ones(n * n), np.zeros(n * n))
        cost = np.empty(2 * n * n, np.int64)
        cost[0::2], cost[1::2] = c.ravel(), -c.ravel()
        supply = np.concatenate([np.ones(n), -np.ones(n)]).astype(np.int64)
        tot, _, _ = oracle.mincost_flow(2 * n, tail, head, cap, cost, supply)
        assert tot == oracle.assign(c)[1]


def test_max_flow_is_a_special_case():
    """Zero supplies, zero costs and an arc t -> s of cost -1: the least-cost
    circulation sends the maximum flow round it, so its cost is -|f*|."""
    for seed in range(3):
        n, tail, head, cap, s, t = synth.graph_random(40, 160, seed=seed)
        tail = np.append(tail, [t, s]).astype(np.int32)
        head = np.append(head, [s, t]).astype(np.int32)
        cap = np.append(cap, [1 << 20, 0]).astype(np.int64)
        cost = np.zeros(len(tail), np.int64)
        cost[-2:] = [-1, 1]
        tot, _, _ = oracle.mincost_flow(n, tail, head, cap, cost, np.zeros(n))
        assert tot == -oracle.graph_maxflow(*synth.graph_random(40, 160, seed=seed))[0]


def test_rejects_bad_input():
    n, tail, head, cap, cost, supply = synth.mcf_random(5, 6, seed=1)
    bad = cost.copy()
    bad[1] = bad[0] + 1
    with pytest.raises(ValueError):
        oracle.mincost_flow(n, tail, head, cap, bad, supply)
    s2 = supply.copy()
    s2[0] += 1
    with pytest.raises(ValueError):
        oracle.mincost_flow(n, tail, head, cap, cost, s2)
