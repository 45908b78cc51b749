"""GPU parity for minimum-cost flow with supplies (cost scaling, Algorithm
5.0) on arbitrary networks: the HIP library against the CPU oracle
(successive shortest paths).

Optimal flows are not unique; the optimal total cost is, and must equal the
oracle's exactly.  The returned flow must conserve every supply, respect the
capacities and cost that total, and the returned prices must certify it:
every residual arc has scaled reduced cost >= -1 (costs scaled by n + 1),
which makes the flow optimal without the oracle.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1110_6231_amd import lpr  # noqa: E402


def check(g, opts=None):
    n, tail, head, cap, cost, supply = g
    print(f"[mcf] n={n} m={len(tail)} {opts}", flush=True)
    want = oracle.mincost_flow(*g)
    assert want is not None
    tot, res, prices, st = lpr.lpr_mincost_flow(*g, opts=opts)
    assert tot == want[0], (tot, want[0], st)
    res = res.cpu().numpy().astype(np.int64)
    p = prices.cpu().numpy()
    tail, head = np.asarray(tail), np.asarray(head)
    cap = np.asarray(cap, np.int64)
    cost = np.asarray(cost, np.int64)
    f = cap - res
    assert np.all(res >= 0) and np.all(f[0::2] == -f[1::2])
    out = np.zeros(n, np.int64)
    np.add.at(out, tail[0::2], f[0::2])
    np.add.at(out, head[0::2], -f[0::2])
    assert np.array_equal(out, np.asarray(supply, np.int64))
    assert int((f[0::2] * cost[0::2]).sum()) == tot
    red = cost * (n + 1) + p[tail] - p[head]
    assert np.all(red[res > 0] >= -1)
    return st


@pytest.mark.parametrize("n,edges", [(1, 0), (2, 1), (3, 4), (10, 40), (100, 400),
                                     (1000, 5000), (2500, 10000)])
def test_random_networks(n, edges):
    for seed in range(2 if n < 2000 else 1):
        check(synth.mcf_random(n, edges, seed=seed))


def test_costs_and_capacities_at_the_limits():
    check(synth.mcf_random(300, 1500, seed=4, max_cost=lpr.LPR_MCF_MAX_COST,
                           max_cap=1 << 20, two_way=0.5))
    check(synth.mcf_random(50, 400, seed=5, max_cost=1, max_cap=1))


def test_transportation():
    check(synth.mcf_transport(30, 40, seed=1))
    st = check(synth.mcf_transport(100, 150, seed=2, max_supply=1000))
    print("[mcf] transport stats", st, flush=True)


def test_assignment_special_case():
    n = 60
    c = synth.assign_random_small(n, 7, lo=-500, hi=500)
    u = np.repeat(np.arange(n), n)
    v = n + np.tile(np.arange(n), n)
    tail, head, cap = synth.pairs_to_arcs(u, v, np.ones(n * n), np.zeros(n * n))
    cost = np.empty(2 * n * n, np.int32)
    cost[0::2], cost[1::2] = c.ravel(), -c.ravel()
    supply = np.concatenate([np.ones(n), -np.ones(n)]).astype(np.int32)
    tot, _, _, _ = lpr.lpr_mincost_flow(2 * n, tail, head, cap, cost, supply)
    assert tot == oracle.assign(c)[1]


def test_circulations():
    """Zero supplies: the least-cost circulation (negative cycles saturated),
    and a max-flow as a circulation through an arc t -> s of cost -1."""
    n, tail, head, cap, cost, _ = synth.mcf_random(200, 800, seed=6)
    check((n, tail, head, cap, cost, np.zeros(n, np.int32)))
    n, tail, head, cap, s, t = synth.graph_random(300, 1500, seed=2)
    tail = np.append(tail, [t, s]).astype(np.int32)
    head = np.append(head, [s, t]).astype(np.int32)
    cap = np.append(cap, [1 << 20, 0]).astype(np.int32)
    cost = np.zeros(len(tail), np.int32)
    cost[-2:] = [-1, 1]
    tot, _, _, _ = lpr.lpr_mincost_flow(n, tail, head, cap, cost, np.zeros(n, np.int32))
    assert tot == -oracle.graph_maxflow(*synth.graph_random(300, 1500, seed=2))[0]


@pytest.mark.parametrize("alpha,per", [(2, 1), (16, 64), (4, 3)])
def test_options(alpha, per):
    check(synth.mcf_random(500, 2500, seed=8), opts=lpr.make_mcf_opts(alpha, per))


def test_infeasible_and_errors():
    n, tail, head, cap, cost, supply = synth.mcf_random(12, 20, seed=3, max_cap=3)
    s2 = np.zeros(n, np.int32)
    s2[0], s2[1] = 1000, -1000
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_mincost_flow(n, tail, head, cap, cost, s2)
    assert e.value.status == lpr.LPR_EINFEASIBLE
    g = synth.mcf_random(30, 100, seed=9)
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_mincost_flow(*g, opts=lpr.make_mcf_opts(max_iters=1, iters_per_check=1))
    assert e.value.status == lpr.LPR_EBUDGET
    n, tail, head, cap, cost, supply = g
    bad = cost.copy()
    bad[3] += 1
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_mincost_flow(n, tail, head, cap, bad, supply)
    assert e.value.status == lpr.LPR_EINVAL
    big = cost.copy()
    big[0], big[1] = 1 << 16, -(1 << 16)
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_mincost_flow(n, tail, head, cap, big, supply)
    assert e.value.status == lpr.LPR_ERANGE
    s3 = supply.copy()
    s3[0] += 1
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_mincost_flow(n, tail, head, cap, cost, s3)
    assert e.value.status == lpr.LPR_EINVAL
    wrong = head.copy()
    wrong[1] = (wrong[1] + 1) % n
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_mincost_flow(n, tail, wrong, cap, cost, supply)
    assert e.value.status == lpr.LPR_EINVAL


def test_large_network_by_certificate():
    """20 000 nodes, 80 000 edges: too large for the oracle in a test, so the
    checks are the ones that need none: the flow conserves every supply
    within the capacities, and the prices certify it optimal (every
    residual arc has scaled reduced cost >= -1, and a residual cycle has at
    most n arcs, so none has negative cost)."""
    n, tail, head, cap, cost, supply = synth.mcf_random(20000, 80000, seed=3)
    print(f"[mcf] n={n} m={len(tail)} certificate only", flush=True)
    tot, res, prices, st = lpr.lpr_mincost_flow(n, tail, head, cap, cost, supply)
    res = res.cpu().numpy().astype(np.int64)
    p = prices.cpu().numpy()
    f = cap.astype(np.int64) - res
    assert np.all(res >= 0) and np.all(f[0::2] == -f[1::2])
    out = np.zeros(n, np.int64)
    np.add.at(out, tail[0::2], f[0::2])
    np.add.at(out, head[0::2], -f[0::2])
    assert np.array_equal(out, supply.astype(np.int64))
    assert int((f[0::2] * cost[0::2].astype(np.int64)).sum()) == tot
    red = cost.astype(np.int64) * (n + 1) + p[tail] - p[head]
    assert np.all(red[res > 0] >= -1)
    print("[mcf] large network stats", st, flush=True)
