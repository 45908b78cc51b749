"""Pins for the assignment oracles (CPU only).

The Hungarian oracle is tied to exhaustive search, to scipy's independent
linear_sum_assignment, to LP duality (its integer duals), to closed forms and
to invariances of the assignment definition (Section 3).  The sequential
cost-scaling oracle (the paper's Algorithms 5.0/5.2/5.4 in FIFO order) is
tied to the Hungarian optimum and to the scaled 1-optimality certificate.
"""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import oracle
import synth
from oracle import brute
from certificates import (hungarian_duals_ok, is_permutation,
                          scaled_eps_certificate)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_bruteforce(n):
    for seed in range(8 if n < 7 else 3):
        c = synth.assign_random_small(n, seed)
        want, _ = brute.assign_bruteforce(c)
        r2c, tot, u, v = oracle.hungarian(c)
        assert tot == want
        assert is_permutation(r2c, n)
        assert hungarian_duals_ok(c, r2c, u, v)
        r2c_cs, tot_cs, prices, _ = oracle.cost_scaling(c)
        assert tot_cs == want
        assert is_permutation(r2c_cs, n)
        assert scaled_eps_certificate(c, r2c_cs, prices)


def test_bruteforce_n8_max():
    c = synth.assign_random_small(8, 3, lo=0, hi=1000)
    want, _ = brute.assign_bruteforce(-c.astype(np.int64))
    r2c, tot = oracle.assign(c, maximize=True)
    assert -tot == want
    assert oracle.cost_scaling(c, maximize=True)[1] == tot


@pytest.mark.parametrize("n", [10, 37, 128, 300])
def test_matches_scipy(n):
    for seed in range(3):
        c = synth.assign_random_small(n, seed, lo=0, hi=1000)
        rows, cols = linear_sum_assignment(c)
        want = int(c[rows, cols].astype(np.int64).sum())
        r2c, tot, u, v = oracle.hungarian(c)
        assert tot == want
        assert hungarian_duals_ok(c, r2c, u, v)
        _, tot_cs, prices, _ = oracle.cost_scaling(c)
        assert tot_cs == want


def test_points_config_matches_scipy():
    for inst in range(3):
        c = synth.assign_points(200 + 37 * inst, seed=0, instance=inst + 1)
        rows, cols = linear_sum_assignment(c)
        want = int(c[rows, cols].astype(np.int64).sum())
        assert oracle.assign(c)[1] == want
        r2c, tot, prices, _ = oracle.cost_scaling(c)
        assert tot == want
        assert scaled_eps_certificate(c, r2c, prices)


def test_uniform_max_config_matches_scipy():
    c = synth.assign_uniform(256, seed=2)
    rows, cols = linear_sum_assignment(c, maximize=True)
    want = int(c[rows, cols].astype(np.int64).sum())
    assert oracle.assign(c, maximize=True)[1] == want
    assert oracle.cost_scaling(c, maximize=True)[1] == want


def test_closed_form_constant():
    for n in (1, 5, 33):
        c = np.full((n, n), 17, np.int32)
        assert oracle.assign(c)[1] == 17 * n
        assert oracle.cost_scaling(c)[1] == 17 * n


def test_closed_form_rank_one_rearrangement():
    """c_ij = a_i * b_j with a, b >= 0: by the rearrangement inequality the
    minimum pairs a ascending with b descending."""
    g = np.random.default_rng(3)
    for n in (4, 19, 64):
        a = g.integers(0, 60, n)
        b = g.integers(0, 60, n)
        c = np.outer(a, b).astype(np.int32)
        want = int((np.sort(a) * np.sort(b)[::-1]).sum())
        assert oracle.assign(c)[1] == want
        assert oracle.cost_scaling(c)[1] == want


def test_closed_form_one_dimensional_distance():
    """c_ij = |a_i - b_j|: matching both sorted sequences in order is optimal."""
    g = np.random.default_rng(4)
    for n in (3, 25, 90):
        a = g.integers(-500, 500, n)
        b = g.integers(-500, 500, n)
        c = np.abs(a[:, None] - b[None, :]).astype(np.int32)
        want = int(np.abs(np.sort(a) - np.sort(b)).sum())
        assert oracle.assign(c)[1] == want
        assert oracle.cost_scaling(c)[1] == want


def test_closed_form_identity_dominant():
    g = np.random.default_rng(6)
    n = 40
    c = g.integers(1, 100, (n, n)).astype(np.int32)
    np.fill_diagonal(c, 0)
    r2c, tot = oracle.assign(c)
    assert tot == 0 and np.array_equal(r2c, np.arange(n))
    assert oracle.cost_scaling(c)[1] == 0


def test_invariances():
    g = np.random.default_rng(8)
    c = synth.assign_random_small(45, 1, lo=-300, hi=300)
    base = oracle.assign(c)[1]
    pr, pc = g.permutation(45), g.permutation(45)
    assert oracle.assign(c[pr][:, pc])[1] == base
    r = g.integers(-50, 50, 45)
    k = g.integers(-50, 50, 45)
    shifted = (c + r[:, None] + k[None, :]).astype(np.int32)
    assert oracle.assign(shifted)[1] == base + int(r.sum() + k.sum())
    assert oracle.cost_scaling(shifted)[1] == base + int(r.sum() + k.sum())


@pytest.mark.parametrize("alpha", [2, 8, 10, 16])
def test_cost_scaling_alpha_and_warm_start(alpha):
    """Refine recomputes row prices, so any column prices (including garbage)
    and any alpha still reach the optimum."""
    g = np.random.default_rng(alpha)
    c = synth.assign_points(120, seed=9, instance=2)
    want = oracle.assign(c)[1]
    for init in (None, g.integers(-10**7, 10**7, 120)):
        r2c, tot, prices, _ = oracle.cost_scaling(c, alpha=alpha,
                                                  init_col_prices=init)
        assert tot == want
        assert scaled_eps_certificate(c, r2c, prices)


def test_cost_scaling_small_eps0():
    c = synth.assign_random_small(30, 2)
    want = oracle.assign(c)[1]
    for eps0 in (1, 2, 9, 100):
        assert oracle.cost_scaling(c, eps0=eps0)[1] == want


def test_certificate_rejects_suboptimal():
    """The checker itself must reject a non-optimal matching."""
    c = synth.assign_random_small(12, 4, lo=0, hi=100)
    r2c, tot, prices, _ = oracle.cost_scaling(c)
    bad = r2c.copy()
    bad[[0, 1]] = bad[[1, 0]]
    if int(c[np.arange(12), bad].sum()) > tot:
        assert not scaled_eps_certificate(c, bad, prices)


def _sparse_bruteforce(n, row_ptr, col, cost, maximize):
    """Every permutation that uses listed arcs only, each pair at the best of
    its parallel arcs; None when there is none."""
    import itertools
    best_arc = {}
    for x in range(n):
        for k in range(row_ptr[x], row_ptr[x + 1]):
            y, c = int(col[k]), int(cost[k])
            key = (x, y)
            if key not in best_arc or (c > best_arc[key] if maximize else c < best_arc[key]):
                best_arc[key] = c
    best = None
    for p in itertools.permutations(range(n)):
        if all((x, p[x]) in best_arc for x in range(n)):
            t = sum(best_arc[(x, p[x])] for x in range(n))
            if best is None or (t > best if maximize else t < best):
                best = t
    return best


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_sparse_oracle_bruteforce(n):
    """Section 3's problem on listed arcs: the oracle against every
    permutation, with parallel arcs, with and without a planted perfect
    matching (so that some instances have none), both senses."""
    infeasible = 0
    for seed in range(12):
        planted = seed % 3 != 0
        inst = synth.assign_sparse(n, 1 + seed % 3, seed=seed, lo=-40, hi=40,
                                   planted=planted, parallel=0.3)
        for maximize in (False, True):
            want = _sparse_bruteforce(n, *inst, maximize)
            got = oracle.assign_sparse(n, *inst, maximize=maximize)
            if want is None:
                assert got is None
                infeasible += 1
            else:
                r2c, tot = got
                assert tot == want
                assert sorted(r2c.tolist()) == list(range(n))
    if n >= 3:
        assert infeasible > 0  # the no-matching branch is exercised


def test_sparse_oracle_complete_graph_is_dense():
    """Listing every arc of the complete graph gives the dense problem."""
    for n, seed in ((7, 1), (40, 2)):
        c = synth.assign_random_small(n, seed, lo=-500, hi=500)
        row_ptr = (np.arange(n + 1) * n).astype(np.int32)
        col = np.tile(np.arange(n), n).astype(np.int32)
        for maximize in (False, True):
            _, tot = oracle.assign_sparse(n, row_ptr, col, c.ravel(), maximize)
            assert tot == oracle.assign(c, maximize)[1]
