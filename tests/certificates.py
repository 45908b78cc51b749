"""Independent numpy certificate checks (test helpers).

These restate definitions from Section 3 directly and share no code with the
oracle or the GPU library.
"""
from __future__ import annotations

import numpy as np


def grid_cut_value(inst, side) -> int:
    """Capacity of the s-t cut whose source side is {s} u {p : side[p]}:
    source arcs into T, sink arcs out of S and neighbour arcs from S to T."""
    H, W = inst.H, inst.W
    S = np.asarray(side).astype(bool).reshape(H, W)
    c = lambda a: np.asarray(a, np.int64).reshape(H, W)
    val = int(c(inst.cap_src)[~S].sum()) + int(c(inst.cap_snk)[S].sum())
    if W > 1:
        a, b = S[:, :-1], S[:, 1:]
        val += int(c(inst.cap_right)[:, :-1][a & ~b].sum())
        val += int(c(inst.cap_left)[:, 1:][b & ~a].sum())
    if H > 1:
        a, b = S[:-1, :], S[1:, :]
        val += int(c(inst.cap_down)[:-1, :][a & ~b].sum())
        val += int(c(inst.cap_up)[1:, :][b & ~a].sum())
    return val


def hungarian_duals_ok(cost, row_to_col, u, v) -> bool:
    """u_i + v_j <= c_ij everywhere, equality on the assignment, and
    sum(u) + sum(v) equals the assignment's cost (LP duality)."""
    cost = np.asarray(cost, np.int64)
    n = cost.shape[0]
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    red = cost - u[:, None] - v[None, :]
    if red.min() < 0:
        return False
    if np.any(red[np.arange(n), row_to_col] != 0):
        return False
    return int(u.sum() + v.sum()) == int(cost[np.arange(n), row_to_col].sum())


def is_permutation(row_to_col, n) -> bool:
    r = np.asarray(row_to_col)
    return r.shape == (n,) and np.array_equal(np.sort(r), np.arange(n))


def scaled_eps_certificate(cost_min, row_to_col, col_prices, eps=1) -> bool:
    """Does some row-price vector make every residual arc's reduced cost at
    least -eps, for costs scaled by S = 2n+1 and the given column prices?

    Residual arcs of a perfect matching M: (x,y) for y != M(x), reduced cost
    S*c(x,y) + p(x) - p(y) >= -eps; and (M(x),x), reduced cost
    -S*c(x,M(x)) + p(M(x)) - p(x) >= -eps.  A feasible p(x) exists iff, with
    g(x,y) = p(y) - S*c(x,y), g(x,M(x)) >= max_{y != M(x)} g(x,y) - 2*eps.
    With eps = 1 this certifies optimality: a residual cycle has at most 2n
    arcs, so its scaled cost is > -(2n+1) and, being a multiple of 2n+1,
    non-negative."""
    c = np.asarray(cost_min, np.int64)
    n = c.shape[0]
    S = 2 * n + 1
    g = np.asarray(col_prices, np.int64)[None, :] - S * c
    rows = np.arange(n)
    m = np.asarray(row_to_col)
    gm = g[rows, m].copy()
    g[rows, m] = np.iinfo(np.int64).min
    if n == 1:
        return True
    return bool(np.all(gm >= g.max(axis=1) - 2 * eps))


def scaled_eps_certificate_sparse(n, row_ptr, col, cost_min, row_to_col,
                                  col_prices, eps=1) -> bool:
    """scaled_eps_certificate on a sparse graph: only listed arcs are
    residual arcs (of parallel arcs, the cheapest), so the condition is
    g(x,M(x)) >= max over the row's other listed columns of g(x,y) - 2 eps.
    A residual cycle still has at most 2n arcs, so eps = 1 certifies
    optimality among the perfect matchings of the listed arcs."""
    S = 2 * n + 1
    row_ptr = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int64)
    c = np.asarray(cost_min, np.int64)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    best = np.full((n, n), np.iinfo(np.int64).max, np.int64)
    np.minimum.at(best, (rows, col), c)
    listed = best != np.iinfo(np.int64).max
    m = np.asarray(row_to_col, np.int64)
    r = np.arange(n)
    if not listed[r, m].all():
        return False
    p = np.asarray(col_prices, np.int64)
    g = np.where(listed, p[None, :] - S * np.where(listed, best, 0),
                 np.iinfo(np.int64).min)
    gm = g[r, m].copy()
    g[r, m] = np.iinfo(np.int64).min
    other = g.max(axis=1)
    alone = other == np.iinfo(np.int64).min  # the row lists one column only
    return bool(np.all(alone | (gm >= np.where(alone, 0, other) - 2 * eps)))
