"""Seeded dense assignment instances (int32 n x n cost, row-major).

Rows are the set X, columns the set Y of the complete bipartite graph.
"""
from __future__ import annotations

import numpy as np

CONFIG_ASSIGN_UNIFORM = 4
CONFIG_ASSIGN_POINTS = 5
# Extra SeedSequence entropy word that separates training instances (used to
# fit the price network) from evaluation instances of the same generator.
TRAIN_BRANCH = 7919


def _rng(config_id: int, instance_id: int, seed: int, *extra: int):
    return np.random.default_rng(
        np.random.SeedSequence([config_id, instance_id, seed, *extra]))


def assign_uniform(n: int = 1024, seed: int = 0, instance: int = 0,
                   hi: int = 1000) -> np.ndarray:
    """Weights uniform in {0..hi}; solved as a max-weight assignment."""
    g = _rng(CONFIG_ASSIGN_UNIFORM, instance, seed)
    return np.ascontiguousarray(g.integers(0, hi + 1, (n, n)).astype(np.int32))


def assign_points(n: int, seed: int = 0, instance: int = 0,
                  train: bool = False, noise: float = 0.05,
                  scale: float = 1e4) -> np.ndarray:
    """Optical-flow-like costs: P uniform in the unit square, Q = P moved by
    N(0, noise^2) per coordinate then row-permuted; c_ij = rint(scale *
    ||P_i - Q_j||).  Draw order: P (n,2), displacement (n,2), permutation."""
    extra = (TRAIN_BRANCH,) if train else ()
    g = _rng(CONFIG_ASSIGN_POINTS, instance, seed, *extra)
    P = g.random((n, 2))
    Q = P + g.normal(0.0, noise, (n, 2))
    Q = Q[g.permutation(n)]
    d = np.sqrt(((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1))
    return np.ascontiguousarray(np.rint(scale * d).astype(np.int32))


def assign_batch(seed: int = 0, count: int = 256, lo: int = 64, hi: int = 512,
                 train: bool = False):
    """Batched optical-flow-like instances with n ~ U{lo..hi}.  Sizes come from
    instance slot 0; instance k uses slot k+1."""
    extra = (TRAIN_BRANCH,) if train else ()
    g = _rng(CONFIG_ASSIGN_POINTS, 0, seed, *extra)
    ns = g.integers(lo, hi + 1, count)
    return [assign_points(int(n), seed=seed, instance=k + 1, train=train)
            for k, n in enumerate(ns)]


def assign_random_small(n: int, seed: int, lo: int = -50, hi: int = 50):
    """Small general cost matrix for pins (negative entries allowed)."""
    g = np.random.default_rng(np.random.SeedSequence([901, n, seed]))
    return np.ascontiguousarray(g.integers(lo, hi + 1, (n, n)).astype(np.int32))


CONFIG_ASSIGN_SPARSE = 16


def assign_sparse(n: int, degree: int, seed: int = 0, instance: int = 0,
                  lo: int = 0, hi: int = 1000, planted: bool = True,
                  parallel: float = 0.0):
    """Sparse bipartite instance in CSR by row: every row gets `degree`
    uniform random columns (repeats possible) and, with `planted`, the column
    of a random permutation, so that a perfect matching exists; a fraction
    `parallel` of the arcs is listed twice with another cost.  Costs uniform
    in {lo..hi}.  Returns (row_ptr, col, cost), int32."""
    g = _rng(CONFIG_ASSIGN_SPARSE, instance, seed)
    perm = g.permutation(n)
    cols = [g.integers(0, n, (n, degree))]
    if planted:
        cols.append(perm[:, None])
    c = np.concatenate(cols, axis=1) if n else np.zeros((0, 0), np.int64)
    rows = [list(r) for r in c]
    if parallel > 0:
        for r in rows:
            extra = [y for y in r if g.random() < parallel]
            r.extend(extra)
    for r in rows:
        g.shuffle(r)
    deg = np.array([len(r) for r in rows], np.int64)
    row_ptr = np.zeros(n + 1, np.int64)
    row_ptr[1:] = np.cumsum(deg)
    col = np.array([y for r in rows for y in r], np.int64)
    cost = g.integers(lo, hi + 1, len(col))
    return row_ptr.astype(np.int32), col.astype(np.int32), cost.astype(np.int32)
