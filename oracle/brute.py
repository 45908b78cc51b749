"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Exhaustive definitions for tiny inputs, used to pin the compiled oracle.

* ``grid_min_cut_bruteforce``: enumerate every source side S of the pixels of
  a grid with at most ~12 pixels; cut(S) = sum_{p not in S} cap_src(p) +
  sum_{p in S} cap_snk(p) + sum_{p in S, q not in S} u(p, q).  The minimum is
  |f*| (max-flow / min-cut, Section 3); the minimal minimum cut is the
  intersection of all minimisers, which must itself be a minimiser (minimum
  cuts form a lattice).
* ``assign_bruteforce``: minimum over all n! permutations.
"""
from __future__ import annotations

import itertools

import numpy as np


def _pair_list(inst):
    H, W = inst.H, inst.W
    pairs = []  # (p, q, u(p,q))
    for i in range(H):
        for j in range(W):
            p = i * W + j
            if j + 1 < W:
                pairs.append((p, p + 1, int(inst.cap_right[p])))
                pairs.append((p + 1, p, int(inst.cap_left[p + 1])))
            if i + 1 < H:
                pairs.append((p, p + W, int(inst.cap_down[p])))
                pairs.append((p + W, p, int(inst.cap_up[p + W])))
    return pairs


def grid_cut_value(inst, side):
    """Capacity of the cut whose source side is {s} u {p : side[p]}."""
    side = np.asarray(side).astype(bool)
    val = int(inst.cap_src[~side].astype(np.int64).sum())
    val += int(inst.cap_snk[side].astype(np.int64).sum())
    for p, q, c in _pair_list(inst):
        if side[p] and not side[q]:
            val += c
    return val


def grid_min_cut_bruteforce(inst):
    """(min cut value, minimal source side) by enumeration of 2^HW sets."""
    HW = inst.H * inst.W
    assert HW <= 14, "brute force is exponential"
    best = None
    minimisers = []
    for mask in range(1 << HW):
        side = np.array([(mask >> p) & 1 for p in range(HW)], bool)
        v = grid_cut_value(inst, side)
        if best is None or v < best:
            best, minimisers = v, [side]
        elif v == best:
            minimisers.append(side)
    inter = np.logical_and.reduce(minimisers)
    assert grid_cut_value(inst, inter) == best, "min cuts must form a lattice"
    return best, inter.astype(np.uint8)


def assign_bruteforce(cost):
    """(minimum total, one optimal permutation) over all n! permutations."""
    cost = np.asarray(cost, np.int64)
    n = cost.shape[0]
    assert n <= 9
    best, arg = None, None
    rows = np.arange(n)
    for perm in itertools.permutations(range(n)):
        v = int(cost[rows, list(perm)].sum())
        if best is None or v < best:
            best, arg = v, perm
    return best, np.array(arg, np.int32)
