"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU implementations of what the GPU library
computes.  Only ``tests/``, the smoke check and the benchmark's
``cpu_baseline`` leg may import this package; the product path
(``paper_1110_6231_amd``) never does, and no code is shared between the two
(only the seeded generators in ``synth`` feed both).

Max-flow (Section 3 definitions; Sections 4.1-4.2 algorithms):
  * ``grid_maxflow(inst, method)`` -- |f*| (int64) and the minimal source
    side S_min of a minimum cut, by Edmonds-Karp (``"ek"``) or FIFO
    push-relabel with global and gap relabelling (``"fifo"``), on the explicit
    arc list of the 4-connected grid network.
  * S_min is computed from a maximum preflow as the residual closure of {s}
    together with every node of positive excess: for a preflow f and a cut
    (S,T), u(S,T) >= sum_{v in T} e(v) >= e(t), with equality iff no residual
    arc leaves S and no node of T other than t holds excess; hence the
    minimum cuts are exactly the residual-closed S containing s and all excess
    nodes, and their intersection is that closure.

Assignment (Section 3 definition; Section 5 method):
  * ``hungarian(cost)`` -- O(n^3) Hungarian method with integer duals.
  * ``assign_sparse(n, row_ptr, col, cost)`` -- the same problem on listed
    arcs only (CSR by row): the Hungarian method on the complete matrix with
    missing arcs at a prohibitive cost.
  * ``mincost_flow(n, tail, head, cap, cost, supply)`` -- minimum-cost flow
    with node supplies (the problem Algorithm 5.0 solves) by successive
    shortest paths.
  * ``cost_scaling(cost, ...)`` -- the paper's refine (Algorithm 5.2) with the
    push/relabel operation of Algorithm 5.4, run sequentially in FIFO order.

Pins: see ``tests/test_oracle_*.py`` (brute force, scipy, closed forms,
metamorphic relations, dual certificates).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def _sources_newer(target: str) -> bool:
    if not os.path.exists(target):
        return True
    t = os.path.getmtime(target)
    return any(os.path.getmtime(os.path.join(_HERE, s)) > t
               for s in _build.SOURCES)


def lib():
    """Load (building first if missing or stale) the oracle library."""
    global _lib
    if _lib is None:
        if _sources_newer(_build.TARGET):
            _build.build()
        L = ctypes.CDLL(_build.TARGET)
        L.oracle_maxflow_ek.argtypes = [
            ctypes.c_int, ctypes.c_int, _i32p, _i32p, _i64p, ctypes.c_int,
            ctypes.c_int, ctypes.POINTER(ctypes.c_int64), _u8p]
        L.oracle_maxflow_fifo.argtypes = [
            ctypes.c_int, ctypes.c_int, _i32p, _i32p, _i64p, ctypes.c_int,
            ctypes.c_int, ctypes.POINTER(ctypes.c_int64), _u8p, _i64p]
        L.oracle_hungarian.argtypes = [
            ctypes.c_int, _i32p, _i32p, ctypes.POINTER(ctypes.c_int64),
            _i64p, _i64p]
        L.oracle_cost_scaling.argtypes = [
            ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_void_p,
            ctypes.c_int64, _i32p, ctypes.POINTER(ctypes.c_int64), _i64p,
            _i64p]
        L.oracle_mincost_flow.argtypes = [
            ctypes.c_int, ctypes.c_int, _i32p, _i32p, _i64p, _i64p, _i64p,
            _i64p, ctypes.POINTER(ctypes.c_int64), _i64p]
        for f in (L.oracle_maxflow_ek, L.oracle_maxflow_fifo,
                  L.oracle_hungarian, L.oracle_cost_scaling,
                  L.oracle_mincost_flow):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# Max-flow
# --------------------------------------------------------------------------
def graph_maxflow(n, tail, head, cap, s, t, method="fifo"):
    """Max-flow on an explicit arc list in mate pairs (arc a^1 reverses a).

    Returns (value, source_side uint8[n], stats or None)."""
    tail = np.ascontiguousarray(tail, np.int32)
    head = np.ascontiguousarray(head, np.int32)
    cap = np.ascontiguousarray(cap, np.int64)
    m = len(tail)
    val = ctypes.c_int64(0)
    side = np.zeros(n, np.uint8)
    if method == "ek":
        rc = lib().oracle_maxflow_ek(n, m, tail, head, cap, s, t,
                                     ctypes.byref(val), side)
        stats = None
    elif method == "fifo":
        stats = np.zeros(3, np.int64)
        rc = lib().oracle_maxflow_fifo(n, m, tail, head, cap, s, t,
                                       ctypes.byref(val), side, stats)
    else:
        raise ValueError(method)
    if rc != 0:
        raise ValueError(f"oracle max-flow rejected its input (rc={rc})")
    return int(val.value), side, stats


def grid_arcs(inst):
    """Explicit arc list (mate pairs) of a grid network.

    Nodes: pixels 0..HW-1, s = HW, t = HW+1.  Pairs: (s->p, p->s) with
    capacities (cap_src, 0); (p->t, t->p) with (cap_snk, 0); (p->p+1,
    p+1->p) with (cap_right[p], cap_left[p+1]); (p->p+W, p+W->p) with
    (cap_down[p], cap_up[p+W])."""
    H, W = inst.H, inst.W
    HW = H * W
    s, t = HW, HW + 1
    pix = np.arange(HW, dtype=np.int64).reshape(H, W)
    tails, heads, caps = [], [], []

    def add(a, b, cab, cba):
        a = np.asarray(a, np.int64).ravel()
        b = np.asarray(b, np.int64).ravel()
        k = len(a)
        tt = np.empty(2 * k, np.int64)
        hh = np.empty(2 * k, np.int64)
        cc = np.empty(2 * k, np.int64)
        tt[0::2], tt[1::2] = a, b
        hh[0::2], hh[1::2] = b, a
        cc[0::2] = np.asarray(cab, np.int64).ravel()
        cc[1::2] = np.asarray(cba, np.int64).ravel()
        tails.append(tt)
        heads.append(hh)
        caps.append(cc)

    allp = pix.ravel()
    add(np.full(HW, s), allp, inst.cap_src, np.zeros(HW))
    add(allp, np.full(HW, t), inst.cap_snk, np.zeros(HW))
    if W > 1:
        a = pix[:, :-1].ravel()
        add(a, a + 1, inst.cap_right[a], inst.cap_left[a + 1])
    if H > 1:
        a = pix[:-1, :].ravel()
        add(a, a + W, inst.cap_down[a], inst.cap_up[a + W])
    return (HW + 2, np.concatenate(tails), np.concatenate(heads),
            np.concatenate(caps), s, t)


def grid_maxflow(inst, method="fifo", with_stats=False):
    """|f*| and S_min (uint8 per pixel, 1 = source side) of a grid network."""
    n, tail, head, cap, s, t = grid_arcs(inst)
    val, side, stats = graph_maxflow(n, tail, head, cap, s, t, method)
    assert side[s] == 1 and side[t] == 0
    out = (val, side[: inst.H * inst.W].copy())
    return out + (stats,) if with_stats else out


# --------------------------------------------------------------------------
# Assignment
# --------------------------------------------------------------------------
def hungarian(cost):
    """Min-cost perfect matching: (row_to_col int32[n], total int, u, v)."""
    cost = np.ascontiguousarray(cost, np.int32)
    n = cost.shape[0]
    assert cost.shape == (n, n)
    r2c = np.zeros(n, np.int32)
    tot = ctypes.c_int64(0)
    u = np.zeros(n, np.int64)
    v = np.zeros(n, np.int64)
    rc = lib().oracle_hungarian(n, cost, r2c, ctypes.byref(tot), u, v)
    if rc != 0:
        raise ValueError("oracle hungarian rejected its input")
    return r2c, int(tot.value), u, v


def _oriented(cost, maximize):
    cost = np.asarray(cost)
    if maximize:
        return np.ascontiguousarray(-cost.astype(np.int64)).astype(np.int32)
    return np.ascontiguousarray(cost, np.int32)


def assign(cost, maximize=False):
    """Optimal assignment: (row_to_col, total of the given entries).  For
    maximize=True the weights are negated and minimised (Section 3 states
    the problem as maximum weight)."""
    r2c, tot, _, _ = hungarian(_oriented(cost, maximize))
    return r2c, (-tot if maximize else tot)


def mincost_flow(n, tail, head, cap, cost, supply):
    """Minimum-cost flow meeting node supplies on mate-pair arcs (arc a^1
    reverses a, cost[a^1] = -cost[a]) by successive shortest paths.

    Returns (total cost, residual capacities int64[m], potentials int64[n])
    or None when no flow meets the supplies."""
    tail = np.ascontiguousarray(tail, np.int32)
    head = np.ascontiguousarray(head, np.int32)
    cap = np.ascontiguousarray(cap, np.int64)
    cost = np.ascontiguousarray(cost, np.int64)
    supply = np.ascontiguousarray(supply, np.int64)
    m = len(tail)
    res = np.zeros(max(m, 1), np.int64)
    pi = np.zeros(n, np.int64)
    tot = ctypes.c_int64(0)
    rc = lib().oracle_mincost_flow(n, m, tail, head, cap, cost, supply, res,
                                   ctypes.byref(tot), pi)
    if rc < 0:
        raise ValueError("oracle min-cost flow rejected its input")
    if rc == 1:
        return None
    return int(tot.value), res[:m], pi


def assign_sparse(n, row_ptr, col, cost, maximize=False):
    """Optimal assignment on a sparse bipartite graph given in CSR by row
    (Section 3's problem restricted to the listed arcs; of parallel arcs the
    best one counts).  Returns (row_to_col, total) or None when no perfect
    matching exists.

    By definition: the complete matrix with every missing arc at a cost M
    larger than n times the spread of the real costs, so that any perfect
    matching of real arcs is cheaper than every assignment using an M arc;
    the Hungarian method then finds the optimum, which uses an M arc exactly
    when no perfect matching of real arcs exists."""
    row_ptr = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int64)
    w = np.asarray(cost, np.int64)
    c = -w if maximize else w
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    spread = int(c.max() - c.min()) if len(c) else 0
    big = int(c.max() if len(c) else 0) + n * (spread + 1) + 1
    dense = np.full((n, n), big, np.int64)
    np.minimum.at(dense, (rows, col), c)
    real = np.zeros((n, n), bool)
    real[rows, col] = True
    assert big < 2**31, "costs too large for the int32 Hungarian oracle"
    r2c, _, _, _ = hungarian(dense)
    if not real[np.arange(n), r2c].all():
        return None
    tot = int(dense[np.arange(n), r2c].sum())
    return r2c, (-tot if maximize else tot)


def cost_scaling(cost, maximize=False, alpha=8, init_col_prices=None,
                 eps0=0):
    """Sequential cost scaling (Algorithms 5.0/5.2/5.4) on scaled costs.

    Returns (row_to_col, total, col_prices (scaled, of the minimised cost),
    stats [pushes, relabels, refines])."""
    c = _oriented(cost, maximize)
    n = c.shape[0]
    r2c = np.zeros(n, np.int32)
    tot = ctypes.c_int64(0)
    prices = np.zeros(n, np.int64)
    stats = np.zeros(3, np.int64)
    ip = None
    if init_col_prices is not None:
        ipa = np.ascontiguousarray(init_col_prices, np.int64)
        ip = ipa.ctypes.data_as(ctypes.c_void_p)
    rc = lib().oracle_cost_scaling(n, c, alpha, ip, int(eps0), r2c,
                                   ctypes.byref(tot), prices, stats)
    if rc != 0:
        raise ValueError("oracle cost scaling rejected its input")
    total = int(tot.value)
    return r2c, (-total if maximize else total), prices, stats
