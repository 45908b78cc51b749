"""Seeded directed networks as arc lists in mate pairs.

Arc 2k and arc 2k+1 are each other's reverse; cap[2k] is the capacity of the
edge's direction tail[2k] -> head[2k] and cap[2k+1] that of the opposite
direction (0 for a one-way arc).  Only random draws and layout live here.
"""
from __future__ import annotations

import numpy as np

CONFIG_GRAPH_RANDOM = 11
CONFIG_GRAPH_LAYERED = 12
CONFIG_GRAPH_BIPARTITE = 13


def _rng(config_id: int, instance_id: int, seed: int):
    return np.random.default_rng(np.random.SeedSequence([config_id, instance_id, seed]))


def pairs_to_arcs(u, v, cap_uv, cap_vu):
    """Edges (u[k], v[k]) with capacities in both directions -> mate-pair arcs."""
    k = len(u)
    tail = np.empty(2 * k, np.int32)
    head = np.empty(2 * k, np.int32)
    cap = np.empty(2 * k, np.int32)
    tail[0::2], head[0::2], cap[0::2] = u, v, cap_uv
    tail[1::2], head[1::2], cap[1::2] = v, u, cap_vu
    return tail, head, cap


def graph_random(n: int, edges: int, seed: int = 0, instance: int = 0,
                 max_cap: int = 100, two_way: float = 0.3):
    """Uniform random edges over n nodes (self-loops and parallel edges kept);
    a fraction `two_way` also gets a reverse capacity.  s = 0, t = n - 1.
    Returns (n, tail, head, cap, s, t)."""
    g = _rng(CONFIG_GRAPH_RANDOM, instance, seed)
    u = g.integers(0, n, edges)
    v = g.integers(0, n, edges)
    c = g.integers(0, max_cap + 1, edges)
    back = g.random(edges) < two_way
    cr = np.where(back, g.integers(0, max_cap + 1, edges), 0)
    return (n, *pairs_to_arcs(u, v, c, cr), 0, n - 1)


def graph_layered(layers: int, width: int, degree: int, seed: int = 0,
                  instance: int = 0, max_cap: int = 1000):
    """s, `layers` layers of `width` nodes, t: s feeds every node of the
    first layer, every node sends `degree` arcs to random nodes of the next
    layer, the last layer feeds t (long augmenting paths).  One-way arcs.
    Returns (n, tail, head, cap, s, t)."""
    g = _rng(CONFIG_GRAPH_LAYERED, instance, seed)
    n = layers * width + 2
    s, t = 0, n - 1
    us, vs, cs = [], [], []
    first = 1 + np.arange(width)
    us.append(np.full(width, s))
    vs.append(first)
    cs.append(g.integers(1, max_cap + 1, width))
    for l in range(layers - 1):
        src = 1 + l * width + np.repeat(np.arange(width), degree)
        dst = 1 + (l + 1) * width + g.integers(0, width, width * degree)
        us.append(src)
        vs.append(dst)
        cs.append(g.integers(1, max_cap + 1, width * degree))
    last = 1 + (layers - 1) * width + np.arange(width)
    us.append(last)
    vs.append(np.full(width, t))
    cs.append(g.integers(1, max_cap + 1, width))
    u, v, c = (np.concatenate(x) for x in (us, vs, cs))
    return (n, *pairs_to_arcs(u, v, c, np.zeros_like(c)), s, t)


def graph_bipartite(nx: int, ny: int, edges: int, seed: int = 0, instance: int = 0):
    """Unit-capacity matching network: s -> X, X -> Y (random edges), Y -> t.
    The flow value is the size of a maximum matching.
    Returns (n, tail, head, cap, s, t)."""
    g = _rng(CONFIG_GRAPH_BIPARTITE, instance, seed)
    n = nx + ny + 2
    s, t = 0, n - 1
    xs = 1 + np.arange(nx)
    ys = 1 + nx + np.arange(ny)
    eu = 1 + g.integers(0, nx, edges)
    ev = 1 + nx + g.integers(0, ny, edges)
    u = np.concatenate([np.full(nx, s), eu, ys])
    v = np.concatenate([xs, ev, np.full(ny, t)])
    c = np.ones(len(u), np.int64)
    return (n, *pairs_to_arcs(u, v, c, np.zeros_like(c)), s, t)


def grid_to_arcs(inst):
    """A grid instance as a mate-pair arc list: pixels 0..HW-1 (row-major),
    s = HW, t = HW + 1; edges s-p (cap_src, 0), p-t (cap_snk, 0), p-right
    (cap_right[p], cap_left[p+1]) and p-down (cap_down[p], cap_up[p+W]).
    Returns (n, tail, head, cap, s, t)."""
    H, W = inst.H, inst.W
    HW = H * W
    s, t = HW, HW + 1
    pix = np.arange(HW).reshape(H, W)
    us, vs, cf, cb = [], [], [], []
    allp = pix.ravel()
    us += [np.full(HW, s), allp]
    vs += [allp, np.full(HW, t)]
    cf += [inst.cap_src, inst.cap_snk]
    cb += [np.zeros(HW, np.int64), np.zeros(HW, np.int64)]
    if W > 1:
        a = pix[:, :-1].ravel()
        us.append(a)
        vs.append(a + 1)
        cf.append(inst.cap_right[a])
        cb.append(inst.cap_left[a + 1])
    if H > 1:
        a = pix[:-1, :].ravel()
        us.append(a)
        vs.append(a + W)
        cf.append(inst.cap_down[a])
        cb.append(inst.cap_up[a + W])
    u, v, c1, c2 = (np.concatenate(x) for x in (us, vs, cf, cb))
    return (HW + 2, *pairs_to_arcs(u, v, c1, c2), s, t)


CONFIG_GRID_3D = 14
CONFIG_GRID_8 = 15


def _terminals(g, npix, tmax):
    """Terminal arcs drawn as in the 64 x 64 grid workload: t uniform in
    [-tmax, tmax]; t > 0 is a source arc of capacity t, else a sink arc of
    capacity -t."""
    tt = g.integers(-tmax, tmax + 1, npix)
    return np.where(tt > 0, tt, 0), np.where(tt < 0, -tt, 0)


def grid3d_arcs(D: int, H: int, W: int, seed: int = 0, instance: int = 0,
                tmax: int = 100, pmax: int = 50):
    """6-connected D x H x W volume as a mate-pair arc list: voxels
    0..DHW-1 (z-major, then rows), s = DHW, t = DHW + 1; every neighbour
    pair gets one capacity drawn uniformly from [0, pmax], the same in both
    directions.  Returns (n, tail, head, cap, s, t)."""
    g = _rng(CONFIG_GRID_3D, instance, seed)
    N = D * H * W
    s, t = N, N + 1
    vox = np.arange(N).reshape(D, H, W)
    src, snk = _terminals(g, N, tmax)
    us, vs, cs = [np.full(N, s), vox.ravel()], [vox.ravel(), np.full(N, t)], [src, snk]
    backs = [np.zeros(N, np.int64), np.zeros(N, np.int64)]
    for a, b in ((vox[:, :, :-1], vox[:, :, 1:]), (vox[:, :-1, :], vox[:, 1:, :]),
                 (vox[:-1, :, :], vox[1:, :, :])):
        a, b = a.ravel(), b.ravel()
        c = g.integers(0, pmax + 1, len(a))
        us.append(a)
        vs.append(b)
        cs.append(c)
        backs.append(c)
    u, v, c1, c2 = (np.concatenate(x) for x in (us, vs, cs, backs))
    return (N + 2, *pairs_to_arcs(u, v, c1, c2), s, t)


def grid8_arcs(H: int, W: int, seed: int = 0, instance: int = 0,
               tmax: int = 100, pmax: int = 50):
    """8-connected H x W grid (the 4 axis neighbours and the 4 diagonals) as
    a mate-pair arc list: pixels row-major, s = HW, t = HW + 1; every
    neighbour pair gets one capacity drawn uniformly from [0, pmax], the
    same in both directions.  Returns (n, tail, head, cap, s, t)."""
    g = _rng(CONFIG_GRID_8, instance, seed)
    N = H * W
    s, t = N, N + 1
    pix = np.arange(N).reshape(H, W)
    src, snk = _terminals(g, N, tmax)
    us, vs, cs = [np.full(N, s), pix.ravel()], [pix.ravel(), np.full(N, t)], [src, snk]
    backs = [np.zeros(N, np.int64), np.zeros(N, np.int64)]
    for a, b in ((pix[:, :-1], pix[:, 1:]), (pix[:-1, :], pix[1:, :]),
                 (pix[:-1, :-1], pix[1:, 1:]), (pix[:-1, 1:], pix[1:, :-1])):
        a, b = a.ravel(), b.ravel()
        c = g.integers(0, pmax + 1, len(a))
        us.append(a)
        vs.append(b)
        cs.append(c)
        backs.append(c)
    u, v, c1, c2 = (np.concatenate(x) for x in (us, vs, cs, backs))
    return (N + 2, *pairs_to_arcs(u, v, c1, c2), s, t)


CONFIG_MCF_RANDOM = 17
CONFIG_MCF_TRANSPORT = 18


def mcf_random(n: int, edges: int, seed: int = 0, instance: int = 0,
               max_cap: int = 50, max_cost: int = 100, two_way: float = 0.3):
    """Random network with costs and supplies met by a planted flow: uniform
    random edges (self-loops and parallel edges kept), forward capacity
    U{0..max_cap}, a share `two_way` also with a reverse capacity, cost
    U{-max_cost..max_cost} along the edge (its reverse the negative); a flow
    drawn uniformly in [-reverse cap, forward cap] on every edge defines the
    supplies (out-flow minus in-flow), so a feasible flow exists.
    Returns (n, tail, head, cap, cost, supply)."""
    g = _rng(CONFIG_MCF_RANDOM, instance, seed)
    u = g.integers(0, n, edges)
    v = g.integers(0, n, edges)
    c = g.integers(0, max_cap + 1, edges)
    back = g.random(edges) < two_way
    cr = np.where(back, g.integers(0, max_cap + 1, edges), 0)
    w = g.integers(-max_cost, max_cost + 1, edges)
    f = np.floor(g.random(edges) * (c + cr + 1)).astype(np.int64) - cr
    supply = np.zeros(n, np.int64)
    np.add.at(supply, u, f)
    np.add.at(supply, v, -f)
    tail, head, cap = pairs_to_arcs(u, v, c, cr)
    cost = np.empty(2 * edges, np.int32)
    cost[0::2], cost[1::2] = w, -w
    return n, tail, head, cap, cost, supply.astype(np.int32)


def mcf_transport(sources: int, sinks: int, seed: int = 0, instance: int = 0,
                  max_cost: int = 1000, max_supply: int = 100, cap: int = 1 << 20):
    """Transportation problem: every source (nodes 0..sources-1) joined to
    every sink (the rest) by an arc of capacity `cap` and cost
    U{0..max_cost}; source supplies U{1..max_supply}, their total split over
    the sinks uniformly at random as demands.
    Returns (n, tail, head, cap, cost, supply)."""
    g = _rng(CONFIG_MCF_TRANSPORT, instance, seed)
    n = sources + sinks
    s = g.integers(1, max_supply + 1, sources)
    demand = np.bincount(g.integers(0, sinks, int(s.sum())), minlength=sinks)
    supply = np.concatenate([s, -demand]).astype(np.int32)
    u = np.repeat(np.arange(sources), sinks)
    v = sources + np.tile(np.arange(sinks), sources)
    w = g.integers(0, max_cost + 1, len(u))
    tail, head, caps = pairs_to_arcs(u, v, np.full(len(u), cap), np.zeros(len(u), np.int64))
    cost = np.empty(2 * len(u), np.int32)
    cost[0::2], cost[1::2] = w, -w
    return n, tail, head, caps, cost, supply
