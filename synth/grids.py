"""Seeded 4-connected grid max-flow instances (int32, row-major, SoA).

A grid instance has H*W pixel nodes plus a source s and a sink t.  Per pixel
p = i*W + j there is one terminal capacity towards s (``cap_src``: arc s->p)
and one towards t (``cap_snk``: arc p->t), and four directional neighbour
capacities: ``cap_right`` (p->p+1), ``cap_left`` (p->p-1), ``cap_down``
(p->p+W), ``cap_up`` (p->p-W).  Entries whose arc would leave the grid are 0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

CONFIG_GRID_UNIFORM = 1
CONFIG_GRID_BLOBS = 2
CONFIG_GRID_BATCH = 3


@dataclass
class GridInstance:
    H: int
    W: int
    cap_src: np.ndarray
    cap_snk: np.ndarray
    cap_right: np.ndarray
    cap_left: np.ndarray
    cap_down: np.ndarray
    cap_up: np.ndarray
    name: str = ""

    @property
    def n_pixels(self) -> int:
        return self.H * self.W

    def arrays(self):
        """The six capacity arrays in library argument order."""
        return (self.cap_src, self.cap_snk, self.cap_right, self.cap_left,
                self.cap_down, self.cap_up)


def _rng(config_id: int, instance_id: int, seed: int, *extra: int):
    return np.random.default_rng(
        np.random.SeedSequence([config_id, instance_id, seed, *extra]))


def grid_from_pairs(H, W, cap_src, cap_snk, horiz_fwd, horiz_bwd,
                    vert_fwd, vert_bwd, name="") -> GridInstance:
    """Lay out pair capacities as the four directional SoA arrays.

    horiz_fwd[i, j] is the capacity of (i,j)->(i,j+1), horiz_bwd[i, j] that
    of (i,j+1)->(i,j); shapes (H, W-1).  vert_* likewise with shape (H-1, W)
    for (i,j)->(i+1,j) and back.
    """
    r = np.zeros((H, W), np.int32)
    l = np.zeros((H, W), np.int32)
    d = np.zeros((H, W), np.int32)
    u = np.zeros((H, W), np.int32)
    if W > 1:
        r[:, :-1] = horiz_fwd
        l[:, 1:] = horiz_bwd
    if H > 1:
        d[:-1, :] = vert_fwd
        u[1:, :] = vert_bwd
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.int32).reshape(-1))
    return GridInstance(H, W, f(cap_src), f(cap_snk), f(r), f(l), f(d), f(u),
                        name)


def grid_uniform(H: int = 64, W: int = 64, seed: int = 0,
                 instance: int = 0) -> GridInstance:
    """Uniform random grid: per-pixel t ~ U{-100..100}; t>0 is a source arc
    of capacity t, otherwise a sink arc of capacity -t; each neighbour pair
    gets one capacity ~ U{0..50}, the same in both directions.  Draw order:
    t (H,W), horizontal pairs (H,W-1), vertical pairs (H-1,W)."""
    g = _rng(CONFIG_GRID_UNIFORM, instance, seed)
    t = g.integers(-100, 101, (H, W))
    hp = g.integers(0, 51, (H, W - 1))
    vp = g.integers(0, 51, (H - 1, W))
    src = np.where(t > 0, t, 0)
    snk = np.where(t > 0, 0, -t)
    return grid_from_pairs(H, W, src, snk, hp, hp, vp, vp,
                           name=f"uniform{H}x{W}/s{seed}/i{instance}")


def blob_image(H: int, W: int, g: np.random.Generator,
               n_blobs: int = 32) -> np.ndarray:
    """Sum of Gaussian blobs, min-max normalised, plus N(0, 0.1^2) noise,
    clipped to [0, 1].  Draw order: centres (n,2) in [0,H)x[0,W), sigma
    fractions U[0.03,0.15) of min(H,W), amplitudes U[0.5,1), signs, noise."""
    cen = g.random((n_blobs, 2)) * np.array([H, W], np.float64)
    sig = g.uniform(0.03, 0.15, n_blobs) * min(H, W)
    amp = g.uniform(0.5, 1.0, n_blobs)
    sign = np.where(g.random(n_blobs) < 0.5, -1.0, 1.0)
    noise = g.normal(0.0, 0.1, (H, W))
    ys = np.arange(H, dtype=np.float64)
    xs = np.arange(W, dtype=np.float64)
    img = np.zeros((H, W), np.float64)
    for k in range(n_blobs):
        gy = np.exp(-((ys - cen[k, 0]) ** 2) / (2.0 * sig[k] ** 2))
        gx = np.exp(-((xs - cen[k, 1]) ** 2) / (2.0 * sig[k] ** 2))
        img += (amp[k] * sign[k]) * np.outer(gy, gx)
    lo, hi = img.min(), img.max()
    img = (img - lo) / (hi - lo) if hi > lo else np.zeros_like(img)
    return np.clip(img + noise, 0.0, 1.0)


def grid_blobs(H: int = 1024, W: int = 1024, seed: int = 0,
               instance: int = 0, pair_scale: float = 50.0,
               config_id: int = CONFIG_GRID_BLOBS) -> GridInstance:
    """Graph-cut grid from a blob image I: terminal k = rint(100|I-0.5|), a
    source arc if I > 0.5 else a sink arc; symmetric pair weight
    rint(pair_scale * exp(-dI^2 / (2 * 0.05^2)))."""
    g = _rng(config_id, instance, seed)
    img = blob_image(H, W, g)
    k = np.rint(100.0 * np.abs(img - 0.5)).astype(np.int64)
    src = np.where(img > 0.5, k, 0)
    snk = np.where(img > 0.5, 0, k)
    w = lambda d: np.rint(pair_scale * np.exp(-(d * d) / (2.0 * 0.05 ** 2)))
    hp = w(img[:, 1:] - img[:, :-1]).astype(np.int64)
    vp = w(img[1:, :] - img[:-1, :]).astype(np.int64)
    return grid_from_pairs(H, W, src, snk, hp, hp, vp, vp,
                           name=f"blobs{H}x{W}x{pair_scale:g}/s{seed}/i{instance}")


def grid_batch(seed: int = 0, n_small: int = 64, lo: int = 128, hi: int = 512,
               big: int = 2048, big_pair_scale: float = 200.0,
               include_big: bool = True):
    """Batched graph cuts: n_small blob grids with H, W ~ U{lo..hi}, plus one
    big x big blob grid whose pair weights are scaled x4 (pair scale 200).
    Sizes are drawn from instance slot 0; grid k uses instance slot k+1."""
    g = _rng(CONFIG_GRID_BATCH, 0, seed)
    hw = g.integers(lo, hi + 1, (n_small, 2))
    out = [grid_blobs(int(h), int(w), seed=seed, instance=k + 1,
                      config_id=CONFIG_GRID_BATCH)
           for k, (h, w) in enumerate(hw)]
    if include_big:
        out.append(grid_blobs(big, big, seed=seed, instance=n_small + 1,
                              pair_scale=big_pair_scale,
                              config_id=CONFIG_GRID_BATCH))
    return out


def grid_random_small(H: int, W: int, seed: int, max_cap: int = 20,
                      max_term: int = 30, both_terminals: bool = True,
                      density: float = 0.8) -> GridInstance:
    """Small general grid for pins and edge cases: independent directional
    capacities (asymmetric), optional both terminals per pixel, and zeroed
    arcs with probability 1-density."""
    g = np.random.default_rng(np.random.SeedSequence([900, H, W, seed]))
    def caps(shape, hi):
        c = g.integers(0, hi + 1, shape)
        return np.where(g.random(shape) < density, c, 0)
    src = caps((H, W), max_term)
    snk = caps((H, W), max_term)
    if not both_terminals:
        keep_src = g.random((H, W)) < 0.5
        src = np.where(keep_src, src, 0)
        snk = np.where(keep_src, 0, snk)
    hf, hb = caps((H, W - 1), max_cap), caps((H, W - 1), max_cap)
    vf, vb = caps((H - 1, W), max_cap), caps((H - 1, W), max_cap)
    return grid_from_pairs(H, W, src, snk, hf, hb, vf, vb,
                           name=f"small{H}x{W}/s{seed}")
