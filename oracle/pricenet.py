"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Float64 reference of the learned warm start for cost scaling: the column
features, the permutation-equivariant price network, its loss and the
gradients.  The paper has no learned component; the definitions below are
the specification the GPU kernels implement, so this module restates them as
plainly as possible (numpy, no batching tricks).

Features of an n x n cost matrix c (minimised), for every column y; all of
them are symmetric functions over the rows x (invariant to row order) and
move with their column (equivariant to column order):
  sc      = mean |c| over the matrix (1 if that is 0); z = c / sc
  rr(x,y) = z(x,y) - min_y' z(x,y')               (row-reduced cost)
  f0..f7  = the 8 smallest z(., y), ascending (the largest repeats if n < 8)
  f8, f9  = mean and (population) standard deviation of z(., y)
  f10,f11 = the 2 smallest rr(., y)
  f12     = mean rr(., y)
  f13     = v2(y) - mean_y v2, where u2(x) = min_y (z(x,y) - f10(y)) and
            v2(y) = min_x (z(x,y) - u2(x))  (two alternating min passes of
            the dual problem started from f10)
  f14     = g(y) - mean_y g: the column potential of the entropic (Sinkhorn)
            dual of the assignment with costs z after SINK_ITERS alternating
            updates at a falling temperature tau_k = max(SINK_TAU_MIN,
            SINK_TAU0 SINK_RATE^k), k = 0, 1, ..., from g = 0:
              f(x) = -tau log sum_y exp(-(z(x,y) - g(y)) / tau)   (rows)
              g(y) = -tau log sum_x exp(-(z(x,y) - f(x)) / tau)   (columns)
            As tau falls, f + g tends to an optimal dual of the assignment
            LP (every column update leaves z - f - g >= 0), which is what
            the network is asked to predict.
  f15     = log(n) / 6

Network (DeepSets-style, equivariant over columns; H0 = features [n, 16]):
  H_l = relu(H_{l-1} W_l + 1 mean_y(H_{l-1}) U_l + 1 b_l),  l = 1, 2, 3
  q   = H_3 w_o + b_o + f14               (normalised price per column)
The last term is a skip connection: the network predicts the correction to
the Sinkhorn potential, so its bf16 rounding falls on the correction and the
potential reaches the prices at full precision.
Widths: 16 -> 128 -> 128 -> 128 -> 1.  Parameter vector layout (float32 on
the device): W1 [16,128], U1 [16,128], b1 [128], W2, U2 [128,128], b2,
W3, U3 [128,128], b3, w_o [128], b_o [1] -- each row-major, concatenated.

Loss over a batch of instances with centred targets t (normalised prices),
q including the skip term (which does not depend on the parameters):
  L = (1 / sum_i n_i) sum_i sum_y ((q_y - mean_i q) - t_y)^2
Scaled integer start prices for the solver: p(y) = rint((q_y - mean q) sc
(2n+1)), and the starting epsilon max(1, rint(kappa sc (2n+1))).
"""
from __future__ import annotations

import numpy as np

F_IN = 16
WIDTH = 128
SINK_TAU0 = 0.3
SINK_RATE = 0.7
SINK_TAU_MIN = 0.003
SINK_ITERS = 16
LAYERS = [(F_IN, WIDTH), (WIDTH, WIDTH), (WIDTH, WIDTH)]


def param_shapes():
    shapes = []
    for (k, m) in LAYERS:
        shapes += [("W", (k, m)), ("U", (k, m)), ("b", (m,))]
    shapes += [("wo", (WIDTH,)), ("bo", (1,))]
    return shapes


def param_count():
    return int(sum(np.prod(s) for _, s in param_shapes()))


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, off = [], 0
    for _, s in param_shapes():
        k = int(np.prod(s))
        out.append(theta[off:off + k].reshape(s))
        off += k
    assert off == len(theta)
    return out


def init_params(seed=0):
    """He-style initialisation (float32 values)."""
    g = np.random.default_rng(np.random.SeedSequence([77, seed]))
    parts = []
    for name, s in param_shapes():
        if name in ("W", "U"):
            parts.append(g.normal(0, np.sqrt(1.0 / s[0]), s).ravel())
        elif name == "wo":
            parts.append(g.normal(0, np.sqrt(1.0 / s[0]), s).ravel())
        else:
            parts.append(np.zeros(s).ravel())
    return np.concatenate(parts).astype(np.float32)


def sinkhorn_potentials(z, tau0=SINK_TAU0, rate=SINK_RATE, tau_min=SINK_TAU_MIN,
                        iters=SINK_ITERS):
    """Row and column potentials (f, g) of the entropic dual of the
    assignment with cost matrix z: `iters` alternating exact updates, each
    a log-sum-exp at temperature tau, computed around its minimum,
        f(x) = -tau log sum_y exp(-(z(x,y) - g(y)) / tau)
        g(y) = -tau log sum_x exp(-(z(x,y) - f(x)) / tau),
    from g = 0, with tau = tau0 first and multiplied by `rate` after every
    iteration down to tau_min.  Returns (f, g, last tau)."""
    z = np.asarray(z, np.float64)
    n = z.shape[0]
    f = np.zeros(n)
    g = np.zeros(n)
    tau = tau0
    last = tau
    for _ in range(iters):
        a = z - g[None, :]
        m = a.min(axis=1)
        f = m - tau * np.log(np.exp(-(a - m[:, None]) / tau).sum(axis=1))
        b = z - f[:, None]
        m = b.min(axis=0)
        g = m - tau * np.log(np.exp(-(b - m[None, :]) / tau).sum(axis=0))
        last = tau
        tau = max(tau_min, tau * rate)
    return f, g, last


def features(cost, maximize=False):
    """[n, 16] float64 features and the cost scale sc (see module doc)."""
    c = np.asarray(cost, np.float64)
    if maximize:
        c = -c
    n = c.shape[0]
    sc = np.abs(c).mean()
    if sc == 0:
        sc = 1.0
    z = c / sc
    rr = z - z.min(axis=1, keepdims=True)
    f = np.zeros((n, F_IN))
    zs = np.sort(z, axis=0)
    rs = np.sort(rr, axis=0)
    for k in range(8):
        f[:, k] = zs[min(k, n - 1)]
    f[:, 8] = z.mean(axis=0)
    f[:, 9] = z.std(axis=0)
    f[:, 10] = rs[0]
    f[:, 11] = rs[min(1, n - 1)]
    f[:, 12] = rr.mean(axis=0)
    u2 = (z - f[:, 10][None, :]).min(axis=1)
    v2 = (z - u2[:, None]).min(axis=0)
    f[:, 13] = v2 - v2.mean()
    _, gs, _ = sinkhorn_potentials(z)
    f[:, 14] = gs - gs.mean()
    f[:, 15] = np.log(n) / 6.0
    return f, sc


def forward(theta, feats_list):
    """Network outputs H_3 w_o + b_o per instance (without the skip term)
    and the cache for backward."""
    P = unpack(theta)
    outs, caches = [], []
    for X in feats_list:
        H = np.asarray(X, np.float64)
        cache = []
        for l in range(3):
            W, U, b = P[3 * l], P[3 * l + 1], P[3 * l + 2]
            Z = H @ W + H.mean(axis=0, keepdims=True) @ U + b[None, :]
            cache.append((H, Z))
            H = np.maximum(Z, 0.0)
        q = H @ P[9] + P[10][0]
        outs.append(q)
        caches.append((cache, H))
    return outs, caches


def _skips(feats_list, skip_list):
    if skip_list is not None:
        return [np.asarray(s, np.float64) for s in skip_list]
    return [np.asarray(X, np.float64)[:, 14] for X in feats_list]


def predict_q(theta, feats_list, skip_list=None):
    """Normalised price prediction per instance: the network output plus
    the skip term f14 (taken from skip_list when given, else from the
    features)."""
    outs = forward(theta, feats_list)[0]
    return [q + sk for q, sk in zip(outs, _skips(feats_list, skip_list))]


def loss_and_grad(theta, feats_list, targets, skip_list=None):
    """Shift-invariant MSE over a batch and its gradient (float64); the
    prediction includes the skip term, which has no parameters."""
    P = unpack(theta)
    outs, caches = forward(theta, feats_list)
    N = sum(len(t) for t in targets)
    L = 0.0
    grads = [np.zeros_like(p) for p in P]
    for q0, sk, t, (cache, H3) in zip(outs, _skips(feats_list, skip_list), targets,
                                      caches):
        q = q0 + sk
        r = (q - q.mean()) - (np.asarray(t, np.float64) - np.mean(t))
        L += (r ** 2).sum() / N
        dq = 2.0 * r / N            # d/dq of the centred residual (sum r = 0)
        grads[9] += H3.T @ dq
        grads[10][0] += dq.sum()
        dH = np.outer(dq, P[9])
        for l in (2, 1, 0):
            W, U = P[3 * l], P[3 * l + 1]
            Hin, Z = cache[l]
            dZ = dH * (Z > 0)
            n = Hin.shape[0]
            grads[3 * l] += Hin.T @ dZ
            grads[3 * l + 1] += np.outer(Hin.mean(axis=0), dZ.sum(axis=0))
            grads[3 * l + 2] += dZ.sum(axis=0)
            dH = dZ @ W.T + np.outer(np.ones(n), dZ.sum(axis=0) @ U.T) / n
    return L, np.concatenate([g.ravel() for g in grads])


def predict_prices(theta, cost, maximize=False):
    """Integer scaled start prices for one instance: the centred prediction
    (network output plus f14) in units of sc, scaled by the solver's cost
    scale S = 2n+1 and rounded half to even."""
    f, sc = features(cost, maximize)
    q = predict_q(theta, [f])[0]
    q = q - q.mean()
    n = f.shape[0]
    return np.rint(q * sc * (2 * n + 1)).astype(np.int64)


def start_epsilon(cost, kappa, maximize=False):
    """Starting epsilon of a warm-started solve, in the solver's scaled
    units: kappa (the network's error in units of sc) times sc (2n+1),
    rounded half to even, at least 1."""
    f, sc = features(cost, maximize)
    n = f.shape[0]
    return max(1, int(np.rint(kappa * sc * (2 * n + 1))))


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
