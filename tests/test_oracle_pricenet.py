"""Pins for the float64 price-network oracle (CPU only).

The network is this project's addition, so its oracle is pinned by
properties: central finite differences of the loss, exact column
equivariance / row invariance, closed-form features of a constant matrix,
library routines for order statistics and deviations, shift invariance of
the loss, and torch's own bfloat16 rounding.
"""
import heapq
import math
import statistics

import numpy as np
import pytest

import synth
from oracle import brute
from oracle import pricenet as P


def _batch(seed, sizes):
    feats = [P.features(synth.assign_random_small(n, seed + n, lo=0, hi=60))[0]
             for n in sizes]
    g = np.random.default_rng(seed)
    targets = [g.normal(0, 1, n) for n in sizes]
    targets = [t - t.mean() for t in targets]
    return feats, targets


def test_param_layout():
    assert P.param_count() == 70145
    theta = P.init_params(0)
    parts = P.unpack(theta)
    assert [p.shape for p in parts] == [s for _, s in P.param_shapes()]


def test_finite_differences():
    feats, targets = _batch(3, [5, 9])
    theta = P.init_params(1).astype(np.float64)
    g = np.random.default_rng(2)
    theta += g.normal(0, 0.05, theta.shape)   # move off the init symmetry
    L, grad = P.loss_and_grad(theta, feats, targets)
    assert L > 0
    idx = np.concatenate([g.choice(len(theta), 60, replace=False),
                          [70016, 70144, 4096, 69888]])
    h = 1e-6

    def relu_pattern(th):
        # which pre-activations are positive: the loss is smooth in theta
        # only where this pattern does not change
        _, caches = P.forward(th, feats)
        return [Z > 0 for cache, _ in caches for _, Z in cache]

    checked = 0
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        if any((a != b).any() for a, b in zip(relu_pattern(tp), relu_pattern(tm))):
            continue   # a ReLU kink inside [-h, h]: no derivative to compare
        fd = (P.loss_and_grad(tp, feats, targets)[0] -
              P.loss_and_grad(tm, feats, targets)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, grad[i])
        checked += 1
    assert checked >= len(idx) - 4


def test_equivariance_and_invariance():
    c = synth.assign_points(40, seed=1, instance=3)
    f, sc = P.features(c)
    g = np.random.default_rng(0)
    pc = g.permutation(40)
    pr = g.permutation(40)
    fc, _ = P.features(c[:, pc])
    np.testing.assert_allclose(fc, f[pc], rtol=1e-12, atol=1e-12)
    fr, _ = P.features(c[pr])
    np.testing.assert_allclose(fr, f, rtol=1e-12, atol=1e-12)
    theta = P.init_params(4)
    q = P.forward(theta, [f])[0][0]
    qc = P.forward(theta, [fc])[0][0]
    np.testing.assert_allclose(qc, q[pc], rtol=1e-10, atol=1e-10)


def test_constant_matrix_features():
    n = 12
    f, sc = P.features(np.full((n, n), 7))
    assert sc == 7
    np.testing.assert_allclose(f[:, :9], 1.0)
    np.testing.assert_allclose(f[:, 9:15], 0.0, atol=1e-12)
    np.testing.assert_allclose(f[:, 15], math.log(n) / 6)


def test_features_against_library_routines():
    c = synth.assign_random_small(23, 9, lo=-40, hi=90)
    f, sc = P.features(c)
    z = c / np.abs(c).mean()
    rr = z - z.min(axis=1, keepdims=True)
    for y in (0, 5, 22):
        col = [float(v) for v in z[:, y]]
        np.testing.assert_allclose(f[y, :8], heapq.nsmallest(8, col))
        assert math.isclose(f[y, 8], math.fsum(col) / len(col))
        assert math.isclose(f[y, 9], statistics.pstdev(col), rel_tol=1e-9)
        rcol = [float(v) for v in rr[:, y]]
        np.testing.assert_allclose(f[y, 10:12], heapq.nsmallest(2, rcol))
    # the two alternating min passes of f13 by explicit loops
    n = 23
    v1 = [min(rr[x, y] for x in range(n)) for y in range(n)]
    u2 = [min(z[x, y] - v1[y] for y in range(n)) for x in range(n)]
    v2 = np.array([min(z[x, y] - u2[x] for x in range(n)) for y in range(n)])
    np.testing.assert_allclose(f[:, 13], v2 - v2.mean(), atol=1e-12)


def test_sinkhorn_feature_on_additive_costs():
    """Costs c(x,y) = a(x) + b(y): every update keeps f = a/sc + const and
    g = b/sc + const whatever the temperature (the exponent separates), so
    f14 is the centred b/sc exactly.  A swapped orientation, a sign or a
    dropped term shows up here."""
    g = np.random.default_rng(11)
    for n in (1, 2, 7, 40):
        a = g.integers(-30, 60, n)
        b = g.integers(0, 90, n)
        c = a[:, None] + b[None, :]
        f, sc = P.features(c)
        np.testing.assert_allclose(f[:, 14], (b - b.mean()) / sc, atol=1e-9)
        fr, fc, _ = P.sinkhorn_potentials(c / sc)
        np.testing.assert_allclose(fr - fr.mean(), (a - a.mean()) / sc, atol=1e-9)


def test_sinkhorn_potentials_reach_the_assignment_dual():
    """LP duality: for potentials with z - f - g >= 0 everywhere (which every
    column update leaves), sum f + sum g is at most the optimal assignment
    cost, and as the temperature falls it must reach it, to within
    n tau log n.  The optimum is taken by exhaustive permutations."""
    for seed in range(6):
        c = synth.assign_random_small(seed % 5 + 3, seed, lo=0, hi=60)
        n = c.shape[0]
        sc = np.abs(c).mean()
        z = c / sc
        opt = brute.assign_bruteforce(c)[0] / sc
        for tau_min, iters in ((1e-4, 150), (1e-6, 200)):
            f, g, last = P.sinkhorn_potentials(z, tau0=1.0, rate=0.8, tau_min=tau_min,
                                               iters=iters)
            assert last == tau_min
            assert (z - f[:, None] - g[None, :]).min() >= -1e-12
            gap = opt - (f.sum() + g.sum())
            assert -1e-9 <= gap <= n * tau_min * math.log(max(n, 2)) + 1e-9, (seed, gap)


def test_loss_shift_invariance():
    feats, targets = _batch(5, [7, 11])
    theta = P.init_params(2).astype(np.float64)
    L0, _ = P.loss_and_grad(theta, feats, targets)
    L1, _ = P.loss_and_grad(theta, feats, [t + 3.0 for t in targets])
    theta2 = theta.copy(); theta2[-1] += 5.0     # output bias
    L2, _ = P.loss_and_grad(theta2, feats, targets)
    assert math.isclose(L0, L1, rel_tol=1e-12) and math.isclose(L0, L2, rel_tol=1e-12)
    q = P.predict_q(theta, feats)
    Lz, _ = P.loss_and_grad(theta, feats, [qq - qq.mean() for qq in q])
    assert Lz < 1e-20
    # the skip term is the feature f14: a zero network predicts it alone
    zero = np.zeros_like(theta)
    for qq, X in zip(P.predict_q(zero, feats), feats):
        np.testing.assert_array_equal(qq, X[:, 14])


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).normal(0, 3, 1000).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(P.bf16_round(x), ref)


def _one_hot_net(feature, sign_in=1.0, sign_out=1.0):
    """Parameters of a network whose output is sign_out * relu(sign_in *
    f_feature): unit 0 of every layer carries the feature, every other
    weight is 0 (all values exact in bf16)."""
    theta = np.zeros(P.param_count(), np.float32)
    parts = P.unpack(theta.astype(np.float64))
    offs, off = [], 0
    for p in parts:
        offs.append(off)
        off += p.size
    W1 = offs[0]
    theta[W1 + feature * P.WIDTH + 0] = sign_in
    for l in (1, 2):
        theta[offs[3 * l] + 0] = 1.0      # W_l[0, 0]
    theta[offs[9] + 0] = sign_out         # w_o[0]
    return theta


def _exact_round(fr):
    """Round a Fraction half to even."""
    from fractions import Fraction
    fl = fr.numerator // fr.denominator
    rem = fr - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return fl


def test_predict_prices_closed_forms():
    """Start prices of hand-set networks against closed forms in exact
    rational arithmetic, on additive costs c(x,y) = a(x) + b(y), where the
    skip term f14 is the centred b / sc exactly: a zero head gives
    p(y) = round((b(y) - mean b) (2n+1)) whatever the bias; a network
    passing the column mean of z = c / sc (centred, also (b - mean b) / sc)
    doubles it; maximising negates the costs, and the same network read
    through -f gives the negated closed form; a network reading another
    feature (the column std, constant here) gives the skip term alone."""
    from fractions import Fraction
    g = np.random.default_rng(5)
    n = 13
    a = g.integers(0, 200, n)
    b = g.integers(0, 200, n)
    c = (a[:, None] + b[None, :]).astype(np.int64)
    tb = int(b.sum())

    def closed(mult):
        return np.array([_exact_round(Fraction(mult * (n * int(v) - tb) * (2 * n + 1), n))
                         for v in b], np.int64)

    theta = P.init_params(3)
    theta[-129:-1] = 0.0                  # w_o = 0
    theta[-1] = 7.25                      # b_o
    np.testing.assert_array_equal(P.predict_prices(theta, c), closed(1))
    want = closed(2)
    np.testing.assert_array_equal(P.predict_prices(_one_hot_net(8), c), want)
    # maximise: z = -c / sc, f8 = -colmean / sc; relu(-f8) then a head of -1
    got = P.predict_prices(_one_hot_net(8, -1.0, -1.0), c, maximize=True)
    np.testing.assert_array_equal(got, closed(-2))
    # a different feature index would be caught: f9 (column std) is constant
    np.testing.assert_array_equal(P.predict_prices(_one_hot_net(9), c), closed(1))
    assert not np.array_equal(P.predict_prices(_one_hot_net(9), c), want)


def test_start_epsilon_closed_form():
    c = np.full((10, 10), 7)
    assert P.start_epsilon(c, 1.0) == 7 * 21
    assert P.start_epsilon(c, 0.5) == 74          # 73.5 rounds to even 74
    assert P.start_epsilon(c, 1e-9) == 1
    assert P.start_epsilon(-c, 2.0, maximize=True) == 2 * 7 * 21
