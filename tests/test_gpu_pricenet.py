"""GPU checks of the price network: features against the float64 oracle,
forward and gradient against the oracle fed the same BF16-rounded inputs and
weights (forward tolerance set by the bf16 mantissa, 2^-8; the gradient's by
the error bf16 operand rounding alone causes in float64), training reduces
the loss, and warm-started solves stay exact."""
import numpy as np
import pytest

import oracle
import synth
from certificates import is_permutation, scaled_eps_certificate
from oracle import pricenet as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1110_6231_amd import lpr  # noqa: E402


def _packed(mats):
    return lpr.PackedAssign.from_matrices(mats)


def _cpu_inputs(theta32, feats_gpu, offs):
    """The oracle's view of what the GPU multiplies: bf16 features, bf16 W;
    U, biases and the head stay float32."""
    th = theta32.astype(np.float64).copy()
    for off, size in ((0, 2048), (4224, 16384), (37120, 16384)):
        th[off:off + size] = P.bf16_round(theta32[off:off + size])
    fb = P.bf16_round(feats_gpu)
    return th, [fb[offs[k]:offs[k + 1]] for k in range(len(offs) - 1)]


def _skips(feats_gpu, offs):
    """The skip term as the GPU adds it: its own float32 f14, not rounded."""
    f = np.asarray(feats_gpu, np.float64)
    return [f[offs[k]:offs[k + 1], 14] for k in range(len(offs) - 1)]


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _loss_and_grad_bf16_operands(theta, feats_list, targets, skips):
    """The oracle's loss and gradient with the hidden activations and the
    back-propagated pre-activation gradients rounded to bf16 where they enter
    a product, as the GPU's BF16 GEMM operands are: the error this rounding
    alone causes sets the scale of the gradient comparison (it grows when the
    residual's contributions cancel)."""
    B = P.bf16_round
    Pp = P.unpack(theta)
    N = sum(len(t) for t in targets)
    grads = [np.zeros_like(x) for x in Pp]
    for X, t, sk in zip(feats_list, targets, skips):
        H = B(X)
        cache = []
        for l in range(3):
            W, U, b = Pp[3 * l], Pp[3 * l + 1], Pp[3 * l + 2]
            Z = H @ W + H.mean(axis=0, keepdims=True) @ U + b[None, :]
            cache.append((H, Z))
            H = B(np.maximum(Z, 0.0))
        q = H @ Pp[9] + Pp[10][0] + sk
        r = (q - q.mean()) - (np.asarray(t, np.float64) - np.mean(t))
        dq = 2.0 * r / N
        grads[9] += H.T @ dq
        grads[10][0] += dq.sum()
        dH = np.outer(dq, Pp[9])
        for l in (2, 1, 0):
            W, U = Pp[3 * l], Pp[3 * l + 1]
            Hin, Z = cache[l]
            dZ = dH * (Z > 0)
            n = Hin.shape[0]
            grads[3 * l] += Hin.T @ B(dZ)
            grads[3 * l + 1] += np.outer(Hin.mean(axis=0), dZ.sum(axis=0))
            grads[3 * l + 2] += dZ.sum(axis=0)
            dH = B(dZ) @ W.T + np.outer(np.ones(n), dZ.sum(axis=0) @ U.T) / n
    return np.concatenate([g.ravel() for g in grads])


def test_features_match_oracle():
    mats = [synth.assign_points(n, seed=2, instance=k + 1)
            for k, n in enumerate([64, 150, 333])]
    mats.append(synth.assign_random_small(5, 3, lo=0, hi=9))
    # the smallest instances: one padded cost group per row
    mats.append(synth.assign_random_small(1, 5, lo=0, hi=9))
    mats.append(synth.assign_random_small(2, 6, lo=-9, hi=9))
    # costs past the int16 range: the feature passes read the int32 input
    mats.append(synth.assign_random_small(70, 4, lo=-100000, hi=900000))
    packed = _packed(mats)
    print("[net] features", packed.ns, flush=True)
    F, sc = lpr.lpr_pricenet_features(packed)
    F = F.cpu().numpy()
    sc = sc.cpu().numpy()
    for k, m in enumerate(mats):
        fw, scw = P.features(m)
        a, b = packed.row_offset[k], packed.row_offset[k + 1]
        assert abs(sc[k] - scw) <= 1e-5 * scw
        np.testing.assert_allclose(F[a:b], fw, atol=3e-3, rtol=1e-3)


def test_sinkhorn_column_nobody_wants():
    """One column far dearer than the rest for every row: its mass under the
    row-normalised plan underflows float32 at once, so the GPU takes that
    column's update directly from the row potentials (its own minimum and
    sum).  f14 must still match the oracle; the other instances of the
    batch, of all three row-length classes of the Sinkhorn launch, too."""
    c = synth.assign_random_small(64, 7, lo=0, hi=100).copy()
    c[:, 5] = 30000
    mats = [c, synth.assign_points(600, seed=4, instance=1),
            synth.assign_points(1100, seed=4, instance=2)]
    packed = _packed(mats)
    print("[net] sinkhorn fallback", packed.ns, flush=True)
    F, _ = lpr.lpr_pricenet_features(packed)
    F = F.cpu().numpy()
    for k, m in enumerate(mats):
        fw, _ = P.features(m)
        a, b = packed.row_offset[k], packed.row_offset[k + 1]
        np.testing.assert_allclose(F[a:b, 14], fw[:, 14], atol=3e-3, rtol=1e-3)


def test_forward_and_gradient_match_oracle():
    mats = [synth.assign_points(n, seed=3, instance=k + 1)
            for k, n in enumerate([64, 97, 200])]
    packed = _packed(mats)
    theta = P.init_params(7)
    g = np.random.default_rng(1)
    theta = (theta + g.normal(0, 0.02, theta.shape)).astype(np.float32)
    params = torch.as_tensor(theta, device="cuda")
    print("[net] forward/backward", packed.ns, flush=True)
    q, prices, _ = lpr.lpr_pricenet_infer(packed, params)
    F, sc = lpr.lpr_pricenet_features(packed)
    th, feats = _cpu_inputs(theta, F.cpu().numpy(), packed.row_offset)
    skips = _skips(F.cpu().numpy(), packed.row_offset)
    q_cpu = P.predict_q(th, feats, skips)
    q_gpu = q.cpu().numpy()
    offs = packed.row_offset
    for k in range(len(mats)):
        assert rel(q_gpu[offs[k]:offs[k + 1]], q_cpu[k]) < 3e-2
    # targets: optimal column prices in the solver's scaled convention from
    # the oracle's sequential cost scaling (optimal duals are not unique; fixed
    # oracle duals keep this check of the backward pass independent of the
    # GPU solver's schedule)
    tp = []
    for m in mats:
        _, _, p, _ = oracle.cost_scaling(m)
        tp.append(torch.as_tensor(p, device="cuda"))
    tgt = torch.cat(tp)
    loss, grad = lpr.lpr_pricenet_train_step(packed, tgt, params, step=0,
                                             want_grad=True)
    scn = sc.cpu().numpy()
    targets = []
    for k, m in enumerate(mats):
        n = m.shape[0]
        t = tp[k].cpu().numpy().astype(np.float64)
        targets.append((t - t.mean()) / (scn[k] * (2 * n + 1)))
    L_cpu, g_cpu = P.loss_and_grad(th, feats, targets, skips)
    assert abs(loss - L_cpu) <= 3e-2 * L_cpu
    g_gpu = grad.cpu().numpy().astype(np.float64)
    g_emu = _loss_and_grad_bf16_operands(th, feats, targets, skips)
    # within a small multiple of what bf16 operand rounding alone causes (the
    # GPU also rounds its transposed copies and sums in another order), and
    # under fixed ceilings whatever that emulated error is
    r_all, r_emu = rel(g_gpu, g_cpu), rel(g_emu, g_cpu)
    print(f"[net] gradient rel {r_all:.4f} (bf16 operand emulation {r_emu:.4f})",
          flush=True)
    assert r_all < 2.5 * r_emu + 5e-3
    assert r_all < 5e-2
    # every parameter block, not just the norm of the whole vector
    off = 0
    for name, shape in P.param_shapes():
        size = int(np.prod(shape))
        if name != "bo":
            a, b = g_gpu[off:off + size], g_cpu[off:off + size]
            rb = rel(a, b)
            assert rb < 2.5 * rel(g_emu[off:off + size], b) + 1e-2, name
            assert rb < 8e-2, (name, off, rb)
        off += size


def test_gradient_with_uncorrelated_targets():
    """The backward pass on targets the network's output does not track
    (unit normal prices).  The gradient of the column-centred loss sums
    residuals that add up to zero against activations that share a large
    common part, so the bf16 rounding of the activations alone moves the
    float64 gradient by tens of percent here (measured on the CPU by the
    emulation below); no bf16 implementation can be held to a fixed bound
    against the exact float64 gradient on such inputs.  The GPU
    is held instead to the oracle fed the same bf16-rounded operands: it must
    agree with that to the error of fp32 accumulation in another order and of
    the rounded transposed copies (2e-2 overall, 4e-2 per block)."""
    mats = [synth.assign_points(n, seed=8, instance=k + 1)
            for k, n in enumerate([80, 211])]
    packed = _packed(mats)
    theta = P.init_params(11)
    g = np.random.default_rng(4)
    theta = (theta + g.normal(0, 0.02, theta.shape)).astype(np.float32)
    params = torch.as_tensor(theta, device="cuda")
    F, sc = lpr.lpr_pricenet_features(packed)
    scn = sc.cpu().numpy()
    th, feats = _cpu_inputs(theta, F.cpu().numpy(), packed.row_offset)
    skips = _skips(F.cpu().numpy(), packed.row_offset)
    tp, targets = [], []
    for k, m in enumerate(mats):
        n = m.shape[0]
        t = np.rint(g.normal(0, 1, n) * scn[k] * (2 * n + 1)).astype(np.int64)
        tp.append(torch.as_tensor(t, device="cuda"))
        tt = t.astype(np.float64)
        targets.append((tt - tt.mean()) / (scn[k] * (2 * n + 1)))
    print("[net] gradient, uncorrelated targets", packed.ns, flush=True)
    loss, grad = lpr.lpr_pricenet_train_step(packed, torch.cat(tp), params, step=0,
                                             want_grad=True)
    L_cpu, g_cpu = P.loss_and_grad(th, feats, targets, skips)
    g_emu = _loss_and_grad_bf16_operands(th, feats, targets, skips)
    g_gpu = grad.cpu().numpy().astype(np.float64)
    r_emu = rel(g_gpu, g_emu)
    print(f"[net] loss {loss:.5f} / {L_cpu:.5f}, gradient rel to float64 "
          f"{rel(g_gpu, g_cpu):.4f} (emulation {rel(g_emu, g_cpu):.4f}), "
          f"rel to bf16-operand emulation {r_emu:.4f}", flush=True)
    assert abs(loss - L_cpu) <= 1e-2 * L_cpu
    assert r_emu < 2e-2
    off = 0
    for name, shape in P.param_shapes():
        size = int(np.prod(shape))
        if name != "bo":  # its true value is 0 (the residual sums to zero)
            rb = rel(g_gpu[off:off + size], g_emu[off:off + size])
            assert rb < 4e-2, (name, off, rb)
        off += size


def _designed_instance(n, seed):
    """Column-constant costs a(y) in {1, 2, 3}, as many 1s as 3s, so that
    sc = mean|c| = 2 and every z = c / sc is 0.5, 1 or 1.5: exact in bf16 and
    float32, so the network below computes the same q on both sides."""
    g = np.random.default_rng(seed)
    k = n // 4
    a = np.array([1] * k + [3] * k + [2] * (n - 2 * k), np.int32)
    a = a[g.permutation(n)]
    return np.repeat(a[None, :], n, axis=0)


def _one_hot_net(feature, sign_in=1.0, sign_out=1.0):
    """q = sign_out * relu(sign_in * f_feature) through unit 0 of all three
    layers, plus a pooled, biased unit 1 that only shifts q by a constant
    (every weight exact in bf16)."""
    theta = np.zeros(P.param_count(), np.float32)
    offs, off = [], 0
    for _, shape in P.param_shapes():
        offs.append(off)
        off += int(np.prod(shape))
    W = P.WIDTH
    theta[offs[0] + feature * W + 0] = sign_in     # W1[f, 0]
    theta[offs[1] + feature * W + 1] = 0.5         # U1[f, 1]: pooled feature
    theta[offs[2] + 1] = 0.25                      # b1[1]
    for l in (1, 2):
        theta[offs[3 * l] + 0] = 1.0               # W_l[0, 0]
        theta[offs[3 * l] + W + 1] = 1.0           # W_l[1, 1]
    theta[offs[9] + 0] = sign_out                  # w_o[0]
    theta[offs[9] + 1] = 2.0                       # w_o[1]
    theta[offs[10]] = -3.0                         # b_o
    return theta


def test_start_prices_exact_on_designed_network():
    """Integer start prices and starting epsilon of lpr_pricenet_infer equal
    the oracle's predict_prices and start_epsilon element by element, on
    inputs where every value is exact in bf16 (both senses)."""
    for n, maximize in ((64, False), (128, True), (96, False)):
        c = _designed_instance(n, seed=n)
        # maximising negates the costs, so f8 = -colmean / sc is read as -f8
        theta = _one_hot_net(8, -1.0, -1.0) if maximize else _one_hot_net(8)
        packed = _packed([c])
        params = torch.as_tensor(theta, device="cuda")
        print(f"[net] designed start prices n={n} max={maximize}", flush=True)
        _, prices, eps = lpr.lpr_pricenet_infer(packed, params, maximize=maximize,
                                                kappa=0.03125)
        want = P.predict_prices(theta, c, maximize=maximize)
        assert np.abs(want).max() > 0
        np.testing.assert_array_equal(prices.cpu().numpy(), want)
        assert int(eps.cpu().numpy()[0]) == P.start_epsilon(c, 0.03125, maximize)


def test_start_prices_match_oracle_committed_weights():
    """The committed network on optical-flow-like instances: the GPU's
    integer start prices against the oracle's predict_prices fed the same
    bf16-rounded weights.  The GPU also rounds its features and activations
    to bf16, so the two agree to the forward tolerance of q (relative 3e-2 of
    the centred prices, in units of sc (2n+1)); the starting epsilon to +-1
    (float32 against float64 sc)."""
    from paper_1110_6231_amd.train_pricenet import load_weights
    theta, kappa, _ = load_weights()
    mats = [synth.assign_points(n, seed=9, instance=k + 1)
            for k, n in enumerate([64, 250, 512])]
    packed = _packed(mats)
    params = torch.as_tensor(theta, device="cuda")
    print("[net] committed-weight start prices", packed.ns, flush=True)
    _, prices, eps = lpr.lpr_pricenet_infer(packed, params, kappa=kappa)
    prices = prices.cpu().numpy()
    eps = eps.cpu().numpy()
    th, _ = _cpu_inputs(theta, np.zeros((1, 16), np.float32), [0, 1])
    offs = packed.row_offset
    for k, m in enumerate(mats):
        want = P.predict_prices(th, m)
        got = prices[offs[k]:offs[k + 1]]
        r = rel(got.astype(np.float64), want.astype(np.float64))
        print(f"[net] n={m.shape[0]} start-price rel {r:.4f}", flush=True)
        assert r < 3e-2
        assert abs(int(eps[k]) - P.start_epsilon(m, kappa)) <= 1


def test_prediction_without_network_equals_zero_head():
    """params NULL (the selected model is the zero correction): the library
    skips the network and the features only it reads, and must return the
    same start prices and epsilons as the network with a zero head, whose
    output is exactly its skip term f14."""
    mats = [synth.assign_points(n, seed=11, instance=k + 1)
            for k, n in enumerate([64, 333, 512, 700])]
    packed = _packed(mats)
    theta = P.init_params(1)
    theta[-129:] = 0.0
    params = torch.as_tensor(theta, device="cuda")
    print("[net] prediction without network", packed.ns, flush=True)
    q0, p0, e0 = lpr.lpr_pricenet_infer(packed, params, kappa=1 / 1024)
    q1, p1, e1 = lpr.lpr_pricenet_infer(packed, None, kappa=1 / 1024)
    assert torch.equal(p0, p1)
    assert torch.equal(e0, e1)
    assert torch.equal(q0, q1)


def test_training_reduces_loss_and_solves_stay_exact():
    mats = synth.assign_batch(seed=0, count=12, train=True)
    packed = _packed(mats)
    _, _, tp, _ = lpr.lpr_assign_solve_batched(packed)
    params = torch.as_tensor(P.init_params(0), device="cuda")
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    first = None
    for step in range(1, 61):
        loss, _ = lpr.lpr_pricenet_train_step(packed, tp, params, m, v,
                                              step=step, lr=2e-3)
        first = first if first is not None else loss
    print(f"[net] loss {first:.4f} -> {loss:.4f}", flush=True)
    assert loss < 0.85 * first
    q, prices, eps = lpr.lpr_pricenet_infer(packed, params, kappa=64.0)
    sc = [np.abs(m).mean() for m in mats]
    want = [max(1, round(64.0 * s * (2 * m.shape[0] + 1))) for s, m in zip(sc, mats)]
    got = eps.cpu().numpy()
    for g_, w_ in zip(got, want):
        assert abs(int(g_) - w_) <= 1e-5 * w_ + 1
    opts = lpr.make_assign_opts(init_col_prices=prices, eps0_per_instance=eps)
    r2c, tots, _, st = lpr.lpr_assign_solve_batched(packed, opts=opts)
    tots = tots.cpu().numpy()
    for k, mat in enumerate(mats):
        assert tots[k] == oracle.assign(mat)[1]


def test_learned_start_gain_on_held_out_instances():
    """The committed network (trained by train_pricenet.py on the training
    branch) against the plain start on evaluation instances it never saw:
    both exact; the learned start must need fewer push/relabel operations.
    The measured ratios are printed."""
    import time
    from paper_1110_6231_amd.train_pricenet import learned_solve, load_predictor

    params, kappa, meta = load_predictor("cuda")
    mats = synth.assign_batch(seed=0, count=64)
    packed = _packed(mats)
    _, tot_p, _, st_p = lpr.lpr_assign_solve_batched(packed)
    _, tot_l, _, st_l = learned_solve(packed, params, kappa, lpr)
    assert torch.equal(tot_p, tot_l)
    want = np.array([oracle.assign(m)[1] for m in mats[:8]])
    np.testing.assert_array_equal(tot_l.cpu().numpy()[:8], want)
    ops_p = st_p["pushes"] + st_p["relabels"]
    ops_l = st_l["pushes"] + st_l["relabels"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        lpr.lpr_assign_solve_batched(packed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(3):
        learned_solve(packed, params, kappa, lpr)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"[net] held-out ops plain {ops_p} learned {ops_l} "
          f"({ops_p / ops_l:.2f}x); time plain {(t1 - t0) / 3 * 1e3:.1f} ms "
          f"learned {(t2 - t1) / 3 * 1e3:.1f} ms", flush=True)
    assert ops_l < ops_p


@pytest.mark.parametrize("seed", range(5))
def test_full_batched_workload_against_oracle(seed):
    """The batched assignment workload at full size (256 optical-flow-like
    instances, n ~ U{64..512}, one launch), from the plain start and from the
    committed network's start: every total equals the Hungarian oracle's,
    every assignment is a permutation costing that total, and every returned
    price vector certifies 1-optimality."""
    from paper_1110_6231_amd.train_pricenet import learned_solve, load_predictor
    params, kappa, _ = load_predictor("cuda")
    mats = synth.assign_batch(seed=seed)
    packed = _packed(mats)
    print(f"[net] full batched workload seed {seed}: {len(mats)} instances, "
          f"sum n^2 = {int(packed.cost_offset[-1])}", flush=True)
    want = np.array([oracle.assign(m)[1] for m in mats])
    runs = {"plain": lpr.lpr_assign_solve_batched(packed),
            "learned": learned_solve(packed, params, kappa, lpr)}
    offs = packed.row_offset
    for name, (r2c, tots, prices, st) in runs.items():
        print(f"[net] {name}: ops {st['pushes'] + st['relabels']}, "
              f"restarts {st['warm_restarts']}", flush=True)
        np.testing.assert_array_equal(tots.cpu().numpy(), want, err_msg=name)
        r2c, prices = r2c.cpu().numpy(), prices.cpu().numpy()
        for k, m in enumerate(mats):
            a, b = offs[k], offs[k + 1]
            assert is_permutation(r2c[a:b], m.shape[0]), (name, k)
            assert int(m[np.arange(m.shape[0]), r2c[a:b]].astype(np.int64).sum()) == want[k]
            assert scaled_eps_certificate(m, r2c[a:b], prices[a:b]), (name, k)


def test_learned_solve_in_one_call_matches_two_calls_and_oracle():
    """lpr_assign_solve_learned (prediction and warm-started solve in one
    call, the solve's cost copies on the library's second stream) against
    lpr_pricenet_infer followed by lpr_assign_solve_batched, on a batch that
    spans the three Sinkhorn launch classes and both cost widths: equal
    totals, equal to the Hungarian oracle, permutations with certified
    prices; then a second, smaller batch through the same call, and a call
    on a stream of the caller's own."""
    from paper_1110_6231_amd.train_pricenet import load_predictor
    params, kappa, _ = load_predictor("cuda")
    sizes = [700, 512, 300, 64, 33, 1, 1100, 257]
    mats = [synth.assign_points(n, seed=3, instance=k + 1) for k, n in enumerate(sizes)]
    mats[2] = mats[2] * 1000  # beyond int16: the int32 cost path
    for rnd, batch in enumerate((mats, mats[3:6])):
        packed = _packed(batch)
        print(f"[net] one-call learned solve, batch {rnd}: n = {packed.ns}", flush=True)
        want = np.array([oracle.assign(m)[1] for m in batch])
        _, prices0, eps0 = lpr.lpr_pricenet_infer(packed, params, kappa=kappa)
        two = lpr.lpr_assign_solve_batched(
            packed, opts=lpr.make_assign_opts(init_col_prices=prices0,
                                              eps0_per_instance=eps0))
        one = lpr.lpr_assign_solve_learned(packed, params, kappa)
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            own = lpr.lpr_assign_solve_learned(packed, params, kappa, stream=side)
        side.synchronize()
        offs = packed.row_offset
        for name, (r2c, tots, prices, st) in (("two calls", two), ("one call", one),
                                               ("own stream", own)):
            np.testing.assert_array_equal(tots.cpu().numpy(), want, err_msg=name)
            r2c, prices = r2c.cpu().numpy(), prices.cpu().numpy()
            for k, m in enumerate(batch):
                a, b = offs[k], offs[k + 1]
                assert is_permutation(r2c[a:b], m.shape[0]), (name, k)
                assert scaled_eps_certificate(m, r2c[a:b], prices[a:b]), (name, k)
        assert one[3]["refines"] == two[3]["refines"]


def test_learned_solve_in_one_call_rejects_bad_arguments():
    """kappa <= 0, start fields already set in the options and a workspace
    smaller than lpr_assign_learned_workspace are rejected before any work
    is enqueued; options the solve rejects after the prediction was enqueued
    end the call cleanly; a valid call afterwards is exact."""
    from paper_1110_6231_amd.train_pricenet import load_predictor
    params, kappa, _ = load_predictor("cuda")
    packed = _packed([synth.assign_points(40, seed=0, instance=1)])
    print("[net] one-call learned solve argument checks", flush=True)
    with pytest.raises(lpr.LprError):
        lpr.lpr_assign_solve_learned(packed, params, 0.0)
    with pytest.raises(lpr.LprError):
        lpr.lpr_assign_solve_learned(packed, params, kappa,
                                     opts=lpr.make_assign_opts(eps0=5))
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(lpr.LprError):
        lpr.lpr_assign_solve_learned(packed, params, kappa, workspace=small)
    # rejected by the solve after the prediction was enqueued
    with pytest.raises(lpr.LprError):
        lpr.lpr_assign_solve_learned(packed, params, kappa,
                                     opts=lpr.make_assign_opts(alpha=1))
    r2c, tots, _, _ = lpr.lpr_assign_solve_learned(packed, params, kappa)
    mat = synth.assign_points(40, seed=0, instance=1)
    assert int(tots[0]) == oracle.assign(mat)[1]
    assert is_permutation(r2c.cpu().numpy(), 40)
    # without the price output (col_prices NULL)
    r2c, tots, pr, _ = lpr.lpr_assign_solve_learned(packed, params, kappa,
                                                     want_prices=False)
    assert pr is None and int(tots[0]) == oracle.assign(mat)[1]
