"""GPU parity for dense assignment: the HIP library against the CPU oracle.

The optimal total is unique and must equal the Hungarian oracle exactly; the
returned permutation must be valid and cost that total; the returned scaled
column prices must certify 1-optimality (hence optimality) independently of
the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from certificates import is_permutation, scaled_eps_certificate
from oracle import brute

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1110_6231_amd import lpr  # noqa: E402


def check(cost, maximize=False, opts=None):
    n = cost.shape[0]
    print(f"[assign] n={n} max={maximize}", flush=True)
    r2c, tot, prices, st = lpr.lpr_assign_solve(cost, maximize=maximize,
                                                opts=opts)
    r2c = r2c.cpu().numpy()
    want = oracle.assign(cost, maximize=maximize)[1]
    assert tot == want, (n, tot, want, st)
    assert is_permutation(r2c, n)
    assert int(cost[np.arange(n), r2c].astype(np.int64).sum()) == tot
    cmin = -cost.astype(np.int64) if maximize else cost
    assert scaled_eps_certificate(cmin, r2c, prices.cpu().numpy())
    return st


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_bruteforce(n):
    for seed in range(4):
        c = synth.assign_random_small(n, seed)
        want, _ = brute.assign_bruteforce(c)
        r2c, tot, _, _ = lpr.lpr_assign_solve(c)
        assert tot == want


@pytest.mark.parametrize("n", [63, 64, 65, 100, 257, 700])
def test_random_sizes(n):
    check(synth.assign_random_small(n, seed=n, lo=-1000, hi=1000))
    check(synth.assign_random_small(n, seed=n + 1, lo=0, hi=1000), maximize=True)


def test_uniform_config_n1024():
    """The dense n = 1024 max-weight workload (weights U{0..1000}) on seeds
    0-4, at the workload's alpha 8 and at the built-in schedule: totals equal
    to the Hungarian oracle's, permutations, certified prices."""
    for seed in range(5):
        c = synth.assign_uniform(1024, seed=seed)
        st = check(c, maximize=True, opts=lpr.make_assign_opts(alpha=8))
        st_b = check(c, maximize=True)
        print(f"[assign] n=1024 seed {seed}: alpha 8 {st['refines']} refines, "
              f"built-in alpha {st_b['alpha']} {st_b['refines']} refines", flush=True)


def test_points_config():
    for k in range(4):
        check(synth.assign_points(64 + 149 * k, seed=0, instance=k + 1))


def test_closed_forms():
    n = 90
    check(np.full((n, n), 17, np.int32))
    g = np.random.default_rng(3)
    a, b = g.integers(0, 60, n), g.integers(0, 60, n)
    c = np.outer(a, b).astype(np.int32)
    r2c, tot, _, _ = lpr.lpr_assign_solve(c)
    assert tot == int((np.sort(a) * np.sort(b)[::-1]).sum())
    a, b = g.integers(-500, 500, n), g.integers(-500, 500, n)
    c = np.abs(a[:, None] - b[None, :]).astype(np.int32)
    r2c, tot, _, _ = lpr.lpr_assign_solve(c)
    assert tot == int(np.abs(np.sort(a) - np.sort(b)).sum())
    # a single popular column: every row bids for it first
    c = np.full((n, n), 500, np.int32)
    c[:, 7] = g.integers(0, 10, n)
    check(c)


def test_alpha_eps_and_warm_start():
    c = synth.assign_points(300, seed=4, instance=9)
    for alpha in (2, 10, 16):
        check(c, opts=lpr.make_assign_opts(alpha=alpha))
    # a small starting epsilon skips the coarse refines (any eps0 is exact;
    # a single refine at eps = 1 from zero prices is only cheap when small)
    check(c, opts=lpr.make_assign_opts(eps0=5000))
    check(synth.assign_random_small(30, 5, lo=0, hi=40),
          opts=lpr.make_assign_opts(eps0=1))
    g = np.random.default_rng(0)
    garbage = torch.as_tensor(g.integers(-10**9, 10**9, 300), device="cuda")
    check(c, opts=lpr.make_assign_opts(init_col_prices=garbage))
    # column prices spread just past and just within the 2^29 window of the
    # 32-bit row scans (past it the scans run in int64 until a rebase fits)
    for spread in (2**29 + 5, 2**29 - 5 * 10**6):
        edge = np.zeros(300, np.int64)
        edge[::2] = -spread
        check(c, opts=lpr.make_assign_opts(
            init_col_prices=torch.as_tensor(edge, device="cuda")))


@pytest.mark.parametrize("n", [64, 257, 700])
def test_arc_fixing_stays_exact(n):
    """Arc fixing (Section 5) with the bound (4n+2) eps: same optimum, and the
    final all-arcs check never has to rerun a refine."""
    fix = lpr.make_assign_opts(flags=lpr.LPR_ASSIGN_ARC_FIXING)
    st = check(synth.assign_random_small(n, seed=n + 7, lo=0, hi=1000), opts=fix)
    assert st["fixing_reruns"] == 0
    st = check(synth.assign_points(n, seed=1, instance=n), opts=fix)
    assert st["fixing_reruns"] == 0
    st = check(synth.assign_random_small(n, seed=n, lo=-1000, hi=1000), maximize=True,
               opts=fix)
    assert st["fixing_reruns"] == 0


def test_arc_fixing_uniform_n1024():
    fix = lpr.make_assign_opts(flags=lpr.LPR_ASSIGN_ARC_FIXING)
    st = check(synth.assign_uniform(1024, seed=1), maximize=True, opts=fix)
    assert st["fixing_reruns"] == 0


def test_arc_fixing_rerun_path():
    """A bound shrunk far below the theorem's drops arcs the optimum needs:
    the final check must catch it and the rerun with full scans must still
    return the optimum."""
    # costs up to 30000: the first lists are built after a refine at an eps
    # of several cost units, whose matching is not yet optimal; with only
    # the matched arc kept, the later refines cannot improve it
    c = synth.assign_random_small(300, seed=11, lo=0, hi=30000)
    st = check(c, opts=lpr.make_assign_opts(flags=lpr.LPR_ASSIGN_ARC_FIXING,
                                            fixing_shift=63))
    assert st["fixing_reruns"] == 1
    with pytest.raises(lpr.LprError):
        lpr.lpr_assign_solve(c, opts=lpr.make_assign_opts(fixing_shift=64))


@pytest.mark.parametrize("tail,flags,period", [
    (1, 0, 0), (2, lpr.LPR_ASSIGN_NO_START_UPDATE, 0), (64, 0, 1),
    (4096, 0, 0), (8, 0, -1), (0, lpr.LPR_ASSIGN_NO_START_UPDATE, -1),
    (16, 0, 37)])
def test_schedule_options_stay_exact(tail, flags, period):
    """Serial-tail threshold (from every row to the whole refine), the
    refine-start price update on or off, and price updates after every push,
    never, or at an odd period: all are admissible schedules of the same
    operations, so the optimum and its certificate must not change."""
    opts = lpr.make_assign_opts(tail_rows=tail, flags=flags,
                                price_update_period=period)
    check(synth.assign_points(257, seed=6, instance=3), opts=opts)
    check(synth.assign_random_small(130, seed=9, lo=0, hi=300), maximize=True,
          opts=opts)
    check(synth.assign_random_small(7, seed=2, lo=-5, hi=5), opts=opts)


def test_costs_at_the_limit():
    """|c| up to LPR_ASSIGN_MAX_COST (2^24 - 1): the int32 row scans and the
    price update over the int32 column-major copy, scaled costs near 2^36 and
    prices in int64; totals must match the oracle."""
    big = lpr.LPR_ASSIGN_MAX_COST
    for n, seed in ((40, 1), (130, 2), (300, 3)):
        c = synth.assign_random_small(n, seed=seed, lo=-big, hi=big)
        st = check(c)
        assert n < 100 or st["price_updates"] > 0, st
        check(c, maximize=True)


@pytest.mark.parametrize("period", [1, 37, -1])
def test_int32_costs_schedules(period):
    """Price updates after every push, at an odd period and never, on costs
    that need int32: the same optimum and certificate."""
    opts = lpr.make_assign_opts(price_update_period=period)
    c = synth.assign_random_small(257, seed=8, lo=0, hi=1 << 22)
    st = check(c, maximize=True, opts=opts)
    assert (st["price_updates"] == 0) == (period < 0), st
    check(synth.assign_points(200, seed=4, instance=2, scale=5e6), opts=opts)


def test_batched_mixed_cost_widths():
    """Instances whose costs fit int16 next to instances that need int32: the
    int32 column-major copy fills the instance's whole share of the copy
    buffer, which must not reach its neighbours."""
    specs = [(65, 1000), (200, 1 << 23), (64, 300), (129, 40000), (8, 1 << 20),
             (300, 32767)]
    mats = [synth.assign_random_small(n, seed=20 + k, lo=-hi, hi=hi)
            for k, (n, hi) in enumerate(specs)]
    packed = lpr.PackedAssign.from_matrices(mats)
    print("[assign] batched mixed widths", packed.ns, flush=True)
    for flags in (0, lpr.LPR_ASSIGN_ARC_FIXING):
        opts = lpr.make_assign_opts(flags=flags)
        r2c, tots, prices, _ = lpr.lpr_assign_solve_batched(packed, opts=opts)
        r2c, prices, tots = (r2c.cpu().numpy(), prices.cpu().numpy(),
                             tots.cpu().numpy())
        for k, m in enumerate(mats):
            a, b = packed.row_offset[k], packed.row_offset[k + 1]
            assert tots[k] == oracle.assign(m)[1], (k, flags)
            assert is_permutation(r2c[a:b], m.shape[0])
            assert scaled_eps_certificate(m, r2c[a:b], prices[a:b])


def test_maximum_size_n2048():
    """n = LPR_ASSIGN_MAX_N (the largest LDS footprint).  The Hungarian oracle
    is too slow here, so the checks are a closed form and the certificate:
    for c = a_i b_j the minimum pairs a ascending with b descending
    (rearrangement inequality), and for random costs the returned prices must
    certify 1-optimality of the returned permutation, which proves it
    optimal without the oracle."""
    n = lpr.LPR_ASSIGN_MAX_N
    g = np.random.default_rng(11)
    a, b = g.integers(0, 180, n), g.integers(0, 180, n)
    c = np.outer(a, b).astype(np.int32)
    print("[assign] n=2048 rank one", flush=True)
    r2c, tot, prices, _ = lpr.lpr_assign_solve(c)
    assert tot == int((np.sort(a) * np.sort(b)[::-1]).astype(np.int64).sum())
    assert is_permutation(r2c.cpu().numpy(), n)
    assert scaled_eps_certificate(c, r2c.cpu().numpy(), prices.cpu().numpy())
    c = synth.assign_random_small(n, seed=12, lo=0, hi=5000)
    print("[assign] n=2048 random", flush=True)
    r2c, tot, prices, _ = lpr.lpr_assign_solve(c, maximize=True)
    r2c = r2c.cpu().numpy()
    assert is_permutation(r2c, n)
    assert int(c[np.arange(n), r2c].astype(np.int64).sum()) == tot
    assert scaled_eps_certificate(-c.astype(np.int64), r2c, prices.cpu().numpy())
    # int32 costs (|c| >= 2^15 takes the int32 row scans and column copy)
    c = synth.assign_random_small(n, seed=13, lo=0, hi=1 << 20)
    print("[assign] n=2048 int32 costs", flush=True)
    r2c, tot, prices, _ = lpr.lpr_assign_solve(c)
    r2c = r2c.cpu().numpy()
    assert is_permutation(r2c, n)
    assert scaled_eps_certificate(c, r2c, prices.cpu().numpy())


def test_batched():
    mats = [synth.assign_points(n, seed=1, instance=k + 1)
            for k, n in enumerate([64, 300, 129, 512, 77, 200])]
    packed = lpr.PackedAssign.from_matrices(mats)
    print("[assign] batched", packed.ns, flush=True)
    r2c, tots, prices, st = lpr.lpr_assign_solve_batched(packed)
    r2c = r2c.cpu().numpy()
    prices = prices.cpu().numpy()
    tots = tots.cpu().numpy()
    for k, m in enumerate(mats):
        a, b = packed.row_offset[k], packed.row_offset[k + 1]
        assert tots[k] == oracle.assign(m)[1]
        assert is_permutation(r2c[a:b], m.shape[0])
        assert scaled_eps_certificate(m, r2c[a:b], prices[a:b])


def test_warm_start_fallback():
    """A start that costs more than its budget restarts from the plain start
    (p = 0, eps = max|c| (2n+1)) and still ends at the optimum.  eps0 = 1 on
    an n = 300 instance and garbage prices with eps0 = 1 both exhaust even the
    whole-solve budget (64 n^2 + 2^20 operations) without the fallback."""
    c = synth.assign_points(300, seed=4, instance=9)
    st = check(c, opts=lpr.make_assign_opts(eps0=1))
    print("[assign] eps0=1 fallback", st, flush=True)
    assert st["warm_restarts"] == 1
    g = np.random.default_rng(5)
    garbage = torch.as_tensor(g.integers(-10**9, 10**9, 300), device="cuda")
    st = check(c, opts=lpr.make_assign_opts(init_col_prices=garbage, eps0=1))
    assert st["warm_restarts"] == 1
    # a plain start never restarts; neither does a warm start within budget
    assert check(c)["warm_restarts"] == 0
    assert check(c, opts=lpr.make_assign_opts(eps0=5000))["warm_restarts"] == 0
    # without the fallback the same start runs into the whole-solve budget
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_assign_solve(c, opts=lpr.make_assign_opts(eps0=1, warm_max_ops=-1,
                                                          max_ops=400000))
    assert e.value.status == lpr.LPR_EBUDGET
    # in a batch, only the instances with a bad start restart
    mats = [synth.assign_points(n, seed=6, instance=k + 1)
            for k, n in enumerate([200, 96, 300, 150])]
    packed = lpr.PackedAssign.from_matrices(mats)
    eps = torch.tensor([1, 0, 1, 0], dtype=torch.int64, device="cuda")
    r2c, tots, prices, st = lpr.lpr_assign_solve_batched(
        packed, opts=lpr.make_assign_opts(eps0_per_instance=eps))
    print("[assign] batched fallback", st, flush=True)
    assert 1 <= st["warm_restarts"] <= 2
    r2c, tots, prices = r2c.cpu().numpy(), tots.cpu().numpy(), prices.cpu().numpy()
    for k, m in enumerate(mats):
        a, b = packed.row_offset[k], packed.row_offset[k + 1]
        assert tots[k] == oracle.assign(m)[1]
        assert is_permutation(r2c[a:b], m.shape[0])
        assert scaled_eps_certificate(m, r2c[a:b], prices[a:b])


def test_errors():
    c = synth.assign_random_small(20, 0)
    big = c.copy()
    big[3, 4] = lpr.LPR_ASSIGN_MAX_COST + 1
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_assign_solve(big)
    assert e.value.status == lpr.LPR_ERANGE
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_assign_solve(synth.assign_uniform(300, seed=1), maximize=True,
                             opts=lpr.make_assign_opts(max_ops=50))
    assert e.value.status == lpr.LPR_EBUDGET
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_assign_solve(c, opts=lpr.make_assign_opts(alpha=1))
    assert e.value.status == lpr.LPR_EINVAL
    check(c)


def test_autotuner_is_exact_and_sets_default():
    """lpr_assign_tune: every schedule it tries gives the oracle's totals, the
    winner is one of the searched schedules, and later solves of that size
    class and kind of start use it when their options leave the fields 0;
    options that set a field still override it."""
    mats = [synth.assign_random_small(n, seed=n, lo=0, hi=500) for n in (33, 47, 61, 70)]
    packed = lpr.PackedAssign.from_matrices(mats)
    want = [oracle.assign(m)[1] for m in mats]
    print("[assign] tuner on 4 instances", flush=True)
    sched, ms, tots = lpr.lpr_assign_tune(packed, reps=1)
    assert tots.cpu().numpy().tolist() == want
    assert sched["alpha"] in (4, 6, 8, 16)
    assert sched["price_update_quarters"] in (1, 2, 4, 8)
    assert sched["tail_rows"] in (0, 8, 32)
    assert ms > 0
    _, tot, _, st = lpr.lpr_assign_solve_batched(packed)
    assert tot.cpu().numpy().tolist() == want
    # a tuned 0 is the built-in rule: a 32-row tail for instances up to 512
    assert (st["alpha"], st["price_update_quarters"], st["tail_rows"]) == (
        sched["alpha"], sched["price_update_quarters"], sched["tail_rows"] or 32)
    o = lpr.make_assign_opts(alpha=5, price_update_quarters=3, tail_rows=12)
    _, tot, _, st = lpr.lpr_assign_solve_batched(packed, opts=o)
    assert tot.cpu().numpy().tolist() == want
    assert (st["alpha"], st["price_update_quarters"], st["tail_rows"]) == (5, 3, 12)
    # a warm start is its own kind: untuned, it keeps the built-in rules
    # (instances up to n = 512: alpha 8, q 1, tail 32)
    eps = torch.full((len(mats),), 1 << 12, dtype=torch.int64, device="cuda")
    _, tot, _, st = lpr.lpr_assign_solve_batched(
        packed, opts=lpr.make_assign_opts(eps0_per_instance=eps))
    assert tot.cpu().numpy().tolist() == want
    assert (st["alpha"], st["price_update_quarters"], st["tail_rows"]) == (8, 1, 32)


def test_builtin_schedule_rules():
    """With no tuned schedule for the size class, the built-in rules apply:
    a dense batch whose largest instance has n <= 512 runs alpha 16 and a
    32-row tail from the plain start, alpha 8, q 1 and a 32-row tail from a
    warm start; n = 1024 runs alpha 6 with the per-instance period and
    tail; the totals equal the oracle's under each."""
    mats = [synth.assign_random_small(n, seed=n, lo=0, hi=900) for n in (100, 200)]
    packed = lpr.PackedAssign.from_matrices(mats)
    want = [oracle.assign(m)[1] for m in mats]
    print("[assign] built-in schedule rules", flush=True)
    _, tot, _, st = lpr.lpr_assign_solve_batched(packed)
    assert tot.cpu().numpy().tolist() == want
    assert (st["alpha"], st["price_update_quarters"], st["tail_rows"]) == (16, 0, 32)
    eps = torch.full((2,), 1 << 10, dtype=torch.int64, device="cuda")
    _, tot, _, st = lpr.lpr_assign_solve_batched(
        packed, opts=lpr.make_assign_opts(eps0_per_instance=eps))
    assert tot.cpu().numpy().tolist() == want
    assert (st["alpha"], st["price_update_quarters"], st["tail_rows"]) == (8, 1, 32)
    big = synth.assign_uniform(1024, seed=3)
    _, tot1, _, st = lpr.lpr_assign_solve(big, maximize=True)
    assert tot1 == oracle.assign(big, maximize=True)[1]
    assert (st["alpha"], st["price_update_quarters"], st["tail_rows"]) == (6, 0, 0)
