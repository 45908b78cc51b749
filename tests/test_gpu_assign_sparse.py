"""GPU parity for sparse assignment (arcs in CSR by row): the HIP library
against the CPU oracle (the Hungarian method with missing arcs priced out).

The optimal total is unique and must equal the oracle's exactly; the returned
permutation must use listed arcs only and cost that total; the returned
scaled column prices must certify 1-optimality over the listed arcs; an
instance without a perfect matching must give LPR_ENOMATCH exactly when the
oracle finds none.
"""
import numpy as np
import pytest

import oracle
import synth
from certificates import is_permutation, scaled_eps_certificate_sparse

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1110_6231_amd import lpr  # noqa: E402


def check(n, inst, maximize=False, opts=None):
    row_ptr, col, cost = inst
    print(f"[sparse] n={n} m={len(col)} max={maximize}", flush=True)
    want = oracle.assign_sparse(n, row_ptr, col, cost, maximize=maximize)
    assert want is not None
    r2c, tot, prices, st = lpr.lpr_assign_sparse_solve(n, row_ptr, col, cost,
                                                       maximize=maximize, opts=opts)
    r2c = r2c.cpu().numpy()
    assert tot == want[1], (n, tot, want[1], st)
    assert is_permutation(r2c, n)
    cmin = -cost.astype(np.int64) if maximize else cost.astype(np.int64)
    assert scaled_eps_certificate_sparse(n, row_ptr, col, cmin, r2c,
                                         prices.cpu().numpy())
    return st


@pytest.mark.parametrize("n,degree", [(1, 1), (2, 1), (7, 2), (64, 3), (257, 8),
                                      (1000, 16)])
def test_random_sparse(n, degree):
    for seed in range(2):
        inst = synth.assign_sparse(n, degree, seed=seed, lo=-1000, hi=1000,
                                   parallel=0.2)
        check(n, inst)
        check(n, inst, maximize=True)


def test_full_range_costs_and_n2048():
    """Costs over the whole int16 range; n = LPR_ASSIGN_MAX_N."""
    inst = synth.assign_sparse(300, 6, seed=3, lo=-32767, hi=32767)
    check(300, inst)
    inst = synth.assign_sparse(2048, 32, seed=1, lo=0, hi=32767)
    st = check(2048, inst)
    print("[sparse] n=2048 stats", st, flush=True)


def test_planted_only_is_the_planted_permutation():
    """Degree 0 plus the planted column: the only perfect matching."""
    n = 500
    row_ptr, col, cost = synth.assign_sparse(n, 0, seed=4, lo=0, hi=100)
    r2c, tot, _, _ = lpr.lpr_assign_sparse_solve(n, row_ptr, col, cost)
    assert np.array_equal(r2c.cpu().numpy(), col)
    assert tot == int(cost.astype(np.int64).sum())


def test_complete_graph_equals_dense_solver():
    n = 200
    c = synth.assign_random_small(n, seed=5, lo=-3000, hi=3000)
    row_ptr = (np.arange(n + 1) * n).astype(np.int32)
    col = np.tile(np.arange(n), n).astype(np.int32)
    for maximize in (False, True):
        _, tot, _, _ = lpr.lpr_assign_sparse_solve(n, row_ptr, col, c.ravel(),
                                                   maximize=maximize)
        _, tot_d, _, _ = lpr.lpr_assign_solve(c, maximize=maximize)
        assert tot == tot_d


def test_no_perfect_matching():
    found = 0
    for seed in range(6):
        n = 40 + seed
        inst = synth.assign_sparse(n, 1, seed=seed, planted=False)
        want = oracle.assign_sparse(n, *inst)
        print(f"[sparse] infeasible? n={n} seed={seed} {want is None}", flush=True)
        if want is None:
            found += 1
            with pytest.raises(lpr.LprError) as e:
                lpr.lpr_assign_sparse_solve(n, *inst)
            assert e.value.status == lpr.LPR_ENOMATCH
        else:
            check(n, inst)
    assert found > 0
    # a row without arcs
    row_ptr = np.array([0, 1, 1, 3], np.int32)
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_assign_sparse_solve(3, row_ptr, np.array([0, 1, 2], np.int32),
                                    np.array([1, 2, 3], np.int32))
    assert e.value.status == lpr.LPR_ENOMATCH


@pytest.mark.parametrize("period,flags", [(1, 0), (-1, 0), (37, 0),
                                          (0, lpr.LPR_ASSIGN_NO_START_UPDATE),
                                          (0, lpr.LPR_ASSIGN_ARC_FIXING)])
def test_schedules_stay_exact(period, flags):
    opts = lpr.make_assign_opts(price_update_period=period, flags=flags)
    check(400, synth.assign_sparse(400, 5, seed=7, lo=0, hi=5000, parallel=0.1),
          maximize=True, opts=opts)


def test_invalid_inputs_are_rejected():
    row_ptr = np.array([0, 2, 3, 4], np.int32)
    col = np.array([0, 1, 2, 0], np.int32)
    cost = np.array([1, 2, 3, 4], np.int32)
    for rp, cl, cs, status in (
            (np.array([1, 2, 3, 4], np.int32), col, cost, lpr.LPR_EINVAL),
            (np.array([0, 2, 3, 3], np.int32), col, cost, lpr.LPR_EINVAL),
            (np.array([0, 3, 2, 4], np.int32), col, cost, lpr.LPR_EINVAL),
            (row_ptr, np.array([0, 1, 3, 0], np.int32), cost, lpr.LPR_EINVAL),
            (row_ptr, np.array([0, -1, 2, 0], np.int32), cost, lpr.LPR_EINVAL),
            (row_ptr, col, np.array([1, 32768, 3, 4], np.int32), lpr.LPR_ERANGE),
            (row_ptr, col, np.array([1, -32768, 3, 4], np.int32), lpr.LPR_ERANGE)):
        with pytest.raises(lpr.LprError) as e:
            lpr.lpr_assign_sparse_solve(3, rp, cl, cs)
        assert e.value.status == status
