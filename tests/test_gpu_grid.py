"""GPU parity for grid max-flow: the HIP library against the CPU oracle.

Flow value and the minimal source side S_min are unique, so both must match
the oracle exactly (int64 value, byte-for-byte side).  Sizes span several
64 x TH tiles with ragged right and bottom tails; the full 1024 x 1024
graph-cut workload runs in the benchmark's launch configuration (defaults).
Most cases run under both relabel modes: the global relabel between the
sweeps (Algorithm 4.8) and the asynchronous one beside them (ARG).
"""
import numpy as np
import pytest

import oracle
import synth
from certificates import grid_cut_value
from oracle import brute

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1110_6231_amd import lpr  # noqa: E402


SYNC = lpr.LPR_GRID_SYNC_RELABEL
ASYNC = lpr.LPR_GRID_ASYNC_RELABEL
MODES = pytest.mark.parametrize("mode", [SYNC, ASYNC], ids=["sync", "async"])


def gpu_solve(inst, opts=None, want_cut=True):
    print(f"[grid] {inst.name} {inst.H}x{inst.W}", flush=True)
    v, side, st = lpr.lpr_grid_maxflow(inst.H, inst.W, *inst.arrays(),
                                       want_cut=want_cut, opts=opts)
    return v, (side.cpu().numpy() if side is not None else None), st


def check_against_oracle(inst, opts=None):
    want_v, want_side = oracle.grid_maxflow(inst, "fifo")
    v, side, st = gpu_solve(inst, opts)
    assert v == want_v, (inst.name, v, want_v, st)
    np.testing.assert_array_equal(side, want_side, err_msg=inst.name)
    return st


@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (2, 1), (2, 2), (3, 3),
                                   (1, 9), (3, 4)])
def test_tiny_bruteforce(shape):
    H, W = shape
    for seed in range(4):
        inst = synth.grid_random_small(H, W, seed)
        want_v, want_side = brute.grid_min_cut_bruteforce(inst)
        v, side, _ = gpu_solve(inst)
        assert v == want_v
        np.testing.assert_array_equal(side, want_side)


@pytest.mark.parametrize("seed", range(5))
def test_uniform64_config(seed):
    check_against_oracle(synth.grid_uniform(64, 64, seed))


@MODES
@pytest.mark.parametrize("H,W", [(37, 70), (100, 129), (17, 200), (130, 65)])
@pytest.mark.parametrize("tile_rows", [4, 8, 16, 32])
def test_ragged_shapes_all_tiles(H, W, tile_rows, mode):
    inst = synth.grid_random_small(H, W, seed=H + W, max_cap=40, max_term=60)
    check_against_oracle(inst, lpr.make_grid_opts(tile_rows=tile_rows, flags=mode))


@MODES
@pytest.mark.parametrize("K,L", [(1, 1), (3, 2), (16, 64), (64, 4)])
def test_schedules(K, L, mode):
    inst = synth.grid_blobs(150, 170, seed=4)
    check_against_oracle(inst, lpr.make_grid_opts(sweeps_per_relabel=K,
                                                  local_iters=L, flags=mode))


@MODES
@pytest.mark.parametrize("R", [1, 3, 16])
def test_rounds_per_check(R, mode):
    """Rounds enqueued between two reads of the device status: retired
    instances and finished relabels turn the surplus rounds into no-ops."""
    inst = synth.grid_blobs(210, 190, seed=8)
    st = check_against_oracle(inst, lpr.make_grid_opts(rounds_per_check=R,
                                                       flags=mode))
    assert st["rounds_per_check"] == R
    assert st["async_relabel"] == (1 if mode == ASYNC else 0)


@MODES
def test_rounds_without_graph_replay(mode):
    inst = synth.grid_blobs(180, 140, seed=6)
    check_against_oracle(inst, lpr.make_grid_opts(flags=lpr.LPR_GRID_NO_GRAPH | mode))
    check_against_oracle(inst, lpr.make_grid_opts(flags=lpr.LPR_GRID_TIME_KERNELS | mode))


@MODES
def test_blobs_medium_and_long_paths(mode):
    o = lpr.make_grid_opts(flags=mode)
    check_against_oracle(synth.grid_blobs(256, 300, seed=2), o)
    check_against_oracle(synth.grid_blobs(200, 260, seed=3, pair_scale=200.0), o)


def serpentine(H, W, seed):
    """One path through every pixel: full rows joined at alternating ends,
    one weak arc in the middle row; the BFS labels run up to H*W."""
    g = np.random.default_rng(seed)
    hf = g.integers(60, 100, (H, W - 1))
    hf[H // 2, W // 2] = 30
    vf = np.zeros((H - 1, W), np.int64)
    for r in range(H - 1):
        vf[r, W - 1 if r % 2 == 0 else 0] = g.integers(60, 100)
    src = np.zeros((H, W), np.int32)
    snk = np.zeros((H, W), np.int32)
    src[0, 0] = 77
    snk[H - 1, W - 1 if (H - 1) % 2 == 0 else 0] = 91
    return synth.grid_from_pairs(H, W, src, snk, hf, hf, vf, vf, f"serpentine{H}x{W}")


@MODES
@pytest.mark.parametrize("scan", [0, lpr.LPR_GRID_SEGMENTED_SCAN],
                         ids=["offset", "segmented"])
def test_row_scan_forms(scan, mode):
    """The relaxation's two forms of row scan (labels offset per segment, or
    a lane test per step) reach the same least fixpoint: the oracle's flow
    and minimal cut on rows cut into many segments (sparse arcs), on a path
    through every pixel and on a blob image."""
    o = lpr.make_grid_opts(flags=mode | scan)
    check_against_oracle(synth.grid_random_small(100, 129, seed=5, max_cap=4,
                                                 max_term=12, density=0.5), o)
    check_against_oracle(synth.grid_random_small(67, 200, seed=6, density=0.9), o)
    st = check_against_oracle(serpentine(33, 130, seed=7), o)
    assert st["rounds"] >= 1
    check_against_oracle(synth.grid_blobs(200, 260, seed=3, pair_scale=200.0), o)


def test_closed_forms():
    H, W = 70, 90
    z = np.zeros(H * W, np.int32)
    zero = synth.GridInstance(H, W, z, z, z, z, z, z, "zero")
    v, side, _ = gpu_solve(zero)
    assert v == 0 and side.sum() == 0
    base = synth.grid_uniform(H, W, seed=7)
    iso = synth.GridInstance(H, W, base.cap_src, base.cap_snk, z, z, z, z, "iso")
    v, side, _ = gpu_solve(iso)
    assert v == 0
    np.testing.assert_array_equal(side, (base.cap_src > 0).astype(np.uint8))
    g = np.random.default_rng(1)
    src = g.integers(0, 40, H * W).astype(np.int32)
    snk = g.integers(0, 40, H * W).astype(np.int32)
    both = synth.GridInstance(H, W, src, snk, z, z, z, z, "both")
    v, side, _ = gpu_solve(both)
    assert v == int(np.minimum(src, snk).astype(np.int64).sum())
    np.testing.assert_array_equal(side, (src > snk).astype(np.uint8))


def test_chain_long_path():
    W = 1000
    src = np.zeros(W, np.int32)
    snk = np.zeros(W, np.int32)
    src[0], snk[-1] = 77, 91
    g = np.random.default_rng(3)
    right = g.integers(60, 100, W - 1)
    inst = synth.grid_from_pairs(1, W, src, snk, right[None], right[None],
                                 np.zeros((0, W)), np.zeros((0, W)), "chain")
    v, side, _ = gpu_solve(inst)
    assert v == min(77, 91, int(right.min()))
    want_v, want_side = oracle.grid_maxflow(inst, "fifo")
    np.testing.assert_array_equal(side, want_side)


@MODES
def test_batched_matches_single(mode):
    insts = [synth.grid_random_small(40 + 13 * k, 30 + 29 * k, seed=k,
                                     max_cap=30) for k in range(5)]
    insts.append(synth.grid_blobs(150, 200, seed=1))
    insts.append(synth.grid_uniform(64, 64, seed=2))
    Hs = [i.H for i in insts]
    Ws = [i.W for i in insts]
    caps = [torch.as_tensor(np.concatenate([getattr(i, f) for i in insts]),
                            device="cuda")
            for f in ("cap_src", "cap_snk", "cap_right", "cap_left",
                      "cap_down", "cap_up")]
    print("[grid] batched", list(zip(Hs, Ws)), flush=True)
    flows, side, st = lpr.lpr_grid_maxflow_batched(
        Hs, Ws, caps, opts=lpr.make_grid_opts(flags=mode))
    flows = flows.cpu().numpy()
    side = side.cpu().numpy()
    off = 0
    for k, inst in enumerate(insts):
        want_v, want_side = oracle.grid_maxflow(inst, "fifo")
        assert flows[k] == want_v, k
        np.testing.assert_array_equal(side[off:off + inst.n_pixels], want_side)
        off += inst.n_pixels


@pytest.mark.parametrize("mode", [0, ASYNC], ids=["default", "async"])
def test_full_size_graph_cut_1024(mode):
    """The 1024 x 1024 graph-cut workload at the benchmark's configuration:
    exact flow value and S_min against the oracle, and the cut certificate."""
    inst = synth.grid_blobs(1024, 1024, seed=0)
    want_v, want_side = oracle.grid_maxflow(inst, "fifo")
    v, side, st = gpu_solve(inst, lpr.make_grid_opts(flags=mode) if mode else None)
    print("[grid] 1024^2 stats", st, flush=True)
    assert v == want_v
    np.testing.assert_array_equal(side, want_side)
    assert grid_cut_value(inst, side) == v


def test_capacities_at_the_limit():
    """Every capacity near LPR_GRID_MAX_CAP (2^26 - 1): a pixel's excess can
    reach five times that, close to the int32 range, and heights stay below
    the packed-key range; the flow value (int64) and S_min must still match
    the oracle."""
    big = lpr.LPR_GRID_MAX_CAP
    inst = synth.grid_random_small(45, 77, seed=21, max_cap=big, max_term=big,
                                   density=1.0)
    st = check_against_oracle(inst)
    print("[grid] limit caps", st, flush=True)
    z = np.zeros(9, np.int32)
    full = np.full(9, big, np.int32)
    # a pixel fed at the limit from the source and all four neighbours
    src = full.copy()
    snk = z.copy()
    snk[4] = big
    inst = synth.GridInstance(3, 3, src, snk, full, full, full, full, "star")
    check_against_oracle(inst)


def test_errors():
    inst = synth.grid_uniform(20, 20, seed=0)
    arrs = [a.copy() for a in inst.arrays()]
    arrs[2][5] = -1
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_grid_maxflow(20, 20, *arrs)
    assert e.value.status == lpr.LPR_EINVAL
    arrs = [a.copy() for a in inst.arrays()]
    arrs[0][7] = lpr.LPR_GRID_MAX_CAP + 1
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_grid_maxflow(20, 20, *arrs)
    assert e.value.status == lpr.LPR_ERANGE
    small_ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_grid_maxflow(20, 20, *inst.arrays(), workspace=small_ws)
    assert e.value.status == lpr.LPR_ENOMEM
    big = synth.grid_blobs(300, 300, seed=5)
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_grid_maxflow(300, 300, *big.arrays(),
                             opts=lpr.make_grid_opts(max_rounds=1,
                                                     sweeps_per_relabel=1,
                                                     local_iters=1))
    assert e.value.status == lpr.LPR_EBUDGET
    for bad in (lpr.make_grid_opts(flags=SYNC | ASYNC),
                lpr.make_grid_opts(rounds_per_check=17)):
        with pytest.raises(lpr.LprError) as e:
            lpr.lpr_grid_maxflow(20, 20, *inst.arrays(), opts=bad)
        assert e.value.status == lpr.LPR_EINVAL
    o = lpr.make_grid_opts()
    o.reserved[1] = 3
    with pytest.raises(lpr.LprError) as e:
        lpr.lpr_grid_maxflow(20, 20, *inst.arrays(), opts=o)
    assert e.value.status == lpr.LPR_EINVAL
    # the library stays usable after every error
    check_against_oracle(synth.grid_uniform(64, 64, seed=1))


def _pack(insts):
    return [torch.as_tensor(np.concatenate([getattr(i, f) for i in insts]),
                            device="cuda")
            for f in ("cap_src", "cap_snk", "cap_right", "cap_left",
                      "cap_down", "cap_up")]


@pytest.mark.parametrize("mode", [0, SYNC, ASYNC], ids=["default", "sync", "async"])
def test_full_batched_workload_against_golden(mode):
    """The batched graph-cut workload: 64 blob grids with H, W in
    [128, 512] plus one 2048 x 2048 grid with pair weights x4, in one batched
    call, at the library's default schedule.  Flow values and S_min must
    match the oracle's stored values (tests/golden/make_grid_golden.py)."""
    import hashlib
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "grid_golden.json")))["batch_seed0"]
    insts = synth.grid_batch(seed=0)
    Hs = [i.H for i in insts]
    Ws = [i.W for i in insts]
    print("[grid] full batched workload", len(insts), sum(i.n_pixels for i in insts),
          flush=True)
    flows, side, st = lpr.lpr_grid_maxflow_batched(
        Hs, Ws, _pack(insts), opts=lpr.make_grid_opts(flags=mode) if mode else None)
    print("[grid] batched stats", st, flush=True)
    flows = flows.cpu().numpy()
    side = side.cpu().numpy()
    off = 0
    for k, (inst, rec) in enumerate(zip(insts, gold)):
        assert rec["name"] == inst.name
        assert flows[k] == rec["flow"], (k, inst.name)
        s = side[off:off + inst.n_pixels]
        assert hashlib.sha256(s.tobytes()).hexdigest() == rec["source_side_sha256"], k
        off += inst.n_pixels


@pytest.mark.parametrize("seed", [1, 2])
def test_full_batched_workload_other_seeds(seed):
    """The batched graph-cut workload drawn with other seeds (64 blob grids
    plus the 2048 x 2048 grid with pair weights x4, 10.5 M pixels, one
    call): every flow value and every minimal source side equal to the FIFO
    oracle's, computed here over a pool of host threads (one instance per
    task, largest first)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    insts = synth.grid_batch(seed=seed)
    Hs = [i.H for i in insts]
    Ws = [i.W for i in insts]
    print(f"[grid] full batched workload seed {seed}: {len(insts)} grids, "
          f"{sum(i.n_pixels for i in insts)} pixels", flush=True)
    flows, side, st = lpr.lpr_grid_maxflow_batched(Hs, Ws, _pack(insts))
    flows = flows.cpu().numpy()
    side = side.cpu().numpy()
    print(f"[grid] seed {seed} solved ({st['rounds']} global relabels); oracle next",
          flush=True)
    oracle.lib()
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    order = sorted(range(len(insts)), key=lambda k: -insts[k].n_pixels)
    with ThreadPoolExecutor(cores) as ex:
        got = dict(zip(order, ex.map(lambda k: oracle.grid_maxflow(insts[k], "fifo"),
                                     order)))
    off = 0
    for k, inst in enumerate(insts):
        want_v, want_side = got[k]
        assert flows[k] == want_v, (seed, k, inst.name)
        assert np.array_equal(side[off:off + inst.n_pixels], want_side), (seed, k)
        off += inst.n_pixels


def test_autotuner_is_exact_and_sets_default():
    insts = [synth.grid_blobs(160 + 40 * k, 230, seed=k) for k in range(3)]
    Hs = [i.H for i in insts]
    Ws = [i.W for i in insts]
    caps = _pack(insts)
    sched, ms, flows = lpr.lpr_grid_tune(Hs, Ws, caps, reps=1)
    print("[grid] tuned", sched, ms, flush=True)
    assert sched["tile_rows"] in (4, 8, 16, 32) and ms > 0
    want = [oracle.grid_maxflow(i, "fifo")[0] for i in insts]
    assert list(flows.cpu().numpy()) == want
    f2, _, st = lpr.lpr_grid_maxflow_batched(Hs, Ws, caps, want_cut=False)
    assert list(f2.cpu().numpy()) == want
    assert (st["tile_rows"], st["local_iters"]) == (sched["tile_rows"],
                                                    sched["local_iters"])
    k = sched["sweeps_per_relabel"]
    assert st["sweeps_per_relabel"] == k


def test_same_pixel_count_other_shape_reuses_buffers():
    """Grids with the same pixel count and sweep-tile count but another
    relaxation tiling (32 x 64, 8 x 256 and 16 x 128: 1, 4 and 2 relaxation
    tiles of 64 x 32, against 4 sweep tiles of the default 64 x 8 each),
    solved back to back through the same capacity tensors and workspace with
    round graphs replayed: each must match the oracle, so no captured round
    of one shape is replayed for the other."""
    shapes = [(32, 64), (8, 256), (16, 128), (32, 64), (8, 256)]
    N = 2048
    need = max(lpr.lpr_grid_maxflow_workspace(H, W) for H, W in shapes)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    caps = [torch.empty(N, dtype=torch.int32, device="cuda") for _ in range(6)]
    for k, (H, W) in enumerate(shapes):
        inst = synth.grid_random_small(H, W, seed=50 + k, max_cap=30, max_term=60)
        for dst, src in zip(caps, inst.arrays()):
            dst.copy_(torch.as_tensor(src))
        print(f"[grid] shared buffers {H}x{W}", flush=True)
        v, side, st = lpr.lpr_grid_maxflow(H, W, *caps, workspace=ws)
        want_v, want_side = oracle.grid_maxflow(inst, "fifo")
        assert v == want_v, (H, W, v, want_v, st)
        np.testing.assert_array_equal(side.cpu().numpy(), want_side)
        assert st["rounds"] >= 2, st   # at least one replayed round


def test_instance_past_the_offset_scan_limit():
    """An instance of more than 2^25 - 66 pixels, whose labels the offset
    row scans cannot hold, solved through the segmented scans the library
    picks for it: 16 400 independent rows of 2 048 pixels, each a chain from
    a source arc a at column 0 to a sink arc b at the last column through
    horizontal arcs of capacity 50.  Closed forms: the row's flow is
    min(a, b, 50); its minimal source side is empty when a is the least,
    column 0 when 50 is, the whole row when b is."""
    H, W, c = 16400, 2048, 50
    assert H * W > (1 << 25) - 66
    r = np.arange(H)
    a = np.array([31, 41, 61, 71])[r % 4]
    b = np.array([33, 47, 53, 67, 77])[r % 5]
    src = np.zeros((H, W), np.int32)
    snk = np.zeros((H, W), np.int32)
    src[:, 0] = a
    snk[:, -1] = b
    horiz = np.full((H, W - 1), c, np.int32)
    vert = np.zeros((H - 1, W), np.int32)
    inst = synth.grid_from_pairs(H, W, src, snk, horiz, horiz, vert, vert, "chains")
    del src, snk, horiz, vert
    v, side, st = gpu_solve(inst)
    flow = np.minimum(np.minimum(a, b), c)
    assert v == int(flow.sum())
    side = side.reshape(H, W)
    want = np.zeros((H, W), np.uint8)
    want[flow == c, 0] = 1
    want[flow == b, :] = 1
    np.testing.assert_array_equal(side, want)
