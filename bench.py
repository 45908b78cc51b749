"""Benchmark: lock-free push-relabel on one MI355X.

One step = one complete solve of the 1024 x 1024 graph-cut grid (32 Gaussian
blobs plus N(0, 0.1^2) noise, int32 capacities): init, push sweeps, global
relabels with gap, termination, flow value and the minimal cut.  Inputs are
resident in HBM before the timed region; outputs and workspace are
preallocated.  The JSON line also carries the dense assignment leg (n = 1024,
weights U{0..1000}, max-weight) and the batched assignment leg (256
optical-flow-like instances), max-flow on two arbitrary networks (a layered
network and a 512 x 512 cut as an arc list), the roofline of the dominant
kernel (the push
sweep or the global-relabel relaxation, whichever takes more time), the push
update rate against a measured atomic-add ceiling, and the CPU oracles timed
on this host (FIFO push-relabel for the grid, Hungarian for the assignment
legs).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       python bench.py --assign-only   (the n = 1024 assignment alone, for
                                        counter profiles of its kernel)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid maxflow Mvertex/s + assignment solves/s, learned vs plain; HBM GB/s"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of the push sweep: the seven int32 state words (e, h,
# four neighbour residuals, sink residual) of every pixel of a processed tile,
# plus 4 bytes per relabel (the height) and 16 per push (the four words a push
# updates: both residuals and both excesses).
SWEEP_BYTES_PER_PIXEL = 28
SWEEP_BYTES_PER_RELABEL = 4
SWEEP_BYTES_PER_PUSH = 16
# Bytes one pass of the global-relabel relaxation must move per pixel of a
# relaxed tile: the height and the four neighbour residuals read, the height
# written.
RELAX_BYTES_PER_PIXEL = 24


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle baseline")
    ap.add_argument("--no-assign", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-batched-grid", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the arbitrary-network max-flow leg")
    ap.add_argument("--assign-only", action="store_true",
                    help="only time the n = 1024 assignment (for counter "
                         "profiles of the solve kernel) and print its JSON")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run plain copies of a known size (counter "
                         "calibration) and exit")
    return ap.parse_args()


def grid_leg(args, torch, lpr, synth):
    inst = synth.grid_blobs(1024, 1024, seed=0)
    dev = torch.device("cuda:0")
    caps = [torch.as_tensor(a, device=dev) for a in inst.arrays()]
    HW = inst.H * inst.W
    ws = torch.empty(lpr.lpr_grid_maxflow_workspace(inst.H, inst.W),
                     dtype=torch.uint8, device=dev)
    opts = lpr.make_grid_opts()
    for _ in range(args.warmup):
        v, _, _ = lpr.lpr_grid_maxflow(inst.H, inst.W, *caps, opts=opts,
                                       workspace=ws)
    print(f"[bench] grid warmup done, flow={v}", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        v, side, st = lpr.lpr_grid_maxflow(inst.H, inst.W, *caps, opts=opts,
                                           workspace=ws, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = wall * 1e3 / args.steps
    # The same K solves again with HIP events around every group of push-sweep
    # and relaxation launches (on the library's stream) for the durations of
    # the two kernels that take the time.
    timed = lpr.make_grid_opts(flags=lpr.LPR_GRID_TIME_KERNELS)
    acc = dict(sweep_ms=0.0, bfs_ms=0.0, tiles_swept=0, tiles_relaxed=0,
               sweeps=0, bfs_passes=0, pushes=0, relabels=0)
    for _ in range(args.steps):
        v, side, st = lpr.lpr_grid_maxflow(inst.H, inst.W, *caps, opts=timed,
                                           workspace=ws, stream=stream)
        for k in acc:
            acc[k] += st[k]
    torch.cuda.synchronize()
    tile_px = st["tile_rows"] * 64
    legs = {
        f"k_sweep<{st['tile_rows']}>": kernel_roofline(
            acc["sweep_ms"], acc["sweeps"], sweep_bytes(acc, tile_px)),
        "k_relax4<false>": kernel_roofline(
            acc["bfs_ms"], acc["bfs_passes"],
            acc["tiles_relaxed"] * st["relax_tile_rows"] * 64 * RELAX_BYTES_PER_PIXEL),
    }
    dominant = max(legs, key=lambda k: legs[k]["total_ms"])
    for name, leg in legs.items():
        leg["traffic"] = traffic_for(name, st["tile_rows"])  # HBM bytes per launch
        leg["traffic_GBps"] = (None if leg["traffic"] is None else
                               round(leg["traffic"] / (leg["avg_launch_us"] * 1e-6) / 1e9, 1))
    roof = dict(legs[dominant])
    roof["kernel"] = dominant
    others = {name: leg for name, leg in legs.items() if name != dominant}
    return dict(inst=inst, flow=v, ms=ms, HW=HW, stats=st, roofline=roof,
                other_kernels=others)


# HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per
# dispatch, averaged over the dispatches of the 1024 x 1024 solve), scaled by
# what the same counters read for a plain copy of known size (FETCH_SIZE
# x 2.0, WRITE_SIZE x 1.0).  Each entry holds the sha256 of the kernel's
# source file at measurement time; a changed source reports null.
MEASURED_TRAFFIC = {
    "k_relax4<false>": {"source_sha256": "101a8f1994ebf72dd6d0b262b2808c23b1c1313a9047be203267bcda5252409d",
                  "bytes_per_launch": 5231326},  # FETCH 2476.6 KiB, WRITE 156.0 KiB
    "k_sweep<8>": {"source_sha256": "101a8f1994ebf72dd6d0b262b2808c23b1c1313a9047be203267bcda5252409d",
                  "bytes_per_launch": 12638952},  # FETCH 3612.6 KiB, WRITE 5118.2 KiB
}


def source_sha(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_for(kernel, tile_rows):
    rec = MEASURED_TRAFFIC.get(kernel)
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_1110_6231_amd", "csrc", "grid_maxflow.hip")
    if source_sha(src) != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


def sweep_bytes(st, tile_px):
    return (st["tiles_swept"] * tile_px * SWEEP_BYTES_PER_PIXEL
            + st["relabels"] * SWEEP_BYTES_PER_RELABEL
            + st["pushes"] * SWEEP_BYTES_PER_PUSH)


def kernel_roofline(total_ms, launches, algo_bytes):
    """Algorithmic bytes per launch / average launch duration (HIP events)."""
    launches = max(launches, 1)
    avg_ms = total_ms / launches
    achieved = (algo_bytes / launches) / max(avg_ms * 1e-3, 1e-12) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(avg_ms * 1e3, 3),
            "bytes_per_launch": int(algo_bytes / launches),
            "launches": launches, "total_ms": round(total_ms, 3)}


def grid_batched_leg(args, torch, lpr, synth):
    """The batched graph-cut workload (64 grids, H, W in [128, 512], plus one
    2048 x 2048 grid with pair weights x4) solved by one batched call."""
    insts = synth.grid_batch(seed=0)
    Hs = [i.H for i in insts]
    Ws = [i.W for i in insts]
    dev = torch.device("cuda:0")
    caps = [torch.as_tensor(np.concatenate([getattr(i, f) for i in insts]),
                            device=dev)
            for f in ("cap_src", "cap_snk", "cap_right", "cap_left",
                      "cap_down", "cap_up")]
    ws = torch.empty(lpr.lpr_grid_maxflow_batched_workspace(Hs, Ws),
                     dtype=torch.uint8, device=dev)
    px = sum(i.n_pixels for i in insts)
    lpr.lpr_grid_maxflow_batched(Hs, Ws, caps, workspace=ws)
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        flows, _, st = lpr.lpr_grid_maxflow_batched(Hs, Ws, caps, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    timed = lpr.make_grid_opts(flags=lpr.LPR_GRID_TIME_KERNELS)
    _, _, sti = lpr.lpr_grid_maxflow_batched(Hs, Ws, caps, opts=timed, workspace=ws)
    tile_px = sti["tile_rows"] * 64
    sweep = kernel_roofline(sti["sweep_ms"], sti["sweeps"], sweep_bytes(sti, tile_px))
    relax = kernel_roofline(sti["bfs_ms"], sti["bfs_passes"],
                            sti["tiles_relaxed"] * sti["relax_tile_rows"] * 64
                            * RELAX_BYTES_PER_PIXEL)
    return {"workload": "64 blob graph cuts (H, W ~ U{128..512}) + one 2048x2048 "
                        "graph cut with pair weights x4, one batched call",
            "pixels": px, "ms_per_batch": round(dt * 1e3, 3),
            "mvertex_per_s": round(px / dt / 1e6, 2),
            "flow_2048": int(flows[-1].item()),
            "global_relabels": st["rounds"], "sweeps": st["sweeps"],
            f"k_sweep<{sti['tile_rows']}>": sweep,
            "k_relax4<false>": relax}


def copy_probe(torch, mib=256, reps=5):
    """Plain device-to-device copies of a known size, for calibrating
    rocprofv3's FETCH_SIZE / WRITE_SIZE counters."""
    n = mib * 2 ** 20 // 4
    a = torch.arange(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "launches": reps}), flush=True)


def assign_single(torch, lpr, synth, reps=3):
    """The dense n = 1024 max-weight assignment, mean of `reps` solves."""
    dev = torch.device("cuda:0")
    cost = torch.as_tensor(synth.assign_uniform(1024, seed=0), device=dev)
    ws = torch.empty(lpr.lpr_assign_workspace(1024), dtype=torch.uint8, device=dev)
    lpr.lpr_assign_solve(cost, maximize=True, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, tot, _, st = lpr.lpr_assign_solve(cost, maximize=True, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return {"workload": "dense assignment n=1024, weights U{0..1000}, "
                        "max-weight, alpha=8, plain start",
            "solves_per_s": round(1.0 / dt, 3), "ms_per_solve": round(dt * 1e3, 3),
            "total": tot, "refines": st["refines"], "phases": st["phases"],
            "pushes": st["pushes"], "relabels": st["relabels"],
            "price_updates": st["price_updates"]}


def assign_leg(args, torch, lpr, synth):
    dev = torch.device("cuda:0")
    out = assign_single(torch, lpr, synth)
    from paper_1110_6231_amd.train_pricenet import learned_solve, load_weights
    mats = synth.assign_batch(seed=0)
    packed = lpr.PackedAssign.from_matrices(mats, device=dev)
    wsb = torch.empty(lpr.lpr_assign_batched_workspace(packed.ns),
                      dtype=torch.uint8, device=dev)
    wsn = torch.empty(lpr.lpr_pricenet_workspace(packed.ns), dtype=torch.uint8,
                      device=dev)
    theta, kappa, _ = load_weights()
    params = torch.as_tensor(theta, device=dev)

    def plain():
        return lpr.lpr_assign_solve_batched(packed, workspace=wsb)

    def learned():
        return learned_solve(packed, params, kappa, lpr, ws_net=wsn, ws_solve=wsb)

    def median_time(fn, k=5):
        fn()
        ts = []
        for _ in range(k):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), r

    tp, (_, tot_p, _, stp) = median_time(plain)
    tl, (_, tot_l, _, stl) = median_time(learned)
    assert torch.equal(tot_p, tot_l), "learned start changed an optimum"
    out["batched"] = {"workload": "256 optical-flow-like instances, "
                                  "n ~ U{64..512}, min-cost",
                      "plain": {"solves_per_s": round(len(mats) / tp, 1),
                                "ms_per_batch": round(tp * 1e3, 3),
                                "ops": stp["pushes"] + stp["relabels"]},
                      "learned": {"solves_per_s": round(len(mats) / tl, 1),
                                  "ms_per_batch": round(tl * 1e3, 3),
                                  "ops": stl["pushes"] + stl["relabels"],
                                  "kappa": kappa},
                      "time_to_optimal_plain_over_learned": round(tp / tl, 3),
                      "ops_plain_over_learned": round(
                          (stp["pushes"] + stp["relabels"]) /
                          (stl["pushes"] + stl["relabels"]), 3)}
    return out


def graph_leg(args, torch, lpr, synth):
    """Form 1 on arbitrary networks (arc lists in mate pairs): a layered
    network with long augmenting paths, a 512 x 512 blob graph cut given as
    an arc list and a 64^3 6-connected volume, each solved three times
    (median)."""
    out = {}
    cases = {
        "layered 64 x 4096, 4 arcs per node": synth.graph_layered(64, 4096, 4, seed=0),
        "512x512 graph cut as an arc list": synth.grid_to_arcs(synth.grid_blobs(512, 512, seed=0)),
        "64x64x64 6-connected volume": synth.grid3d_arcs(64, 64, 64, seed=0),
    }
    for name, (n, tail, head, cap, s, t) in cases.items():
        arrs = [torch.as_tensor(a, device="cuda") for a in (tail, head, cap)]
        ws = torch.empty(lpr.lpr_graph_maxflow_workspace(n, len(tail)), dtype=torch.uint8,
                         device="cuda")
        lpr.lpr_graph_maxflow(n, *arrs, s, t, workspace=ws)
        print(f"[bench] graph warmup done: {name}", file=sys.stderr, flush=True)
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v, _, st = lpr.lpr_graph_maxflow(n, *arrs, s, t, workspace=ws)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        dt = float(np.median(ts))
        out[name] = {"nodes": n, "arcs": len(tail), "flow_value": v,
                     "ms_per_solve": round(dt * 1e3, 3),
                     "mvertex_per_s": round(n / dt / 1e6, 3),
                     "rounds": st["rounds"], "pushes": st["pushes"],
                     "bfs_levels": st["bfs_levels"]}
        if not args.no_cpu:
            # the FIFO push-relabel oracle on one host core, one solve
            import oracle
            t0 = time.perf_counter()
            vc = oracle.graph_maxflow(n, tail, head, cap, s, t)[0]
            assert vc == v, (vc, v)
            out[name]["cpu_oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    return out


def sparse_assign_leg(args, torch, lpr, synth):
    """Sparse assignment: n = 2048 rows of 32 random arcs plus a planted
    permutation, weights U{0..1000}, max-weight; three solves (median), the
    Hungarian oracle (missing arcs priced out) once on one host core."""
    n, d = 2048, 32
    inst = synth.assign_sparse(n, d, seed=0, lo=0, hi=1000)
    rp, cl, cs = (torch.as_tensor(a, device="cuda") for a in inst)
    ws = torch.empty(lpr.lpr_assign_sparse_workspace(n, cl.numel()), dtype=torch.uint8,
                     device="cuda")
    lpr.lpr_assign_sparse_solve(n, rp, cl, cs, maximize=True, workspace=ws)
    print("[bench] sparse assignment warmup done", file=sys.stderr, flush=True)
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, tot, _, st = lpr.lpr_assign_sparse_solve(n, rp, cl, cs, maximize=True,
                                                    workspace=ws)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    out = {"workload": f"sparse assignment n={n}, {d} random arcs per row + a planted "
                       "permutation, weights U{0..1000}, max-weight",
           "arcs": int(cl.numel()), "total": tot, "ms_per_solve": round(dt * 1e3, 3),
           "solves_per_s": round(1.0 / dt, 3), "refines": st["refines"],
           "pushes": st["pushes"], "price_updates": st["price_updates"]}
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        want = oracle.assign_sparse(n, *inst, maximize=True)[1]
        assert want == tot, (want, tot)
        out["cpu_oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    return out


def mincost_leg(args, torch, lpr, synth):
    """Minimum-cost flow with supplies (Algorithm 5.0 on a capacitated
    network): a 200 x 300 transportation problem and random networks of
    2000 and 100000 nodes with planted supplies; three solves (median), the
    successive-shortest-path oracle once on one host core for the two
    smaller ones."""
    out = {}
    cases = {
        "transportation 200 x 300, supplies U{1..1000}, costs U{0..1000}":
            synth.mcf_transport(200, 300, seed=0, max_supply=1000),
        "random network 2000 nodes, 8000 edges, costs U{-100..100}":
            synth.mcf_random(2000, 8000, seed=0),
        "random network 100000 nodes, 400000 edges, costs U{-100..100}":
            synth.mcf_random(100000, 400000, seed=0),
    }
    for name, g in cases.items():
        n = g[0]
        arrs = [torch.as_tensor(a, device="cuda") for a in g[1:]]
        ws = torch.empty(lpr.lpr_mincost_flow_workspace(n, arrs[0].numel()),
                         dtype=torch.uint8, device="cuda")
        lpr.lpr_mincost_flow(n, *arrs, workspace=ws)
        print(f"[bench] min-cost flow warmup done: {name}", file=sys.stderr, flush=True)
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tot, _, _, st = lpr.lpr_mincost_flow(n, *arrs, workspace=ws)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        dt = float(np.median(ts))
        out[name] = {"nodes": n, "arcs": int(arrs[0].numel()), "total_cost": tot,
                     "ms_per_solve": round(dt * 1e3, 3), "refines": st["refines"],
                     "passes": st["iterations"], "pushes": st["pushes"],
                     "relabels": st["relabels"]}
        if not args.no_cpu and n <= 10000:  # the oracle takes minutes beyond
            import oracle
            t0 = time.perf_counter()
            want = oracle.mincost_flow(*g)[0]
            assert want == tot, (want, tot)
            out[name]["cpu_oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    return out


def atomics_leg(torch, lpr, g):
    """Push updates per second of the 1024 x 1024 solve (four atomic word
    updates per push in Algorithm 4.5) next to the measured ceiling of
    non-returning device-scope atomic adds to scattered addresses."""
    log2, blocks, per = 23, 16384, 16        # 32 MiB of counters, 64 M adds
    cnt = torch.zeros(1 << log2, dtype=torch.int32, device="cuda")
    lpr.lpr_atomic_probe(cnt, log2, blocks, per)
    total = blocks * 256 * per
    assert int(cnt.sum().item()) == total
    ms = sorted(lpr.lpr_atomic_probe(cnt, log2, blocks, per) for _ in range(5))[2]
    ceiling = total / (ms * 1e-3)
    pushes = g["stats"]["pushes"]
    rate = 4 * pushes / (g["ms"] * 1e-3)
    return {"push_updates_per_s": round(rate / 1e9, 3), "unit": "G/s",
            "pushes_per_solve": pushes,
            "atomic_add_ceiling_per_s": round(ceiling / 1e9, 3),
            "frac": round(rate / ceiling, 4),
            "probe": f"{total} non-returning 32-bit atomic adds over 2^{log2} "
                     f"int32 counters (xorshift addresses), median of 5: "
                     f"{ms:.3f} ms"}


def cpu_assign_leg(args, synth):
    """The Hungarian oracle on this host: the n = 1024 instance on one core,
    and the batched workload over a thread pool (the oracle releases the GIL)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.lib()
    c = synth.assign_uniform(1024, seed=0)
    t0 = time.perf_counter()
    oracle.assign(c, maximize=True)
    t1024 = time.perf_counter() - t0
    mats = synth.assign_batch(seed=0)
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    per = []

    def one(m):
        ts = time.perf_counter()
        oracle.assign(m)
        return time.perf_counter() - ts

    with ThreadPoolExecutor(cores) as ex:
        per = list(ex.map(one, mats))
    tb = time.perf_counter() - t0
    return {"kind": "oracle", "n1024_solves_per_s": round(1.0 / t1024, 3),
            "n1024_cores": 1,
            "batched_solves_per_s": round(len(mats) / tb, 1),
            "batched_cores": cores,
            "batched_instance_ms_median": round(float(np.median(per)) * 1e3, 3),
            "sample": "Hungarian oracle: one solve of the n=1024 instance on "
                      "one core; the 256 batched instances over a pool of "
                      f"{cores} threads"}


def cpu_leg(args, inst):
    import oracle
    oracle.lib()
    reps, t_used = 0, 0.0
    t0 = time.perf_counter()
    while t_used < args.cpu_seconds and reps < 50:
        v, _ = oracle.grid_maxflow(inst, "fifo")
        reps += 1
        t_used = time.perf_counter() - t0
    mv = inst.H * inst.W * reps / t_used / 1e6
    return {"value": round(mv, 4), "unit": "Mvertex/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{reps} full solves of the same 1024x1024 graph cut by "
                      f"the FIFO push-relabel oracle (global + gap relabel, "
                      f"single thread), {t_used:.1f} s"}, v


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} "
              "is not supported (the batched workloads would shard by "
              "instance across GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_1110_6231_amd import lpr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(torch)
        return
    if args.assign_only:
        print(json.dumps({"assignment": assign_single(torch, lpr, synth)}), flush=True)
        return
    g = grid_leg(args, torch, lpr, synth)
    out = {
        "metric": METRIC,
        "value": round(g["HW"] / (g["ms"] * 1e-3) / 1e6, 3),
        "unit": "Mvertex/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(g["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "4-connected grid graph cut 1024x1024, int32: "
                               "32 Gaussian blobs + N(0,0.1) noise; terminals "
                               "rint(100|I-0.5|), pairs rint(50 exp(-dI^2/"
                               "(2*0.05^2))); seed 0",
                   "pixels": g["HW"], "flow_value": g["flow"],
                   "global_relabels": g["stats"]["rounds"],
                   "sweeps": g["stats"]["sweeps"],
                   "tile": f"64x{g['stats']['tile_rows']}",
                   "local_iters": g["stats"]["local_iters"],
                   "sweeps_per_relabel": g["stats"]["sweeps_per_relabel"]},
        "roofline": g["roofline"],
        "other_kernels": g["other_kernels"],
        "atomics": atomics_leg(torch, lpr, g),
    }
    if not args.no_batched_grid:
        out["grid_batched"] = grid_batched_leg(args, torch, lpr, synth)
    if not args.no_graph:
        out["graph"] = graph_leg(args, torch, lpr, synth)
        out["mincost_flow"] = mincost_leg(args, torch, lpr, synth)
    if not args.no_assign:
        out["assignment"] = assign_leg(args, torch, lpr, synth)
        if not args.no_cpu:
            out["assignment"]["cpu_oracle"] = cpu_assign_leg(args, synth)
        out["assignment"]["sparse"] = sparse_assign_leg(args, torch, lpr, synth)
    if not args.no_cpu:
        cb, cpu_flow = cpu_leg(args, g["inst"])
        assert cpu_flow == g["flow"], (cpu_flow, g["flow"])
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
