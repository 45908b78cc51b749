"""Thin ctypes binding of the C ABI in ``include/lpr.h``.

Argument marshalling only: every step of the solves runs in the HIP library
(``liblpr.so``).  PyTorch is used for device memory (outputs and the
workspace) and for the current stream.  If the library is missing the calls
raise immediately -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblpr.so")

LPR_OK, LPR_EINVAL, LPR_ERANGE, LPR_ENOMEM, LPR_EDEVICE, LPR_EBUDGET = (
    0, -1, -2, -3, -4, -5)
LPR_ENOMATCH = -6
LPR_EINFEASIBLE = -7
STATUS_NAMES = {0: "LPR_OK", -1: "LPR_EINVAL", -2: "LPR_ERANGE",
                -3: "LPR_ENOMEM", -4: "LPR_EDEVICE", -5: "LPR_EBUDGET",
                -6: "LPR_ENOMATCH", -7: "LPR_EINFEASIBLE"}
LPR_MCF_MAX_N = 1 << 20
LPR_MCF_MAX_COST = (1 << 16) - 1
LPR_MCF_MAX_SUPPLY = 1 << 30
LPR_GRID_MAX_CAP = (1 << 26) - 1
LPR_ASSIGN_MAX_COST = (1 << 24) - 1
LPR_ASSIGN_MAX_N = 2048
LPR_ASSIGN_SPARSE_MAX_ARCS = 1 << 26
LPR_GRID_TIME_KERNELS = 0x1
LPR_GRID_NO_GRAPH = 0x2
LPR_GRID_ASYNC_RELABEL = 0x4
LPR_GRID_SYNC_RELABEL = 0x8
LPR_GRID_SEGMENTED_SCAN = 0x10
LPR_ASSIGN_TIME_KERNELS = 0x1
LPR_ASSIGN_NO_START_UPDATE = 0x2
LPR_ASSIGN_ARC_FIXING = 0x4

# Every symbol the header declares (checked by the ABI test).
EXPORTED = [
    "lpr_last_error", "lpr_version",
    "lpr_grid_maxflow_workspace", "lpr_grid_maxflow",
    "lpr_grid_maxflow_noalloc_max_bytes", "lpr_grid_maxflow_noalloc",
    "lpr_grid_maxflow_batched_workspace", "lpr_grid_maxflow_batched",
    "lpr_grid_tune",
    "lpr_assign_workspace", "lpr_assign_solve",
    "lpr_assign_batched_workspace", "lpr_assign_solve_batched", "lpr_assign_tune",
    "lpr_assign_sparse_workspace", "lpr_assign_sparse_solve",
    "lpr_pricenet_param_count", "lpr_pricenet_workspace",
    "lpr_pricenet_features", "lpr_pricenet_infer", "lpr_pricenet_train_step",
    "lpr_assign_learned_workspace", "lpr_assign_solve_learned",
    "lpr_graph_maxflow_workspace", "lpr_graph_maxflow",
    "lpr_mincost_flow_workspace", "lpr_mincost_flow",
    "lpr_atomic_probe",
]
PRICENET_FEATURES = 16
PRICENET_WIDTH = 128


class LprError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GridOpts(ctypes.Structure):
    _fields_ = [("sweeps_per_relabel", ctypes.c_int32),
                ("local_iters", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("rounds_per_check", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class GridStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("sweeps", ctypes.c_int64),
                ("bfs_passes", ctypes.c_int64),
                ("tiles_swept", ctypes.c_int64), ("pushes", ctypes.c_int64),
                ("relabels", ctypes.c_int64), ("cut_passes", ctypes.c_int64),
                ("tiles_relaxed", ctypes.c_int64),
                ("device_atomics", ctypes.c_int64),
                ("tile_rows", ctypes.c_int32), ("local_iters", ctypes.c_int32),
                ("sweeps_per_relabel", ctypes.c_int32),
                ("relax_tile_rows", ctypes.c_int32),
                ("sweep_ms", ctypes.c_double), ("bfs_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double),
                ("async_relabel", ctypes.c_int32),
                ("rounds_per_check", ctypes.c_int32),
                ("bfs_passes_with_work", ctypes.c_int64)]


class AssignOpts(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("eps0", ctypes.c_int64),
                ("init_col_prices", ctypes.c_void_p),
                ("max_ops", ctypes.c_int64),
                ("max_ms", ctypes.c_int64),
                ("eps0_per_instance", ctypes.c_void_p),
                ("price_update_period", ctypes.c_int64),
                ("tail_rows", ctypes.c_int32), ("fixing_shift", ctypes.c_int32),
                ("warm_max_ops", ctypes.c_int64),
                ("price_update_quarters", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class AssignStats(ctypes.Structure):
    _fields_ = [("refines", ctypes.c_int64), ("phases", ctypes.c_int64),
                ("pushes", ctypes.c_int64), ("relabels", ctypes.c_int64),
                ("scans", ctypes.c_int64), ("price_updates", ctypes.c_int64),
                ("price_update_us", ctypes.c_int64),
                ("fixing_reruns", ctypes.c_int64),
                ("warm_restarts", ctypes.c_int64),
                ("scan_entries", ctypes.c_int64),
                ("price_update_steps", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("alpha", ctypes.c_int32),
                ("price_update_quarters", ctypes.c_int32),
                ("tail_rows", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class GraphOpts(ctypes.Structure):
    _fields_ = [("cycle", ctypes.c_int32), ("max_rounds", ctypes.c_int32),
                ("sweeps_per_relabel", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class GraphStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("pushes", ctypes.c_int64),
                ("relabels", ctypes.c_int64), ("bfs_levels", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class McfOpts(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_int32), ("iters_per_check", ctypes.c_int32),
                ("max_iters", ctypes.c_int64)]


class McfStats(ctypes.Structure):
    _fields_ = [("refines", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("pushes", ctypes.c_int64), ("relabels", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


def _struct_dict(s) -> dict:
    return {k: getattr(s, k) for k, _ in s._fields_ if k != "reserved"}


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_1110_6231_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.lpr_last_error.restype = ctypes.c_char_p
    L.lpr_last_error.argtypes = []
    L.lpr_version.restype = ctypes.c_char_p
    L.lpr_version.argtypes = []
    L.lpr_grid_maxflow_workspace.restype = sz
    L.lpr_grid_maxflow_workspace.argtypes = [i32, i32]
    L.lpr_grid_maxflow.restype = ctypes.c_int
    L.lpr_grid_maxflow.argtypes = [i32, i32] + [vp] * 6 + [
        vp, vp, ctypes.POINTER(GridOpts), ctypes.POINTER(GridStats), vp, sz, vp]
    L.lpr_grid_maxflow_noalloc_max_bytes.restype = sz
    L.lpr_grid_maxflow_noalloc_max_bytes.argtypes = []
    L.lpr_grid_maxflow_noalloc.restype = ctypes.c_int
    L.lpr_grid_maxflow_noalloc.argtypes = [i32, i32] + [vp] * 6 + [
        vp, vp, ctypes.POINTER(GridOpts), ctypes.POINTER(GridStats), vp]
    L.lpr_grid_maxflow_batched_workspace.restype = sz
    L.lpr_grid_maxflow_batched_workspace.argtypes = [i32, i32p, i32p]
    L.lpr_grid_maxflow_batched.restype = ctypes.c_int
    L.lpr_grid_maxflow_batched.argtypes = [i32, i32p, i32p, i64p] + [vp] * 6 + [
        vp, vp, ctypes.POINTER(GridOpts), ctypes.POINTER(GridStats), vp, sz, vp]
    L.lpr_grid_tune.restype = ctypes.c_int
    L.lpr_grid_tune.argtypes = [i32, i32p, i32p, i64p] + [vp] * 6 + [
        vp, i32, ctypes.POINTER(GridOpts), ctypes.POINTER(ctypes.c_double), vp, sz, vp]
    L.lpr_assign_workspace.restype = sz
    L.lpr_assign_workspace.argtypes = [i32]
    L.lpr_assign_solve.restype = ctypes.c_int
    L.lpr_assign_solve.argtypes = [i32, vp, i32, vp, vp, vp,
                                   ctypes.POINTER(AssignOpts),
                                   ctypes.POINTER(AssignStats), vp, sz, vp]
    L.lpr_assign_batched_workspace.restype = sz
    L.lpr_assign_batched_workspace.argtypes = [i32, i32p]
    L.lpr_assign_solve_batched.restype = ctypes.c_int
    L.lpr_assign_solve_batched.argtypes = [i32, i32p, i64p, vp, i32, vp, vp, vp,
                                           ctypes.POINTER(AssignOpts),
                                           ctypes.POINTER(AssignStats), vp, sz,
                                           vp]
    L.lpr_assign_tune.restype = ctypes.c_int
    L.lpr_assign_tune.argtypes = [i32, i32p, i64p, vp, i32, vp, vp,
                                  ctypes.POINTER(AssignOpts), i32,
                                  ctypes.POINTER(AssignOpts),
                                  ctypes.POINTER(ctypes.c_double), vp, sz, vp]
    L.lpr_assign_sparse_workspace.restype = sz
    L.lpr_assign_sparse_workspace.argtypes = [i32, i32]
    L.lpr_assign_sparse_solve.restype = ctypes.c_int
    L.lpr_assign_sparse_solve.argtypes = [i32, i32, vp, vp, vp, i32, vp, vp, vp,
                                          ctypes.POINTER(AssignOpts),
                                          ctypes.POINTER(AssignStats), vp, sz, vp]
    L.lpr_pricenet_param_count.restype = sz
    L.lpr_pricenet_param_count.argtypes = []
    L.lpr_pricenet_workspace.restype = sz
    L.lpr_pricenet_workspace.argtypes = [i32, i32p]
    L.lpr_pricenet_features.restype = ctypes.c_int
    L.lpr_pricenet_features.argtypes = [i32, i32p, i64p, vp, i32, vp, vp, vp, sz, vp]
    L.lpr_pricenet_infer.restype = ctypes.c_int
    L.lpr_pricenet_infer.argtypes = [i32, i32p, i64p, vp, i32, vp, ctypes.c_float,
                                     vp, vp, vp, vp, sz, vp]
    L.lpr_assign_learned_workspace.restype = sz
    L.lpr_assign_learned_workspace.argtypes = [i32, i32p]
    L.lpr_assign_solve_learned.restype = ctypes.c_int
    L.lpr_assign_solve_learned.argtypes = [i32, i32p, i64p, vp, i32, vp, ctypes.c_float,
                                           vp, vp, vp, ctypes.POINTER(AssignOpts),
                                           ctypes.POINTER(AssignStats), vp, sz, vp]
    L.lpr_pricenet_train_step.restype = ctypes.c_int
    L.lpr_pricenet_train_step.argtypes = [i32, i32p, i64p, vp, i32, vp, vp, vp, vp,
                                          vp, i32, ctypes.c_float, vp, vp, sz, vp]
    L.lpr_graph_maxflow_workspace.restype = sz
    L.lpr_graph_maxflow_workspace.argtypes = [i32, i32]
    L.lpr_graph_maxflow.restype = ctypes.c_int
    L.lpr_graph_maxflow.argtypes = [i32, i32, vp, vp, vp, i32, i32, i64p, vp,
                                    ctypes.POINTER(GraphOpts),
                                    ctypes.POINTER(GraphStats), vp, sz, vp]
    L.lpr_mincost_flow_workspace.restype = sz
    L.lpr_mincost_flow_workspace.argtypes = [i32, i32]
    L.lpr_mincost_flow.restype = ctypes.c_int
    L.lpr_mincost_flow.argtypes = [i32, i32, vp, vp, vp, vp, vp, i64p, vp, vp,
                                   ctypes.POINTER(McfOpts), ctypes.POINTER(McfStats),
                                   vp, sz, vp]
    L.lpr_atomic_probe.restype = ctypes.c_int
    L.lpr_atomic_probe.argtypes = [vp, i32, i32, i32, ctypes.POINTER(ctypes.c_double), vp]
    _lib = L
    return L


def last_error() -> str:
    return lib().lpr_last_error().decode()


def version() -> str:
    return lib().lpr_version().decode()


def _check(status: int, where: str):
    if status != LPR_OK:
        raise LprError(status, where, last_error())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_i32(a, device):
    import torch
    if isinstance(a, torch.Tensor):
        assert a.dtype == torch.int32 and a.is_contiguous() and a.is_cuda
        return a
    return torch.as_tensor(np.ascontiguousarray(a, np.int32), device=device)


# Host arrays for the C-ABI go through numpy: building a ctypes array element
# by element costs about 0.3 us per entry, which a batch of a few hundred
# instances pays on every call.  The returned pointer keeps its array alive.
def _i32_arr(vals):
    a = np.ascontiguousarray(vals, dtype=np.int32)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _i64_arr(vals):
    a = np.ascontiguousarray(vals, dtype=np.int64)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _workspace(nbytes: int, device):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
# Grid max-flow
# ---------------------------------------------------------------------------
def make_grid_opts(sweeps_per_relabel=0, local_iters=0, tile_rows=0,
                   max_rounds=0, flags=0, rounds_per_check=0) -> GridOpts:
    o = GridOpts()
    o.sweeps_per_relabel = sweeps_per_relabel
    o.local_iters = local_iters
    o.tile_rows = tile_rows
    o.max_rounds = max_rounds
    o.flags = flags
    o.rounds_per_check = rounds_per_check
    return o


def lpr_grid_maxflow_workspace(H: int, W: int) -> int:
    return int(lib().lpr_grid_maxflow_workspace(H, W))


def lpr_grid_maxflow(H, W, cap_src, cap_snk, cap_right, cap_left, cap_down,
                     cap_up, want_cut=True, opts: GridOpts | None = None,
                     workspace=None, stream=None, device="cuda"):
    """Solve one grid (see lpr_grid_maxflow in include/lpr.h).

    Capacities: int32 arrays of H*W (torch CUDA tensors or host arrays, the
    latter are copied to the device first).  Returns (flow_value (int),
    source_side (torch uint8 [H*W] on the device, or None), stats dict)."""
    import torch
    caps = [_dev_i32(a, device) for a in (cap_src, cap_snk, cap_right,
                                          cap_left, cap_down, cap_up)]
    dev = caps[0].device
    for c in caps:
        assert c.numel() == H * W
    flow = torch.zeros(1, dtype=torch.int64, device=dev)
    side = torch.empty(H * W, dtype=torch.uint8, device=dev) if want_cut else None
    need = lpr_grid_maxflow_workspace(H, W)
    ws = workspace if workspace is not None else _workspace(need, dev)
    st = GridStats()
    rc = lib().lpr_grid_maxflow(
        H, W, *[_ptr(c) for c in caps], _ptr(flow), _ptr(side),
        ctypes.byref(opts) if opts is not None else None, ctypes.byref(st),
        _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "lpr_grid_maxflow")
    return int(flow.item()), side, _struct_dict(st)


def lpr_grid_maxflow_noalloc_max_bytes() -> int:
    return int(lib().lpr_grid_maxflow_noalloc_max_bytes())


def lpr_grid_maxflow_noalloc(H, W, caps, flow, side, opts: GridOpts | None = None,
                             stream=None):
    """The allocation-free entry point (lpr_grid_maxflow_noalloc).  The
    caller passes the six int32 capacity tensors and the outputs already on
    the device (flow: int64 [1]; side: uint8 [H*W] or None); nothing is
    allocated here.  Returns the stats dict."""
    for c in caps:
        assert c.numel() == H * W and c.is_contiguous()
    st = GridStats()
    rc = lib().lpr_grid_maxflow_noalloc(
        H, W, *[_ptr(c) for c in caps], _ptr(flow), _ptr(side),
        ctypes.byref(opts) if opts is not None else None, ctypes.byref(st),
        _stream(stream))
    _check(rc, "lpr_grid_maxflow_noalloc")
    return _struct_dict(st)


def lpr_grid_maxflow_batched_workspace(Hs, Ws) -> int:
    return int(lib().lpr_grid_maxflow_batched_workspace(
        len(Hs), _i32_arr(Hs), _i32_arr(Ws)))


def lpr_grid_maxflow_batched(Hs, Ws, caps_packed, want_cut=True,
                             opts: GridOpts | None = None, workspace=None,
                             stream=None):
    """Solve B grids in shared launches (lpr_grid_maxflow_batched).

    caps_packed: six int32 CUDA tensors, each the concatenation of the
    instances' arrays.  Returns (flow_values int64 tensor [B], packed
    source_side uint8 tensor or None, stats dict)."""
    import torch
    B = len(Hs)
    offs = np.zeros(B + 1, np.int64)
    offs[1:] = np.cumsum(np.asarray(Hs, np.int64) * np.asarray(Ws, np.int64))
    caps = list(caps_packed)
    dev = caps[0].device
    for c in caps:
        assert c.dtype == torch.int32 and c.is_contiguous() and c.numel() == offs[-1]
    flows = torch.zeros(B, dtype=torch.int64, device=dev)
    side = (torch.empty(int(offs[-1]), dtype=torch.uint8, device=dev)
            if want_cut else None)
    need = lpr_grid_maxflow_batched_workspace(Hs, Ws)
    ws = workspace if workspace is not None else _workspace(need, dev)
    st = GridStats()
    rc = lib().lpr_grid_maxflow_batched(
        B, _i32_arr(Hs), _i32_arr(Ws), _i64_arr(offs), *[_ptr(c) for c in caps],
        _ptr(flows), _ptr(side),
        ctypes.byref(opts) if opts is not None else None, ctypes.byref(st),
        _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "lpr_grid_maxflow_batched")
    return flows, side, _struct_dict(st)


def lpr_grid_tune(Hs, Ws, caps_packed, reps=2, workspace=None, stream=None):
    """Schedule search (lpr_grid_tune).  Returns (schedule dict, best ms,
    flow values of the batch as an int64 tensor)."""
    import torch
    B = len(Hs)
    offs = np.zeros(B + 1, np.int64)
    offs[1:] = np.cumsum(np.asarray(Hs, np.int64) * np.asarray(Ws, np.int64))
    caps = list(caps_packed)
    dev = caps[0].device
    flows = torch.zeros(B, dtype=torch.int64, device=dev)
    ws = workspace if workspace is not None else _workspace(
        lpr_grid_maxflow_batched_workspace(Hs, Ws), dev)
    best = GridOpts()
    ms = ctypes.c_double(0.0)
    rc = lib().lpr_grid_tune(B, _i32_arr(Hs), _i32_arr(Ws), _i64_arr(offs),
                             *[_ptr(c) for c in caps], _ptr(flows), int(reps),
                             ctypes.byref(best), ctypes.byref(ms), _ptr(ws),
                             ws.numel(), _stream(stream))
    _check(rc, "lpr_grid_tune")
    sched = {"tile_rows": best.tile_rows, "local_iters": best.local_iters,
             "sweeps_per_relabel": best.sweeps_per_relabel,
             "rounds_per_check": best.rounds_per_check,
             "async_relabel": bool(best.flags & LPR_GRID_ASYNC_RELABEL)}
    return sched, ms.value, flows


# ---------------------------------------------------------------------------
# Assignment
# ---------------------------------------------------------------------------
def make_assign_opts(alpha=0, eps0=0, init_col_prices=None, max_ops=0,
                     flags=0, max_ms=0, eps0_per_instance=None,
                     price_update_period=0, tail_rows=0,
                     fixing_shift=0, warm_max_ops=0,
                     price_update_quarters=0) -> AssignOpts:
    o = AssignOpts()
    o.price_update_quarters = price_update_quarters
    o.warm_max_ops = warm_max_ops
    o.max_ms = max_ms
    o.price_update_period = price_update_period
    o.tail_rows = tail_rows
    o.fixing_shift = fixing_shift
    o.eps0_per_instance = (None if eps0_per_instance is None
                           else eps0_per_instance.data_ptr())
    o.alpha = alpha
    o.eps0 = eps0
    o.init_col_prices = None if init_col_prices is None else init_col_prices.data_ptr()
    o.max_ops = max_ops
    o.flags = flags
    # the struct holds raw device pointers: keep their tensors alive with it
    o._keep = (init_col_prices, eps0_per_instance)
    return o


def lpr_assign_workspace(n: int) -> int:
    return int(lib().lpr_assign_workspace(n))


def lpr_assign_solve(cost, maximize=False, opts: AssignOpts | None = None,
                     want_prices=True, workspace=None, stream=None,
                     device="cuda"):
    """Solve one n x n assignment (lpr_assign_solve).  Returns (row_to_col
    int32 tensor, total (int), col_prices int64 tensor or None, stats)."""
    import torch
    c = _dev_i32(cost, device)
    n = int(c.shape[0])
    assert c.numel() == n * n
    dev = c.device
    r2c = torch.empty(n, dtype=torch.int32, device=dev)
    tot = torch.zeros(1, dtype=torch.int64, device=dev)
    prices = torch.empty(n, dtype=torch.int64, device=dev) if want_prices else None
    ws = workspace if workspace is not None else _workspace(lpr_assign_workspace(n), dev)
    st = AssignStats()
    rc = lib().lpr_assign_solve(
        n, _ptr(c), int(bool(maximize)), _ptr(r2c), _ptr(tot), _ptr(prices),
        ctypes.byref(opts) if opts is not None else None, ctypes.byref(st),
        _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "lpr_assign_solve")
    return r2c, int(tot.item()), prices, _struct_dict(st)


def lpr_assign_sparse_workspace(n: int, m: int) -> int:
    return int(lib().lpr_assign_sparse_workspace(n, m))


def lpr_assign_sparse_solve(n, row_ptr, col, cost, maximize=False,
                            opts: AssignOpts | None = None, want_prices=True,
                            workspace=None, stream=None, device="cuda"):
    """Solve one sparse assignment given in CSR by row
    (lpr_assign_sparse_solve).  Returns (row_to_col int32 tensor, total (int),
    col_prices int64 tensor or None, stats)."""
    import torch
    rp = _dev_i32(row_ptr, device)
    cl = _dev_i32(col, device)
    cs = _dev_i32(cost, device)
    m = int(cl.numel())
    assert rp.numel() == n + 1 and cs.numel() == m
    dev = rp.device
    r2c = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    tot = torch.zeros(1, dtype=torch.int64, device=dev)
    prices = (torch.empty(max(n, 1), dtype=torch.int64, device=dev)
              if want_prices else None)
    ws = (workspace if workspace is not None
          else _workspace(lpr_assign_sparse_workspace(n, m), dev))
    st = AssignStats()
    rc = lib().lpr_assign_sparse_solve(
        n, m, _ptr(rp), _ptr(cl if m else None), _ptr(cs if m else None),
        int(bool(maximize)), _ptr(r2c), _ptr(tot), _ptr(prices),
        ctypes.byref(opts) if opts is not None else None, ctypes.byref(st),
        _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "lpr_assign_sparse_solve")
    return r2c[:n], int(tot.item()), None if prices is None else prices[:n], \
        _struct_dict(st)


def lpr_assign_batched_workspace(ns) -> int:
    return int(lib().lpr_assign_batched_workspace(len(ns), _i32_arr(ns)))


@dataclass
class PackedAssign:
    """Instances packed for lpr_assign_solve_batched."""
    ns: list
    cost_offset: np.ndarray
    row_offset: np.ndarray
    costs: object  # int32 CUDA tensor

    @staticmethod
    def from_matrices(mats, device="cuda"):
        import torch
        ns = [int(m.shape[0]) for m in mats]
        co = np.zeros(len(ns) + 1, np.int64)
        co[1:] = np.cumsum(np.asarray(ns, np.int64) ** 2)
        ro = np.zeros(len(ns) + 1, np.int64)
        ro[1:] = np.cumsum(ns)
        flat = np.concatenate([np.ascontiguousarray(m, np.int32).ravel()
                               for m in mats])
        return PackedAssign(ns, co, ro, torch.as_tensor(flat, device=device))


def lpr_assign_solve_batched(packed: PackedAssign, maximize=False,
                             opts: AssignOpts | None = None, want_prices=True,
                             workspace=None, stream=None):
    """Solve B instances in one launch.  Returns (row_to_col packed int32,
    totals int64 tensor [B], col_prices packed or None, stats)."""
    import torch
    B = len(packed.ns)
    dev = packed.costs.device
    rows = int(packed.row_offset[-1])
    r2c = torch.empty(rows, dtype=torch.int32, device=dev)
    tots = torch.zeros(B, dtype=torch.int64, device=dev)
    prices = torch.empty(rows, dtype=torch.int64, device=dev) if want_prices else None
    ws = workspace if workspace is not None else _workspace(
        lpr_assign_batched_workspace(packed.ns), dev)
    st = AssignStats()
    rc = lib().lpr_assign_solve_batched(
        B, _i32_arr(packed.ns), _i64_arr(packed.cost_offset), _ptr(packed.costs),
        int(bool(maximize)), _ptr(r2c), _ptr(tots), _ptr(prices),
        ctypes.byref(opts) if opts is not None else None, ctypes.byref(st),
        _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "lpr_assign_solve_batched")
    return r2c, tots, prices, _struct_dict(st)


def lpr_assign_tune(packed: PackedAssign, maximize=False,
                    base: AssignOpts | None = None, reps=2, workspace=None,
                    stream=None):
    """Schedule search (lpr_assign_tune).  Returns (schedule dict, best ms,
    totals of the batch as an int64 tensor)."""
    import torch
    B = len(packed.ns)
    dev = packed.costs.device
    rows = int(packed.row_offset[-1])
    r2c = torch.empty(rows, dtype=torch.int32, device=dev)
    tots = torch.zeros(B, dtype=torch.int64, device=dev)
    ws = workspace if workspace is not None else _workspace(
        lpr_assign_batched_workspace(packed.ns), dev)
    best = AssignOpts()
    ms = ctypes.c_double(0.0)
    rc = lib().lpr_assign_tune(
        B, _i32_arr(packed.ns), _i64_arr(packed.cost_offset), _ptr(packed.costs),
        int(bool(maximize)), _ptr(r2c), _ptr(tots),
        ctypes.byref(base) if base is not None else None, int(reps),
        ctypes.byref(best), ctypes.byref(ms), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "lpr_assign_tune")
    sched = {"alpha": best.alpha, "price_update_quarters": best.price_update_quarters,
             "tail_rows": best.tail_rows}
    return sched, ms.value, tots


# ---------------------------------------------------------------------------
# Learned warm start (price network)
# ---------------------------------------------------------------------------
def lpr_pricenet_param_count() -> int:
    return int(lib().lpr_pricenet_param_count())


def lpr_pricenet_workspace(ns) -> int:
    return int(lib().lpr_pricenet_workspace(len(ns), _i32_arr(ns)))


def _net_ws(packed, workspace):
    if workspace is not None:
        return workspace
    return _workspace(lpr_pricenet_workspace(packed.ns), packed.costs.device)


def lpr_pricenet_features(packed: PackedAssign, maximize=False, workspace=None,
                          stream=None):
    """Column features [sum n, 16] (float32) and cost scales [B]."""
    import torch
    dev = packed.costs.device
    R = int(packed.row_offset[-1])
    B = len(packed.ns)
    feats = torch.empty((R, PRICENET_FEATURES), dtype=torch.float32, device=dev)
    scales = torch.empty(B, dtype=torch.float32, device=dev)
    ws = _net_ws(packed, workspace)
    rc = lib().lpr_pricenet_features(
        B, _i32_arr(packed.ns), _i64_arr(packed.cost_offset), _ptr(packed.costs),
        int(bool(maximize)), _ptr(feats), _ptr(scales), _ptr(ws), ws.numel(),
        _stream(stream))
    _check(rc, "lpr_pricenet_features")
    return feats, scales


def lpr_pricenet_infer(packed: PackedAssign, params, maximize=False,
                       kappa=None, workspace=None, stream=None):
    """Network output q (float32 [sum n]), scaled start prices (int64
    [sum n]) and, when kappa is given, the per-instance starting epsilon
    (int64 [B]); otherwise the third value is None."""
    import torch
    dev = packed.costs.device
    R = int(packed.row_offset[-1])
    q = torch.empty(R, dtype=torch.float32, device=dev)
    prices = torch.empty(R, dtype=torch.int64, device=dev)
    eps = (torch.empty(len(packed.ns), dtype=torch.int64, device=dev)
           if kappa is not None else None)
    ws = _net_ws(packed, workspace)
    rc = lib().lpr_pricenet_infer(
        len(packed.ns), _i32_arr(packed.ns), _i64_arr(packed.cost_offset),
        _ptr(packed.costs), int(bool(maximize)), _ptr(params),
        float(kappa or 0.0), _ptr(q), _ptr(prices), _ptr(eps), _ptr(ws),
        ws.numel(), _stream(stream))
    _check(rc, "lpr_pricenet_infer")
    return q, prices, eps


def lpr_assign_learned_workspace(ns) -> int:
    return int(lib().lpr_assign_learned_workspace(len(ns), _i32_arr(ns)))


def lpr_assign_solve_learned(packed: PackedAssign, params, kappa, maximize=False,
                             opts: AssignOpts | None = None, want_prices=True,
                             workspace=None, stream=None):
    """Predicted start (params None: f14 alone) and the warm-started batched
    solve in one library call.  Returns (row_to_col packed int32, totals
    int64 tensor [B], col_prices packed or None, stats)."""
    import torch
    B = len(packed.ns)
    dev = packed.costs.device
    rows = int(packed.row_offset[-1])
    r2c = torch.empty(rows, dtype=torch.int32, device=dev)
    tots = torch.zeros(B, dtype=torch.int64, device=dev)
    prices = torch.empty(rows, dtype=torch.int64, device=dev) if want_prices else None
    ws = workspace if workspace is not None else _workspace(
        lpr_assign_learned_workspace(packed.ns), dev)
    st = AssignStats()
    rc = lib().lpr_assign_solve_learned(
        B, _i32_arr(packed.ns), _i64_arr(packed.cost_offset), _ptr(packed.costs),
        int(bool(maximize)), _ptr(params), float(kappa), _ptr(r2c), _ptr(tots),
        _ptr(prices), ctypes.byref(opts) if opts is not None else None,
        ctypes.byref(st), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "lpr_assign_solve_learned")
    return r2c, tots, prices, _struct_dict(st)


def lpr_pricenet_train_step(packed: PackedAssign, target_prices, params,
                            adam_m=None, adam_v=None, step=0, lr=1e-3,
                            maximize=False, want_grad=False, workspace=None,
                            stream=None):
    """One training step (step 0: loss and gradient only).  Returns
    (loss float, gradient tensor or None)."""
    import torch
    dev = packed.costs.device
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    grad = (torch.empty(lpr_pricenet_param_count(), dtype=torch.float32,
                        device=dev) if want_grad else None)
    ws = _net_ws(packed, workspace)
    rc = lib().lpr_pricenet_train_step(
        len(packed.ns), _i32_arr(packed.ns), _i64_arr(packed.cost_offset),
        _ptr(packed.costs), int(bool(maximize)), _ptr(target_prices),
        _ptr(params), _ptr(grad), _ptr(adam_m), _ptr(adam_v), int(step),
        float(lr), _ptr(loss), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "lpr_pricenet_train_step")
    return float(loss.item()), grad


def lpr_atomic_probe(counters, log2_counters, blocks, per_thread, stream=None):
    """Kernel time (ms) of blocks * 256 * per_thread non-returning atomic adds
    into the device int32 tensor `counters` (2^log2_counters entries)."""
    assert counters.numel() == (1 << log2_counters) and counters.dtype.itemsize == 4
    ms = ctypes.c_double(0)
    rc = lib().lpr_atomic_probe(_ptr(counters), int(log2_counters), int(blocks),
                                int(per_thread), ctypes.byref(ms), _stream(stream))
    _check(rc, "lpr_atomic_probe")
    return ms.value


def lpr_graph_maxflow_workspace(n: int, m: int) -> int:
    return int(lib().lpr_graph_maxflow_workspace(int(n), int(m)))


def make_graph_opts(cycle=0, max_rounds=0, sweeps_per_relabel=0) -> GraphOpts:
    o = GraphOpts()
    o.cycle = cycle
    o.max_rounds = max_rounds
    o.sweeps_per_relabel = sweeps_per_relabel
    return o


def lpr_graph_maxflow(n, tail, head, cap, s, t, want_cut=True,
                      opts: GraphOpts | None = None, workspace=None, stream=None,
                      device="cuda"):
    """Maximum s-t flow of the network whose arcs come in mate pairs (see
    lpr_graph_maxflow in include/lpr.h).  tail, head, cap: int32 arrays of m
    entries (torch CUDA tensors or host arrays).  Returns (flow_value (int),
    source_side (torch uint8 [n] on the device, or None), stats dict)."""
    import torch
    arrs = [_dev_i32(a, device) for a in (tail, head, cap)]
    m = arrs[0].numel()
    dev = arrs[0].device
    side = torch.empty(n, dtype=torch.uint8, device=dev) if want_cut else None
    need = lpr_graph_maxflow_workspace(n, m)
    ws = workspace if workspace is not None else _workspace(max(need, 1), dev)
    flow = ctypes.c_int64(0)
    st = GraphStats()
    rc = lib().lpr_graph_maxflow(
        int(n), int(m), *[_ptr(a) for a in arrs], int(s), int(t),
        ctypes.byref(flow), _ptr(side),
        ctypes.byref(opts) if opts is not None else None, ctypes.byref(st),
        _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "lpr_graph_maxflow")
    return int(flow.value), side, _struct_dict(st)


def make_mcf_opts(alpha=0, iters_per_check=0, max_iters=0) -> McfOpts:
    o = McfOpts()
    o.alpha, o.iters_per_check, o.max_iters = alpha, iters_per_check, max_iters
    return o


def lpr_mincost_flow_workspace(n: int, m: int) -> int:
    return int(lib().lpr_mincost_flow_workspace(n, m))


def lpr_mincost_flow(n, tail, head, cap, cost, supply, want_residual=True,
                     want_prices=True, opts: McfOpts | None = None,
                     workspace=None, stream=None, device="cuda"):
    """Minimum-cost flow meeting the supplies (lpr_mincost_flow).  Arrays are
    int32 (torch CUDA tensors or host arrays).  Returns (total cost (int),
    residual int32 tensor [m] or None, prices int64 tensor [n] or None,
    stats dict)."""
    import torch
    arrs = [_dev_i32(a, device) for a in (tail, head, cap, cost)]
    sup = _dev_i32(supply, device)
    m = arrs[0].numel()
    dev = sup.device
    res = torch.empty(max(m, 1), dtype=torch.int32, device=dev) if want_residual else None
    pr = torch.empty(n, dtype=torch.int64, device=dev) if want_prices else None
    ws = (workspace if workspace is not None
          else _workspace(lpr_mincost_flow_workspace(n, m), dev))
    tot = ctypes.c_int64(0)
    st = McfStats()
    rc = lib().lpr_mincost_flow(
        int(n), int(m), *[_ptr(a if m else None) for a in arrs], _ptr(sup),
        ctypes.byref(tot), _ptr(res if m else None), _ptr(pr),
        ctypes.byref(opts) if opts is not None else None, ctypes.byref(st),
        _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "lpr_mincost_flow")
    return int(tot.value), None if res is None else res[:m], pr, _struct_dict(st)
