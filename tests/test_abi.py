"""C-ABI contract checks that need no GPU: the library builds and loads,
exports every function include/lpr.h declares, and its host-side sizing
functions and constants agree with the header."""
import os
import re

import pytest

from paper_1110_6231_amd import lpr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lpr_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_expected_api():
    assert declared_functions() == sorted(lpr.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = lpr.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_version_and_empty_error():
    assert lpr.version().startswith("lpr ")
    assert isinstance(lpr.last_error(), str)


def test_constants_match_header():
    text = open(HEADER).read()
    assert "#define LPR_GRID_MAX_CAP ((1 << 26) - 1)" in text
    assert lpr.LPR_GRID_MAX_CAP == (1 << 26) - 1
    assert "#define LPR_ASSIGN_MAX_COST ((1 << 24) - 1)" in text
    assert lpr.LPR_ASSIGN_MAX_COST == (1 << 24) - 1
    assert "#define LPR_ASSIGN_MAX_N 2048" in text


def test_workspace_sizes():
    w = lpr.lpr_grid_maxflow_workspace(1024, 1024)
    # at least the seven int32 state arrays
    assert w >= 7 * 4 * 1024 * 1024
    assert lpr.lpr_grid_maxflow_workspace(0, 5) == 0
    assert lpr.lpr_grid_maxflow_workspace(1, 1) > 0
    wb = lpr.lpr_grid_maxflow_batched_workspace([1024], [1024])
    assert wb == w
    w2 = lpr.lpr_grid_maxflow_batched_workspace([100, 37], [64, 129])
    assert w2 >= 7 * 4 * (100 * 64 + 37 * 129)
    assert lpr.lpr_assign_workspace(0) == 0
    assert lpr.lpr_assign_workspace(512) > 0
    assert lpr.lpr_assign_batched_workspace([64, 128, 512]) > 0


STRUCTS = {
    "lpr_grid_opts": "GridOpts", "lpr_grid_stats": "GridStats",
    "lpr_assign_opts": "AssignOpts", "lpr_assign_stats": "AssignStats",
    "lpr_graph_opts": "GraphOpts", "lpr_graph_stats": "GraphStats",
    "lpr_mcf_opts": "McfOpts", "lpr_mcf_stats": "McfStats",
}


def test_struct_layouts(tmp_path):
    """Every field offset and struct size of the ctypes mirrors in the
    binding equals what the C compiler makes of include/lpr.h."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lpr.h"',
             "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(lpr, pyname)
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", f"-I{os.path.join(ROOT, 'include')}",
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True,
                         text=True).stdout.split()
    got = {(out[i], out[i + 1]): int(out[i + 2]) for i in range(0, len(out), 3)}
    for cname, pyname in STRUCTS.items():
        cls = getattr(lpr, pyname)
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)


def test_atomic_probe_rejects_bad_arguments():
    """Argument checks run on the host before anything reaches the device."""
    import ctypes
    L = lpr.lib()
    ms = ctypes.c_double(0)
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below is rejected
    for args in ((None, 10, 1, 1), (fake, 5, 1, 1), (fake, 29, 1, 1),
                 (fake, 10, 0, 1), (fake, 10, 1, 0), (fake, 10, 1, 4097)):
        assert L.lpr_atomic_probe(*args, ctypes.byref(ms), None) == lpr.LPR_EINVAL


def test_sparse_assignment_host_checks():
    """Sizes and argument checks of the sparse assignment entry point, all
    decided on the host before anything reaches the device."""
    import ctypes
    assert lpr.lpr_assign_sparse_workspace(0, 5) == 0
    assert lpr.lpr_assign_sparse_workspace(lpr.LPR_ASSIGN_MAX_N + 1, 5) == 0
    assert lpr.lpr_assign_sparse_workspace(8, -1) == 0
    assert lpr.lpr_assign_sparse_workspace(8, lpr.LPR_ASSIGN_SPARSE_MAX_ARCS + 1) == 0
    w = lpr.lpr_assign_sparse_workspace(1024, 32 * 1024)
    # the dense copy and the assignment workspace at least
    assert w >= 4 * 1024 * 1024 + lpr.lpr_assign_workspace(1024)
    assert "#define LPR_ASSIGN_SPARSE_MAX_ARCS (1 << 26)" in open(HEADER).read()
    assert "LPR_ENOMATCH = -6" in open(HEADER).read()
    L = lpr.lib()
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below is rejected
    f = L.lpr_assign_sparse_solve
    common = (0, fake, fake, None, None, None, fake)
    assert f(0, 4, fake, fake, fake, *common, 1 << 30, None) == lpr.LPR_EINVAL
    assert f(4, -1, fake, fake, fake, *common, 1 << 30, None) == lpr.LPR_EINVAL
    assert f(4, 4, None, fake, fake, *common, 1 << 30, None) == lpr.LPR_EINVAL
    assert f(4, 4, fake, None, fake, *common, 1 << 30, None) == lpr.LPR_EINVAL
    assert f(4, 4, fake, fake, fake, 0, None, fake, None, None, None, fake,
             1 << 30, None) == lpr.LPR_EINVAL  # row_to_col NULL
    assert f(4, 4, fake, fake, fake, *common, 16, None) == lpr.LPR_ENOMEM


def test_assign_tune_host_checks():
    """The assignment tuner rejects, on the host and before anything reaches
    the device, a repetition count outside 1..100, missing sizes or totals,
    and base options that already fix a schedule field; the option checks of
    every solve reject a quarter count outside 0..64 and a nonzero reserved
    field."""
    import ctypes
    L = lpr.lib()
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below is rejected
    n = (ctypes.c_int32 * 1)(4)
    off = (ctypes.c_int64 * 2)(0, 16)
    ms = ctypes.c_double(0)

    def tune(base, reps, nn=n, totals=fake):
        return L.lpr_assign_tune(1, nn, off, fake, 0, fake, totals, base, reps, None,
                                 ctypes.byref(ms), fake, 1 << 30, None)

    assert tune(None, 0) == lpr.LPR_EINVAL
    assert tune(None, 101) == lpr.LPR_EINVAL
    assert tune(None, 1, nn=None) == lpr.LPR_EINVAL
    assert tune(None, 1, totals=None) == lpr.LPR_EINVAL
    for field, value in (("alpha", 4), ("price_update_period", 100),
                         ("price_update_quarters", 2), ("tail_rows", 8)):
        o = lpr.make_assign_opts()
        setattr(o, field, value)
        assert tune(ctypes.byref(o), 1) == lpr.LPR_EINVAL, field
    for field, value in (("price_update_quarters", 65), ("price_update_quarters", -1),
                         ("reserved", 1)):
        o = lpr.make_assign_opts()
        setattr(o, field, value)
        rc = L.lpr_assign_solve(4, fake, 0, fake, fake, None, ctypes.byref(o), None,
                                fake, 1 << 30, None)
        assert rc == lpr.LPR_EINVAL, field


def test_mincost_flow_host_checks():
    """Sizes and argument checks of the min-cost flow entry point, decided on
    the host before anything reaches the device."""
    import ctypes
    assert lpr.lpr_mincost_flow_workspace(0, 4) == 0
    assert lpr.lpr_mincost_flow_workspace(4, 3) == 0
    assert lpr.lpr_mincost_flow_workspace(lpr.LPR_MCF_MAX_N + 1, 4) == 0
    assert lpr.lpr_mincost_flow_workspace(100, 400) >= lpr.lpr_graph_maxflow_workspace(100, 400)
    text = open(HEADER).read()
    assert "#define LPR_MCF_MAX_N (1 << 20)" in text
    assert "#define LPR_MCF_MAX_COST ((1 << 16) - 1)" in text
    assert "LPR_EINFEASIBLE = -7" in text
    assert ctypes.sizeof(lpr.McfOpts) == 16
    assert ctypes.sizeof(lpr.McfStats) == 5 * 8
    L = lpr.lib()
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below is rejected
    tot = ctypes.c_int64(0)
    f = L.lpr_mincost_flow
    arcs = (fake, fake, fake, fake, fake)
    assert f(0, 2, *arcs, ctypes.byref(tot), None, None, None, None, fake, 1 << 30,
             None) == lpr.LPR_EINVAL
    assert f(4, 3, *arcs, ctypes.byref(tot), None, None, None, None, fake, 1 << 30,
             None) == lpr.LPR_EINVAL
    assert f(4, 2, fake, fake, fake, fake, None, ctypes.byref(tot), None, None, None,
             None, fake, 1 << 30, None) == lpr.LPR_EINVAL  # supply NULL
    bad = lpr.make_mcf_opts(alpha=1)
    assert f(4, 2, *arcs, ctypes.byref(tot), None, None, ctypes.byref(bad), None, fake,
             1 << 30, None) == lpr.LPR_EINVAL
    assert f(4, 2, *arcs, ctypes.byref(tot), None, None, None, None, fake, 16,
             None) == lpr.LPR_ENOMEM


def test_learned_solve_host_checks():
    """The one-call learned solve sizes its workspace as the prediction's,
    the start prices and epsilons and the solve's together, and rejects on
    the host, before anything reaches the device, kappa <= 0, start fields
    set in the options, missing sizes and a small workspace."""
    import ctypes
    L = lpr.lib()
    n = (ctypes.c_int32 * 2)(40, 300)
    off = (ctypes.c_int64 * 3)(0, 1600, 1600 + 90000)
    need = L.lpr_assign_learned_workspace(2, n)
    parts = (L.lpr_pricenet_workspace(2, n) + L.lpr_assign_batched_workspace(2, n) +
             8 * (340 + 2))
    assert parts <= need <= parts + 5 * 256
    assert L.lpr_assign_learned_workspace(0, n) == 0
    assert L.lpr_assign_learned_workspace(1, (ctypes.c_int32 * 1)(0)) == 0
    assert L.lpr_assign_learned_workspace(1, (ctypes.c_int32 * 1)(lpr.LPR_ASSIGN_MAX_N + 1)) == 0
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below is rejected

    def solve(kappa, opts=None, nn=n, ws_bytes=1 << 40):
        return L.lpr_assign_solve_learned(2, nn, off, fake, 0, None, kappa, fake, fake,
                                          None, opts, None, fake, ws_bytes, None)

    assert solve(0.0) == lpr.LPR_EINVAL
    assert solve(-1.0) == lpr.LPR_EINVAL
    assert solve(0.01, nn=None) == lpr.LPR_EINVAL
    for field in ("eps0", "init_col_prices", "eps0_per_instance"):
        o = lpr.make_assign_opts()
        setattr(o, field, 8)
        assert solve(0.01, opts=ctypes.byref(o)) == lpr.LPR_EINVAL, field
    assert solve(0.01, ws_bytes=need - 1) == lpr.LPR_ENOMEM


def test_host_array_marshalling():
    """Host size and offset arrays reach the C-ABI as contiguous int32 /
    int64 buffers with the caller's values; a value outside the type's range
    is an error, not a silent wrap."""
    import ctypes
    import numpy as np
    vals = [5, 0, -3, 2 ** 31 - 1]
    p = lpr._i32_arr(vals)
    assert [p[i] for i in range(4)] == vals
    q = lpr._i64_arr(np.array([0, 2 ** 40, -7], dtype=np.int64))
    assert [q[i] for i in range(3)] == [0, 2 ** 40, -7]
    assert isinstance(p, ctypes.POINTER(ctypes.c_int32))
    with pytest.raises(OverflowError):
        lpr._i32_arr([2 ** 31])
    # the sizes a batched call passes: the workspace size of an instance list
    ns = [3, 7, 11]
    assert lpr.lpr_assign_batched_workspace(ns) == lpr.lib().lpr_assign_batched_workspace(
        3, (ctypes.c_int32 * 3)(*ns))
