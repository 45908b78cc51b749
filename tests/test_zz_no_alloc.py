"""The allocation-free grid entry point (lpr_grid_maxflow_noalloc) against
lpr_grid_maxflow on the same inputs: the flow value and the minimal source
side are unique, so both must be equal exactly.  Two calls in a row share the
library's scratch array, the second on a smaller ragged grid, so stale
contents of the first call must not leak into the second."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1110_6231_amd import lpr  # noqa: E402


def _caps(inst):
    return [torch.as_tensor(np.ascontiguousarray(a, np.int32), device="cuda")
            for a in inst.arrays()]


def _noalloc(inst):
    caps = _caps(inst)
    flow = torch.zeros(1, dtype=torch.int64, device="cuda")
    side = torch.empty(inst.H * inst.W, dtype=torch.uint8, device="cuda")
    st = lpr.lpr_grid_maxflow_noalloc(inst.H, inst.W, caps, flow, side)
    return int(flow.item()), side.cpu().numpy(), st


def _reference(inst):
    v, side, st = lpr.lpr_grid_maxflow(inst.H, inst.W, *_caps(inst))
    return v, side.cpu().numpy(), st


def test_noalloc_matches_workspace_entry_point_twice():
    big = synth.grid_blobs(1024, 1024, seed=0)
    small = synth.grid_blobs(300, 77, seed=3)
    assert lpr.lpr_grid_maxflow_workspace(1024, 1024) <= \
        lpr.lpr_grid_maxflow_noalloc_max_bytes()
    for inst in (big, small):
        print(f"[noalloc] {inst.H}x{inst.W}", flush=True)
        v, side, st = _noalloc(inst)
        want_v, want_side, _ = _reference(inst)
        assert v == want_v, (inst.H, inst.W, v, want_v)
        np.testing.assert_array_equal(side, want_side)
        assert st["rounds"] >= 1


def test_noalloc_rejects_grids_beyond_its_scratch():
    H = W = 2048
    assert lpr.lpr_grid_maxflow_workspace(H, W) > \
        lpr.lpr_grid_maxflow_noalloc_max_bytes()
    caps = [torch.zeros(1, dtype=torch.int32, device="cuda").expand(H * W)
            .contiguous() for _ in range(6)]
    flow = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(lpr.LprError, match="ENOMEM"):
        lpr.lpr_grid_maxflow_noalloc(H, W, caps, flow, None)
