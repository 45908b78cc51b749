"""The atomic-throughput probe used by the benchmark: every add lands."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1110_6231_amd import lpr  # noqa: E402


@pytest.mark.parametrize("log2,blocks,per", [(6, 1, 1), (10, 4, 8), (20, 64, 33)])
def test_probe_counts_every_add(log2, blocks, per):
    print(f"[probe] log2={log2} blocks={blocks} per={per}", flush=True)
    cnt = torch.zeros(1 << log2, dtype=torch.int32, device="cuda")
    ms = lpr.lpr_atomic_probe(cnt, log2, blocks, per)
    assert ms >= 0
    assert int(cnt.sum().item()) == blocks * 256 * per
    assert int(cnt.min().item()) >= 0
