"""The read-only streaming reference used by the benchmark (tk_stream_read):
every float4 of the buffer is read exactly once (whole 4 KB blocks and the
tail), checked through its checksums on integer-valued data."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("numel", [4 * 1024 * 1024 + 1000, 1024, 12])
def test_stream_read_reads_every_element_once(numel):
    from paper_2603_21379_amd import binding as B
    x = (torch.arange(numel, device="cuda", dtype=torch.int64) % 7).to(torch.float32)
    parts = torch.zeros(B.stream_read_blocks(), dtype=torch.float64, device="cuda")
    B.stream_read(x, parts)
    torch.cuda.synchronize()
    n4 = numel // 4 * 4   # a tail of fewer than four floats is not read
    assert float(parts.sum()) == float(x[:n4].double().sum())


def test_stream_read_rejects_small_partials():
    from paper_2603_21379_amd import binding as B
    x = torch.ones(1024, device="cuda")
    parts = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(B.TkError):
        B.stream_read(x, parts)
