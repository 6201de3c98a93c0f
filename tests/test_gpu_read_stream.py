"""cs_read_stream (the read-stream measurement aid): reads without writing."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n,blocks", [(4, 0), (4 * 1000 + 4, 3), (1 << 24, 0), (1 << 24, 16384)], ids=str)
def test_read_stream_leaves_the_sink_alone(n, blocks):
    from paper_1203_4587_amd.api import read_stream
    buf = torch.randn(n, dtype=torch.float32, device="cuda")
    sink = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    keep = buf.clone()
    read_stream(buf, sink, blocks=blocks)
    torch.cuda.synchronize()
    assert sink.item() == 7.0
    assert torch.equal(buf, keep)
