"""GPU tests of the calibration probes (include/tt_probe.h): what each
streaming probe reads and writes, and the argument refusals."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def test_stream_probes_move_what_they_claim():
    import torch
    from paper_2601_08217_amd import binding as B
    n = (1 << 20) + 16 * 37  # not a multiple of the grid's stride
    g = np.random.default_rng(1)
    src_h = g.integers(-2**31, 2**31 - 1, size=n // 4, dtype=np.int64).astype(np.int32)
    src = torch.from_numpy(src_h).to("cuda:0")
    dst = torch.zeros(n // 4, dtype=torch.int32, device="cuda:0")
    for nt in (False, True):
        dst.zero_()
        B.probe_stream("copy", dst.data_ptr(), src.data_ptr(), n, 96, nt)
        torch.cuda.synchronize()
        assert np.array_equal(dst.cpu().numpy(), src_h)
        dst.zero_()
        B.probe_stream("write", dst.data_ptr(), 0, n, 96, nt)
        torch.cuda.synchronize()
        assert np.array_equal(dst.cpu().numpy(), np.tile(np.array([7, 8, 9, 10], np.int32), n // 16))
    blocks = 80
    sink = torch.zeros(blocks * 4, dtype=torch.int32, device="cuda:0")
    B.probe_stream("read", sink.data_ptr(), src.data_ptr(), n, blocks, False)
    torch.cuda.synchronize()
    # each workgroup writes the XOR of every word it read; together they read everything once
    per_block = sink.cpu().numpy().reshape(blocks, 4)[:, 0]
    assert np.bitwise_xor.reduce(per_block) == np.bitwise_xor.reduce(src_h)


def test_chunked_write_probe_covers_whole_streams_only():
    import torch
    from paper_2601_08217_amd import binding as B
    chunks, streams = 37, 5  # 7 chunks per stream; the last 2 chunks stay untouched
    n = chunks * 8192
    dst = torch.zeros(n // 4, dtype=torch.int32, device="cuda:0")
    B.probe_chunked_write(dst.data_ptr(), n, streams, 13, False)
    torch.cuda.synchronize()
    d = dst.cpu().numpy().reshape(chunks, 2048)
    covered = (chunks // streams) * streams
    assert np.array_equal(d[:covered], np.tile(np.array([1, 2, 3, 4], np.int32), (covered, 512)))
    assert not d[covered:].any()


def test_probe_refusals():
    import torch
    from paper_2601_08217_amd import binding as B
    buf = torch.zeros(4096, dtype=torch.int32, device="cuda:0")
    with pytest.raises(B.TTError):
        B.probe_stream("copy", buf.data_ptr(), buf.data_ptr(), 100, 4)        # not a multiple of 16
    with pytest.raises(B.TTError):
        B.probe_stream("write", buf.data_ptr(), 0, 4096, 0)                   # no workgroups
    with pytest.raises(B.TTError):
        B.probe_stream("read", buf.data_ptr(), 0, 4096, 4)                    # read without a source
    with pytest.raises(B.TTError):
        B.probe_chunked_write(buf.data_ptr(), 12288, 1, 4)                    # not whole 8 KiB chunks
    with pytest.raises(B.TTError):
        B.probe_chunked_write(buf.data_ptr(), 8192, 2, 4)                     # more streams than chunks
